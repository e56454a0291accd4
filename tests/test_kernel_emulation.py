"""The encoded energy program, executed by a host emulation of the kernels'
algorithm, reproduces the oracle: energies exactly (integer couplings) or
to float64 rounding, and the walked-back configuration attains E*."""
import numpy as np
import pytest

import kernel_emulator as K
from oracle import spinglass as O
from paper_2008_06888_amd import binding as B
from paper_2008_06888_amd import instances as I


def _run(plan, n, e, J, h=None):
    prog = K.load_program(plan)
    info = plan.info()
    ops, fs = plan.ops()
    Jf = J.astype(np.float64)
    hf = None if h is None else h.astype(np.float64)
    states = K.forward(prog, info["width"], Jf, hf if hf is not None else np.zeros(n))
    mx, sigma = K.backward(prog, states, len(fs), fs, n, Jf, hf if hf is not None else np.zeros(n))
    return -mx, sigma


@pytest.mark.parametrize("L,tb", [(3, 7), (5, 7), (6, 7), (9, 7), (10, 8)])
def test_lattice_with_fields(L, tb):
    rng = np.random.default_rng([41, L])
    e = I.square_lattice(L)
    x = I.make(e, L * L, rng, "gauss", field_std=0.3)
    plan = B.Plan(L * L, e, order=list(range(L * L)), has_field=True, tile_bits=tb)
    E, sig = _run(plan, L * L, e, x.J, x.h)
    ref = O.eliminate(L * L, e, x.J, x.h)
    assert abs(E - ref["energy"]) < 1e-9
    assert np.array_equal(sig, ref["sigma"])


@pytest.mark.parametrize("n,seed", [(12, 0), (16, 1), (20, 2), (24, 3), (30, 4)])
def test_regular3_greedy(n, seed):
    rng = np.random.default_rng([42, seed])
    e = I.random_regular(n, 3, rng)
    J = I.pm1(len(e), rng)
    plan = B.Plan(n, e, seed=seed, trials=4, tile_bits=7)
    E, sig = _run(plan, n, e, J)
    ref = O.eliminate(n, e, J, None)
    assert E == ref["energy"]
    assert O.energy(n, e, J, None, sig) == ref["energy"]


@pytest.mark.parametrize("fam", ["chimera12", "tree", "K6", "ring"])
def test_families(fam):
    rng = np.random.default_rng(len(fam) + 50)
    if fam == "chimera12":
        e, n = I.chimera(1, 2), 16
    elif fam == "tree":
        e, n = I.random_tree(14, rng), 14
    elif fam == "K6":
        e, n = I.complete(6), 6
    else:
        e, n = I.ring(11), 11
    J = I.pm1(len(e), rng) * rng.integers(1, 4, len(e)).astype(np.int32)
    plan = B.Plan(n, e, seed=3, trials=4, tile_bits=7)
    E, sig = _run(plan, n, e, J)
    ref = O.eliminate(n, e, J, None)
    assert E == ref["energy"]
    assert O.energy(n, e, J, None, sig) == ref["energy"]


@pytest.mark.parametrize("case", ["isolated", "no_edges", "two_components"])
def test_degenerate_graphs(case):
    rng = np.random.default_rng(7)
    if case == "isolated":
        n, e = 5, np.array([[0, 1], [1, 2]], np.int32)
    elif case == "no_edges":
        n, e = 4, np.zeros((0, 2), np.int32)
    else:
        n, e = 10, np.concatenate([I.ring(5), I.path(5) + 5]).astype(np.int32)
    J = I.pm1(len(e), rng) if len(e) else np.zeros(0, np.int32)
    for order in (None, list(range(n))):
        plan = B.Plan(n, e, order=order, seed=1, trials=2, tile_bits=7)
        E, sig = _run(plan, n, e, J)
        ref = O.eliminate(n, e, J, None)
        assert E == ref["energy"]
        assert O.energy(n, e, J, None, sig) == ref["energy"]

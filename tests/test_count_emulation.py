"""CPU checks of the counting path's encoded program (tt_plan_program parts
10 and 11): the host emulation of the count pass kernel gives the oracle's
E* and exact degeneracy on lattices, random graphs with fields and chimera-free
sweep plans, at several tile sizes."""
import numpy as np
import pytest

import count_emulator as CE
from oracle import spinglass as O
from paper_2008_06888_amd import binding as B
from paper_2008_06888_amd import instances as I


def _cases():
    out = []
    for L, b in ((4, 0), (5, 1), (6, 2)):
        x = I.config_instances(0, batch=b + 1, L=L)[b]
        out.append((x, list(range(L * L))))
    rng = np.random.default_rng([61, 0])
    for n in (10, 14):
        e = I.random_regular(n, 3, rng)
        J = I.pm1(len(e), rng)
        h = rng.integers(-2, 3, n).astype(np.int32)
        out.append((I.Instance(n=n, edges=e, J=J, h=h), None))
    e = I.square_lattice(4)
    out.append((I.Instance(n=16, edges=e, J=np.zeros(len(e), np.int32), h=None), list(range(16))))
    return out


@pytest.mark.parametrize("case", range(6))
@pytest.mark.parametrize("ctile", [7, 9])
def test_encoded_count_program_matches_oracle(case, ctile):
    x, order = _cases()[case]
    plan = B.Plan(x.n, x.edges, order=order, seed=3, has_field=x.h is not None, count_tile_bits=ctile)
    passes, ops = CE.load(plan)
    assert len(passes) == plan.info()["n_count_passes"]
    _, fs = plan.ops()
    best, g = CE.run(passes, ops, x.J, x.h, plan.info()["width"], fs)
    ref = O.eliminate(x.n, x.edges, x.J, x.h, counts="exact", traceback=False)
    assert -best == ref["energy"] and g == ref["count"]


@pytest.mark.parametrize("L,kind", [(8, "pm1"), (9, "pm1"), (10, "pm1"), (9, "zero")])
def test_half_state_count_program(L, kind):
    """Half-state plans (no fields, tiles of 2^7): the same E* and degeneracy
    from half of every state, with every stored entry of every pass written
    (each tile writes its mirror outputs)."""
    n, e = L * L, I.square_lattice(L)
    J = I.pm1(len(e), np.random.default_rng([5, L])) if kind == "pm1" else np.zeros(len(e), np.int32)
    plan = B.Plan(n, e, order=list(range(n)), count_tile_bits=7, z2=True)
    passes, ops = CE.load(plan)
    assert any(P.z2_skip >= 0 for P in passes)
    _, fs = plan.ops()
    best, g = CE.run(passes, ops, J, None, plan.info()["width"], fs, z2=True)
    ref = O.eliminate(n, e, J, None, counts="exact", traceback=False)
    assert -best == ref["energy"] and g == ref["count"]
    if kind == "zero":
        assert g == 2 ** n


@pytest.mark.parametrize("n,seed", [(36, 0), (44, 1)])
def test_half_state_count_random_graphs(n, seed):
    rng = np.random.default_rng([62, seed])
    e = I.random_regular(n, 3, rng)
    J = I.pm1(len(e), rng)
    plan = B.Plan(n, e, seed=seed, count_tile_bits=7, z2=True)
    passes, ops = CE.load(plan)
    _, fs = plan.ops()
    best, g = CE.run(passes, ops, J, None, plan.info()["width"], fs, z2=True)
    ref = O.eliminate(n, e, J, None, counts="exact", traceback=False)
    assert -best == ref["energy"] and g == ref["count"]

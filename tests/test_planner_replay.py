"""The planner's operation list, replayed on the host, reproduces the oracle's
E* and degeneracy on small graphs, for given and greedy spin orders."""
import numpy as np
import pytest

import plan_replay as R
from oracle import spinglass as O
from paper_2008_06888_amd import binding as B
from paper_2008_06888_amd import instances as I


def _check(n, e, J, order=None, seed=0, h=None):
    p = B.Plan(n, e, order=order, seed=seed, trials=4, has_field=h is not None)
    ops, fs = p.ops()
    E, g = R.replay(ops, fs, n, J.astype(np.int64), None if h is None else h.astype(np.int64))
    ref = O.eliminate(n, e, J, h, counts="exact")
    assert E == ref["energy"] and g == ref["count"]
    # every edge absorbed exactly once, every spin introduced once
    used = sorted(int(r[3]) for r in ops if r[0] in (R.GATE, R.DIAG))
    assert used == list(range(len(e)))
    entered = sorted(int(r[5]) for r in ops if r[0] in (R.GATE, R.INTRO))
    assert entered == list(range(n))
    return p


@pytest.mark.parametrize("L", [2, 3, 4, 5])
def test_square_raster(L):
    rng = np.random.default_rng(L)
    e = I.square_lattice(L)
    _check(L * L, e, I.pm1(len(e), rng), order=list(range(L * L)))


@pytest.mark.parametrize("seed", range(4))
def test_greedy_regular3(seed):
    rng = np.random.default_rng([21, seed])
    n = 14
    e = I.random_regular(n, 3, rng)
    _check(n, e, I.pm1(len(e), rng), seed=seed)


@pytest.mark.parametrize("fam", ["chimera12", "K5", "tree", "ring", "path"])
def test_greedy_families(fam):
    rng = np.random.default_rng(len(fam))
    if fam == "chimera12":
        e, n = I.chimera(1, 2), 16
    elif fam == "K5":
        e, n = I.complete(5), 5
    elif fam == "tree":
        e, n = I.random_tree(12, rng), 12
    elif fam == "ring":
        e, n = I.ring(9), 9
    else:
        e, n = I.path(6), 6
    _check(n, e, I.pm1(len(e), rng) * rng.integers(1, 3, len(e)).astype(np.int32))


def test_fields_and_disconnected_graph():
    rng = np.random.default_rng(9)
    e = np.concatenate([I.square_lattice(2, 3), I.ring(4) + 6]).astype(np.int32)
    n = 10
    J = I.pm1(len(e), rng)
    h = rng.integers(-2, 3, n).astype(np.int32)
    _check(n, e, J, h=h)
    _check(n, e, J, h=h, order=list(rng.permutation(n)))


def test_isolated_spin():
    e = np.array([[0, 1]], np.int32)
    _check(3, e, np.array([1], np.int32))

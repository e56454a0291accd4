"""Pins of the 3-state Potts oracle (Appendix C Hamiltonian, doubled energies).

Closed forms fix brute force (the plain definition) independently of the
elimination; the elimination is then checked against brute force on small
graphs, under several orders, and against invariants of the model.
"""
import itertools

import numpy as np
import pytest

from oracle import potts as P
from paper_2008_06888_amd import instances as I


def test_energy2_hand_example():
    # triangle, J = (+1 on (0,1), -1 on (0,2), +1 on (1,2)), labels (0, 0, 1):
    # (0,1) equal: 2*1; (0,2) unequal: -(-1) = 1; (1,2) unequal: -1  ->  2H = 2
    edges = np.array([[0, 1], [0, 2], [1, 2]], np.int32)
    J = np.array([1, -1, 1], np.int32)
    assert P.energy2(3, edges, J, [0, 0, 1]) == 2
    assert P.energy2(3, edges, J, [2, 2, 2]) == 2 * (1 - 1 + 1)
    assert P.energy2(3, edges, J.astype(np.float64) * 0.25, [0, 1, 2]) == pytest.approx(-0.25)


def test_energy2_matches_the_matrix_form():
    # 2H = sum_e J_e * 2 M[s_i][s_j] with M = [[1,-1/2,-1/2],[-1/2,1,-1/2],[-1/2,-1/2,1]]
    M = np.array([[1, -.5, -.5], [-.5, 1, -.5], [-.5, -.5, 1]])
    rng = np.random.default_rng(3)
    e = I.square_lattice(3)
    J = rng.normal(size=len(e))
    for _ in range(20):
        s = rng.integers(0, 3, 9)
        ref = sum(2 * J[k] * M[s[a], s[b]] for k, (a, b) in enumerate(e))
        assert P.energy2(9, e, J, s) == pytest.approx(ref, abs=1e-12)


@pytest.mark.parametrize("n", [2, 4, 7])
def test_ferromagnet(n):
    # J = -1 on every edge of a connected graph: all labels equal, 2H* = -2m, g = 3
    for e in (I.path(n), I.ring(n) if n >= 3 else I.path(n), I.complete(n)):
        J = -np.ones(len(e), np.int32)
        r = P.brute_force(n, e, J)
        assert r["energy2"] == -2 * len(e) and r["count"] == 3


@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_antiferro_path_proper_colourings(n):
    # J = +1: a proper 3-colouring of a path gives every bond -1; there are 3 * 2^(n-1)
    e = I.path(n)
    r = P.brute_force(n, e, np.ones(len(e), np.int32))
    assert r["energy2"] == -(n - 1) and r["count"] == 3 * 2 ** (n - 1)


@pytest.mark.parametrize("n", [3, 4, 5, 6, 9])
def test_antiferro_cycle_chromatic_polynomial(n):
    # proper 3-colourings of C_n: 2^n + 2 (-1)^n (chromatic polynomial at 3), all bonds -1
    e = I.ring(n)
    r = P.brute_force(n, e, np.ones(n, np.int32))
    assert r["energy2"] == -n and r["count"] == 2 ** n + 2 * (-1) ** n


def test_antiferro_k4():
    # K_4 is not 3-colourable: best is one monochromatic pair (6 pairs x 3 x 2 labelings),
    # 2H* = 2 - 5 = -3, g = 36
    e = I.complete(4)
    r = P.brute_force(4, e, np.ones(6, np.int32))
    assert r["energy2"] == -3 and r["count"] == 36


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tree_closed_form(seed):
    # on a tree every bond is satisfied independently: -2 for J = -1 (equal), -1 for J = +1
    # (two unequal choices) -> 2H* = sum(-2 | -1), g = 3 * 2^(#antiferro bonds)
    rng = np.random.default_rng([7, seed])
    n = 9
    e = I.random_tree(n, rng)
    J = (2 * rng.integers(0, 2, len(e)) - 1).astype(np.int32)
    r = P.brute_force(n, e, J)
    assert r["energy2"] == int(np.sum(np.where(J < 0, -2, -1)))
    assert r["count"] == 3 * 2 ** int(np.sum(J > 0))
    o = P.eliminate(n, e, J, counts="exact")
    assert o["energy2"] == r["energy2"] and o["count"] == r["count"]


def _small_cases():
    rng = np.random.default_rng(11)
    cases = []
    for L, Lc in ((2, 3), (3, 3), (3, 4)):
        e = I.square_lattice(L, Lc)
        cases.append((L * Lc, e, (2 * rng.integers(0, 2, len(e)) - 1).astype(np.int32)))
        cases.append((L * Lc, e, rng.normal(size=len(e))))
    for n in (6, 8, 10):
        e = I.random_regular(n, 3, rng)
        cases.append((n, e, (2 * rng.integers(0, 2, len(e)) - 1).astype(np.int32)))
        cases.append((n, e, rng.integers(-3, 4, len(e)).astype(np.int32)))
    return cases


@pytest.mark.parametrize("case", range(12))
def test_elimination_equals_brute_force(case):
    n, e, J = _small_cases()[case]
    bf = P.brute_force(n, e, J)
    integer = np.issubdtype(np.asarray(J).dtype, np.integer)
    orders = [None, list(range(n)), list(range(n))[::-1]]
    for order in orders:
        o = P.eliminate(n, e, J, order=order, counts="exact" if integer else None)
        if integer:
            assert o["energy2"] == bf["energy2"] and o["count"] == bf["count"]
            m = P.eliminate(n, e, J, order=order, counts="mod")
            assert m["count"] == bf["count"]
            assert P.energy2(n, e, J, o["labels"]) == bf["energy2"]
        else:
            assert o["energy2"] == pytest.approx(bf["energy2"], abs=1e-9)
            # label permutations map ground states to ground states (orbits of 3 or 6)
            assert bf["count"] % 3 == 0
            assert P.energy2(n, e, J, o["labels"]) == pytest.approx(bf["energy2"], abs=1e-9)


@pytest.mark.parametrize("seed", range(4))
def test_label_permutation_symmetry(seed):
    # H depends only on whether neighbouring labels agree: permuting the three labels maps
    # ground states to ground states, no configuration is fixed by every permutation, so g % 3 == 0
    rng = np.random.default_rng([9, seed])
    e = I.square_lattice(3, 4)
    J = (2 * rng.integers(0, 2, len(e)) - 1).astype(np.int32)
    o = P.eliminate(12, e, J, counts="exact")
    assert o["count"] % 3 == 0
    for perm in itertools.permutations(range(3)):
        s = np.array(perm)[o["labels"]]
        assert P.energy2(12, e, J, s) == o["energy2"]


def test_disjoint_union():
    rng = np.random.default_rng(5)
    e1, e2 = I.square_lattice(3), I.ring(5)
    J1 = (2 * rng.integers(0, 2, len(e1)) - 1).astype(np.int32)
    J2 = (2 * rng.integers(0, 2, len(e2)) - 1).astype(np.int32)
    a = P.eliminate(9, e1, J1, counts="exact")
    b = P.eliminate(5, e2, J2, counts="exact")
    e = np.concatenate([e1, e2 + 9]).astype(np.int32)
    u = P.eliminate(14, e, np.concatenate([J1, J2]), counts="exact")
    assert u["energy2"] == a["energy2"] + b["energy2"]
    assert u["count"] == a["count"] * b["count"]


def test_order_independence_on_a_lattice():
    rng = np.random.default_rng(6)
    e = I.square_lattice(6)
    J = (2 * rng.integers(0, 2, len(e)) - 1).astype(np.int32)
    ref = P.eliminate(36, e, J, order=list(range(36)), counts="exact")
    for order in (None, list(range(36))[::-1], list(rng.permutation(36))):
        o = P.eliminate(36, e, J, order=order, counts="mod")
        assert o["energy2"] == ref["energy2"] and o["count"] == ref["count"]

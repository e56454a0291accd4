"""Pins of the CPU oracle against facts other than itself.

Brute force is pinned by closed forms (rings, plaquettes, trees, ferromagnets,
J = 0); elimination is pinned by brute force on <= 20 spins, by closed forms at
full size (planted instances, trees, rings) and by invariants (gauge, Z2,
order independence, disjoint union). Gradients are pinned by finite
differences of the oracle energy.
"""
import math

import numpy as np
import pytest

from oracle import spinglass as O
from paper_2008_06888_amd import instances as I


def _trial_prime(p):
    if p < 2:
        return False
    for d in range(2, int(math.isqrt(p)) + 1):
        if p % d == 0:
            return False
    return True


def test_oracle_primes_are_prime_and_distinct():
    assert len(set(O.ORACLE_PRIMES)) == len(O.ORACLE_PRIMES)
    for p in O.ORACLE_PRIMES:
        assert p < 2 ** 31 and _trial_prime(p)


def test_energy_hand_example():
    # 3 spins, edges (0,1) J=2, (1,2) J=-1, fields h = (1, 0, -3)
    edges = np.array([[0, 1], [1, 2]], np.int32)
    J = np.array([2, -1], np.int32)
    h = np.array([1, 0, -3], np.int32)
    # sigma = (+1, -1, -1): -(2*(+1)(-1) + (-1)(-1)(-1)) - (1*1 + 0 + (-3)(-1)) = -(-2 - 1) - (1 + 3) = -1
    assert O.energy(3, edges, J, h, np.array([1, -1, -1])) == -1
    # sigma = (+1, +1, -1): -(2 + 1) - (1 + 3) = -7
    assert O.energy(3, edges, J, h, np.array([1, 1, -1])) == -7


@pytest.mark.parametrize("n", [3, 4, 5, 7, 10])
def test_brute_force_frustrated_ring(n):
    # ring with exactly one antiferro... i.e. one negative bond: frustrated.
    e = I.ring(n)
    J = np.ones(n, np.int32)
    J[0] = -1
    r = O.brute_force(n, e, J, None)
    assert r["energy"] == -(n - 2)
    assert r["count"] == 2 * n


def test_brute_force_plaquette():
    e = I.ring(4)
    J = np.array([1, 1, 1, -1], np.int32)
    r = O.brute_force(4, e, J, None)
    assert r["energy"] == -2 and r["count"] == 8


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_tree_closed_form(seed):
    rng = np.random.default_rng([99, seed])
    n = 12
    e = I.random_tree(n, rng)
    J = I.pm1(len(e), rng) * rng.integers(1, 4, len(e)).astype(np.int32)
    r = O.brute_force(n, e, J, None)
    assert r["energy"] == -int(np.abs(J).sum())
    assert r["count"] == 2


def test_brute_force_ferromagnet_field():
    e = I.square_lattice(3)
    J = np.ones(len(e), np.int32)
    h = np.full(9, 2, np.int32)
    r = O.brute_force(9, e, J, h)
    assert r["energy"] == -len(e) - 18 and r["count"] == 1
    assert np.all(r["sigma"] == 1) and r["index"] == 0


def test_brute_force_zero_couplings():
    e = I.square_lattice(3)
    r = O.brute_force(9, e, np.zeros(len(e), np.int32), None)
    assert r["energy"] == 0 and r["count"] == 2 ** 9


def _small_cases():
    cases = []
    for s in range(3):
        rng = np.random.default_rng([7, s])
        cases.append(("sq4", I.square_lattice(4), 16, "pm1", None, rng))
        cases.append(("sq3x5g", I.square_lattice(3, 5), 15, "gauss", 0.3, rng))
        cases.append(("reg3_16", I.random_regular(16, 3, rng), 16, "pm1", None, rng))
        cases.append(("chim1x2", I.chimera(1, 2), 16, "pm1", None, rng))
        cases.append(("K6g", I.complete(6), 6, "gauss", 0.5, rng))
    return cases


@pytest.mark.parametrize("case", range(15))
def test_elimination_matches_brute_force(case):
    name, e, n, coupling, fstd, rng = _small_cases()[case]
    inst = I.make(e, n, rng, coupling, field_std=fstd)
    bf = O.brute_force(n, e, inst.J, inst.h)
    integer = coupling == "pm1"
    for order in (None, list(range(n)), list(rng.permutation(n))):
        r = O.eliminate(n, e, inst.J, inst.h, order=order,
                        counts="exact" if integer else None)
        if integer:
            assert r["energy"] == bf["energy"]
            assert r["count"] == bf["count"]
            assert O.energy(n, e, inst.J, inst.h, r["sigma"]) == bf["energy"]
        else:
            assert abs(r["energy"] - bf["energy"]) < 1e-9
            assert abs(O.energy(n, e, inst.J, inst.h, r["sigma"]) - bf["energy"]) < 1e-9


def test_mod_counts_match_exact_counts():
    rng = np.random.default_rng(5)
    e = I.square_lattice(5)
    J = I.pm1(len(e), rng)
    a = O.eliminate(25, e, J, None, counts="exact")
    b = O.eliminate(25, e, J, None, counts="mod")
    assert a["count"] == b["count"] and a["energy"] == b["energy"]


def test_zero_couplings_count_exceeds_any_small_modulus():
    # g = 2^N exactly (exact integers), N = 64 on an 8x8 lattice
    e = I.square_lattice(8)
    r = O.eliminate(64, e, np.zeros(len(e), np.int32), None, counts="exact",
                    order=list(range(64)))
    assert r["energy"] == 0 and r["count"] == 2 ** 64


@pytest.mark.parametrize("fam", ["sq12", "chimera2", "reg3_40"])
def test_planted_closed_form_full_elimination(fam):
    rng = np.random.default_rng([11, hash(fam) % 1000])
    if fam == "sq12":
        e, n = I.square_lattice(12), 144
    elif fam == "chimera2":
        e, n = I.chimera(2), 32
    else:
        e, n = I.random_regular(40, 3, rng), 40
    inst, tau = I.planted(e, n, rng)
    r = O.eliminate(n, e, inst.J, None, counts="exact")
    assert r["energy"] == -len(e)
    assert r["count"] == 2
    assert np.all(r["sigma"] == tau) or np.all(r["sigma"] == -tau)


def test_tree_and_ring_closed_forms_elimination():
    rng = np.random.default_rng(3)
    n = 60
    e = I.random_tree(n, rng)
    J = I.pm1(len(e), rng) * 3
    r = O.eliminate(n, e, J, None, counts="exact")
    assert r["energy"] == -3 * (n - 1) and r["count"] == 2
    n = 31
    e = I.ring(n)
    J = np.ones(n, np.int32)
    J[[2, 5, 9]] = -1            # odd number of negative bonds: frustrated
    r = O.eliminate(n, e, J, None, counts="exact")
    assert r["energy"] == -(n - 2) and r["count"] == 2 * n


@pytest.mark.parametrize("seed", range(3))
def test_gauge_invariance_and_z2(seed):
    rng = np.random.default_rng([13, seed])
    e = I.square_lattice(6)
    inst = I.make(e, 36, rng, "pm1")
    tau = (2 * rng.integers(0, 2, 36) - 1).astype(np.int8)
    g = I.gauge(inst, tau)
    a = O.eliminate(36, e, inst.J, None, counts="exact")
    b = O.eliminate(36, e, g.J, None, counts="exact")
    assert a["energy"] == b["energy"] and a["count"] == b["count"]
    assert a["count"] % 2 == 0                       # Z2 at h = 0
    assert O.energy(36, e, g.J, None, tau * a["sigma"]) == a["energy"]
    assert O.energy(36, e, inst.J, None, -a["sigma"]) == a["energy"]


def test_disjoint_union():
    rng = np.random.default_rng(17)
    e1 = I.square_lattice(3, 4)
    e2 = I.random_regular(10, 3, rng)
    J1, J2 = I.pm1(len(e1), rng), I.pm1(len(e2), rng)
    a = O.eliminate(12, e1, J1, None, counts="exact")
    b = O.eliminate(10, e2, J2, None, counts="exact")
    e = np.concatenate([e1, e2 + 12]).astype(np.int32)
    c = O.eliminate(22, e, np.concatenate([J1, J2]), None, counts="exact")
    assert c["energy"] == a["energy"] + b["energy"]
    assert c["count"] == a["count"] * b["count"]


@pytest.mark.parametrize("seed", range(3))
def test_gradient_by_finite_differences(seed):
    rng = np.random.default_rng([19, seed])
    L = 5
    e = I.square_lattice(L)
    inst = I.make(e, L * L, rng, "gauss", field_std=0.3)
    J = inst.J.astype(np.float64)
    h = inst.h.astype(np.float64)
    r = O.eliminate(L * L, e, J, h)
    dJ, dh = O.ground_state_gradient(e, r["sigma"])
    eps = 1e-6
    for k in rng.choice(len(e), 6, replace=False):
        Jp, Jm = J.copy(), J.copy()
        Jp[k] += eps
        Jm[k] -= eps
        fp = (O.eliminate(L * L, e, Jp, h, traceback=False)["energy"] - r["energy"]) / eps
        fm = (r["energy"] - O.eliminate(L * L, e, Jm, h, traceback=False)["energy"]) / eps
        assert abs(fp - fm) < 1e-6            # non-degenerate: both slopes agree
        assert abs(fp - dJ[k]) < 1e-6
    for i in rng.choice(L * L, 6, replace=False):
        hp = h.copy()
        hp[i] += eps
        fp = (O.eliminate(L * L, e, J, hp, traceback=False)["energy"] - r["energy"]) / eps
        assert abs(fp - dh[i]) < 1e-6


def test_crt_roundtrip():
    P = O.ORACLE_PRIMES
    for x in [0, 1, 12345678901234567890, 2 ** 200 + 17, math.prod(P) - 1]:
        assert O.crt([x % p for p in P], P) == x


def test_induced_width_of_raster_order():
    # raster elimination of an open L x L lattice joins at most L + 1 spins
    for L in (3, 5, 8):
        w = O.induced_width(L * L, I.square_lattice(L), list(range(L * L)))
        assert w == L + 1


def test_golden_small_cases_reproduce():
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "small_cases.json")
    gold = json.load(open(path))
    for b in range(4):
        inst = I.config_instances(0, batch=4)[b]
        g = gold[f"square4x4_pm1_{b}"]
        assert g["J"] == inst.J.tolist()
        r = O.eliminate(inst.n, inst.edges, inst.J, None, counts="exact")
        assert r["energy"] == g["energy"] and r["count"] == g["count"]

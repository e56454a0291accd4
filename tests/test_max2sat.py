"""#Max-2-SAT through the Ising mapping.

CPU: the mapping against direct clause counting over every assignment (small
formulas), and against the oracle's elimination. GPU: the library's counting
path gives the maximum number of satisfied clauses and the number of optimal
assignments, checked by brute force (n <= 18) and against the oracle.
"""
import itertools
import sys

import numpy as np
import pytest

from oracle import spinglass as O
from paper_2008_06888_amd import max2sat as M


def brute(inst):
    best, count = None, 0
    for bits in itertools.product((1, -1), repeat=inst.n):
        v = M.violated(inst, np.array(bits))
        if best is None or v < best:
            best, count = v, 1
        elif v == best:
            count += 1
    return len(inst.clauses) - best, count


def formula(n, m, rng, units=0):
    cl = []
    for _ in range(m):
        i, j = rng.choice(n, 2, replace=False)
        cl.append((int((i + 1) * rng.choice([-1, 1])), int((j + 1) * rng.choice([-1, 1]))))
    for _ in range(units):
        i = int(rng.integers(n))
        s = int(rng.choice([-1, 1]))
        cl.append((s * (i + 1), s * (i + 1)))
    cl.append((1, -1))   # a tautology
    return cl


@pytest.mark.parametrize("seed", range(6))
def test_mapping_energy_is_four_violations(seed):
    rng = np.random.default_rng([61, seed])
    n = 8
    inst = M.to_ising(n, formula(n, 14, rng, units=2))
    for bits in itertools.product((1, -1), repeat=n):
        s = np.array(bits, np.int8)
        assert O.energy(n, inst.edges, inst.J, inst.h, s) + inst.const == 4 * M.violated(inst, s)


@pytest.mark.parametrize("seed", range(4))
def test_mapping_optimum_and_count_match_brute_force(seed):
    rng = np.random.default_rng([62, seed])
    n = 10
    inst = M.to_ising(n, formula(n, 20, rng, units=1))
    best, count = brute(inst)
    ref = O.eliminate(n, inst.edges, inst.J, inst.h, counts="exact")
    assert M.max_satisfied(inst, ref["energy"]) == best
    assert ref["count"] == count


def test_regular_formula_shape():
    rng = np.random.default_rng(63)
    cl = M.random_regular_formula(20, rng)
    assert len(cl) == 30
    inst = M.to_ising(20, cl)
    deg = np.bincount(inst.edges.ravel(), minlength=20)
    assert np.all(deg == 3)


torch = pytest.importorskip("torch")


@pytest.mark.gpu
@pytest.mark.parametrize("n,seed", [(12, 0), (16, 1), (18, 2)])
def test_gpu_count_matches_brute_force(n, seed):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_06888_amd import binding as B
    rng = np.random.default_rng([64, seed])
    inst = M.to_ising(n, M.random_regular_formula(n, rng))
    print("[case] max2sat brute", n, seed, flush=True)
    sys.stdout.flush()
    plan = B.Plan(n, inst.edges, has_field=True, seed=seed)
    E, res, g = B.count(plan, torch.tensor(inst.J[None], device="cuda:0"),
                        torch.tensor(inst.h[None], device="cuda:0"))
    best, count = brute(inst)
    assert M.max_satisfied(inst, int(E[0])) == best and g[0] == count


@pytest.mark.gpu
@pytest.mark.parametrize("n,seed", [(60, 3), (100, 4)])
def test_gpu_count_matches_oracle(n, seed):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_06888_amd import binding as B
    rng = np.random.default_rng([65, seed])
    inst = M.to_ising(n, M.random_regular_formula(n, rng))
    print("[case] max2sat oracle", n, seed, flush=True)
    sys.stdout.flush()
    plan = B.Plan(n, inst.edges, has_field=True, seed=seed)
    E, res, g = B.count(plan, torch.tensor(inst.J[None], device="cuda:0"),
                        torch.tensor(inst.h[None], device="cuda:0"))
    ref = O.eliminate(n, inst.edges, inst.J, inst.h, counts="exact")
    assert int(E[0]) == ref["energy"] and g[0] == ref["count"]

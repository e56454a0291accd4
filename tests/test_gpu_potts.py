"""GPU parity of the 3-state Potts path (Appendix C) against the CPU oracle.

Doubled energies 2H* of integer couplings and all degeneracies are compared
exactly; float32 energies of Gaussian couplings within |dH| <= 1e-5 N of the
float64 oracle. Sizes span several passes and tiles, with ragged lattice
shapes; the 18 x 18 lattice of the paper's largest Potts runs is checked by
closed forms (ferromagnet) and invariants (label symmetry, energy path =
counting path, tile sizes agree).
"""
import sys

import numpy as np
import pytest

from oracle import potts as OP
from paper_2008_06888_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2008_06888_amd import binding as B  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), device=DEV)


@pytest.mark.parametrize("L,Lc,batch", [(3, 3, 3), (4, 5, 4), (6, 6, 2), (7, 9, 3), (10, 10, 2)])
def test_potts_pm1_lattice_energy_and_count(L, Lc, batch):
    insts = I.potts_lattice(L, batch=batch, Lc=Lc)
    n = L * Lc
    plan = B.Plan(n, insts[0].edges, order=list(range(n)), q=3)
    say("potts pm1", L, Lc, "batch", batch, "width", plan.info()["width"], "passes", plan.info()["n_passes"])
    J = dev(np.stack([x.J for x in insts]))
    E = B.potts_contract(plan, J).cpu().numpy()
    E2, _, g = B.potts_count(plan, J)
    for b, x in enumerate(insts):
        ref = OP.eliminate(n, x.edges, x.J, counts="mod", traceback=False)
        assert 2 * E[b] == ref["energy2"], (b, E[b], ref["energy2"])
        assert E2[b] == ref["energy2"] and g[b] == ref["count"], (b, E2[b], g[b], ref)
        assert g[b] % 3 == 0


@pytest.mark.parametrize("L,Lc", [(5, 5), (8, 11), (12, 12)])
def test_potts_gauss_lattice_energy(L, Lc):
    insts = I.potts_lattice(L, batch=3, Lc=Lc, coupling="gauss")
    n = L * Lc
    plan = B.Plan(n, insts[0].edges, order=list(range(n)), q=3)
    say("potts gauss", L, Lc)
    E = B.potts_contract(plan, dev(np.stack([x.J for x in insts]))).cpu().numpy()
    for b, x in enumerate(insts):
        ref = OP.eliminate(n, x.edges, x.J, traceback=False)
        assert abs(E[b] - ref["energy"]) <= 1e-5 * n, (b, E[b], ref["energy"])


@pytest.mark.parametrize("n,seed", [(20, 0), (30, 1), (40, 2)])
def test_potts_random_regular_greedy(n, seed):
    rng = np.random.default_rng([22, seed])
    e = I.random_regular(n, 3, rng)
    insts = [I.make(e, n, np.random.default_rng([22, seed, b]), "pm1") for b in range(3)]
    plan = B.Plan(n, e, seed=seed, q=3)
    say("potts reg3", n, "width", plan.info()["width"])
    J = dev(np.stack([x.J for x in insts]))
    E = B.potts_contract(plan, J).cpu().numpy()
    E2, _, g = B.potts_count(plan, J)
    for b, x in enumerate(insts):
        ref = OP.eliminate(n, e, x.J, counts="mod", traceback=False)
        assert 2 * E[b] == ref["energy2"] and E2[b] == ref["energy2"] and g[b] == ref["count"], b


@pytest.mark.parametrize("tiles", [(2, 2), (3, 3), (4, 2)])
def test_potts_tile_sizes_agree(tiles):
    insts = I.potts_lattice(9, batch=2, Lc=7)
    plan = B.Plan(63, insts[0].edges, order=list(range(63)), q=3, tile_bits=tiles[0], count_tile_bits=tiles[1])
    say("potts tiles", tiles)
    J = dev(np.stack([x.J for x in insts]))
    E = B.potts_contract(plan, J).cpu().numpy()
    E2, _, g = B.potts_count(plan, J)
    for b, x in enumerate(insts):
        ref = OP.eliminate(63, x.edges, x.J, counts="mod", traceback=False)
        assert 2 * E[b] == ref["energy2"] and E2[b] == ref["energy2"] and g[b] == ref["count"]


def test_potts_degenerate_graphs():
    # isolated spins: 2H* = 0, g = 3^n; a path: proper colourings 3 * 2^(n-1) (antiferro)
    plan = B.Plan(5, np.zeros((0, 2), np.int32), q=3)
    J = torch.zeros((1, 0), dtype=torch.int32, device=DEV)
    E2, _, g = B.potts_count(plan, J)
    assert E2[0] == 0 and g[0] == 3 ** 5
    assert B.potts_contract(plan, J).cpu().numpy()[0] == 0
    e = I.path(9)
    plan = B.Plan(9, e, q=3)
    J = dev(np.ones((2, 8), np.int32))
    E2, _, g = B.potts_count(plan, J)
    assert list(E2) == [-8, -8] and g == [3 * 2 ** 8] * 2


def test_potts_input_checks():
    e = I.square_lattice(4)
    plan = B.Plan(16, e, q=3)
    J = np.ones((2, len(e)), np.float32)
    J[1, 3] = np.inf
    with pytest.raises(B.TTError) as ei:
        B.potts_contract(plan, dev(J))
    assert ei.value.code == B.TT_E_INVAL
    Ji = np.ones((1, len(e)), np.int32) * (1 << 19)           # sum |J| = 24 * 2^19 >= 2^23
    with pytest.raises(B.TTError) as ei:
        B.potts_contract(plan, dev(Ji))
    assert ei.value.code == B.TT_E_RANGE
    with pytest.raises(B.TTError) as ei:
        B.potts_count(plan, dev(Ji))
    assert ei.value.code == B.TT_E_RANGE
    # an Ising call on the 3-state plan is refused
    with pytest.raises(B.TTError):
        B.contract(plan, dev(np.ones((1, len(e)), np.int32)))


def test_potts_18x18_ferromagnet_closed_form():
    # J = -1 everywhere: all labels equal, 2H* = -2m, g = 3 (exact count: n = 324 > 115, guard plane on)
    e = I.square_lattice(18)
    m = len(e)
    plan = B.Plan(324, e, order=list(range(324)), q=3)
    say("potts 18x18 ferro, width", plan.info()["width"])
    J = dev(-np.ones((1, m), np.int32))
    E = B.potts_contract(plan, J).cpu().numpy()
    E2, _, g, exact = B.potts_count(plan, J, flags=True)
    assert 2 * E[0] == -2 * m and E2[0] == -2 * m and g[0] == 3 and exact[0]


def test_potts_18x18_pm1_invariants():
    insts = I.potts_lattice(18, batch=2)
    e = insts[0].edges
    plan = B.Plan(324, e, order=list(range(324)), q=3)
    J = dev(np.stack([x.J for x in insts]))
    say("potts 18x18 pm1 energy")
    E = B.potts_contract(plan, J).cpu().numpy()
    say("potts 18x18 pm1 count")
    E2, _, g, exact = B.potts_count(plan, J, flags=True)
    for b in range(2):
        assert 2 * E[b] == E2[b] and exact[b] and g[b] % 3 == 0 and g[b] > 0
        # a lower bound: every bond at its best value (-2 for J = -1, -1 for J = +1)
        Jb = insts[b].J
        assert E2[b] >= int(np.sum(np.where(Jb < 0, -2, -1)))
    # reversing the order of the sweep gives the same energy and count
    rplan = B.Plan(324, e, order=list(range(324))[::-1], q=3)
    say("potts 18x18 pm1 reversed order")
    Er = B.potts_contract(rplan, J).cpu().numpy()
    E2r, _, gr = B.potts_count(rplan, J)
    assert np.array_equal(Er, E) and np.array_equal(E2r, E2) and gr == g

"""GPU parity of half-state plans (z2: h = 0, half of every energy-path
state stored, reads and writes at the stored address, half the tiles of a
pass run): energies equal to the full-state plan's and to the oracle (stored
values for the 64 headline lattices), ground states that attain E*, exact
gradients, over tile sizes, greedy plans, int16 couplings, the two-part
path, graph replays, the unfused final maximum, uneven batches and the
autotuner; and the counting path on half states: E* and exact degeneracies
equal to the oracle's, the stored values, the full-state path and closed
forms (J = 0: g = 2^n; planted 32 x 32: g = 2), the overflow flag
included."""
import json
import os
import sys

import numpy as np
import pytest

from oracle import spinglass as O
from paper_2008_06888_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2008_06888_amd import binding as B  # noqa: E402

DEV = "cuda:0"
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "parity_large.json")))


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dt=None):
    t = torch.tensor(np.ascontiguousarray(x), device=DEV)
    return t.to(dt) if dt is not None else t


def check_configs(n, e, J, E, sig, dJ, tol=0.0):
    for b in range(J.shape[0]):
        assert abs(O.energy(n, e, J[b], None, sig[b]) - E[b]) <= tol, b
        assert np.array_equal(dJ[b], O.ground_state_gradient(e, sig[b])[0].astype(np.float32)), b


@pytest.mark.parametrize("tile", [7, 9, 11, 12, 14])
@pytest.mark.parametrize("coupling", ["pm1", "gauss"])
def test_square_lattices(tile, coupling):
    L = 12
    n, e = L * L, I.square_lattice(L)
    insts = [I.make(e, n, np.random.default_rng([71, tile, b]), coupling) for b in range(3)]
    J = np.stack([x.J for x in insts])
    full = B.Plan(n, e, order=list(range(n)), tile_bits=tile)
    half = B.Plan(n, e, order=list(range(n)), tile_bits=tile, z2=True)
    say("z2 12x12", coupling, "tile", tile)
    Ef = B.contract(full, dev(J)).cpu().numpy()
    E = B.contract(half, dev(J)).cpu().numpy()
    Eb, sig, dJ, _ = [x.cpu().numpy() if x is not None else None for x in B.backward(half, dev(J))]
    assert np.array_equal(E, Ef) and np.array_equal(Eb, Ef)
    check_configs(n, e, J, Ef, sig, dJ, tol=1e-5 * n if coupling == "gauss" else 0.0)
    for b, x in enumerate(insts):
        ref = O.eliminate(n, e, x.J, None, traceback=False)
        assert abs(E[b] - ref["energy"]) <= (1e-5 * n if coupling == "gauss" else 0.0), b


def test_headline_pm1_b64_against_stored_oracle():
    insts = I.config_instances(0, batch=64, L=16)
    gold = GOLD["square16_pm1_b64"]["cases"]
    n = 256
    J = np.stack([x.J for x in insts])
    for tile in (12, 13):
        plan = B.Plan(n, insts[0].edges, order=list(range(n)), tile_bits=tile, z2=True)
        say("z2 headline b64 tile", tile)
        E, sig, dJ, _ = [x.cpu().numpy() if x is not None else None for x in B.backward(plan, dev(J))]
        Ec = B.contract(plan, dev(J)).cpu().numpy()
        assert np.array_equal(E, Ec)
        for b in range(64):
            assert E[b] == gold[str(b)]["energy"], b
        check_configs(n, insts[0].edges, J, E, sig, dJ)
        E16, sig16, _, _ = B.backward(plan, dev(J, torch.int16))
        assert np.array_equal(E16.cpu().numpy(), E)
        assert np.array_equal(sig16.cpu().numpy(), sig)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_greedy_random_regular(seed):
    n = 70
    rng = np.random.default_rng([72, seed])
    e = I.random_regular(n, 3, rng)
    J = np.stack([I.gauss(len(e), rng) for _ in range(4)])
    plan = B.Plan(n, e, seed=seed, z2=True)
    full = B.Plan(n, e, seed=seed)
    say("z2 reg3 n=70 seed", seed, "width", plan.info()["width"])
    E, sig, dJ, _ = [x.cpu().numpy() if x is not None else None for x in B.backward(plan, dev(J))]
    assert np.array_equal(E, B.contract(full, dev(J)).cpu().numpy())
    check_configs(n, e, J, E, sig, dJ, tol=1e-5 * n)
    for tie in (1, 777):
        Et, st, _, _ = B.backward_tie(plan, dev(J), tie=tie)
        assert np.array_equal(Et.cpu().numpy(), E)
        for b in range(4):
            assert abs(O.energy(n, e, J[b], None, st.cpu().numpy()[b]) - E[b]) <= 1e-5 * n


def test_graph_replays_match_eager():
    insts = I.config_instances(0, batch=4, L=10)
    plan = B.Plan(100, insts[0].edges, order=list(range(100)), z2=True)
    J = dev(np.stack([x.J for x in insts]))
    first = [x.cpu().numpy() for x in B.backward(plan, J)[:3]]
    for _ in range(4):
        again = [x.cpu().numpy() for x in B.backward(plan, J)[:3]]
        for a, b in zip(first, again):
            assert np.array_equal(a, b)
        torch.cuda.synchronize()


def test_unfused_final_maximum():
    L = 26
    x = I.config_instances(0, batch=1, L=L)[0]
    full = B.Plan(L * L, x.edges, order=list(range(L * L)), tile_bits=12)
    half = B.Plan(L * L, x.edges, order=list(range(L * L)), tile_bits=12, z2=True)
    say("z2 26x26 unfused final maximum")
    assert np.array_equal(B.contract(half, dev(x.J[None])).cpu().numpy(),
                          B.contract(full, dev(x.J[None])).cpu().numpy())


def test_uneven_batch_and_count():
    rng = np.random.default_rng(73)
    graphs = [(n, I.random_regular(n, 3, rng)) for n in (30, 44, 58)]
    plans = [B.Plan(n, e, seed=1, z2=True) for n, e in graphs]
    Jints = [I.pm1(len(e), rng) for _, e in graphs]
    Js = [dev(j.astype(np.float32)) for j in Jints]
    res = B.contract_uneven(plans, Js)
    Eu = res[0].cpu().numpy()
    for i, ((n, e), p, J, Ji) in enumerate(zip(graphs, plans, Js, Jints)):
        E1 = B.contract(p, J[None].contiguous()).cpu().numpy()[0]
        assert Eu[i] == E1
        assert O.energy(n, e, Ji, None, res[1][i].cpu().numpy()) == E1
        ref = O.eliminate(n, e, Ji, None, counts="exact", traceback=False)
        assert E1 == ref["energy"]
        Ec, _, g = B.count(p, dev(Ji[None]))   # half-state counting
        assert Ec[0] == ref["energy"] and g[0] == ref["count"]


def test_autotune_half_state():
    insts = I.config_instances(0, batch=8, L=12)
    plan = B.Plan(144, insts[0].edges, order=list(range(144)), z2=True)
    J = dev(np.stack([x.J for x in insts]))
    ref = B.backward(plan, J)[0].cpu().numpy()
    bits, _ = B.autotune(plan, J, config=True)
    say("z2 autotune", bits)
    assert np.array_equal(B.backward(plan, J)[0].cpu().numpy(), ref)


@pytest.mark.parametrize("z2", [False, True])
def test_autotune_chooses_parts_on_the_headline_batch(z2):
    """A large batch with the part count left to the library: the autotuner
    times one and two parts per tile and keeps the faster; results are those
    of the stored oracle either way, and an explicit part count is kept."""
    insts = I.config_instances(0, batch=64, L=16)
    gold = GOLD["square16_pm1_b64"]["cases"]
    J = dev(np.stack([x.J for x in insts]))
    plan = B.Plan(256, insts[0].edges, order=list(range(256)), z2=z2)
    bits, _ = B.autotune(plan, J, config=True)
    parts = plan.info()["parts"]
    say("autotune headline z2", z2, "tile", bits, "parts", parts)
    assert parts in (1, 2)
    E = B.backward(plan, J)[0].cpu().numpy()
    assert all(E[b] == gold[str(b)]["energy"] for b in range(64))
    fixed = B.Plan(256, insts[0].edges, order=list(range(256)), z2=z2, parts=2)
    B.autotune(fixed, J, config=True)
    assert fixed.info()["parts"] == 2


# ----------------------------------------------------------------------------
# counting on half states
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("ctile", [7, 9, 12])
def test_count_square_lattices(ctile):
    L = 12
    n, e = L * L, I.square_lattice(L)
    J = np.stack([I.pm1(len(e), np.random.default_rng([74, ctile, b])) for b in range(3)])
    full = B.Plan(n, e, order=list(range(n)), count_tile_bits=ctile)
    half = B.Plan(n, e, order=list(range(n)), count_tile_bits=ctile, z2=True)
    say("z2 count 12x12 tile", ctile)
    Ef, rf, gf = B.count(full, dev(J))
    Eh, rh, gh = B.count(half, dev(J))
    assert np.array_equal(Eh, Ef) and np.array_equal(rh, rf) and gh == gf
    for b in range(3):
        ref = O.eliminate(n, e, J[b], None, counts="exact", traceback=False)
        assert Eh[b] == ref["energy"] and gh[b] == ref["count"], b


def test_count_headline_b64_against_stored_oracle():
    insts = I.config_instances(0, batch=64, L=16)
    gold = GOLD["square16_pm1_b64"]["cases"]
    plan = B.Plan(256, insts[0].edges, order=list(range(256)), z2=True)
    say("z2 count headline b64")
    Ec, _, g = B.count(plan, dev(np.stack([x.J for x in insts])))
    for b in range(64):
        assert Ec[b] == gold[str(b)]["energy"] and g[b] == int(gold[str(b)]["count"]), b


@pytest.mark.parametrize("L", [12, 16])
def test_count_zero_couplings(L):
    """J = 0: E* = 0 and g = 2^n, exact for n <= 182 (12 x 12); for 16 x 16
    (2^256, beyond the moduli) the flag is cleared and the residues equal the
    full-state path's."""
    n, e = L * L, I.square_lattice(L)
    J = dev(np.zeros((1, len(e)), np.int32))
    half = B.Plan(n, e, order=list(range(n)), z2=True)
    say("z2 count J=0", L)
    Eh, rh, gh, xh = B.count_with_flags(half, J)
    assert Eh[0] == 0
    if n <= 182:
        assert xh[0] and gh[0] == 2 ** n
    else:
        Ef, rf, gf, xf = B.count_with_flags(B.Plan(n, e, order=list(range(n))), J)
        assert not xh[0] and not xf[0] and np.array_equal(rh, rf)


def test_count_planted_square32_full_size():
    """32 x 32 planted instance (J_ij = tau_i tau_j): E* = -m, g = 2, on the
    half state (2^31 stored entries of the widest state)."""
    L = 32
    n, e = L * L, I.square_lattice(L)
    x, tau = I.planted(e, n, np.random.default_rng([32, 1024]))
    plan = B.Plan(n, e, order=list(range(n)), z2=True)
    say("z2 count 32x32 planted")
    Ec, _, g, ex = B.count_with_flags(plan, dev(x.J[None]))
    plan.close()
    assert Ec[0] == -len(e) and ex[0] and g[0] == 2


# ----------------------------------------------------------------------------
# chimera plans on half states
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("rows,cols,tb", [(2, 2, 0), (3, 3, 0), (3, 3, 8), (2, 4, 0), (3, 4, 9), (4, 4, 10)])
def test_chimera_half_state_against_oracle(rows, cols, tb):
    """E*, sigma (E(sigma) = E*, dE/dJ), exact g against the oracle and the
    full-state chimera plan, float32 and int16 couplings."""
    n = 8 * rows * cols
    e = I.chimera(rows, cols)
    insts = [I.make(e, n, I.rng_for(95, b), "pm1") for b in range(3 if rows * cols < 16 else 1)]
    J = np.stack([x.J for x in insts])
    half = B.Plan(n, e, chimera=(rows, cols), tile_bits=tb, z2=True)
    full = B.Plan(n, e, chimera=(rows, cols), tile_bits=tb)
    say("z2 chimera", rows, cols, "tile", tb)
    E, sig, dJ, _ = [x.cpu().numpy() if x is not None else None for x in B.backward(half, dev(J))]
    E16, sig16, _, _ = B.backward(half, dev(J, torch.int16))
    Ec, res, g = B.count(half, dev(J))
    Efull = B.contract(full, dev(J.astype(np.float32))).cpu().numpy()
    _, resf, gf = B.count(full, dev(J))
    assert np.array_equal(E, Efull) and np.array_equal(E16.cpu().numpy(), E)
    assert np.array_equal(res, resf) and g == gf
    for b, x in enumerate(insts):
        ref = O.eliminate(n, e, x.J, None, counts="exact")
        assert E[b] == ref["energy"] and Ec[b] == ref["energy"] and g[b] == ref["count"], b
        assert O.energy(n, e, x.J, None, sig[b]) == ref["energy"], b
        assert O.energy(n, e, x.J, None, sig16.cpu().numpy()[b]) == ref["energy"], b
        assert np.array_equal(dJ[b], -(sig[b][e[:, 0]].astype(np.float32) * sig[b][e[:, 1]])), b


def test_chimera_half_state_full_size_planted():
    """8 x 8 cells on the half state (2^31 stored entries): the Mattis
    instance's E* = -m, sigma = +-tau and g = 2."""
    e = I.chimera(8)
    x, tau = I.planted(e, 512, np.random.default_rng(96))
    plan = B.Plan(512, e, chimera=(8, 8), z2=True)
    say("z2 chimera 8x8 planted: backward")
    E, sig, _, _ = B.backward(plan, dev(x.J[None]))
    s = sig[0].cpu().numpy()
    assert E[0].item() == -len(e)
    assert np.array_equal(s, tau) or np.array_equal(s, -tau)
    say("z2 chimera 8x8 planted: count")
    Ec, _, g = B.count(plan, dev(x.J[None]))
    plan.close()
    assert Ec[0] == -len(e) and g[0] == 2


def test_chimera_half_state_full_size_random():
    """8 x 8 random +-J: the half-state plan's E*, residues and g equal the
    full-state plan's; E(sigma) = E*."""
    x = I.config_instances(4)[0]
    e = x.edges
    half = B.Plan(512, e, chimera=(8, 8), z2=True)
    say("z2 chimera 8x8 pm1: backward and count")
    E, sig, _, _ = B.backward(half, dev(x.J[None]))
    E = E[0].item()
    assert O.energy(512, e, x.J, None, sig[0].cpu().numpy()) == E
    Ec, res, g = B.count(half, dev(x.J[None]))
    half.close()
    full = B.Plan(512, e, chimera=(8, 8))
    say("z2 chimera 8x8 pm1: full-state reference")
    Ef = B.contract(full, dev(x.J[None]).float().contiguous()).cpu().numpy()[0]
    Ecf, resf, gf = B.count(full, dev(x.J[None]))
    full.close()
    assert E == Ef and Ec[0] == Ecf[0] and np.array_equal(res, resf) and g[0] == gf[0]


@pytest.mark.parametrize("case", ["edge", "path3", "ring4", "star5", "zero_ring6"])
def test_tiny_graphs(case):
    """Degenerate widths (a 1- or 2-bit state, J = 0 ties): E*, a ground
    state and g against the oracle on the half state."""
    graphs = {"edge": (2, [(0, 1)]), "path3": (3, [(0, 1), (1, 2)]), "ring4": (4, [(0, 1), (1, 2), (2, 3), (0, 3)]),
              "star5": (5, [(0, 1), (0, 2), (0, 3), (0, 4)]), "zero_ring6": (6, [(i, (i + 1) % 6) for i in range(6)])}
    n, el = graphs[case]
    e = np.array(sorted((min(a, b), max(a, b)) for a, b in el), dtype=np.int32)
    rng = np.random.default_rng([97, n])
    J = np.zeros((2, len(e)), np.int32) if case.startswith("zero") else np.stack([I.pm1(len(e), rng) for _ in range(2)])
    plan = B.Plan(n, e, seed=0, z2=True)
    say("z2 tiny", case, "width", plan.info()["width"])
    E, sig, dJ, _ = [x.cpu().numpy() if x is not None else None for x in B.backward(plan, dev(J))]
    Ec, _, g = B.count(plan, dev(J))
    for b in range(2):
        ref = O.eliminate(n, e, J[b], None, counts="exact", traceback=False)
        assert E[b] == ref["energy"] and Ec[b] == ref["energy"] and g[b] == ref["count"], b
        assert O.energy(n, e, J[b], None, sig[b]) == ref["energy"], b


def test_uneven_batch_mixing_half_and_full_state_plans():
    """One uneven call over half-state and full-state plans (launches hold
    both kinds of items): E* and sigma equal to one call per instance."""
    rng = np.random.default_rng(98)
    graphs = [(n, I.random_regular(n, 3, rng)) for n in (24, 36, 48, 60)]
    plans = [B.Plan(n, e, seed=2, z2=(k % 2 == 0)) for k, (n, e) in enumerate(graphs)]
    Js = [dev(I.gauss(len(e), rng).astype(np.float32)) for _, e in graphs]
    say("z2 uneven mixed")
    res = B.contract_uneven(plans, Js)
    Eu = res[0].cpu().numpy()
    for i, ((n, e), p, J) in enumerate(zip(graphs, plans, Js)):
        E1, s1, _, _ = B.backward(p, J[None].contiguous())
        assert abs(Eu[i] - E1.cpu().numpy()[0]) <= 1e-5 * n, i
        assert abs(O.energy(n, e, J.cpu().numpy(), None, res[1][i].cpu().numpy()) - Eu[i]) <= 1e-5 * n, i

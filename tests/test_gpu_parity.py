"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Energies of integer instances and all counts are compared exactly; float32
energies within |dE| <= 1e-5 * N of the float64 oracle (the tolerance the
headline workload states); configurations exactly where the ground state is
unique (Gaussian couplings with fields), else by E(sigma) = E*.
"""
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


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), device=DEV)


def stack(insts, attr):
    return np.stack([getattr(x, attr) for x in insts])


def tol(n):
    return 1e-5 * n


# ----------------------------------------------------------------------------
# 4 x 4 open square lattice, J = +-1: brute force over 2^16 configurations
# ----------------------------------------------------------------------------
def test_square4x4_pm1_energy_sigma_count():
    insts = I.config_instances(0, batch=8)
    say("square4x4_pm1 batch 8")
    plan = B.Plan(16, insts[0].edges, order=list(range(16)))
    Ji = dev(stack(insts, "J"))
    Ef = B.contract(plan, Ji.float().contiguous()).cpu().numpy()
    Ei = B.contract(plan, Ji).cpu().numpy()
    E2, sig, dJ, _ = B.backward(plan, Ji)
    Ec, res, g = B.count(plan, Ji)
    sig = sig.cpu().numpy()
    dJ = dJ.cpu().numpy()
    for b, x in enumerate(insts):
        bf = O.brute_force(16, x.edges, x.J, None)
        assert Ef[b] == bf["energy"] and Ei[b] == bf["energy"] and E2[b].item() == bf["energy"]
        assert Ec[b] == bf["energy"] and g[b] == bf["count"]
        assert O.energy(16, x.edges, x.J, None, sig[b]) == bf["energy"]
        ref_dJ, _ = O.ground_state_gradient(x.edges, sig[b])
        assert np.array_equal(dJ[b], ref_dJ.astype(np.float32))


# ----------------------------------------------------------------------------
# Gaussian couplings with fields: unique ground states
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("shape,tile_bits", [((3, 3), 0), ((5, 5), 7), ((6, 6), 7), ((3, 7), 8),
                                             ((10, 10), 7), ((10, 10), 8), ((9, 11), 9)])
def test_lattice_gauss_field_parity(shape, tile_bits):
    Lr, Lc = shape
    n = Lr * Lc
    e = I.square_lattice(Lr, Lc)
    rng = np.random.default_rng([5, Lr, Lc])
    insts = [I.make(e, n, np.random.default_rng([5, Lr, Lc, b]), "gauss", field_std=0.3) for b in range(3)]
    say("lattice", shape, "tile_bits", tile_bits)
    plan = B.Plan(n, e, order=list(range(n)), has_field=True, tile_bits=tile_bits)
    J, h = dev(stack(insts, "J")), dev(stack(insts, "h"))
    E0 = B.contract(plan, J, h).cpu().numpy()
    E, sig, dJ, dh = B.backward(plan, J, h)
    E, sig, dJ, dh = E.cpu().numpy(), sig.cpu().numpy(), dJ.cpu().numpy(), dh.cpu().numpy()
    assert np.array_equal(E0, E)
    for b, x in enumerate(insts):
        ref = O.eliminate(n, e, x.J, x.h)
        assert abs(E[b] - ref["energy"]) <= tol(n)
        assert np.array_equal(sig[b], ref["sigma"])
        gJ, gh = O.ground_state_gradient(e, ref["sigma"])
        assert np.array_equal(dJ[b], gJ.astype(np.float32)) and np.array_equal(dh[b], gh.astype(np.float32))
    del rng


# ----------------------------------------------------------------------------
# general graphs with greedy orders: energies and counts exact
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("fam,n", [("reg3", 16), ("reg3", 20), ("reg3", 24), ("chim", 16), ("chim", 32),
                                   ("sq", 20)])
def test_greedy_pm1_energy_count(fam, n):
    rng = np.random.default_rng([6, n, len(fam)])
    if fam == "reg3":
        e = I.random_regular(n, 3, rng)
    elif fam == "chim":
        e = I.chimera(1, 2) if n == 16 else I.chimera(2, 2)
    else:
        e = I.square_lattice(4, 5)
    insts = [I.make(e, n, np.random.default_rng([6, n, b]), "pm1") for b in range(4)]
    J = dev(stack(insts, "J"))
    results = []
    for seed in (0, 1, 2):
        say(fam, n, "seed", seed)
        plan = B.Plan(n, e, seed=seed, trials=4, tile_bits=7, count_tile_bits=7)
        Ec, _, g = B.count(plan, J)
        E, sig, _, _ = B.backward(plan, J)
        results.append((Ec.tolist(), g))
        sig = sig.cpu().numpy()
        for b, x in enumerate(insts):
            assert O.energy(n, e, x.J, None, sig[b]) == Ec[b]
            assert E[b].item() == Ec[b]
    for b, x in enumerate(insts):
        ref = O.eliminate(n, e, x.J, None, counts="exact")
        for Ec, g in results:
            assert Ec[b] == ref["energy"] and g[b] == ref["count"]


def test_gauge_and_z2_invariance():
    L = 8
    e = I.square_lattice(L)
    rng = np.random.default_rng(31)
    x = I.make(e, L * L, rng, "pm1")
    tau = (2 * rng.integers(0, 2, L * L) - 1).astype(np.int8)
    y = I.gauge(x, tau)
    say("gauge 8x8")
    plan = B.Plan(L * L, e, order=list(range(L * L)), count_tile_bits=7, tile_bits=7)
    Ec, _, g = B.count(plan, dev(np.stack([x.J, y.J])))
    assert Ec[0] == Ec[1] and g[0] == g[1] and g[0] % 2 == 0
    ref = O.eliminate(L * L, e, x.J, None, counts="exact")
    assert Ec[0] == ref["energy"] and g[0] == ref["count"]


def test_zero_couplings_count_two_to_n():
    L = 8
    e = I.square_lattice(L)
    say("zero couplings 8x8")
    plan = B.Plan(L * L, e, order=list(range(L * L)), count_tile_bits=7)
    Ec, res, g = B.count(plan, dev(np.zeros((1, len(e)), np.int32)))
    assert Ec[0] == 0 and g[0] == 2 ** 64


# ----------------------------------------------------------------------------
# the headline workload: 16 x 16, Gaussian J, h ~ N(0, 0.1^2), batch 64
# ----------------------------------------------------------------------------
def test_square16_gauss_b64_sampled():
    insts = I.config_instances(1)
    say("square16 gauss b64")
    plan = B.Plan(256, insts[0].edges, order=list(range(256)), has_field=True)
    J, h = dev(stack(insts, "J")), dev(stack(insts, "h"))
    E, sig, dJ, dh = B.backward(plan, J, h)
    E, sig = E.cpu().numpy(), sig.cpu().numpy()
    for b, x in enumerate(insts):        # every configuration attains its energy
        assert abs(O.energy(256, x.edges, x.J, x.h, sig[b]) - E[b]) <= tol(256)
    for b in (0, 17, 42, 63):            # sampled instances against the oracle
        x = insts[b]
        ref = O.eliminate(256, x.edges, x.J, x.h, order=list(range(256)))
        assert abs(E[b] - ref["energy"]) <= tol(256)
        assert np.array_equal(sig[b], ref["sigma"])


@pytest.mark.parametrize("tile_bits", [13, 14])
def test_square16_wide_tiles_backward(tile_bits):
    """Tiles of 2^13 / 2^14: the passes eliminate 13 / 14 spins, so the
    backward scores exactly one / two full batches of 8 x 1024 candidates per
    pass (the second batch is loaded inside the scoring loop)."""
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    import kernel_emulator as KE
    insts = I.config_instances(1, batch=3)
    say("square16 gauss tile_bits", tile_bits, "batch 3")
    plan = B.Plan(256, insts[0].edges, order=list(range(256)), has_field=True, tile_bits=tile_bits)
    assert max(p.n_cand for p in KE.load_program(plan)["passes"]) == tile_bits
    J, h = dev(stack(insts, "J")), dev(stack(insts, "h"))
    E, sig, dJ, dh = B.backward(plan, J, h)
    E, sig, dJ, dh = E.cpu().numpy(), sig.cpu().numpy(), dJ.cpu().numpy(), dh.cpu().numpy()
    for b, x in enumerate(insts):
        ref = O.eliminate(256, x.edges, x.J, x.h, order=list(range(256)))
        assert abs(E[b] - ref["energy"]) <= tol(256)
        assert np.array_equal(sig[b], ref["sigma"])
        gJ, gh = O.ground_state_gradient(x.edges, ref["sigma"])
        assert np.array_equal(dJ[b], gJ.astype(np.float32)) and np.array_equal(dh[b], gh.astype(np.float32))


@pytest.mark.parametrize("tile_bits", [7, 8])
def test_square14_many_passes_backward(tile_bits):
    """14x14 at tiles 2^7 / 2^8: 182 / 91 passes, more than the 64 a chunk of
    the backward stages in LDS at once, so the walk crosses chunk boundaries."""
    sys.path.insert(0, __file__.rsplit("/", 1)[0])
    import kernel_emulator as KE
    L = 14
    e = I.square_lattice(L)
    insts = [I.make(e, L * L, np.random.default_rng([11, b]), "gauss", field_std=0.3) for b in range(3)]
    say("square14 gauss tile_bits", tile_bits, "batch 3")
    plan = B.Plan(L * L, e, order=list(range(L * L)), has_field=True, tile_bits=tile_bits)
    assert len(KE.load_program(plan)["passes"]) > 64
    J, h = dev(stack(insts, "J")), dev(stack(insts, "h"))
    E, sig, dJ, dh = B.backward(plan, J, h)
    E, sig, dJ, dh = E.cpu().numpy(), sig.cpu().numpy(), dJ.cpu().numpy(), dh.cpu().numpy()
    for b, x in enumerate(insts):
        ref = O.eliminate(L * L, e, x.J, x.h, order=list(range(L * L)))
        assert abs(E[b] - ref["energy"]) <= tol(L * L)
        assert np.array_equal(sig[b], ref["sigma"])
        gJ, gh = O.ground_state_gradient(e, ref["sigma"])
        assert np.array_equal(dJ[b], gJ.astype(np.float32)) and np.array_equal(dh[b], gh.astype(np.float32))


def test_split_batch_odd_size_matches_single_calls():
    # 17 x 2^16 state entries: the call runs as two parts (8 and 9 instances)
    # on two streams; every instance must equal its own single-instance call
    insts = I.config_instances(1, batch=17)
    say("square16 gauss b17 split")
    plan = B.Plan(256, insts[0].edges, order=list(range(256)), has_field=True)
    J, h = dev(stack(insts, "J")), dev(stack(insts, "h"))
    E, sig, dJ, dh = B.backward(plan, J, h)
    Ec = B.contract(plan, J, h)
    E, sig, Ec = E.cpu().numpy(), sig.cpu().numpy(), Ec.cpu().numpy()
    assert np.array_equal(E, Ec)
    for b in (0, 7, 8, 16):
        E1, sig1, _, _ = B.backward(plan, J[b:b + 1].contiguous(), h[b:b + 1].contiguous())
        assert E1.cpu().numpy()[0] == E[b]
        assert np.array_equal(sig1.cpu().numpy()[0], sig[b])
    x = insts[8]
    ref = O.eliminate(256, x.edges, x.J, x.h, order=list(range(256)))
    assert abs(E[8] - ref["energy"]) <= tol(256) and np.array_equal(sig[8], ref["sigma"])


def test_square16_gradient_finite_differences():
    insts = I.config_instances(1, batch=2)
    plan = B.Plan(256, insts[0].edges, order=list(range(256)), has_field=True)
    J, h = dev(stack(insts, "J")), dev(stack(insts, "h"))
    say("square16 FD")
    E, sig, dJ, dh = B.backward(plan, J, h)
    rng = np.random.default_rng(3)
    eps = 1e-2
    for k in rng.choice(plan.m, 6, replace=False):
        Jp, Jm = J.clone(), J.clone()
        Jp[:, k] += eps
        Jm[:, k] -= eps
        fd = (B.contract(plan, Jp, h) - B.contract(plan, Jm, h)).cpu().numpy() / (2 * eps)
        assert np.all(np.abs(fd - dJ[:, k].cpu().numpy()) < 2e-2)


# ----------------------------------------------------------------------------
# full size: 32 x 32 planted (Mattis) instance, closed form E* = -m, g = 2
# ----------------------------------------------------------------------------
def test_square32_planted_energy_and_count():
    L = 32
    e = I.square_lattice(L)
    x, tau = I.planted(e, L * L, np.random.default_rng(77))
    say("square32 planted")
    plan = B.Plan(L * L, e, order=list(range(L * L)))
    E = B.contract(plan, dev(x.J[None])).cpu().numpy()
    assert E[0] == -len(e)
    Ec, res, g = B.count(plan, dev(x.J[None]))
    assert Ec[0] == -len(e) and g[0] == 2


# ----------------------------------------------------------------------------
# uneven batch of different graphs
# ----------------------------------------------------------------------------
def test_uneven_regular3_small():
    insts = []
    for b, n in enumerate([18, 22, 26, 30]):
        rng = np.random.default_rng([8, b])
        insts.append(I.make(I.random_regular(n, 3, rng), n, rng, "gauss"))
    say("uneven reg3")
    plans = [B.Plan(x.n, x.edges, seed=1, trials=8, tile_bits=7) for x in insts]
    E, sig, dJ = B.contract_uneven(plans, [dev(x.J) for x in insts])
    E = E.cpu().numpy()
    for b, x in enumerate(insts):
        ref = O.eliminate(x.n, x.edges, x.J, None)
        assert abs(E[b] - ref["energy"]) <= tol(x.n)
        s = sig[b].cpu().numpy()
        assert abs(O.energy(x.n, x.edges, x.J, None, s) - ref["energy"]) <= tol(x.n)
        assert np.array_equal(s, ref["sigma"]) or np.array_equal(s, -ref["sigma"])


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
    say("degenerate", case)
    plan = B.Plan(n, e, seed=1, trials=2, tile_bits=7, count_tile_bits=7)
    Jd = dev(J[None].astype(np.int32)) if len(e) else torch.zeros((1, 0), dtype=torch.int32, device=DEV)
    E, sig, _, _ = B.backward(plan, Jd)
    Ec, _, g = B.count(plan, Jd)
    ref = O.eliminate(n, e, J, None, counts="exact")
    assert E[0].item() == ref["energy"] and Ec[0] == ref["energy"] and g[0] == ref["count"]
    assert O.energy(n, e, J, None, sig[0].cpu().numpy()) == ref["energy"]


def test_uneven_matches_per_instance_calls():
    insts = I.config_instances(3, batch=5, L=None)[:5]
    small = []
    for b, n in enumerate([20, 26, 32, 40, 24]):
        rng = np.random.default_rng([9, b])
        small.append(I.make(I.random_regular(n, 3, rng), n, rng, "gauss"))
    say("uneven vs per-instance")
    plans = [B.Plan(x.n, x.edges, seed=2, trials=8, tile_bits=8) for x in small]
    E, sig, dJ = B.contract_uneven(plans, [dev(x.J) for x in small])
    for b, x in enumerate(small):
        p1 = B.Plan(x.n, x.edges, seed=2, trials=8, tile_bits=8)
        E1, s1, dJ1, _ = B.backward(p1, dev(x.J[None]))
        assert E1[0].item() == E[b].item()
        assert torch.equal(s1[0], sig[b]) and torch.equal(dJ1[0], dJ[b])
    del insts


def test_graph_replays_match_eager():
    insts = I.config_instances(1, batch=16, L=8)
    plan = B.Plan(64, insts[0].edges, order=list(range(64)), has_field=True, tile_bits=7)
    J, h = dev(stack(insts, "J")), dev(stack(insts, "h"))
    say("graph replays")
    B.graphs_enable(False)
    ref = [t.clone() for t in B.backward(plan, J, h)]
    B.graphs_enable(True)
    E = torch.empty(16, dtype=torch.float64, device=DEV)
    sig = torch.empty(16, 64, dtype=torch.int8, device=DEV)
    dJ = torch.empty(16, plan.m, dtype=torch.float32, device=DEV)
    dh = torch.empty(16, 64, dtype=torch.float32, device=DEV)
    lib = B.lib()
    import ctypes as C
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    for rep in range(6):                       # 1st eager, 2nd captured, then replays
        E.zero_()
        sig.zero_()
        rc = lib.tt_backward(plan.handle, 16, B.TT_F32, C.c_void_p(J.data_ptr()), C.c_void_p(h.data_ptr()),
                             C.c_void_p(E.data_ptr()), C.c_void_p(sig.data_ptr()), C.c_void_p(dJ.data_ptr()),
                             C.c_void_p(dh.data_ptr()), st)
        assert rc == 0
        x = torch.randn(256, 256, device=DEV) @ torch.randn(256, 256, device=DEV)   # eager work between
        torch.cuda.synchronize()
        assert torch.equal(E, ref[0]) and torch.equal(sig, ref[1]) and torch.equal(dJ, ref[2])
        assert torch.equal(dh, ref[3])
        del x
    # a replay reads the current inputs: change J in place and compare to eager
    J.mul_(-1.0)
    for rep in range(2):
        rc = lib.tt_backward(plan.handle, 16, B.TT_F32, C.c_void_p(J.data_ptr()), C.c_void_p(h.data_ptr()),
                             C.c_void_p(E.data_ptr()), C.c_void_p(sig.data_ptr()), C.c_void_p(dJ.data_ptr()),
                             C.c_void_p(dh.data_ptr()), st)
        assert rc == 0
    torch.cuda.synchronize()
    B.graphs_enable(False)
    ref2 = B.backward(plan, J, h)
    B.graphs_enable(True)
    assert torch.equal(E, ref2[0]) and torch.equal(sig, ref2[1])


def test_kernel_timing_with_graphs_enabled():
    """Kernel timing on: repeated calls run eagerly, every launch is timed, results are exact."""
    insts = I.config_instances(1, batch=8, L=8)
    plan = B.Plan(64, insts[0].edges, order=list(range(64)), has_field=True, tile_bits=7)
    J, h = dev(stack(insts, "J")), dev(stack(insts, "h"))
    say("graph replays with kernel timing")
    B.graphs_enable(False)
    ref = [t.clone() for t in B.backward(plan, J, h)]
    B.graphs_enable(True)
    B.prof_enable(True)
    try:
        B.prof_reset()
        for rep in range(5):                   # never captured while timing is on
            out = B.backward(plan, J, h)
            torch.cuda.synchronize()
            assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]) and torch.equal(out[2], ref[2])
        ms, n = B.prof_read("sweep_pass")
        nb = plan.info()["n_passes"]
        assert n == 5 * nb and ms > 0
        msb, nbw = B.prof_read("sweep_backward")
        assert nbw == 5 and msb > 0
    finally:
        B.prof_enable(False)


# ----------------------------------------------------------------------------
# tile-size autotuner: the chosen tiles give the same results
# ----------------------------------------------------------------------------
def test_autotune_keeps_results():
    insts = I.config_instances(1, batch=8, L=10)
    say("autotune square10 gauss batch 8")
    plan = B.Plan(100, insts[0].edges, order=list(range(100)), has_field=True)
    J = dev(np.stack([x.J for x in insts]))
    h = dev(np.stack([x.h for x in insts]))
    E0 = B.contract(plan, J, h).cpu().numpy()
    bits, ms = B.autotune(plan, J, h)
    assert 7 <= bits <= 14 and ms > 0
    E1, sig, _, _ = B.backward(plan, J, h)
    assert np.array_equal(E0, E1.cpu().numpy())
    say("autotune backward square10 gauss batch 8")
    bits2, ms2 = B.autotune(plan, J, h, config=True)
    assert 7 <= bits2 <= 14 and ms2 > 0
    E2, sig2, _, _ = B.backward(plan, J, h)
    assert np.array_equal(E0, E2.cpu().numpy())
    with pytest.raises(ValueError):
        B.autotune(plan, J, h, count=True, config=True)
    say("autotune count reg3 n=24")
    rng = np.random.default_rng(5)
    e = I.random_regular(24, 3, rng)
    Jp = I.pm1(len(e), rng)
    cplan = B.Plan(24, e, seed=1)
    Ec0, res0, _ = B.count(cplan, dev(Jp[None]))
    cbits, _ = B.autotune(cplan, dev(Jp[None]), count=True)
    assert 7 <= cbits <= 12
    Ec1, res1, _ = B.count(cplan, dev(Jp[None]))
    assert Ec0[0] == Ec1[0] and np.array_equal(res0, res1)


# ----------------------------------------------------------------------------
# full size: 32 x 32 random +-J (the counting workload) -- properties that
# hold at any size: forward energy = counting energy, g even (spin flip at
# h = 0), E* and the residues unchanged by a gauge transform
# ----------------------------------------------------------------------------
def test_square32_random_pm1_count_properties():
    x = I.config_instances(2)[0]
    L = 32
    tau = (2 * np.random.default_rng(78).integers(0, 2, L * L) - 1).astype(np.int8)
    xg = I.gauge(x, tau)
    plan = B.Plan(L * L, x.edges, order=list(range(L * L)))
    say("square32 pm1: contract")
    E = B.contract(plan, dev(x.J[None])).cpu().numpy()[0]
    say("square32 pm1: count")
    Ec, res, g = B.count(plan, dev(x.J[None]))
    say("square32 pm1: count gauged")
    Eg, resg, gg = B.count(plan, dev(xg.J[None]))
    plan.close()
    assert Ec[0] == E and Eg[0] == E
    assert np.array_equal(res, resg) and g[0] == gg[0]
    assert g[0] % 2 == 0 and g[0] >= 2

"""GPU tests of the backward with recomputed pass inputs (Sec. IV: trading
time for memory by checkpointing): a device budget too small for every pass
input makes tt_backward keep a few snapshots and recompute the rest segment by
segment. The walk is the same computation, so sigma, the gradients and E*
must equal those of the store-everything path bit for bit, at every number of
snapshots, including none (one pass at a time, each recomputed from the start).
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


def widest(batch, width, esz=4):
    """Bytes of one state of the widest pass (256-byte aligned): width is log2
    of the entries stored per instance, esz the bytes of one entry."""
    return ((batch << width) * esz + 255) & ~255


def solve(L, insts, tile, max_bytes=0):
    n = L * L
    has_h = insts[0].h is not None
    plan = B.Plan(n, insts[0].edges, order=list(range(n)), has_field=has_h, tile_bits=tile, max_bytes=max_bytes,
                  parts=1)
    J = dev(np.stack([x.J for x in insts]))
    h = dev(np.stack([x.h for x in insts])) if has_h else None
    E, sig, dJ, dh = B.backward(plan, J, h)
    out = [E.cpu().numpy(), sig.cpu().numpy(), dJ.cpu().numpy(), None if dh is None else dh.cpu().numpy()]
    return plan, out


@pytest.mark.parametrize("snapshots", [0, 1, 3, 6])
def test_recompute_20x20_gauss_identical_to_store_all(snapshots):
    L, batch = 20, 2
    insts = I.config_instances(1, batch=batch, L=L)
    ref_plan, ref = solve(L, insts, 12)
    info = ref_plan.info()
    budget = (snapshots + 2) * widest(batch, info["width"])
    say("recompute 20x20 gauss, passes", info["n_passes"], "snapshots", snapshots, "budget", budget)
    _, got = solve(L, insts, 12, max_bytes=budget)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    for k, x in enumerate(insts):
        o = O.eliminate(L * L, x.edges, x.J, x.h, order=list(range(L * L)))
        assert np.array_equal(got[1][k], o["sigma"]) and abs(got[0][k] - o["energy"]) <= 1e-5 * L * L


@pytest.mark.parametrize("snapshots", [0, 2, 5])
def test_recompute_many_passes_pm1(snapshots):
    # 14 x 14 at tile 2^8: 91 passes, several levels of splitting
    L, batch = 14, 3
    insts = I.config_instances(0, batch=batch, L=L)
    ref_plan, ref = solve(L, insts, 8)
    info = ref_plan.info()
    say("recompute 14x14 pm1, passes", info["n_passes"], "snapshots", snapshots)
    _, got = solve(L, insts, 8, max_bytes=(snapshots + 2) * widest(batch, info["width"]))
    for a, b in zip(ref[:3], got[:3]):
        assert np.array_equal(a, b)
    for k, x in enumerate(insts):
        assert O.energy(L * L, x.edges, x.J, None, got[1][k]) == got[0][k]


def test_recompute_budget_below_two_states_rejected():
    insts = I.config_instances(0, batch=1, L=10)
    plan = B.Plan(100, insts[0].edges, order=list(range(100)), max_bytes=widest(1, 10))
    with pytest.raises(B.TTError) as ei:
        B.backward(plan, dev(insts[0].J[None]))
    assert ei.value.code == B.TT_E_TOOBIG


def test_square32_pm1_ground_state_by_recomputation():
    # every pass input of the 32 x 32 sweep would need about 2 TB; with snapshots
    # the ground state fits the GPU
    x = I.config_instances(2)[0]
    plan = B.Plan(1024, x.edges, order=list(range(1024)))
    J = dev(x.J[None])
    say("square32 pm1 energy")
    E0 = B.contract(plan, J).cpu().numpy()[0]
    say("square32 pm1 backward with recomputation")
    E, sig, dJ, _ = B.backward(plan, J)
    E, s = E.cpu().numpy()[0], sig.cpu().numpy()[0]
    assert E == E0
    assert O.energy(1024, x.edges, x.J, None, s) == E0 and O.energy(1024, x.edges, x.J, None, -s) == E0
    assert np.array_equal(dJ.cpu().numpy()[0], O.ground_state_gradient(x.edges, s)[0].astype(np.float32))


@pytest.mark.parametrize("snapshots", [0, 2, 5])
@pytest.mark.parametrize("kind", ["half", "int16", "half_int16"])
def test_recompute_half_state_and_int16(kind, snapshots):
    # half-state plans (h = 0: half of every state stored) and int16 states:
    # snapshots of the stored entries in the state's element type; the walk is
    # that of the store-all backward of the same plan and dtype
    L, batch = 14, 3
    n = L * L
    z2, i16 = kind.startswith("half"), kind.endswith("int16")
    insts = I.config_instances(0, batch=batch, L=L)
    J = np.stack([x.J for x in insts])
    Jd = dev(J.astype(np.int16)) if i16 else dev(J)

    def run(max_bytes):
        plan = B.Plan(n, insts[0].edges, order=list(range(n)), tile_bits=8, parts=1, z2=z2, max_bytes=max_bytes)
        return plan, [t.cpu().numpy() for t in B.backward(plan, Jd)[:3]]

    ref_plan, ref = run(0)
    info = ref_plan.info()
    per = widest(batch, info["width"] - (1 if z2 else 0), 2 if i16 else 4)
    say("recompute 14x14 pm1", kind, "passes", info["n_passes"], "snapshots", snapshots, "state bytes", per)
    _, got = run((snapshots + 2) * per)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    full = B.Plan(n, insts[0].edges, order=list(range(n)), tile_bits=8)
    E32 = B.contract(full, dev(J)).cpu().numpy()
    assert np.array_equal(got[0], E32)
    for k, x in enumerate(insts):
        assert O.energy(n, x.edges, x.J, None, got[1][k]) == got[0][k]
        assert np.array_equal(got[2][k], O.ground_state_gradient(x.edges, got[1][k])[0].astype(np.float32))


def test_square32_pm1_ground_state_half_state_int16_by_recomputation():
    # the half-state plan with int16 couplings keeps snapshots of 4 GiB (2^31
    # stored entries of two bytes) instead of 16 GiB
    x = I.config_instances(2)[0]
    say("square32 pm1 energy, full state, float32 couplings")
    E32 = B.contract(B.Plan(1024, x.edges, order=list(range(1024))), dev(x.J[None])).cpu().numpy()[0]
    plan = B.Plan(1024, x.edges, order=list(range(1024)), z2=True)
    J = dev(x.J[None].astype(np.int16))
    say("square32 pm1 backward with recomputation, half state, int16")
    E, sig, dJ, _ = B.backward(plan, J)
    E, s = E.cpu().numpy()[0], sig.cpu().numpy()[0]
    assert E == E32
    assert O.energy(1024, x.edges, x.J, None, s) == E32 and O.energy(1024, x.edges, x.J, None, -s) == E32
    assert np.array_equal(dJ.cpu().numpy()[0], O.ground_state_gradient(x.edges, s)[0].astype(np.float32))
    # a second call keeps the snapshot buffer the first one allocated: same results
    say("square32 pm1 backward with recomputation, second call")
    E2, sig2, dJ2, _ = B.backward(plan, J)
    assert E2.cpu().numpy()[0] == E and np.array_equal(sig2.cpu().numpy()[0], s)
    assert np.array_equal(dJ2.cpu().numpy(), dJ.cpu().numpy())

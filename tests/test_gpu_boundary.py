"""GPU tests of the C-ABI's error paths and count guard, and of the
torch.autograd.Function over tt_backward.

Every error here is forced from the host side (inputs the device check or the
host check rejects); the kernels themselves always run to completion.
"""
import ctypes as C
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
from paper_2008_06888_amd.autograd import ground_state_energy  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), device=DEV)


# ----------------------------------------------------------------------------
# input checks: non-finite couplings / fields, integer range
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("what", ["nan_J", "inf_J", "ninf_h", "nan_h"])
def test_nonfinite_inputs_rejected(what):
    say("nonfinite", what)
    insts = I.config_instances(1, batch=4, L=6)
    plan = B.Plan(36, insts[0].edges, order=list(range(36)), has_field=True, tile_bits=7)
    J = np.stack([x.J for x in insts])
    h = np.stack([x.h for x in insts])
    if what == "nan_J":
        J[2, 5] = np.nan
    elif what == "inf_J":
        J[0, 0] = np.inf
    elif what == "ninf_h":
        h[3, 7] = -np.inf
    else:
        h[1, 35] = np.nan
    Jd, hd = dev(J), dev(h)
    for call in (lambda: B.contract(plan, Jd, hd), lambda: B.backward(plan, Jd, hd)):
        with pytest.raises(B.TTError) as ei:
            call()
        assert ei.value.code == B.TT_E_INVAL and "finite" in str(ei.value)
    # the library stays usable: the same call on valid inputs is correct
    J2 = dev(np.stack([x.J for x in insts]))
    h2 = dev(np.stack([x.h for x in insts]))
    E = B.contract(plan, J2, h2).cpu().numpy()
    for b, x in enumerate(insts):
        ref = O.eliminate(36, x.edges, x.J, x.h, order=list(range(36)))
        assert abs(E[b] - ref["energy"]) <= 1e-5 * 36


def test_int32_range_rejected():
    say("int32 range")
    e = I.square_lattice(4)
    plan = B.Plan(16, e, order=list(range(16)))
    J = np.ones((2, len(e)), np.int32)
    J[1, :] = 1 << 20                       # 24 edges x 2^20 >= 2^24
    for call in (lambda: B.contract(plan, dev(J)), lambda: B.backward(plan, dev(J)), lambda: B.count(plan, dev(J))):
        with pytest.raises(B.TTError) as ei:
            call()
        assert ei.value.code == B.TT_E_RANGE
    J[1, :] = (1 << 24) // len(e) - 1       # just inside the exact range
    E = B.contract(plan, dev(J)).cpu().numpy()
    assert E[0] == -len(e) and E[1] == -len(e) * ((1 << 24) // len(e) - 1)


def test_uneven_batch_input_checks():
    say("uneven nonfinite")
    small = []
    for b, n in enumerate([12, 16, 20]):
        rng = np.random.default_rng([42, b])
        small.append(I.make(I.random_regular(n, 3, rng), n, rng, "gauss"))
    plans = [B.Plan(x.n, x.edges, seed=1, trials=4, tile_bits=7) for x in small]
    Js = [dev(x.J) for x in small]
    Js[2][3] = float("nan")
    with pytest.raises(B.TTError) as ei:
        B.contract_uneven(plans, Js)
    assert ei.value.code == B.TT_E_INVAL and "instance 2" in str(ei.value)


def test_budget_exceeded_before_device_work():
    say("TT_E_TOOBIG")
    insts = I.config_instances(1, batch=2, L=8)
    plan = B.Plan(64, insts[0].edges, order=list(range(64)), has_field=True, max_bytes=1 << 10)
    J, h = dev(np.stack([x.J for x in insts])), dev(np.stack([x.h for x in insts]))
    for call in (lambda: B.contract(plan, J, h), lambda: B.backward(plan, J, h)):
        with pytest.raises(B.TTError) as ei:
            call()
        assert ei.value.code == B.TT_E_TOOBIG


# ----------------------------------------------------------------------------
# count guard (Eq. 4 counts are unbounded; residues are exact below ~2^183)
# ----------------------------------------------------------------------------
def test_count_exact_below_182_spins():
    say("count 8x8 J=0")
    L = 8
    e = I.square_lattice(L)
    plan = B.Plan(L * L, e, order=list(range(L * L)), count_tile_bits=7)
    Ec, res, g, ex = B.count_with_flags(plan, dev(np.zeros((1, len(e)), np.int32)))
    assert Ec[0] == 0 and g[0] == 2 ** 64 and ex[0]


@pytest.mark.parametrize("case", ["path200_zero", "path200_pm1", "tree300_pm1"])
def test_count_guard_beyond_182_spins(case):
    say("count guard", case)
    rng = np.random.default_rng([43, len(case)])
    if case.startswith("path"):
        n, e = 200, I.path(200)
    else:
        n, e = 300, I.random_tree(300, rng)
    J = np.zeros(len(e), np.int32) if case.endswith("zero") else I.pm1(len(e), rng)
    plan = B.Plan(n, e, seed=1, trials=2, count_tile_bits=8)
    Ec, res, g, ex = B.count_with_flags(plan, dev(J[None]))
    if case.endswith("zero"):
        M = int(np.prod([int(p) for p in B.moduli()], dtype=object))
        assert Ec[0] == 0 and not ex[0]
        assert g[0] == (2 ** n) % M          # only g mod M is known
        with pytest.raises(B.TTError) as ei:  # strict mode refuses it
            B.count(plan, dev(J[None]))
        assert ei.value.code == B.TT_E_COUNT_OVERFLOW
    else:
        # a tree at h = 0 has no frustration: E* = -sum |J|, g = 2
        assert Ec[0] == -int(np.abs(J).sum()) and ex[0] and g[0] == 2


def test_count_guard_square32_zero_couplings():
    """32 x 32, J = 0: E* = 0 and g = 2^1024, far beyond the moduli."""
    say("count guard 32x32 J=0")
    L = 32
    e = I.square_lattice(L)
    plan = B.Plan(L * L, e, order=list(range(L * L)))
    Ec, res, g, ex = B.count_with_flags(plan, dev(np.zeros((1, len(e)), np.int32)))
    plan.close()
    assert Ec[0] == 0 and not ex[0]


# ----------------------------------------------------------------------------
# torch.autograd.Function: E* as a function of J and h
# ----------------------------------------------------------------------------
def test_autograd_ground_state_energy():
    say("autograd 6x6 gauss + h")
    insts = I.config_instances(1, batch=4, L=6)
    n = 36
    plan = B.Plan(n, insts[0].edges, order=list(range(n)), has_field=True, tile_bits=7)
    J = dev(np.stack([x.J for x in insts])).requires_grad_(True)
    h = dev(np.stack([x.h for x in insts])).requires_grad_(True)
    w = torch.tensor([1.0, -2.0, 0.5, 3.0], dtype=torch.float64, device=DEV)
    E = ground_state_energy(J, h, plan)
    (w * E).sum().backward()
    Jg, hg = J.grad.cpu().numpy(), h.grad.cpu().numpy()
    for b, x in enumerate(insts):
        ref = O.eliminate(n, x.edges, x.J, x.h, order=list(range(n)))
        assert abs(E[b].item() - ref["energy"]) <= 1e-5 * n
        gJ, gh = O.ground_state_gradient(x.edges, ref["sigma"])
        assert np.array_equal(Jg[b], (w[b].item() * gJ).astype(np.float32))
        assert np.array_equal(hg[b], (w[b].item() * gh).astype(np.float32))


def test_autograd_without_fields():
    say("autograd 5x5 pm1 (float) h = 0")
    insts = I.config_instances(0, batch=3, L=5)
    n = 25
    plan = B.Plan(n, insts[0].edges, order=list(range(n)), tile_bits=7)
    J = dev(np.stack([x.J for x in insts]).astype(np.float32)).requires_grad_(True)
    E = ground_state_energy(J, None, plan)
    E.sum().backward()
    for b, x in enumerate(insts):
        sig = -J.grad[b].cpu().numpy()          # -dE/dJ_ij = sigma_i sigma_j of the returned state
        assert np.all(np.abs(sig) == 1)
        ref = O.eliminate(n, x.edges, x.J, None, counts="exact")
        assert E[b].item() == ref["energy"]

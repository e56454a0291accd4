"""GPU test of the allocation-free contraction (tt_contract_noalloc) against
tt_contract, called through the C-ABI on the same inputs.

Two calls in a row share the one per-GPU workspace, the second with a smaller
input (fewer instances of a smaller graph), so a stale region left by the first
call would show. The energies must equal tt_contract's exactly (same kernels,
same per-instance arithmetic: every max is exact and every sum is taken in the
same order) and the float64 oracle's within 1e-5 N.
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

DEV = "cuda:0"


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), device=DEV)


def noalloc(plan, J, h, out):
    """The entry point itself, through ctypes (no binding logic in between)."""
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    dt = B.TT_F32 if J.dtype == torch.float32 else B.TT_I32
    hp = None if h is None else C.c_void_p(h.data_ptr())
    return B._lib.tt_contract_noalloc(plan.handle, J.shape[0], dt, C.c_void_p(J.data_ptr()), hp,
                                      C.c_void_p(out.data_ptr()), stream)


def run_case(L, batch, coupling, tile_bits):
    n = L * L
    insts = I.config_instances(1 if coupling == "gauss" else 0, batch=batch, L=L)
    has_h = insts[0].h is not None
    plan = B.Plan(n, insts[0].edges, order=list(range(n)), has_field=has_h, tile_bits=tile_bits)
    J = dev(np.stack([x.J for x in insts]))
    h = dev(np.stack([x.h for x in insts])) if has_h else None
    out = torch.full((batch,), float("nan"), dtype=torch.float64, device=DEV)
    say("noalloc", coupling, f"{L}x{L}", "batch", batch, "tile", tile_bits, "width", plan.info()["width"])
    assert noalloc(plan, J, h, out) == B.TT_OK, B.last_error()
    ref = B.contract(plan, J, h)
    torch.cuda.synchronize()
    E, Er = out.cpu().numpy(), ref.cpu().numpy()
    assert np.array_equal(E, Er), (E, Er)
    for b in (0, batch - 1):
        x = insts[b]
        Eo = O.eliminate(n, x.edges, x.J, x.h, order=list(range(n)), traceback=False)["energy"]
        assert abs(E[b] - Eo) <= 1e-5 * n, (b, E[b], Eo)
    return E


def test_noalloc_matches_contract_twice_second_smaller():
    # 16x16 Gaussian with fields, 48 instances (24 MiB of state), then 10x10 +-J, 5 instances
    run_case(16, 48, "gauss", 12)
    run_case(10, 5, "pm1", 9)
    # and once more at the first size: the smaller call's leftovers must not matter either
    run_case(16, 48, "gauss", 12)


def test_noalloc_rejects_a_batch_beyond_the_workspace():
    insts = I.config_instances(0, batch=2, L=16)
    plan = B.Plan(256, insts[0].edges, order=list(range(256)))
    batch = (B.NOALLOC_MAX_BYTES // (2 * 4 << 16)) + 1      # two states of batch x 2^16 floats
    J = dev(np.tile(insts[0].J, (batch, 1)))
    out = torch.empty(batch, dtype=torch.float64, device=DEV)
    say("noalloc too big, batch", batch)
    assert noalloc(plan, J, None, out) == B.TT_E_TOOBIG
    assert "workspace" in B.last_error()
    # the same plan still works at a size that fits
    run_case(16, 4, "pm1", 12)


def test_noalloc_input_checks():
    insts = I.config_instances(1, batch=3, L=6)
    plan = B.Plan(36, insts[0].edges, order=list(range(36)), has_field=True, tile_bits=7)
    J = np.stack([x.J for x in insts])
    h = np.stack([x.h for x in insts])
    J[1, 3] = np.nan
    out = torch.empty(3, dtype=torch.float64, device=DEV)
    say("noalloc nonfinite")
    assert noalloc(plan, dev(J), dev(h), out) == B.TT_E_INVAL
    J[1, 3] = 0.5
    assert noalloc(plan, dev(J), dev(h), out) == B.TT_OK

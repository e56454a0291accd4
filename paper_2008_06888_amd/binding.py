"""ctypes binding of libtt.so (C-ABI in include/tt.h). Argument marshalling only.

Every compute step runs inside the HIP library; this module only converts
torch tensors (device memory and the current stream) into pointers. If the
library has not been built, importing this module raises: there is no
fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np
# torch first: its HIP and HSA runtime libraries then satisfy the library's
# dependencies, so the process holds one runtime. Loading the library first
# would bring in a second HIP/HSA runtime beside torch's, and the second one
# to initialise finds no device.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtt.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2008_06888_amd.build`")

_lib = C.CDLL(LIB_PATH)

TT_OK = 0
TT_E_INVAL, TT_E_DTYPE, TT_E_RANGE, TT_E_TOOBIG = -1, -2, -3, -4
TT_E_COUNT_OVERFLOW, TT_E_DEVICE, TT_E_NOMEM = -5, -6, -7
TT_F32, TT_I32, TT_I16 = 0, 1, 2
NOALLOC_MAX_BYTES = 64 << 20      # workspace of tt_contract_noalloc per GPU (TT_NOALLOC_MAX_BYTES)
ORDER_GREEDY, ORDER_GIVEN, ORDER_CHIMERA = 0, 1, 2

#: every symbol the header declares (checked by the CPU tests)
EXPORTS = ("tt_plan_create", "tt_plan_info", "tt_plan_order", "tt_plan_destroy", "tt_contract",
           "tt_backward", "tt_count", "tt_count_moduli", "tt_count_to_decimal", "tt_contract_uneven",
           "tt_prof_enable", "tt_prof_reset", "tt_prof_read", "tt_last_error", "tt_plan_ops",
           "tt_plan_program", "tt_graphs_enable", "tt_tgemm", "tt_plan_autotune", "tt_contract_noalloc",
           "tt_potts_contract", "tt_potts_count", "tt_backward_tie", "tt_config_fd",
           "tt_sample_ground_state", "tt_count_log", "tt_contract_uneven_fields", "tt_plan_create_sliced",
           "tt_plan_slice_info")


class PlanOpts(C.Structure):
    _fields_ = [("kind", C.c_int32), ("order", C.POINTER(C.c_int32)), ("seed", C.c_uint64),
                ("trials", C.c_int32), ("has_field", C.c_int32), ("tile_bits", C.c_int32),
                ("count_tile_bits", C.c_int32), ("chimera_rows", C.c_int32),
                ("chimera_cols", C.c_int32), ("max_bytes", C.c_int64), ("parts", C.c_int32),
                ("q", C.c_int32), ("z2", C.c_int32)]


class PlanStats(C.Structure):
    _fields_ = [("n_spins", C.c_int32), ("n_edges", C.c_int64), ("width", C.c_int32),
                ("n_ops", C.c_int32), ("n_passes", C.c_int32), ("n_count_passes", C.c_int32),
                ("terms", C.c_double), ("elementwise", C.c_double), ("reduce_ops", C.c_double),
                ("entry_updates", C.c_double), ("parts", C.c_int32)]


_vp = C.c_void_p
_lib.tt_plan_create.argtypes = [C.c_int32, C.c_int64, _vp, C.POINTER(PlanOpts), C.POINTER(_vp)]
_lib.tt_plan_create_sliced.argtypes = [C.c_int32, C.c_int64, _vp, C.POINTER(PlanOpts), C.c_int32, _vp,
                                       C.POINTER(_vp)]
_lib.tt_plan_slice_info.argtypes = [_vp, _vp]
_lib.tt_plan_info.argtypes = [_vp, C.POINTER(PlanStats)]
_lib.tt_plan_order.argtypes = [_vp, _vp]
_lib.tt_plan_ops.argtypes = [_vp, _vp, C.c_int64, _vp, _vp]
_lib.tt_plan_program.argtypes = [_vp, C.c_int32, _vp, C.c_int64]
_lib.tt_plan_program.restype = C.c_int64
_lib.tt_plan_destroy.argtypes = [_vp]
_lib.tt_plan_destroy.restype = None
_lib.tt_contract.argtypes = [_vp, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp]
_lib.tt_contract_noalloc.argtypes = [_vp, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp]
_lib.tt_backward.argtypes = [_vp, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.tt_count.argtypes = [_vp, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.tt_backward_tie.argtypes = [_vp, C.c_int32, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, C.c_uint64, _vp]
_lib.tt_config_fd.argtypes = [_vp, _vp, _vp, C.c_double, _vp, _vp, _vp, _vp]
_lib.tt_sample_ground_state.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.tt_count_log.argtypes = [_vp, _vp]
_lib.tt_potts_contract.argtypes = [_vp, C.c_int32, C.c_int32, _vp, _vp, _vp]
_lib.tt_potts_count.argtypes = [_vp, C.c_int32, _vp, _vp, _vp, _vp, _vp]
_lib.tt_count_moduli.argtypes = [_vp]
_lib.tt_count_to_decimal.argtypes = [_vp, C.c_char_p, C.c_size_t]
_lib.tt_contract_uneven.argtypes = [C.c_int32, _vp, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
_lib.tt_prof_enable.argtypes = [C.c_int32]
_lib.tt_graphs_enable.argtypes = [C.c_int32]
_lib.tt_contract_uneven_fields.argtypes = [C.c_int32, _vp, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                           _vp]
_lib.tt_tgemm.argtypes = [C.c_int32, C.c_int64, C.c_int64, C.c_int64, _vp, C.c_int64, C.c_int64, _vp, C.c_int64,
                          C.c_int64, _vp, C.c_int64, C.c_int64, _vp]
_lib.tt_plan_autotune.argtypes = [_vp, C.c_int32, C.c_int32, _vp, _vp, C.c_int32, _vp, _vp, _vp]
_lib.tt_prof_read.argtypes = [C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
_lib.tt_last_error.restype = C.c_char_p


class TTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tt error {code}: {msg}")
        self.code = code


def last_error() -> str:
    """Message of the last failed call on this thread."""
    return _lib.tt_last_error().decode()


def _check(code: int):
    if code != TT_OK:
        raise TTError(code, _lib.tt_last_error().decode())


def lib():
    return _lib


class Plan:
    """A contraction plan (host object owned by the library)."""

    def __init__(self, n: int, edges, *, order: Optional[Sequence[int]] = None, kind: Optional[int] = None,
                 has_field: bool = False, seed: int = 0, trials: int = 32, tile_bits: int = 0,
                 count_tile_bits: int = 0, chimera: Optional[tuple] = None, max_bytes: int = 0,
                 parts: int = 0, q: int = 2, n_fixed: int = 0, fixed: Optional[Sequence[int]] = None,
                 z2: bool = False):
        """n_fixed / fixed: a sliced plan (tt_plan_create_sliced) with that many
        fixed spins, given or (fixed None) chosen by the planner."""
        self.n = int(n)
        self.edges = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
        self.m = int(self.edges.shape[0])
        self.has_field = bool(has_field)
        o = PlanOpts()
        if kind is None:
            kind = ORDER_GIVEN if order is not None else (ORDER_CHIMERA if chimera else ORDER_GREEDY)
        o.kind = kind
        self._order_buf = None
        if order is not None:
            self._order_buf = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
            o.order = self._order_buf.ctypes.data_as(C.POINTER(C.c_int32))
        o.seed, o.trials, o.has_field = seed, trials, int(has_field)
        o.tile_bits, o.count_tile_bits, o.max_bytes, o.parts = tile_bits, count_tile_bits, max_bytes, parts
        if chimera:
            o.chimera_rows, o.chimera_cols = chimera
        o.q = q
        o.z2 = int(bool(z2))
        self.q = q
        h = _vp()
        if fixed is not None or n_fixed:
            fx = None if fixed is None else np.ascontiguousarray(np.asarray(fixed, dtype=np.int32))
            nf = int(n_fixed) if fx is None else int(fx.size)
            _check(_lib.tt_plan_create_sliced(self.n, self.m, self.edges.ctypes.data, C.byref(o), nf,
                                              None if fx is None else fx.ctypes.data, C.byref(h)))
        else:
            _check(_lib.tt_plan_create(self.n, self.m, self.edges.ctypes.data, C.byref(o), C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        s = PlanStats()
        _check(_lib.tt_plan_info(self._h, C.byref(s)))
        return {f: getattr(s, f) for f, _ in PlanStats._fields_}

    def order(self) -> np.ndarray:
        out = np.zeros(self.n, np.int32)
        _check(_lib.tt_plan_order(self._h, out.ctypes.data))
        return out

    def fixed(self) -> np.ndarray:
        """Fixed spins of a sliced plan (empty when unsliced)."""
        k = _lib.tt_plan_slice_info(self._h, None)
        if k < 0:
            _check(k)
        out = np.zeros(max(k, 1), np.int32)
        _lib.tt_plan_slice_info(self._h, out.ctypes.data)
        return out[:k]

    def ops(self):
        """(ops int32 [n_ops, 8], final_slot_spin int32 [final_width]); see tt_plan_ops."""
        n = _lib.tt_plan_ops(self._h, None, 0, None, None)
        if n < 0:
            _check(n)
        out = np.zeros((max(n, 1), 8), np.int32)
        fw = C.c_int32()
        _lib.tt_plan_ops(self._h, out.ctypes.data, n, None, C.byref(fw))
        fs = np.zeros(max(fw.value, 1), np.int32)
        _lib.tt_plan_ops(self._h, out.ctypes.data, n, fs.ctypes.data, C.byref(fw))
        return out[:n], fs[:fw.value]

    def program(self, which: int) -> bytes:
        """Raw bytes of one part of the encoded energy program (see tt_plan_program)."""
        n = _lib.tt_plan_program(self._h, which, None, 0)
        if n < 0:
            _check(int(n))
        buf = C.create_string_buffer(max(int(n), 1))
        _lib.tt_plan_program(self._h, which, buf, n)
        return buf.raw[:n]

    def close(self):
        if getattr(self, "_h", None):
            _lib.tt_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def moduli() -> List[int]:
    buf = (C.c_uint64 * 3)()
    _check(_lib.tt_count_moduli(buf))
    return [int(x) for x in buf]


def residues_to_int(res) -> int:
    arr = (C.c_uint64 * 3)(*[int(x) for x in res])
    buf = C.create_string_buffer(128)
    _check(_lib.tt_count_to_decimal(arr, buf, 128))
    return int(buf.value.decode())


# ---------------------------------------------------------------------------
# compute calls (torch tensors on the current HIP device)
# ---------------------------------------------------------------------------

def count_log(res) -> float:
    """ln g from the three residues of a count (the residual entropy is ln g / n)."""
    r = np.ascontiguousarray(np.asarray(res, dtype=np.uint64).reshape(3))
    out = C.c_double()
    _check(_lib.tt_count_log(r.ctypes.data, C.byref(out)))
    return out.value


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return TT_F32
    if t.dtype == torch.int32:
        return TT_I32
    if t.dtype == torch.int16:
        return TT_I16
    raise TypeError(f"J must be float32, int32 or int16, got {t.dtype}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_inputs(plan: Plan, J, h):
    if not J.is_cuda or not J.is_contiguous() or J.dim() != 2 or J.shape[1] != plan.m:
        raise ValueError(f"J must be a contiguous device tensor [batch, {plan.m}]")
    if plan.has_field:
        if h is None or not h.is_cuda or not h.is_contiguous() or tuple(h.shape) != (J.shape[0], plan.n) \
                or h.dtype != J.dtype:
            raise ValueError(f"h must be a contiguous device tensor [batch, {plan.n}] of J's dtype")
    elif h is not None:
        raise ValueError("plan was built without fields")


def contract(plan: Plan, J, h=None):
    """E* of every instance (device float64 [batch])."""
    torch = _torch()
    _check_inputs(plan, J, h)
    B = J.shape[0]
    energy = torch.empty(B, dtype=torch.float64, device=J.device)
    _check(_lib.tt_contract(plan.handle, B, _dtype_code(J), _ptr(J), _ptr(h), _ptr(energy), _stream()))
    return energy


def contract_noalloc(plan: Plan, J, h=None, out=None):
    """E* through the allocation-free entry point (its workspace is the
    library's fixed per-GPU array); ``out`` (device float64 [batch]) may be
    given so that the call allocates nothing at all. Returns after the stream
    has synchronised."""
    torch = _torch()
    _check_inputs(plan, J, h)
    B = J.shape[0]
    energy = out if out is not None else torch.empty(B, dtype=torch.float64, device=J.device)
    if energy.dtype != torch.float64 or not energy.is_cuda or energy.numel() < B or not energy.is_contiguous():
        raise ValueError("out must be a contiguous device float64 tensor of at least batch entries")
    _check(_lib.tt_contract_noalloc(plan.handle, B, _dtype_code(J), _ptr(J), _ptr(h), _ptr(energy), _stream()))
    return energy[:B]


def backward_tie(plan: Plan, J, h=None, tie: int = 1, want_grad: bool = True):
    """tt_backward with another tie rule (1: the last maximiser, other: pseudo-random per pass)."""
    torch = _torch()
    _check_inputs(plan, J, h)
    B = J.shape[0]
    dev = J.device
    energy = torch.empty(B, dtype=torch.float64, device=dev)
    sigma = torch.empty(B, plan.n, dtype=torch.int8, device=dev)
    dJ = torch.empty(B, plan.m, dtype=torch.float32, device=dev) if want_grad else None
    dh = torch.empty(B, plan.n, dtype=torch.float32, device=dev) if (want_grad and plan.has_field) else None
    _check(_lib.tt_backward_tie(plan.handle, B, _dtype_code(J), _ptr(J), _ptr(h), _ptr(energy), _ptr(sigma),
                                _ptr(dJ), _ptr(dh), int(tie), _stream()))
    return energy, sigma, dJ, dh


def config_fd(plan: Plan, J, h=None, delta: float = 2.0 ** -5):
    """(E*, sigma, consistent) of one float32 instance by finite differences of the fields."""
    torch = _torch()
    if J.dim() != 1 or J.dtype != torch.float32 or not J.is_cuda or J.shape[0] != plan.m:
        raise ValueError(f"J must be a device float32 tensor [{plan.m}]")
    if h is not None and (h.dim() != 1 or h.dtype != torch.float32 or h.shape[0] != plan.n):
        raise ValueError(f"h must be a device float32 tensor [{plan.n}]")
    energy = torch.empty(1, dtype=torch.float64, device=J.device)
    sigma = torch.empty(plan.n, dtype=torch.int8, device=J.device)
    ok = C.c_uint8(0)
    _check(_lib.tt_config_fd(plan.handle, _ptr(J), _ptr(h), float(delta), _ptr(energy), _ptr(sigma),
                             C.byref(ok), _stream()))
    return energy, sigma, bool(ok.value)


def sample_ground_state(plan: Plan, J, h=None, u=None):
    """(E*, sigma int8 numpy [n]) drawn uniformly from the ground states; u: n numbers in [0, 1)."""
    torch = _torch()
    if J.dim() != 1 or J.dtype != torch.int32 or not J.is_cuda or J.shape[0] != plan.m:
        raise ValueError(f"J must be a device int32 tensor [{plan.m}]")
    u = np.ascontiguousarray(np.asarray(u, dtype=np.float64))
    if u.shape != (plan.n,):
        raise ValueError(f"u must hold {plan.n} numbers")
    sigma = np.zeros(plan.n, np.int8)
    energy = C.c_int64(0)
    _check(_lib.tt_sample_ground_state(plan.handle, _ptr(J), _ptr(h), u.ctypes.data, sigma.ctypes.data,
                                       C.byref(energy), _stream()))
    return energy.value, sigma


def _check_potts(plan: Plan, J):
    if plan.q != 3:
        raise ValueError("plan was not built for 3-state labels (q=3)")
    if not J.is_cuda or not J.is_contiguous() or J.dim() != 2 or J.shape[1] != plan.m:
        raise ValueError(f"J must be a contiguous device tensor [batch, {plan.m}]")


def potts_contract(plan: Plan, J):
    """Ground-state energy H* of 3-state Potts glasses (device float64 [batch])."""
    torch = _torch()
    _check_potts(plan, J)
    B = J.shape[0]
    energy = torch.empty(B, dtype=torch.float64, device=J.device)
    _check(_lib.tt_potts_contract(plan.handle, B, _dtype_code(J), _ptr(J), _ptr(energy), _stream()))
    return energy


def potts_count(plan: Plan, J, flags: bool = False):
    """(2H* int64 [batch], residues [batch, 3], g as Python ints[, exact flags]) for int32 couplings."""
    torch = _torch()
    _check_potts(plan, J)
    if J.dtype != torch.int32:
        raise TypeError("counting needs int32 couplings")
    B = J.shape[0]
    energy2 = np.zeros(B, np.int64)
    res = np.zeros((B, 3), np.uint64)
    exact = np.zeros(B, np.uint8)
    _check(_lib.tt_potts_count(plan.handle, B, _ptr(J), energy2.ctypes.data, res.ctypes.data,
                               exact.ctypes.data if flags else None, _stream()))
    g = [residues_to_int(r) for r in res]
    return (energy2, res, g, exact.astype(bool)) if flags else (energy2, res, g)


def backward(plan: Plan, J, h=None, want_grad: bool = True):
    """(E*, sigma, dE/dJ, dE/dh) with sigma int8 [batch, n] in {+1, -1}."""
    torch = _torch()
    _check_inputs(plan, J, h)
    B = J.shape[0]
    dev = J.device
    energy = torch.empty(B, dtype=torch.float64, device=dev)
    sigma = torch.empty(B, plan.n, dtype=torch.int8, device=dev)
    dJ = torch.empty(B, plan.m, dtype=torch.float32, device=dev) if want_grad else None
    dh = torch.empty(B, plan.n, dtype=torch.float32, device=dev) if (want_grad and plan.has_field) else None
    _check(_lib.tt_backward(plan.handle, B, _dtype_code(J), _ptr(J), _ptr(h), _ptr(energy), _ptr(sigma),
                            _ptr(dJ), _ptr(dh), _stream()))
    return energy, sigma, dJ, dh


def _count(plan: Plan, J, h, flags: bool):
    torch = _torch()
    _check_inputs(plan, J, h)
    if J.dtype != torch.int32:
        raise TypeError("counting needs int32 couplings")
    B = J.shape[0]
    energy = np.zeros(B, np.int64)
    res = np.zeros((B, 3), np.uint64)
    exact = np.zeros(B, np.uint8)
    _check(_lib.tt_count(plan.handle, B, _ptr(J), _ptr(h), energy.ctypes.data, res.ctypes.data,
                         exact.ctypes.data if flags else None, _stream()))
    return energy, res, [residues_to_int(r) for r in res], exact.astype(bool)


def count(plan: Plan, J, h=None):
    """(E* int64 numpy [batch], residues uint64 numpy [batch, 3], g as Python ints).

    Strict: raises TTError (TT_E_COUNT_OVERFLOW) when a count may exceed the
    product of the moduli instead of returning it modulo that product."""
    return _count(plan, J, h, False)[:3]


def count_with_flags(plan: Plan, J, h=None):
    """(E*, residues, g mod M as Python ints, exact bool numpy [batch]): g is exact where the flag is set."""
    return _count(plan, J, h, True)


def contract_uneven(plans: Sequence[Plan], J_list, want_sigma: bool = True):
    """Forward (+ backward) of instances with different graphs. J_list: device tensors [m_i]."""
    torch = _torch()
    n = len(plans)
    if n != len(J_list) or n == 0:
        raise ValueError("one J per plan")
    dt = J_list[0].dtype
    Jcat = torch.cat([j.reshape(-1) for j in J_list]).contiguous()
    j_off = np.zeros(n, np.int64)
    s_off = np.zeros(n, np.int64)
    for i in range(1, n):
        j_off[i] = j_off[i - 1] + plans[i - 1].m
        s_off[i] = s_off[i - 1] + plans[i - 1].n
    for p, j in zip(plans, J_list):
        if j.numel() != p.m or j.dtype != dt or p.has_field:
            raise ValueError("J sizes / dtypes must match the plans (no fields)")
    handles = (C.c_void_p * n)(*[p.handle for p in plans])
    energy = torch.empty(n, dtype=torch.float64, device=Jcat.device)
    sigma = torch.empty(int(sum(p.n for p in plans)), dtype=torch.int8, device=Jcat.device) if want_sigma else None
    dJ = torch.empty_like(Jcat, dtype=torch.float32) if want_sigma else None
    _check(_lib.tt_contract_uneven(n, handles, _dtype_code(Jcat), _ptr(Jcat), j_off.ctypes.data, _ptr(energy),
                                   _ptr(sigma), s_off.ctypes.data, _ptr(dJ), _stream()))
    if not want_sigma:
        return energy, None, None
    sig = [sigma[s_off[i]:s_off[i] + plans[i].n] for i in range(n)]
    dj = [dJ[j_off[i]:j_off[i] + plans[i].m] for i in range(n)]
    return energy, sig, dj


def contract_uneven_fields(plans: Sequence[Plan], J_list, h_list, want_sigma: bool = True):
    """contract_uneven with fields: h_list[i] is a device tensor [n_i] for plans with fields, else None.
    Returns (E*, sigma list, dE/dJ list, dE/dh list (None where a plan has no fields))."""
    torch = _torch()
    n = len(plans)
    if n != len(J_list) or n != len(h_list) or n == 0:
        raise ValueError("one J and one h (or None) per plan")
    dt = J_list[0].dtype
    Jcat = torch.cat([j.reshape(-1) for j in J_list]).contiguous()
    hs = [h.reshape(-1) for h in h_list if h is not None]
    hcat = torch.cat(hs).contiguous() if hs else None
    j_off, s_off, h_off = np.zeros(n, np.int64), np.zeros(n, np.int64), np.zeros(n, np.int64)
    hpos = 0
    for i in range(n):
        if i:
            j_off[i] = j_off[i - 1] + plans[i - 1].m
            s_off[i] = s_off[i - 1] + plans[i - 1].n
        p, j, h = plans[i], J_list[i], h_list[i]
        if j.numel() != p.m or j.dtype != dt or (h is not None) != p.has_field:
            raise ValueError("J / h sizes, dtypes and fields must match the plans")
        if h is not None:
            if h.numel() != p.n or h.dtype != dt:
                raise ValueError("h sizes / dtypes must match the plans")
            h_off[i] = hpos
            hpos += p.n
    handles = (C.c_void_p * n)(*[p.handle for p in plans])
    energy = torch.empty(n, dtype=torch.float64, device=Jcat.device)
    sigma = torch.empty(int(sum(p.n for p in plans)), dtype=torch.int8, device=Jcat.device) if want_sigma else None
    dJ = torch.empty_like(Jcat, dtype=torch.float32) if want_sigma else None
    dh = torch.empty_like(hcat, dtype=torch.float32) if (want_sigma and hcat is not None) else None
    _check(_lib.tt_contract_uneven_fields(n, handles, _dtype_code(Jcat), _ptr(Jcat), j_off.ctypes.data, _ptr(hcat),
                                          h_off.ctypes.data, _ptr(energy), _ptr(sigma), s_off.ctypes.data, _ptr(dJ),
                                          _ptr(dh), _stream()))
    if not want_sigma:
        return energy, None, None, None
    sig = [sigma[s_off[i]:s_off[i] + plans[i].n] for i in range(n)]
    dj = [dJ[j_off[i]:j_off[i] + plans[i].m] for i in range(n)]
    dhl = [dh[h_off[i]:h_off[i] + plans[i].n] if plans[i].has_field else None for i in range(n)]
    return energy, sig, dj, dhl


def tgemm(A, B, out=None):
    """Tropical product C = max_k A[..., i, k] + B[..., k, j] of float32 device tensors (2-D or batched 3-D)."""
    torch = _torch()
    if A.dtype != torch.float32 or B.dtype != torch.float32 or not (A.is_cuda and B.is_cuda):
        raise TypeError("tgemm takes float32 device tensors")
    batched = A.dim() == 3
    A3 = A if batched else A.unsqueeze(0)
    B3 = B if batched else B.unsqueeze(0)
    A3, B3 = A3.contiguous(), B3.contiguous()
    nb, M, K = A3.shape
    nb2, K2, N = B3.shape
    if nb != nb2 or K != K2:
        raise ValueError("shape mismatch")
    C3 = torch.empty(nb, M, N, dtype=torch.float32, device=A.device) if out is None else out.view(nb, M, N)
    _check(_lib.tt_tgemm(nb, M, N, K, _ptr(A3), K, M * K, _ptr(B3), N, K * N, _ptr(C3), N, M * N, _stream()))
    return C3 if batched else C3[0]


TUNE_ENERGY, TUNE_COUNT, TUNE_BACKWARD = 0, 1, 2


def autotune(plan: Plan, J, h=None, count: bool = False, config: bool = False):
    """Times every tile size on these instances and keeps the fastest in the plan; returns (bits, ms per call).

    Times the call the tiles are for: contract (default), count (count=True)
    or backward (config=True: energy, configuration and gradients)."""
    _check_inputs(plan, J, h)
    if count and config:
        raise ValueError("count and config exclude each other")
    if count and J.dtype != _torch().int32:
        raise TypeError("counting needs int32 couplings")
    mode = TUNE_COUNT if count else (TUNE_BACKWARD if config else TUNE_ENERGY)
    bits = C.c_int32(0)
    ms = C.c_double(0.0)
    _check(_lib.tt_plan_autotune(plan.handle, J.shape[0], _dtype_code(J), _ptr(J), _ptr(h), mode,
                                 C.byref(bits), C.byref(ms), _stream()))
    return bits.value, ms.value


def graphs_enable(on: bool = True):
    """Replay repeated calls as HIP graphs (default on)."""
    _check(_lib.tt_graphs_enable(1 if on else 0))


def prof_enable(on: bool = True):
    _check(_lib.tt_prof_enable(1 if on else 0))


def prof_reset():
    _check(_lib.tt_prof_reset())


def prof_read(name: str):
    ms = C.c_double()
    n = C.c_int64()
    _check(_lib.tt_prof_read(name.encode(), C.byref(ms), C.byref(n)))
    return ms.value, n.value

"""CPU tests of the C-ABI library: it loads, exports every declared symbol,
and its host-side planner and CRT helper behave (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2008_06888_amd import binding as B
from paper_2008_06888_amd import instances as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_header_symbol_is_exported():
    hdr = open(os.path.join(ROOT, "include", "tt.h")).read()
    declared = set(re.findall(r"^\s*(?:int64_t|int|void|const char\*)\s+(tt_\w+)\s*\(", hdr, re.M))
    assert declared == set(B.EXPORTS)
    for name in declared:
        assert hasattr(B.lib(), name), name


def test_moduli_and_crt():
    P = B.moduli()
    assert P == [2 ** 61 - 1, 2 ** 61 - 31, 2 ** 61 - 45]
    for x in [0, 1, 2 ** 64 + 3, 2 ** 150 + 12345, (P[0] * P[1] * P[2]) - 1]:
        assert B.residues_to_int([x % p for p in P]) == x


def test_square_lattice_sweep_width():
    for L in (4, 7, 16, 32):
        p = B.Plan(L * L, I.square_lattice(L), order=list(range(L * L)))
        info = p.info()
        assert info["width"] == L          # the 2^L state of Sec. V
        assert info["n_passes"] >= 1


def test_greedy_plan_is_a_permutation_and_deterministic():
    rng = np.random.default_rng(1)
    e = I.random_regular(60, 3, rng)
    a = B.Plan(60, e, seed=3, trials=8)
    b = B.Plan(60, e, seed=3, trials=8)
    assert sorted(a.order().tolist()) == list(range(60))
    assert a.order().tolist() == b.order().tolist()
    assert a.info()["width"] <= 14


def test_more_restarts_never_widen_the_plan():
    """The greedy restarts of one seed draw from one random stream, so the best
    of 512 includes the first 32 and the width can only fall; on the widest
    graphs of the uneven 3-regular workload (N = 220) it falls by two spins."""
    insts = I.config_instances(3)
    for i in (6, 13):
        x = insts[i]
        w32 = B.Plan(x.n, x.edges, seed=i, trials=32).info()["width"]
        w512 = B.Plan(x.n, x.edges, seed=i, trials=512).info()["width"]
        assert w512 <= w32 - 2 and w512 <= 30


@pytest.mark.parametrize("bad", [
    dict(edges=[[0, 0]]), dict(edges=[[1, 0]]), dict(edges=[[0, 5]]), dict(edges=[[0, 1], [0, 1]]),
])
def test_invalid_graphs_rejected(bad):
    with pytest.raises(B.TTError) as ei:
        B.Plan(3, np.array(bad["edges"]), order=[0, 1, 2])
    assert ei.value.code == B.TT_E_INVAL


def test_invalid_order_rejected():
    with pytest.raises(B.TTError):
        B.Plan(3, I.path(3), order=[0, 0, 1])


def test_tile_bits_option_validated():
    with pytest.raises(B.TTError):
        B.Plan(16, I.square_lattice(4), order=list(range(16)), tile_bits=20)


def test_parts_option_reported_and_validated():
    e = I.square_lattice(4)
    assert B.Plan(16, e, order=list(range(16))).info()["parts"] == 2
    assert B.Plan(16, e, order=list(range(16)), parts=1).info()["parts"] == 1
    with pytest.raises(B.TTError):
        B.Plan(16, e, order=list(range(16)), parts=3)


def test_autotune_mode_validated_before_any_device_work():
    p = B.Plan(16, I.square_lattice(4), order=list(range(16)))
    for mode in (-1, 3):
        assert B.lib().tt_plan_autotune(p.handle, 1, 0, None, None, mode, None, None, None) == B.TT_E_INVAL
    assert B.TUNE_ENERGY == 0 and B.TUNE_COUNT == 1 and B.TUNE_BACKWARD == 2


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus above 1 exits with a message before any device work."""
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


# ----------------------------------------------------------------------------
# failure injection on the host: errors returned before any device work
# ----------------------------------------------------------------------------
FAKE = C.c_void_p(0x1000)   # never dereferenced: the calls fail before touching the device


def _lib_call_contract(plan, batch, dtype, J=FAKE, h=None, energy=FAKE):
    return B.lib().tt_contract(plan.handle, batch, dtype, J, h, energy, None)


def test_dtype_rejected():
    p = B.Plan(16, I.square_lattice(4), order=list(range(16)))
    assert _lib_call_contract(p, 1, 5) == B.TT_E_DTYPE
    assert B.lib().tt_backward(p.handle, 1, 9, FAKE, None, FAKE, FAKE, None, None, None) == B.TT_E_DTYPE
    assert B.lib().tt_contract_uneven(1, (C.c_void_p * 1)(p.handle), 3, FAKE,
                                      np.zeros(1, np.int64).ctypes.data, FAKE, None, None, None, None) == B.TT_E_DTYPE


def test_invalid_arguments_rejected():
    p = B.Plan(16, I.square_lattice(4), order=list(range(16)))
    assert _lib_call_contract(p, 0, B.TT_F32) == B.TT_E_INVAL          # empty batch
    assert _lib_call_contract(p, 1, B.TT_F32, energy=None) == B.TT_E_INVAL
    assert _lib_call_contract(p, 1, B.TT_F32, J=None) == B.TT_E_INVAL
    assert _lib_call_contract(p, 1, B.TT_F32, h=FAKE) == B.TT_E_INVAL   # the plan has no fields
    pf = B.Plan(16, I.square_lattice(4), order=list(range(16)), has_field=True)
    assert _lib_call_contract(pf, 1, B.TT_F32) == B.TT_E_INVAL          # fields missing
    assert B.lib().tt_backward(p.handle, 1, B.TT_F32, FAKE, None, FAKE, None, None, None, None) == B.TT_E_INVAL
    assert B.lib().tt_count(p.handle, 1, FAKE, None, None, FAKE, None, None) == B.TT_E_INVAL
    assert B.lib().tt_count(None, 1, FAKE, None, FAKE, FAKE, None, None) == B.TT_E_INVAL


@pytest.mark.parametrize("call", ["contract", "backward", "count", "uneven"])
def test_budget_checked_before_device_work(call):
    """An explicit max_bytes below the planned state: TT_E_TOOBIG with no device touched."""
    e = I.square_lattice(8)
    p = B.Plan(64, e, order=list(range(64)), max_bytes=1024)
    lib = B.lib()
    if call == "contract":
        rc = lib.tt_contract(p.handle, 4, B.TT_F32, FAKE, None, FAKE, None)
    elif call == "backward":
        rc = lib.tt_backward(p.handle, 4, B.TT_F32, FAKE, None, FAKE, FAKE, None, None, None)
    elif call == "count":
        rc = lib.tt_count(p.handle, 4, FAKE, None, FAKE, FAKE, None, None)
    else:
        rc = lib.tt_contract_uneven(1, (C.c_void_p * 1)(p.handle), B.TT_F32, FAKE,
                                    np.zeros(1, np.int64).ctypes.data, FAKE, None, None, None, None)
    assert rc == B.TT_E_TOOBIG
    assert b"budget" in lib.tt_last_error()


def test_crt_of_reduced_residues_only():
    P = B.moduli()
    with pytest.raises(B.TTError):
        B.residues_to_int([P[0], 0, 0])


def test_count_log_of_known_counts():
    import math
    P = B.moduli()
    for g in (1, 2, 8, 3 ** 40, 2 ** 64, 2 ** 103 + 12345, 7 ** 60):
        res = [g % p for p in P]
        assert abs(B.count_log(res) - math.log(g)) <= 1e-14 * max(1.0, math.log(g)), g
    with pytest.raises(B.TTError):
        B.count_log([0, 0, 0])


def test_int16_refused_where_unsupported_before_device_work():
    """int16 couplings (TT_I16) run on sweep and chimera plans through
    tt_contract / tt_backward; the uneven and allocation-free calls refuse
    them before touching the device."""
    p = B.Plan(16, I.square_lattice(4), order=list(range(16)))
    lib = B.lib()
    assert lib.tt_contract_noalloc(p.handle, 1, B.TT_I16, FAKE, None, FAKE, None) == B.TT_E_DTYPE
    assert lib.tt_contract_uneven(1, (C.c_void_p * 1)(p.handle), B.TT_I16, FAKE,
                                  np.zeros(1, np.int64).ctypes.data, FAKE, None, None, None, None) == B.TT_E_DTYPE
    assert lib.tt_contract(p.handle, 1, 3, FAKE, None, FAKE, None) == B.TT_E_DTYPE     # no dtype 3


@pytest.mark.parametrize("z2,dtype", [(False, "f32"), (True, "f32"), (False, "i16"), (True, "i16")])
def test_backward_budget_counts_stored_entries_in_their_type(z2, dtype):
    """The backward needs at least two states of the widest pass (its working
    states when inputs are recomputed): stored entries (half of them on a
    half-state plan) of the state's element type (two bytes with int16
    couplings), 256-byte aligned. One byte less than that is refused before
    any device work, and the message names the amount."""
    e = I.square_lattice(8)
    p = B.Plan(64, e, order=list(range(64)), z2=z2, max_bytes=1)
    width, batch = p.info()["width"], 4
    esz = 2 if dtype == "i16" else 4
    need = 2 * (((batch << (width - (1 if z2 else 0))) * esz + 255) & ~255)
    q = B.Plan(64, e, order=list(range(64)), z2=z2, max_bytes=need - 1)
    code = B.TT_I16 if dtype == "i16" else B.TT_F32
    rc = B.lib().tt_backward(q.handle, batch, code, FAKE, None, FAKE, FAKE, None, None, None)
    assert rc == B.TT_E_TOOBIG
    assert f"needs {need} bytes".encode() in B.lib().tt_last_error()

"""CPU tests of sliced plans (tt_plan_create_sliced): the fixed spins, the
reduced sweep, its width on the 6 x 6 x 6 lattice, option validation, and
that calls which do not take sliced plans refuse them before any device work
(no GPU needed)."""
import ctypes as C

import numpy as np
import pytest

from paper_2008_06888_amd import binding as B
from paper_2008_06888_amd import instances as I

FAKE = C.c_void_p(0x1000)   # never dereferenced: the calls fail before touching the device


def test_given_fixed_spins_and_order():
    e = I.square_lattice(6)
    fixed = [14, 21, 3]
    p = B.Plan(36, e, order=list(range(36)), n_fixed=3, fixed=fixed)
    assert list(p.fixed()) == fixed
    order = p.order()
    assert list(order[:3]) == fixed                      # fixed spins first
    assert sorted(order.tolist()) == list(range(36))     # then every other spin once
    rest = [v for v in range(36) if v not in fixed]
    assert list(order[3:]) == rest                       # a GIVEN order keeps its sequence


def test_unsliced_plan_reports_no_fixed_spins():
    p = B.Plan(16, I.square_lattice(4), order=list(range(16)))
    assert p.fixed().size == 0


def test_reduced_graph_numbering_in_ops():
    """tt_plan_ops of a sliced plan is the reduced plan's: spins renumbered in
    ascending order without the fixed ones, edges without those touching them."""
    e = I.square_lattice(4)
    fixed = [5, 10]
    p = B.Plan(16, e, order=list(range(16)), fixed=fixed)
    ops, _ = p.ops()
    keep = [v for v in range(16) if v not in fixed]
    red_edges = [k for k, (a, b) in enumerate(e) if a not in fixed and b not in fixed]
    intro = sorted(set(int(o[5]) for o in ops if o[0] in (0, 1) and o[5] >= 0))
    assert intro == list(range(len(keep)))
    gate_edges = [int(o[3]) for o in ops if o[0] in (1, 3)]
    assert sorted(gate_edges) == list(range(len(red_edges)))
    # every reduced spin carries a field op (the bonds to fixed spins become fields)
    assert sorted(int(o[3]) for o in ops if o[0] == 4) == list(range(len(keep)))


def test_slicing_lowers_the_cubic_width():
    """6 x 6 x 6: the greedy sweep holds 2^30 entries; four fixed spins chosen
    by the planner bring the reduced sweep to at most 2^28 per slice."""
    e = I.cubic_lattice(6)
    whole = B.Plan(216, e, seed=0)
    p = B.Plan(216, e, seed=0, n_fixed=4)
    wi, si = whole.info(), p.info()
    assert wi["width"] == 30
    assert si["width"] <= 28
    assert len(set(p.fixed().tolist())) == 4
    assert sorted(p.order().tolist()) == list(range(216))
    # the work per instance is that of all 16 slices
    red = B.Plan(216 - 4, _reduced_edges(e, p.fixed()), order=_reduced_order(p), has_field=True)
    assert si["terms"] == pytest.approx(16 * red.info()["terms"])


def _reduced_edges(e, fixed):
    fixed = set(int(v) for v in fixed)
    rid, k = {}, 0
    for v in range(int(e.max()) + 1):
        if v not in fixed:
            rid[v] = k
            k += 1
    return np.array([(rid[a], rid[b]) for a, b in e if a not in fixed and b not in fixed], np.int32)


def _reduced_order(p):
    fixed = set(p.fixed().tolist())
    keep = [v for v in range(p.n) if v not in fixed]
    rid = {v: i for i, v in enumerate(keep)}
    return [rid[v] for v in p.order()[len(fixed):]]


@pytest.mark.parametrize("kw", [dict(n_fixed=17), dict(fixed=[0, 0]), dict(fixed=[99]), dict(fixed=[-1]),
                                dict(fixed=list(range(16)))])
def test_invalid_slicing_rejected(kw):
    with pytest.raises(B.TTError):
        B.Plan(16, I.square_lattice(4), order=list(range(16)), **kw)


def test_chimera_and_potts_cannot_be_sliced():
    with pytest.raises(B.TTError):
        B.Plan(32, I.chimera_graph(2, 2) if hasattr(I, "chimera_graph") else I.square_lattice(4),
               chimera=(2, 2), n_fixed=2)
    with pytest.raises(B.TTError):
        B.Plan(16, I.square_lattice(4), q=3, n_fixed=2)


def test_other_calls_refuse_sliced_plans_before_device_work():
    e = I.square_lattice(4)
    p = B.Plan(16, e, order=list(range(16)), has_field=True, n_fixed=2)
    lib = B.lib()
    assert lib.tt_contract_noalloc(p.handle, 1, B.TT_F32, FAKE, FAKE, FAKE, None) == B.TT_E_INVAL
    assert b"sliced" in lib.tt_last_error()
    assert lib.tt_config_fd(p.handle, FAKE, FAKE, C.c_double(0.01), FAKE, FAKE, None, None) == B.TT_E_INVAL
    u = np.full(16, 0.5)
    assert lib.tt_sample_ground_state(p.handle, FAKE, FAKE, u.ctypes.data, FAKE, FAKE, None) == B.TT_E_INVAL
    assert lib.tt_plan_autotune(p.handle, 1, 0, FAKE, FAKE, 0, None, None, None) == B.TT_E_INVAL
    assert lib.tt_contract_uneven(1, (C.c_void_p * 1)(p.handle), B.TT_F32, FAKE,
                                  np.zeros(1, np.int64).ctypes.data, FAKE, None, None, None, None) == B.TT_E_INVAL


@pytest.mark.parametrize("call", ["contract", "backward", "count"])
def test_sliced_budget_checked_before_device_work(call):
    """An explicit max_bytes below one slice's state: TT_E_TOOBIG with no device touched."""
    p = B.Plan(64, I.square_lattice(8), order=list(range(64)), max_bytes=1024, n_fixed=2)
    lib = B.lib()
    if call == "contract":
        rc = lib.tt_contract(p.handle, 4, B.TT_F32, FAKE, None, FAKE, None)
    elif call == "backward":
        rc = lib.tt_backward(p.handle, 4, B.TT_F32, FAKE, None, FAKE, FAKE, None, None, None)
    else:
        rc = lib.tt_count(p.handle, 4, FAKE, None, FAKE, FAKE, None, None)
    assert rc == B.TT_E_TOOBIG
    assert b"budget" in lib.tt_last_error()

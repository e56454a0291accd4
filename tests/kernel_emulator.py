"""Host emulation of the energy kernels' algorithm (sweep_kernels.hip) on the
encoded program the library builds (tt_plan_program): tile loads and stores
in per-pass bit layouts, register stages of fused gates, final reduction and
the one-argmax-per-pass backward walk. Used by CPU tests to check the
encoder and the kernel algorithm on small cases before they run on a GPU.
Test infrastructure only; shares no code with the HIP sources.
"""
import ctypes as C

import numpy as np

FK_GATE, FK_CUT, FK_STAR = 1, 2, 3
SLOT_FIXED, NO_POS = 64, 0xFF


class DevPass2(C.Structure):
    _fields_ = [("in_w", C.c_int32), ("out_w", C.c_int32), ("w_max", C.c_int32), ("t", C.c_int32),
                ("stage_begin", C.c_int32), ("n_stages", C.c_int32), ("init", C.c_int32), ("n_free", C.c_int32),
                ("cand_begin", C.c_int32), ("n_cand", C.c_int32), ("term_begin", C.c_int32), ("n_lo", C.c_int32),
                ("n_hi", C.c_int32), ("n_cross", C.c_int32), ("surv_mask", C.c_uint64),
                ("R", C.c_uint8 * 16), ("fre", C.c_uint8 * 48), ("in_pos", C.c_uint8 * 64),
                ("out_pos", C.c_uint8 * 64), ("ld_order", C.c_uint8 * 16), ("st_order", C.c_uint8 * 16),
                ("n_ld", C.c_int32), ("n_st", C.c_int32), ("ld_bti", C.c_uint32 * 16), ("st_bti", C.c_uint32 * 16),
                ("ld_bad", C.c_uint64 * 16), ("st_bad", C.c_uint64 * 16), ("ld_hti", C.c_uint32 * 16),
                ("st_hti", C.c_uint32 * 16), ("ld_had", C.c_uint64 * 16), ("st_had", C.c_uint64 * 16),
                ("tb", C.c_int32), ("z2_skip", C.c_int32), ("fin", C.c_uint8 * 48), ("fout", C.c_uint8 * 48),
                ("op_begin", C.c_int32), ("n_ops", C.c_int32)]


class DevStage(C.Structure):
    _fields_ = [("sb", C.c_uint8 * 4), ("nns", C.c_uint8), ("ns", C.c_uint8 * 15), ("op_begin", C.c_int32),
                ("op_end", C.c_int32), ("pad", C.c_int32 * 2), ("g_lo", C.c_uint16 * 32),
                ("g_hi", C.c_uint16 * 32), ("sg_lo", C.c_uint16 * 32), ("sg_hi", C.c_uint16 * 32),
                ("soff", C.c_uint32 * 16)]


class FOp(C.Structure):
    _fields_ = [("kind", C.c_uint8), ("bit", C.c_uint8), ("lidx", C.c_uint8), ("nt", C.c_uint8),
                ("edge", C.c_int32), ("hspin", C.c_int32), ("w", C.c_uint8 * 4), ("te", C.c_int32 * 4),
                ("wl", C.c_uint8 * 4)]


class BCand(C.Structure):
    _fields_ = [("spin", C.c_int32), ("start_slot", C.c_int32)]


class BTerm(C.Structure):
    _fields_ = [("coef", C.c_int32), ("is_field", C.c_uint8), ("a", C.c_uint8), ("b", C.c_uint8),
                ("pad", C.c_uint8)]


def _records(raw, cls):
    n = len(raw) // C.sizeof(cls)
    assert n * C.sizeof(cls) == len(raw)
    arr = (cls * max(n, 1)).from_buffer_copy(raw + b"\0" * (C.sizeof(cls) * max(n, 1) - len(raw)))
    return [arr[i] for i in range(n)]


def load_program(plan):
    return {
        "passes": _records(plan.program(0), DevPass2),
        "stages": _records(plan.program(1), DevStage),
        "fops": _records(plan.program(2), FOp),
        "cands": _records(plan.program(3), BCand),
        "terms": _records(plan.program(4), BTerm),
        "final_pos": list(plan.program(5)),
        "chain_after": list(np.frombuffer(plan.program(6), dtype=np.int32)),
    }


def _swz(i):
    return i ^ ((i >> 5) & 31)


def _ebit(enc, i, bs):
    return (i >> enc) & 1 if enc < SLOT_FIXED else (bs >> (enc - SLOT_FIXED)) & 1


def z2_addr(a, w):
    """Stored address of entry a of a half-state plan (top bit of w set: complement)."""
    return a ^ ((1 << w) - 1) if w > 0 and (a >> (w - 1)) & 1 else a


def forward(prog, width, J, h, x0=None, after_pass=None, z2=False):
    """Runs every pass; returns the list of pass inputs and the final state.

    x0: initial state (default zeros); after_pass(q, state): called on each
    pass's output state (may modify it in place). z2: the half-state mode
    (h = 0): only the tiles with tile-id bit z2_skip at 0 run, every read and
    write goes to the stored address; every stored entry of each output must
    be written."""
    size = 1 << width
    states = [np.zeros(size) if x0 is None else np.array(x0, dtype=np.float64)]
    for qi, P in enumerate(prog["passes"]):
        src = states[-1]
        dst = np.full(size, np.nan)
        t = P.t
        tb = P.tb
        assert tb == min(10, max(6, t - 4))
        for k in range(P.n_free):
            assert P.fin[k] == P.in_pos[P.fre[k]] and P.fout[k] == P.out_pos[P.fre[k]]
        for tid in range(1 << P.n_free):
            if z2 and P.z2_skip >= 0 and (tid >> P.z2_skip) & 1:
                continue
            bs = in_base = out_base = 0
            stored = True
            for k in range(P.n_free):
                b = (tid >> k) & 1
                s = P.fre[k]
                bs |= b << s
                if P.in_pos[s] != NO_POS:
                    in_base |= b << P.in_pos[s]
                if P.out_pos[s] != NO_POS:
                    out_base |= b << P.out_pos[s]
                elif b:
                    stored = False
            tile = np.full(1 << t, np.nan)
            for u in range(1 << t):
                lo, hi = u & ((1 << tb) - 1), u >> tb
                ti = a = 0
                for k in range(min(t, tb)):
                    if (lo >> k) & 1:
                        ti |= P.ld_bti[k]
                        a |= P.ld_bad[k]
                ti |= P.ld_hti[hi]
                a |= P.ld_had[hi]
                tile[ti] = 0.0 if P.init else src[z2_addr(in_base | a, P.in_w) if z2 else in_base | a]
            assert not np.any(np.isnan(tile))
            if P.n_stages:
                stg = prog["stages"]
                assert P.op_begin == stg[P.stage_begin].op_begin
                assert P.n_ops == stg[P.stage_begin + P.n_stages - 1].op_end - P.op_begin <= 64
            else:
                assert P.n_ops == 0
            for si in range(P.n_stages):
                ST = prog["stages"][P.stage_begin + si]
                sb = [ST.sb[l] for l in range(4)]
                # encoded tables agree with their definitions
                for x in range(32):
                    assert ST.sg_lo[x] == _swz(ST.g_lo[x]) and ST.sg_hi[x] == _swz(ST.g_hi[x])
                for j in range(16):
                    assert ST.soff[j] == _swz(sum((1 << sb[l]) for l in range(4) if (j >> l) & 1))
                for o in range(ST.op_begin, ST.op_end):
                    op = prog["fops"][o]
                    # the op's bit among the stage bits (4: not a stage bit, or a fixed slot)
                    assert op.lidx == (sb.index(op.bit) if op.bit in sb else 4)
                    for k in range(op.nt):
                        if op.w[k] < SLOT_FIXED and op.w[k] in sb:
                            assert op.wl[k] == sb.index(op.w[k])
                        else:
                            assert op.wl[k] == 255
                for g in range((1 << t) >> 4):
                    gb = ST.g_lo[g & 31] | ST.g_hi[g >> 5]
                    ix = [gb | sum((1 << sb[l]) for l in range(4) if (j >> l) & 1) for j in range(16)]
                    v = [tile[i] for i in ix]
                    for o in range(ST.op_begin, ST.op_end):
                        op = prog["fops"][o]
                        h0 = h[op.hspin] if op.hspin >= 0 else 0.0
                        if op.kind == FK_STAR:
                            for j in range(16):
                                sw = h0 + sum((-J[op.te[k]] if _ebit(op.w[k], ix[j], bs) else J[op.te[k]])
                                              for k in range(op.nt))
                                v[j] += -sw if _ebit(op.bit, ix[j], bs) else sw
                            continue
                        L = op.lidx
                        for p in range(8):
                            j0 = ((p >> L) << (L + 1)) | (p & ((1 << L) - 1))
                            j1 = j0 | (1 << L)
                            sw = h0 + sum((-J[op.te[k]] if _ebit(op.w[k], ix[j0], bs) else J[op.te[k]])
                                          for k in range(op.nt))
                            a0, a1 = v[j0], v[j1]
                            if op.kind == FK_GATE:
                                Je = J[op.edge]
                                v[j0] = max(a0 + Je, a1 - Je) + sw
                                v[j1] = max(a0 - Je, a1 + Je) - sw
                            else:
                                v[j0] = v[j1] = max(a0, a1)
                    for j in range(16):
                        tile[ix[j]] = v[j]
            if not stored:
                continue
            for u in range(1 << P.n_st):
                lo, hi = u & ((1 << tb) - 1), u >> tb
                ti = a = 0
                for k in range(min(P.n_st, tb)):
                    if (lo >> k) & 1:
                        ti |= P.st_bti[k]
                        a |= P.st_bad[k]
                ti |= P.st_hti[hi]
                a |= P.st_had[hi]
                o = z2_addr(out_base | a, P.out_w) if z2 else out_base | a
                if z2 and not np.isnan(dst[o]):
                    assert dst[o] == tile[ti], "two tiles wrote different values to one stored entry"
                dst[o] = tile[ti]
        if z2:
            half = (1 << P.out_w) >> 1 if P.out_w > 0 else 1
            assert not np.any(np.isnan(dst[:half])), "a stored entry of the half state was not written"
        if after_pass is not None:
            after_pass(qi, dst)
        states.append(dst)
    return states


def backward(prog, states, final_w, final_slot_spin, n, J, h, z2=False):
    """Final argmax (lowest address) and the walk back; returns (max, sigma).
    z2: half states (the final maximum over the stored half, reads at stored addresses)."""
    fin = states[-1][: (1 << final_w) >> (1 if z2 and final_w > 0 else 0)]
    assert not np.any(np.isnan(fin)), "final state has unwritten entries"
    mx = fin.max()
    addr = int(np.argmax(fin == mx))
    s = np.zeros(n, np.int64)
    t = 0
    for c in range(final_w):
        b = (addr >> prog["final_pos"][c]) & 1
        t |= b << c
        if final_slot_spin[c] >= 0:
            s[final_slot_spin[c]] = b
    for pi in range(len(prog["passes"]) - 1, -1, -1):
        P = prog["passes"][pi]
        nc = P.n_cand
        if nc == 0:
            t &= P.surv_mask
            continue
        cands = prog["cands"][P.cand_begin:P.cand_begin + nc]
        terms = prog["terms"][P.term_begin:P.term_begin + P.n_lo + P.n_hi + P.n_cross]
        base = 0
        for c in range(P.in_w):
            if (P.surv_mask >> c) & 1 and (t >> c) & 1:
                base |= 1 << P.in_pos[c]
        best, best_a = -np.inf, -1
        for a in range(1 << nc):
            ad = base
            for k, cd in enumerate(cands):
                if cd.start_slot >= 0 and P.in_pos[cd.start_slot] != NO_POS and (a >> k) & 1:
                    ad |= 1 << P.in_pos[cd.start_slot]
            val = 0.0 if P.init else states[pi][z2_addr(ad, P.in_w) if z2 else ad]
            assert not np.isnan(val), "backward read an unwritten entry"
            for tm in terms:
                c = h[tm.coef] if tm.is_field else J[tm.coef]
                sa = ((a >> tm.a) & 1) if tm.a < 64 else ((t >> (tm.a - 64)) & 1)
                sg = -1 if sa else 1
                if tm.b != 255:
                    sb_ = ((a >> tm.b) & 1) if tm.b < 64 else ((t >> (tm.b - 64)) & 1)
                    sg *= -1 if sb_ else 1
                val += c * sg
            if val > best:
                best, best_a = val, a
        tin = t & P.surv_mask
        for k, cd in enumerate(cands):
            b = (best_a >> k) & 1
            s[cd.spin] = b
            if cd.start_slot >= 0:
                tin |= b << cd.start_slot
        t = tin
    return mx, (1 - 2 * s).astype(np.int8)

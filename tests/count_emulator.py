"""Host emulation of the counting sweep's pass kernel (count_kernels.hip) on
the encoded counting program (tt_plan_program parts 10 and 11): the tile
load through the deposit tables, the ops applied one after another to the
tile (gates and cuts pairing entries across their tile bit, diagonal and
field terms per entry), the store in the output width, and the final
maximum / count over the entries whose free slots are 0. Counts are exact
Python integers. With z2 the half-state mode of plans without fields: only
the tiles whose z2_skip tile-id bit is 0 run, every read and write goes to
the stored address (the complement when the top address bit is 1), and every
stored entry of each pass output must be written. Test code only: it checks
the counting path's encoding on the CPU.
"""
import ctypes as C

import numpy as np

OP_INTRO, OP_GATE, OP_CUT, OP_DIAG, OP_FIELD = 0, 1, 2, 3, 4
SLOT_FIXED = 64


class DevOp(C.Structure):
    _fields_ = [("kind", C.c_uint8), ("a", C.c_uint8), ("b", C.c_uint8), ("dec", C.c_uint8),
                ("param", C.c_int32), ("g4", C.c_uint8 * 4)]


class DevPass(C.Structure):
    _fields_ = [("in_w", C.c_int32), ("out_w", C.c_int32), ("w_max", C.c_int32), ("t", C.c_int32),
                ("op_begin", C.c_int32), ("n_ops", C.c_int32), ("n_dec", C.c_int32), ("init", C.c_int32),
                ("n_free", C.c_int32), ("reg", C.c_int32), ("merge_src", C.c_int32), ("z2_skip", C.c_int32),
                ("R", C.c_uint8 * 16), ("fre", C.c_uint8 * 48)]


def _records(raw, cls):
    n = len(raw) // C.sizeof(cls)
    assert n * C.sizeof(cls) == len(raw)
    arr = (cls * max(n, 1)).from_buffer_copy(raw + b"\0" * (C.sizeof(cls) * max(n, 1) - len(raw)))
    return [arr[i] for i in range(n)]


def load(plan):
    return _records(plan.program(10), DevPass), _records(plan.program(11), DevOp)


def _bit(enc, i, base):
    return (i >> enc) & 1 if enc < SLOT_FIXED else (base >> (enc - SLOT_FIXED)) & 1


def z2_addr(a, w):
    """Stored address of entry a of a half-state state of width w."""
    return a ^ ((1 << w) - 1) if w > 0 and (a >> (w - 1)) & 1 else a


def run(passes, ops, J, h, width, final_slot_spin, z2=False):
    """(max of the final state = -E*, count of maximisers) with exact Python counts."""
    J = np.asarray(J, dtype=np.int64)
    size_all = 1 << width
    x = np.zeros(size_all, dtype=np.int64)
    n = np.ones(size_all, dtype=object)
    za = (lambda a, w: z2_addr(a, w)) if z2 else (lambda a, w: a)
    for P in passes:
        t = P.t
        size = 1 << t
        R = [P.R[k] for k in range(t)]
        fre = [P.fre[k] for k in range(P.n_free)]
        po = ops[P.op_begin:P.op_begin + P.n_ops]
        xin, nin = x.copy(), n.copy()
        written = {}
        for tile_id in range(1 << P.n_free):
            if z2 and P.z2_skip >= 0 and (tile_id >> P.z2_skip) & 1:
                continue
            base = 0
            for k, s in enumerate(fre):
                base |= ((tile_id >> k) & 1) << s
            idx = np.array([base | sum(((i >> k) & 1) << R[k] for k in range(t)) for i in range(size)], dtype=np.int64)
            src = np.array([za(int(a), P.in_w) for a in idx & ((1 << P.in_w) - 1)], dtype=np.int64)
            tx = np.zeros(size, np.int64) if P.init else xin[src]
            tn = np.ones(size, dtype=object) if P.init else nin[src].copy()
            for op in po:
                if op.kind in (OP_GATE, OP_CUT):
                    Jv = int(J[op.param]) if op.kind == OP_GATE else 0
                    b = op.a
                    assert 0 <= b < t
                    for i0 in range(size):
                        if (i0 >> b) & 1:
                            continue
                        i1 = i0 | (1 << b)
                        a0, a1 = int(tx[i0]), int(tx[i1])
                        c00, c10, c01, c11 = a0 + Jv, a1 - Jv, a0 - Jv, a1 + Jv
                        n0, n1 = tn[i0], tn[i1]
                        tx[i0], tx[i1] = max(c00, c10), max(c01, c11)
                        tn[i0] = n0 if c00 > c10 else (n1 if c10 > c00 else n0 + n1)
                        tn[i1] = n0 if c01 > c11 else (n1 if c11 > c01 else n0 + n1)
                elif op.kind == OP_DIAG:
                    Jv = int(J[op.param])
                    for i in range(size):
                        tx[i] += -Jv if (_bit(op.a, i, base) ^ _bit(op.b, i, base)) else Jv
                elif op.kind == OP_FIELD:
                    hv = int(h[op.param])
                    for i in range(size):
                        tx[i] += -hv if _bit(op.a, i, base) else hv
            for i in range(size):
                if (int(idx[i]) >> P.out_w) != 0:
                    continue
                a = za(int(idx[i]), P.out_w)
                if a in written:   # written twice: the same value
                    assert written[a] == (int(tx[i]), tn[i])
                written[a] = (int(tx[i]), tn[i])
                x[a], n[a] = tx[i], tn[i]
        stored = (1 << (P.out_w - 1)) if (z2 and P.out_w > 0) else (1 << P.out_w)
        assert set(written) == set(range(stored)), "a stored entry of the pass output was not written"
    fw = len(final_slot_spin)
    free = [s for s in range(fw) if final_slot_spin[s] < 0]
    live = [i for i in range(1 << fw) if all(((i >> s) & 1) == 0 for s in free)]
    best = max(x[za(i, fw)] for i in live)
    return best, sum(n[za(i, fw)] for i in live if x[za(i, fw)] == best)

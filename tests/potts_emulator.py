"""Host emulation of the encoded 3-state (Potts) program: the pass records the
library uploads to the GPU (tt_plan_program parts 7-9), executed with numpy in
the order and with the per-thread entry sets the kernels use. Test code only:
it checks the encoder (tile digits, strides, op operands, live digits of the
final reduction) independently of the GPU.
"""
import struct

import numpy as np

MAX_W, MAX_T, MAX_OPS = 20, 4, 48
PASS_FMT = "<6iq" + f"{MAX_T}q" + f"{MAX_W}q" + "".join("4Bi" for _ in range(MAX_OPS))
PASS_SIZE = struct.calcsize(PASS_FMT)
RED_FMT = "<2iq" + f"{MAX_W}q"
OP_GATE, OP_CUT, OP_DIAG = 1, 2, 3


def parse_passes(raw: bytes):
    assert len(raw) % PASS_SIZE == 0, (len(raw), PASS_SIZE)
    out = []
    for k in range(len(raw) // PASS_SIZE):
        f = struct.unpack_from(PASS_FMT, raw, k * PASS_SIZE)
        t, n_nt, n_ops, init, low, _, threads = f[0:7]
        tile_st = list(f[7:7 + MAX_T])[:t]
        nt_st = list(f[7 + MAX_T:7 + MAX_T + MAX_W])[:n_nt]
        if low:   # the tile is slots 0 .. t-1
            assert tile_st == [3 ** r for r in range(t)]
        ops = []
        base = 7 + MAX_T + MAX_W
        for o in range(n_ops):
            kind, a, b, _, edge = f[base + 5 * o:base + 5 * o + 5]
            ops.append((kind, a, b, edge))
        out.append(dict(t=t, n_nt=n_nt, init=init, low=low, threads=threads, tile_st=tile_st, nt_st=nt_st, ops=ops))
    return out


def parse_reduce(raw: bytes):
    f = struct.unpack_from(RED_FMT, raw, 0)
    n_live, contig, combos = f[0:3]
    st = list(f[3:3 + n_live])
    if contig:
        assert st == [3 ** r for r in range(n_live)]
    return dict(n_live=n_live, contig=contig, combos=combos, st=st)


def _digits_offsets(strides):
    """Offsets sum_r d_r strides[r] over all digit assignments, digit 0 fastest."""
    off = np.zeros(1, dtype=np.int64)
    for s in strides:
        off = (off[None, :] + np.arange(3, dtype=np.int64)[:, None] * s).reshape(-1)
    return off


def run(passes, red, J, width, count=False):
    """Returns (max of the final state = -2H*, count of maximisers or None)."""
    J = np.asarray(J, dtype=np.float64)
    size = 3 ** width
    x = np.zeros(size)
    n = np.ones(size, dtype=object) if count else None
    for P in passes:
        t = P["t"]
        base = _digits_offsets(P["nt_st"])             # one per thread
        assert len(base) == P["threads"]
        tile = _digits_offsets(P["tile_st"])           # one per register entry
        idx = base[:, None] + tile[None, :]             # [threads, 3^t]
        v = np.zeros(idx.shape) if P["init"] else x[idx]
        c = None
        if count:
            c = np.empty(idx.shape, dtype=object)
            if P["init"]:
                c.fill(1)
            else:
                c[:] = n[idx]
        shp = (len(base),) + (3,) * t                  # axis 1 + (t - 1 - r) is digit r
        v = v.reshape(shp)
        if count:
            c = c.reshape(shp)
        for kind, a, b, e in P["ops"]:
            ax_a = 1 + (t - 1 - a)
            if kind == OP_DIAG:
                ax_b = 1 + (t - 1 - b)
                da = np.arange(3).reshape([3 if k == ax_a else 1 for k in range(len(shp))])
                db = np.arange(3).reshape([3 if k == ax_b else 1 for k in range(len(shp))])
                v = v + np.where(da == db, -2 * J[e], J[e])
                continue
            vm = np.moveaxis(v, ax_a, -1)
            cm = np.moveaxis(c, ax_a, -1) if count else None
            if kind == OP_CUT:
                y = vm.max(axis=-1, keepdims=True)
                ny = np.repeat(y, 3, axis=-1)
                if count:
                    s = np.where(vm == y, cm, 0).sum(axis=-1, keepdims=True)
                    cm = np.repeat(s, 3, axis=-1)
                vm = ny
            else:   # GATE: new[b] = max_a x[a] + (a == b ? -2J : J)
                T = np.where(np.eye(3, dtype=bool), -2 * J[e], J[e])
                cand = vm[..., :, None] + T                      # [..., a, b]
                y = cand.max(axis=-2)
                if count:
                    cm = np.where(cand == y[..., None, :], cm[..., :, None], 0).sum(axis=-2)
                vm = y
            v = np.moveaxis(vm, -1, ax_a)
            if count:
                c = np.moveaxis(cm, -1, ax_a)
        flat = idx.reshape(-1)
        # entry i of a thread: digit r = (i // 3^r) % 3 -> the C-order flattening of shp
        # lists digit t-1 first, matching axis 1 + (t - 1 - r) for digit r
        x[flat] = v.reshape(len(base), -1).reshape(-1)
        if count:
            n[flat] = c.reshape(len(base), -1).reshape(-1)
    live = _digits_offsets(red["st"])
    best = x[live].max()
    if not count:
        return best, None
    g = sum(int(k) for k in n[live][x[live] == best])
    return best, g

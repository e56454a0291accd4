"""Host replay of a plan's operation list (see tt_plan_ops), for CPU tests of
the planner: the ops are applied in numpy to a dense state of (x, n) tuples
exactly as their definitions state (int64 values, Python-int counts).

This is test infrastructure that checks the planner's op list; it shares no
code with the HIP kernels and is not the oracle.
"""
import numpy as np

INTRO, GATE, CUT, DIAG, FIELD = 0, 1, 2, 3, 4


def _bit(idx, slot):
    return (idx >> slot) & 1


def replay(ops, final_slot_spin, n, J, h=None, counts=True):
    """Returns (E*, g or None, sigma of one ground state by brute recording)."""
    W = int(max([1] + [max(r[6], r[7]) for r in ops]))
    size = 1 << W
    idx = np.arange(size, dtype=np.int64)
    sig = [1 - 2 * _bit(idx, s) for s in range(W)]           # sigma of each slot per entry
    x = np.zeros(size, dtype=np.int64 if np.issubdtype(np.asarray(J).dtype, np.integer) else np.float64)
    cnt = np.ones(size, dtype=object) if counts else None
    for kind, a, b, param, old, new, wb, wa in ops:
        if kind == INTRO:
            continue
        if kind in (GATE, CUT):
            Jv = J[param] if kind == GATE else 0
            lo = idx[_bit(idx, a) == 0]
            hi = lo | (1 << a)
            a0, a1 = x[lo].copy(), x[hi].copy()
            c00, c10, c01, c11 = a0 + Jv, a1 - Jv, a0 - Jv, a1 + Jv
            x[lo] = np.maximum(c00, c10)
            x[hi] = np.maximum(c01, c11)
            if counts:
                n0, n1 = cnt[lo].copy(), cnt[hi].copy()
                cnt[lo] = np.where(c00 > c10, n0, np.where(c10 > c00, n1, n0 + n1))
                cnt[hi] = np.where(c01 > c11, n0, np.where(c11 > c01, n1, n0 + n1))
        elif kind == DIAG:
            x = x + J[param] * sig[a] * sig[b]
        elif kind == FIELD:
            x = x + h[param] * sig[a]
    fw = len(final_slot_spin)
    # entries beyond the final width are copies of free slots: restrict to the final width
    xs = x[: 1 << fw]
    mx = xs.max()
    g = None
    if counts:
        g = int(sum(cnt[: 1 << fw][xs == mx]))
        # free slots inside the final width duplicate each configuration
        free = sum(1 for s in final_slot_spin if s < 0)
        assert g % (1 << free) == 0
        g //= (1 << free)
    return -mx, g

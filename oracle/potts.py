"""CPU oracle for 3-state Potts glasses (the paper's Appendix C).

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything here. The
product path never touches it, and this module imports nothing from the
product package.

Model (Appendix C, the Hamiltonian of the Potts-glass comparison there):
H(s) = sum over edges (i, j) of J_ij M[s_i][s_j], with s_i in {0, 1, 2} (the
paper's labels 1, 2, 3) and M = 1 on the diagonal, -1/2 off it. The ground
state minimises H. Every energy is kept doubled, 2H = sum J_ij (2 if
s_i = s_j else -1), so that integer couplings give exact integers (int64).

What it computes:

* ``energy2``      -- 2H(s) of a configuration.
* ``brute_force``  -- the plain definition: the minimum of 2H over all 3^n
                      configurations, the number of minimisers and the
                      lowest-index one (index = sum_i s_i 3^i).
* ``eliminate``    -- max-sum bucket elimination of the factor graph with one
                      factor per edge, f_e(a, b) = -J_e (2 if a = b else -1)
                      (negative doubled energies, so that the tropical sum
                      max and product + of Eq. (2) give -2H*); with the (x, n)
                      tuple algebra of Eq. (4) for counts, and traceback of the
                      cached tables for one ground state (Sec. IV).

Every function is pinned by tests against closed forms (ferromagnets, proper
3-colourings of paths, cycles and trees, K_4), brute force and invariants
(tests/test_oracle_potts.py). Which degenerate ground state is returned is
parity unpinned: any minimiser is correct.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence

import numpy as np

from .spinglass import ORACLE_PRIMES, crt, min_fill_order

Q = 3


def _values(J):
    """int64 when the couplings are integers, else float64."""
    J = np.asarray(J)
    dt = np.int64 if np.issubdtype(J.dtype, np.integer) else np.float64
    return J.astype(dt), dt


def energy2(n: int, edges, J, s):
    """2H(s) = sum_e J_e (2 if s_i = s_j else -1); int for integer J, else float64."""
    Jv, dt = _values(J)
    s = np.asarray(s, dtype=np.int64)
    if s.shape != (n,) or np.any((s < 0) | (s >= Q)):
        raise ValueError("s must hold n labels in {0, 1, 2}")
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if len(e) == 0:
        return dt(0).item()
    same = s[e[:, 0]] == s[e[:, 1]]
    E = np.sum(np.where(same, 2 * Jv, -Jv))
    return int(E) if dt is np.int64 else float(E)


def labels_from_index(n: int, idx: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.int8)
    for i in range(n):
        out[i] = idx % Q
        idx //= Q
    return out


def brute_force(n: int, edges, J, chunk: int = 1 << 16) -> Dict:
    """Minimum of 2H over {0,1,2}^n, number of minimisers, lowest-index minimiser (n <= 14)."""
    if n > 14:
        raise ValueError("brute force limited to n <= 14")
    Jv, dt = _values(J)
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    total = Q ** n
    pw = Q ** np.arange(n, dtype=np.int64)
    best, count, arg = None, 0, -1
    for start in range(0, total, chunk):
        x = np.arange(start, min(start + chunk, total), dtype=np.int64)
        lab = (x[:, None] // pw[None, :]) % Q                       # [chunk, n]
        E = np.zeros(len(x), dtype=dt)
        for k in range(len(e)):
            same = lab[:, e[k, 0]] == lab[:, e[k, 1]]
            E += np.where(same, 2 * Jv[k], -Jv[k])
        mn = E.min()
        if best is None or mn < best:
            best, count, arg = mn, int(np.count_nonzero(E == mn)), start + int(np.argmax(E == mn))
        elif mn == best:
            count += int(np.count_nonzero(E == mn))
    E2 = int(best) if dt is np.int64 else float(best)
    return {"energy2": E2, "energy": E2 / 2, "count": count, "index": arg,
            "labels": labels_from_index(n, arg)}


class _Factor:
    __slots__ = ("scope", "val", "cnt")

    def __init__(self, scope, val, cnt):
        self.scope = tuple(scope)
        self.val = val
        self.cnt = cnt


def _expand(f: _Factor, U, arr, lead: int = 0):
    shape = list(arr.shape[:lead]) + [Q if u in f.scope else 1 for u in U]
    return arr.reshape(shape)


def eliminate(n: int, edges, J, order: Optional[Sequence[int]] = None, counts: Optional[str] = None,
              moduli: Sequence[int] = ORACLE_PRIMES, traceback: bool = True) -> Dict:
    """Max-sum bucket elimination of the 3-state Potts factor graph.

    For each v in ``order``: join every factor mentioning v by the tropical
    product (addition), then eliminate v by the tropical sum (maximum over its
    three labels); with ``counts`` the entries are (x, n) tuples of Eq. (4):
    products add x and multiply n, sums keep the larger x and add the n's of
    equal x. The scalar left is -2H* (and g). Traceback (Sec. IV): in reverse
    order, s_v is the first argmax of v's joined table given its
    already-assigned neighbours.

    counts: None, "exact" (Python integers) or "mod" (residues mod ``moduli``).
    """
    Jv, dt = _values(J)
    if counts is not None and dt is not np.int64:
        raise ValueError("counting needs integer couplings")
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if order is None:
        order = min_fill_order(n, e)
    order = [int(v) for v in order]
    if sorted(order) != list(range(n)):
        raise ValueError("order must be a permutation of the spins")
    P = np.array(moduli, dtype=np.uint64)

    def ones(shape):
        if counts is None:
            return None
        if counts == "exact":
            c = np.empty(shape, dtype=object)
            c.fill(1)
            return c
        return np.ones((len(P),) + tuple(shape), dtype=np.uint64)

    same = np.eye(Q, dtype=bool)
    factors: List[_Factor] = []
    for k in range(len(e)):
        t = np.where(same, -2 * Jv[k], Jv[k]).astype(dt)           # -(doubled bond energy)
        factors.append(_Factor((int(e[k, 0]), int(e[k, 1])), t, ones((Q, Q))))
    touched = set()
    for f in factors:
        touched.update(f.scope)
    for i in range(n):
        if i not in touched:                                         # an isolated spin: three free labels
            factors.append(_Factor((i,), np.zeros(Q, dtype=dt), ones((Q,))))

    saved = []
    for v in order:
        bucket = [f for f in factors if v in f.scope]
        factors = [f for f in factors if v not in f.scope]
        U = tuple(sorted(set().union(*[f.scope for f in bucket])))
        shape = (Q,) * len(U)
        val = np.zeros(shape, dtype=dt)
        for f in bucket:
            val = val + _expand(f, U, f.val)
        cnt = None
        if counts == "exact":
            cnt = np.empty(shape, dtype=object)
            cnt.fill(1)
            for f in bucket:
                cnt = cnt * _expand(f, U, f.cnt)
        elif counts == "mod":
            cnt = np.ones((len(P),) + shape, dtype=np.uint64)
            pb = P.reshape((-1,) + (1,) * len(U))
            for f in bucket:
                cnt = (cnt * _expand(f, U, f.cnt, lead=1)) % pb
        ax = U.index(v)
        mx = val.max(axis=ax)
        newU = U[:ax] + U[ax + 1:]
        newc = None
        if counts is not None:
            hit = val == np.expand_dims(mx, ax)
            if counts == "exact":
                newc = np.where(hit, cnt, 0).sum(axis=ax)
                if not isinstance(newc, np.ndarray):
                    newc = np.array(newc, dtype=object)
            else:
                newc = np.where(hit[None], cnt, np.uint64(0)).sum(axis=ax + 1) % P.reshape((-1,) + (1,) * len(newU))
        if traceback:
            saved.append((v, U, val))
        factors.append(_Factor(newU, mx, newc))

    total = dt(0)
    cnt_exact = 1
    cnt_mod = np.ones(len(P), dtype=np.uint64)
    for f in factors:
        assert f.scope == ()
        total = total + f.val.reshape(())[()]
        if counts == "exact":
            cnt_exact = cnt_exact * f.cnt.reshape(())[()]
        elif counts == "mod":
            cnt_mod = (cnt_mod * f.cnt.reshape(len(P))) % P
    E2 = -total
    E2 = int(E2) if dt is np.int64 else float(E2)
    out = {"energy2": E2, "energy": E2 / 2, "order": order}
    if counts == "exact":
        out["count"] = int(cnt_exact)
    elif counts == "mod":
        out["residues"] = [int(r) for r in cnt_mod]
        out["moduli"] = [int(p) for p in P]
        out["count"] = crt(out["residues"], out["moduli"])
    if traceback:
        s = np.full(n, -1, dtype=np.int64)
        for v, U, val in reversed(saved):
            idx = []
            for u in U:
                if u == v:
                    idx.append(slice(None))
                else:
                    assert s[u] >= 0, "traceback reached an unassigned neighbour"
                    idx.append(int(s[u]))
            s[v] = int(np.argmax(val[tuple(idx)]))                   # first argmax: lowest label on ties
        out["labels"] = s.astype(np.int8)
    return out

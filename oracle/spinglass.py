"""CPU oracle for tropical tensor-network ground states of Ising spin glasses.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything here. The
product path (the HIP library and its Python binding) never touches it, and
this module imports nothing from the product package.

What it computes (paper sections cited per function):

* ``energy``          -- the Ising energy of Eq. (1).
* ``brute_force``     -- the plain definition: min over all 2^n configurations of
                         Eq. (1), the number of minimisers, and the lowest-index one.
* ``eliminate``       -- max-sum bucket (variable) elimination over the tropical
                         semiring of Eq. (2), the algorithm the paper states the
                         tropical contraction equals on trees and junction trees
                         (Sec. III); with the (x, n) tuple algebra of Eq. (4) for
                         counting; with traceback of cached tables for one ground
                         state (Sec. IV, caching intermediates and backtracking).
* ``crt``             -- exact integer from residues (Chinese remainder theorem).

Encoding: spin index s in {0, 1} with sigma = +1 for s = 0 and -1 for s = 1 (the
field gate diag(h, -h) and the bond matrix [[J, -J], [-J, J]] of Sec. II / App. A).
A configuration's integer index is sum_i s_i 2^i.

Arithmetic: float64 for real couplings, int64 for integer ones; counts either
exact Python integers or residues modulo the oracle's own 31-bit primes (numpy
uint64, so one product of two residues stays below 2^62).

Every function is pinned by tests against brute force, closed forms and
invariants (see tests/test_oracle.py). The choice of *which* degenerate ground
state is returned is parity unpinned: any minimiser is correct.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

# The oracle's own moduli: primes just below 2^31 (checked prime by trial
# division in tests). Their product is about 2^217.
ORACLE_PRIMES = (2147483647, 2147483629, 2147483587, 2147483579,
                 2147483563, 2147483549, 2147483543)


def _is_integer_problem(J, h) -> bool:
    arrs = [np.asarray(J)] + ([] if h is None else [np.asarray(h)])
    return all(np.issubdtype(a.dtype, np.integer) for a in arrs)


def _as_problem(J, h):
    """Values in int64 when every input is an integer array, else float64."""
    dt = np.int64 if _is_integer_problem(J, h) else np.float64
    Jv = np.asarray(J).astype(dt)
    hv = None if h is None else np.asarray(h).astype(dt)
    return Jv, hv, dt


# ----------------------------------------------------------------------------
# Eq. (1)
# ----------------------------------------------------------------------------

def energy(n: int, edges, J, h, sigma) -> float:
    """E(sigma) = -sum_{i<j} J_ij sigma_i sigma_j - sum_i h_i sigma_i (Eq. 1).

    ``sigma`` holds +-1 values. Returns an int for integer inputs, else a float
    accumulated in float64.
    """
    Jv, hv, dt = _as_problem(J, h)
    s = np.asarray(sigma).astype(dt)
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    E = -np.sum(Jv * s[e[:, 0]] * s[e[:, 1]]) if len(e) else dt(0)
    if hv is not None:
        E = E - np.sum(hv * s)
    return int(E) if dt is np.int64 else float(E)


def sigma_from_index(n: int, idx: int) -> np.ndarray:
    s = (idx >> np.arange(n)) & 1
    return (1 - 2 * s).astype(np.int8)


# ----------------------------------------------------------------------------
# brute force: the plain definition of E*, g and an argmin
# ----------------------------------------------------------------------------

def brute_force(n: int, edges, J, h, chunk_bits: int = 16) -> Dict:
    """Minimum of Eq. (1) over {+-1}^n, number of minimisers, lowest-index minimiser.

    Enumerates every configuration index x in [0, 2^n) (n <= 26). Energies are
    exact for integer inputs (int64); for real inputs they are float64 and
    minimisers are counted by exact equality of those float64 values.
    """
    if n > 26:
        raise ValueError("brute force limited to n <= 26")
    Jv, hv, dt = _as_problem(J, h)
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    best = None
    count = 0
    arg = -1
    total = 1 << n
    step = 1 << min(n, chunk_bits)
    for start in range(0, total, step):
        x = np.arange(start, start + step, dtype=np.int64)
        bits = (x[:, None] >> np.arange(n)[None, :]) & 1          # [chunk, n]
        sig = (1 - 2 * bits).astype(dt)
        E = np.zeros(step, dtype=dt)
        for k in range(len(e)):
            E -= Jv[k] * sig[:, e[k, 0]] * sig[:, e[k, 1]]
        if hv is not None:
            for i in range(n):
                E -= hv[i] * sig[:, i]
        mn = E.min()
        if best is None or mn < best:
            best = mn
            count = int(np.count_nonzero(E == mn))
            arg = start + int(np.argmax(E == mn))
        elif mn == best:
            count += int(np.count_nonzero(E == mn))
    Estar = int(best) if dt is np.int64 else float(best)
    return {"energy": Estar, "count": count, "index": arg,
            "sigma": sigma_from_index(n, arg)}


# ----------------------------------------------------------------------------
# elimination orders (the oracle's own; never the GPU planner's)
# ----------------------------------------------------------------------------

def min_fill_order(n: int, edges) -> List[int]:
    """Greedy min-fill elimination order (ties: smaller degree, then smaller index)."""
    adj = [set() for _ in range(n)]
    for a, b in np.asarray(edges, dtype=np.int64).reshape(-1, 2):
        adj[a].add(int(b))
        adj[b].add(int(a))
    alive = set(range(n))
    order = []
    while alive:
        best = None
        for v in alive:
            nb = list(adj[v])
            fill = 0
            for i in range(len(nb)):
                for j in range(i + 1, len(nb)):
                    if nb[j] not in adj[nb[i]]:
                        fill += 1
            key = (fill, len(nb), v)
            if best is None or key < best:
                best = key
        v = best[2]
        nb = list(adj[v])
        for i in range(len(nb)):
            for j in range(i + 1, len(nb)):
                adj[nb[i]].add(nb[j])
                adj[nb[j]].add(nb[i])
        for w in nb:
            adj[w].discard(v)
        adj[v] = set()
        alive.discard(v)
        order.append(v)
    return order


def induced_width(n: int, edges, order: Sequence[int]) -> int:
    """Largest bucket scope (variables joined when eliminating one) along ``order``."""
    adj = [set() for _ in range(n)]
    for a, b in np.asarray(edges, dtype=np.int64).reshape(-1, 2):
        adj[a].add(int(b))
        adj[b].add(int(a))
    done = set()
    w = 0
    for v in order:
        nb = [x for x in adj[v] if x not in done]
        w = max(w, len(nb) + 1)
        for i in range(len(nb)):
            for j in range(i + 1, len(nb)):
                adj[nb[i]].add(nb[j])
                adj[nb[j]].add(nb[i])
        done.add(v)
    return w


# ----------------------------------------------------------------------------
# factors: scope (sorted tuple of spins) + value table (+ optional count table)
# ----------------------------------------------------------------------------

class _Factor:
    __slots__ = ("scope", "val", "cnt")

    def __init__(self, scope, val, cnt):
        self.scope = tuple(scope)
        self.val = val          # ndarray, one axis of length 2 per scope variable
        self.cnt = cnt          # None, or object ndarray (exact), or uint64 [P, ...] residues


def _expand_to(f: _Factor, U: Tuple[int, ...], arr, lead: int = 0):
    """View of ``arr`` (axes = f.scope, after ``lead`` leading axes) broadcastable over U."""
    shape = list(arr.shape[:lead]) + [2 if u in f.scope else 1 for u in U]
    # scope and U are both sorted, so the axis order already agrees
    return arr.reshape(shape)


def eliminate(n: int, edges, J, h, order: Optional[Sequence[int]] = None,
              counts: Optional[str] = None, moduli: Sequence[int] = ORACLE_PRIMES,
              traceback: bool = True) -> Dict:
    """Max-sum bucket elimination of the Ising factor graph (Sec. II-III).

    Factors (negative energies, Sec. II): each edge e = (i, j) gives
    f_e(s_i, s_j) = J_ij sigma_i sigma_j, i.e. the table [[J, -J], [-J, J]];
    each spin with a field gives f_i(s_i) = h_i sigma_i, i.e. (h, -h).
    For each v in ``order``: join every factor mentioning v by the tropical
    product (addition, Eq. 2), then eliminate v by the tropical sum (max).
    With ``counts`` the entries are tuples (x, n) with the product
    (x1 + x2, n1 * n2) and the sum of Eq. (4): keep the larger x, add the
    n's when the x's are equal. The scalar left is -E* (and g).

    counts: None, "exact" (Python integers) or "mod" (residues mod ``moduli``).
    Traceback (Sec. IV): in reverse order, s_v is the first argmax of v's
    joined table given its already-assigned neighbours.
    """
    Jv, hv, dt = _as_problem(J, h)
    if counts is not None and dt is not np.int64:
        raise ValueError("counting needs integer couplings (exact equality in Eq. 4)")
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if order is None:
        order = min_fill_order(n, e)
    order = [int(v) for v in order]
    if sorted(order) != list(range(n)):
        raise ValueError("order must be a permutation of the spins")
    P = np.array(moduli, dtype=np.uint64)

    def one_count(shape):
        if counts is None:
            return None
        if counts == "exact":
            c = np.empty(shape, dtype=object)
            c.fill(1)
            return c
        return np.ones((len(P),) + tuple(shape), dtype=np.uint64)

    factors: List[_Factor] = []
    for k in range(len(e)):
        a, b = int(e[k, 0]), int(e[k, 1])
        t = np.array([[Jv[k], -Jv[k]], [-Jv[k], Jv[k]]], dtype=dt)
        factors.append(_Factor((a, b), t, one_count((2, 2))))
    if hv is not None:
        for i in range(n):
            factors.append(_Factor((i,), np.array([hv[i], -hv[i]], dtype=dt), one_count((2,))))
    # spins with no factor at all still take two values
    touched = set()
    for f in factors:
        touched.update(f.scope)
    for i in range(n):
        if i not in touched:
            factors.append(_Factor((i,), np.zeros(2, dtype=dt), one_count((2,))))

    saved = []        # (v, U, joined values) for traceback
    for v in order:
        bucket = [f for f in factors if v in f.scope]
        factors = [f for f in factors if v not in f.scope]
        U = tuple(sorted(set().union(*[f.scope for f in bucket])))
        shape = (2,) * len(U)
        val = np.zeros(shape, dtype=dt)
        for f in bucket:
            val = val + _expand_to(f, U, f.val)
        cnt = None
        if counts == "exact":
            cnt = np.empty(shape, dtype=object)
            cnt.fill(1)
            for f in bucket:
                cnt = cnt * _expand_to(f, U, f.cnt)
        elif counts == "mod":
            cnt = np.ones((len(P),) + shape, dtype=np.uint64)
            pb = P.reshape((-1,) + (1,) * len(U))
            for f in bucket:
                cnt = (cnt * _expand_to(f, U, f.cnt, lead=1)) % pb
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
                masked = np.where(hit[None], cnt, np.uint64(0))
                newc = masked.sum(axis=ax + 1) % P.reshape((-1,) + (1,) * len(newU))
        if traceback:
            saved.append((v, U, val))
        factors.append(_Factor(newU, mx, newc))

    # every remaining factor is a scalar
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
    Estar = -total
    out = {"energy": int(Estar) if dt is np.int64 else float(Estar),
           "order": order}
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
            line = val[tuple(idx)]
            s[v] = int(np.argmax(line))       # first argmax: lowest s on ties
        sigma = (1 - 2 * s).astype(np.int8)
        out["sigma"] = sigma
    return out


# ----------------------------------------------------------------------------
# residues -> integer
# ----------------------------------------------------------------------------

def crt(residues: Sequence[int], moduli: Sequence[int]) -> int:
    """Smallest non-negative integer with the given residues (pairwise coprime moduli)."""
    x, M = 0, 1
    for r, p in zip(residues, moduli):
        r, p = int(r), int(p)
        # x + M*t = r (mod p)
        t = ((r - x) * pow(M, -1, p)) % p
        x += M * t
        M *= p
    return x


def ground_state_gradient(edges, sigma) -> Tuple[np.ndarray, np.ndarray]:
    """dE*/dJ_ij = -sigma_i sigma_j and dE*/dh_i = -sigma_i at a unique ground state.

    E* is piecewise linear in (J, h) (Sec. IV): on the piece where sigma is the
    minimiser, E* = E(sigma), whose partial derivatives follow from Eq. (1).
    """
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    s = np.asarray(sigma).astype(np.float64)
    return -(s[e[:, 0]] * s[e[:, 1]]), -s

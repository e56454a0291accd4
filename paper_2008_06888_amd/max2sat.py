"""#Max-2-SAT as an Ising ground-state count (App. D of the paper).

A clause (l1 or l2) over literals l = +-(v + 1) is violated exactly when both
literals are false. With sigma_v = +1 for "true" and s_l = +sigma_v for a
positive literal, -sigma_v for a negated one, the number of violated clauses
is sum over clauses of (1 - s_1)(1 - s_2) / 4. Four times that count is an
Ising energy plus a constant:

    4 V(sigma) = C + sum_c (a b sigma_i sigma_j - a sigma_i - b sigma_j)

for a clause on variables i != j with literal signs a, b. With E(sigma) =
-sum J sigma_i sigma_j - sum h sigma_i (Eq. (1)) this is J_ij += -a b,
h_i += a, h_j += b, C += 1. A clause whose two literals are the same
variable is a unit clause (same sign: 4 V = 2 - 2 s, i.e. h_i += 2 a, C += 2)
or always satisfied (opposite signs). All couplings and fields are integers,
so the counting path is exact: the most clauses that can be satisfied is
m - (E* + C) / 4, and the number of assignments reaching it is the ground-state
degeneracy g.

This module only builds the instance (integer J, h and the constant); the
contraction runs in the library (tt_count / tt_backward).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Sequence, Tuple

import numpy as np


@dataclass
class Max2SatInstance:
    n: int                 # variables
    clauses: np.ndarray    # [m][2] literals +-(v + 1)
    edges: np.ndarray      # [k][2] int32, i < j (variable pairs sharing a clause)
    J: np.ndarray          # [k] int32
    h: np.ndarray          # [n] int32
    const: int             # C of 4 V = E + C


def to_ising(n: int, clauses: Sequence[Tuple[int, int]]) -> Max2SatInstance:
    """Ising form of a 2-CNF formula (see the module docstring)."""
    cl = np.asarray(clauses, dtype=np.int64).reshape(-1, 2)
    if np.any(cl == 0) or np.any(np.abs(cl) > n):
        raise ValueError("literals are +-(v + 1) with 0 <= v < n")
    pair = {}
    h = np.zeros(n, np.int64)
    const = 0
    for l1, l2 in cl:
        i, j = abs(int(l1)) - 1, abs(int(l2)) - 1
        a, b = (1 if l1 > 0 else -1), (1 if l2 > 0 else -1)
        if i == j:
            if a == b:          # unit clause
                h[i] += 2 * a
                const += 2
            else:               # tautology: never violated
                pass
            continue
        if i > j:
            i, j, a, b = j, i, b, a
        pair[(i, j)] = pair.get((i, j), 0) - a * b
        h[i] += a
        h[j] += b
        const += 1
    keys = sorted(pair)
    edges = np.array(keys, dtype=np.int32).reshape(-1, 2)
    J = np.array([pair[k] for k in keys], dtype=np.int32)
    return Max2SatInstance(n=n, clauses=cl, edges=edges, J=J, h=h.astype(np.int32), const=const)


def violated(inst: Max2SatInstance, sigma: np.ndarray) -> int:
    """Clauses violated by an assignment (sigma = +1 true, -1 false), counted directly."""
    s = np.asarray(sigma)
    lit = lambda l: s[abs(l) - 1] * (1 if l > 0 else -1)
    return int(sum(1 for l1, l2 in inst.clauses if lit(l1) < 0 and lit(l2) < 0))


def max_satisfied(inst: Max2SatInstance, energy: int) -> int:
    """Most clauses satisfiable, from the Ising ground-state energy E*."""
    v4 = int(energy) + inst.const
    if v4 % 4:
        raise ValueError("E* + C must be a multiple of 4")
    return len(inst.clauses) - v4 // 4


def random_regular_formula(n: int, rng: np.random.Generator, degree: int = 3):
    """One clause per edge of a random d-regular graph, literal signs uniform (App. D)."""
    from .instances import random_regular
    e = random_regular(n, degree, rng)
    signs = np.where(rng.random((len(e), 2)) < 0.5, -1, 1)
    return [(int(signs[k, 0] * (e[k, 0] + 1)), int(signs[k, 1] * (e[k, 1] + 1))) for k in range(len(e))]

"""Seeded synthetic spin-glass instances: graphs, couplings J_ij and fields h_i.

This module holds no contraction arithmetic. It only draws the inputs of the
Ising problem (Eq. 1 of the paper: E(sigma) = -sum_{i<j} J_ij s_i s_j - sum_i h_i s_i)
on the graph families the paper studies (Sec. V and Appendices C, D):

* open L x L square lattices (Sec. V, square-lattice experiments),
* chimera graphs of L x L unit cells of K_{4,4} (Sec. V, chimera experiments),
* random 3-regular graphs (Appendix D),
* small closed-form families used as pins (paths, rings, trees, plaquettes).

Every random draw comes from ``numpy.random.default_rng([config_id, instance_id])``
(or an explicit seed), so the GPU path and the CPU oracle consume the same arrays.

Spin and edge conventions (shared by every consumer):
  * spins are 0..n-1; square-lattice spin (r, c) is r*Lc + c;
  * ``edges`` is int32 [m, 2] with edges[e, 0] < edges[e, 1], no duplicates;
  * ``J`` is [m] (float32 for Gaussian couplings, int32 for +-1 couplings);
  * ``h`` is [n] of the same dtype, or None when the field vanishes.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Instance:
    """One Ising instance: graph plus couplings (Eq. 1)."""

    n: int
    edges: np.ndarray
    J: np.ndarray
    h: Optional[np.ndarray]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.edges.shape[0])


# ----------------------------------------------------------------------------
# graphs
# ----------------------------------------------------------------------------

def _canon(edges) -> np.ndarray:
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    lo = np.minimum(e[:, 0], e[:, 1])
    hi = np.maximum(e[:, 0], e[:, 1])
    out = np.stack([lo, hi], axis=1).astype(np.int32)
    if np.any(out[:, 0] == out[:, 1]):
        raise ValueError("self loop")
    if len({(int(a), int(b)) for a, b in out}) != len(out):
        raise ValueError("duplicate edge")
    return out


def square_lattice(L: int, Lc: Optional[int] = None) -> np.ndarray:
    """Open-boundary L x Lc square lattice; spin (r, c) = r*Lc + c.

    Edge order: for each spin in raster order, its right neighbour (if any)
    then its lower neighbour (if any).
    """
    Lc = L if Lc is None else Lc
    edges = []
    for r in range(L):
        for c in range(Lc):
            i = r * Lc + c
            if c + 1 < Lc:
                edges.append((i, i + 1))
            if r + 1 < L:
                edges.append((i, i + Lc))
    return _canon(edges) if edges else np.zeros((0, 2), np.int32)


def chimera(Lr: int, Lc: Optional[int] = None) -> np.ndarray:
    """Chimera graph of Lr x Lc unit cells, each a complete bipartite K_{4,4}.

    Cell (r, c) holds spins 8*(r*Lc + c) + k, k in 0..7. Spins k < 4 form the
    group coupled vertically to the same k in cell (r+1, c); spins k >= 4 form
    the group coupled horizontally to the same k in cell (r, c+1). Intra-cell
    edges join every k < 4 with every k' >= 4 (16 per cell).
    """
    Lc = Lr if Lc is None else Lc
    edges = []
    for r in range(Lr):
        for c in range(Lc):
            base = 8 * (r * Lc + c)
            for k in range(4):
                for kp in range(4, 8):
                    edges.append((base + k, base + kp))
            if r + 1 < Lr:
                below = 8 * ((r + 1) * Lc + c)
                for k in range(4):
                    edges.append((base + k, below + k))
            if c + 1 < Lc:
                right = 8 * (r * Lc + c + 1)
                for k in range(4, 8):
                    edges.append((base + k, right + k))
    return _canon(edges)


def path(n: int) -> np.ndarray:
    return _canon([(i, i + 1) for i in range(n - 1)]) if n > 1 else np.zeros((0, 2), np.int32)


def ring(n: int) -> np.ndarray:
    if n < 3:
        raise ValueError("ring needs n >= 3")
    return _canon([(i, (i + 1) % n) for i in range(n)])


def complete(n: int) -> np.ndarray:
    return _canon([(i, j) for i in range(n) for j in range(i + 1, n)])


def random_tree(n: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform random recursive tree: vertex v > 0 attaches to a random earlier vertex."""
    return _canon([(int(rng.integers(0, v)), v) for v in range(1, n)]) if n > 1 else np.zeros((0, 2), np.int32)


def _connected(n: int, edges: np.ndarray) -> bool:
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    seen = {0}
    stack = [0]
    while stack:
        v = stack.pop()
        for w in adj[v]:
            if w not in seen:
                seen.add(w)
                stack.append(w)
    return len(seen) == n


def random_regular(n: int, d: int, rng: np.random.Generator, max_tries: int = 10000) -> np.ndarray:
    """Random d-regular simple connected graph by the pairing model with rejection.

    n*d stubs are shuffled and paired; pairings with a loop or a repeated edge
    are rejected and redrawn, as are disconnected graphs.
    """
    if (n * d) % 2:
        raise ValueError("n*d must be even")
    stubs = np.repeat(np.arange(n), d)
    for _ in range(max_tries):
        perm = rng.permutation(stubs)
        pairs = perm.reshape(-1, 2)
        if np.any(pairs[:, 0] == pairs[:, 1]):
            continue
        lo = np.minimum(pairs[:, 0], pairs[:, 1])
        hi = np.maximum(pairs[:, 0], pairs[:, 1])
        keys = lo * n + hi
        if len(np.unique(keys)) != len(keys):
            continue
        e = np.stack([lo, hi], 1).astype(np.int32)
        if not _connected(n, e):
            continue
        order = np.lexsort((e[:, 1], e[:, 0]))
        return e[order]
    raise RuntimeError("pairing model failed")


# ----------------------------------------------------------------------------
# couplings and fields
# ----------------------------------------------------------------------------

def pm1(size: int, rng: np.random.Generator) -> np.ndarray:
    """Independent +-1 with probability 1/2 each, int32."""
    return (2 * rng.integers(0, 2, size=size) - 1).astype(np.int32)


def gauss(size: int, rng: np.random.Generator, std: float = 1.0) -> np.ndarray:
    """N(0, std^2) drawn in float64, rounded to float32."""
    return (rng.standard_normal(size) * std).astype(np.float32)


def make(edges: np.ndarray, n: int, rng: np.random.Generator, coupling: str = "pm1",
         field_std: Optional[float] = None, name: str = "") -> Instance:
    m = edges.shape[0]
    if coupling == "pm1":
        J = pm1(m, rng)
    elif coupling == "gauss":
        J = gauss(m, rng)
    else:
        raise ValueError(coupling)
    h = None
    if field_std is not None:
        h = gauss(n, rng, field_std)
        if coupling == "pm1":
            raise ValueError("integer couplings take no Gaussian field")
    return Instance(n=n, edges=edges, J=J, h=h, name=name)


# ----------------------------------------------------------------------------
# the five workload families (small case, headline case, and three more)
# ----------------------------------------------------------------------------

CONFIG_NAMES = {
    0: "square4x4_pm1",
    1: "square16x16_gauss_h_b64",
    2: "square32x32_pm1",
    3: "regular3_uneven16_gauss",
    4: "chimera8x8_pm1",
}


def rng_for(config_id: int, instance_id: int) -> np.random.Generator:
    return np.random.default_rng([config_id, instance_id])


def config_instances(config_id: int, batch: Optional[int] = None, L: Optional[int] = None) -> List[Instance]:
    """Instances of workload ``config_id``; ``batch``/``L`` shrink it for tests.

    0: 4x4 open square, J = +-1, h = 0, one instance.
    1: 16x16 open square, J ~ N(0,1), h ~ N(0, 0.1^2), float32, batch 64.
    2: 32x32 open square, J = +-1 int32, h = 0, one instance.
    3: 16 random 3-regular graphs, n_i = 100 + 20*(i mod 7), J ~ N(0,1), h = 0.
    4: chimera of 8x8 K_{4,4} cells (512 spins), J = +-1, h = 0.
    """
    out = []
    if config_id == 0:
        L = 4 if L is None else L
        e = square_lattice(L)
        for b in range(1 if batch is None else batch):
            out.append(make(e, L * L, rng_for(0, b), "pm1", name=f"sq{L}_pm1_{b}"))
    elif config_id == 1:
        L = 16 if L is None else L
        e = square_lattice(L)
        for b in range(64 if batch is None else batch):
            out.append(make(e, L * L, rng_for(1, b), "gauss", field_std=0.1, name=f"sq{L}_gauss_{b}"))
    elif config_id == 2:
        L = 32 if L is None else L
        e = square_lattice(L)
        for b in range(1 if batch is None else batch):
            out.append(make(e, L * L, rng_for(2, b), "pm1", name=f"sq{L}_pm1_{b}"))
    elif config_id == 3:
        for b in range(16 if batch is None else batch):
            n = (100 + 20 * (b % 7)) if L is None else L
            rng = rng_for(3, b)
            e = random_regular(n, 3, rng)
            out.append(make(e, n, rng, "gauss", name=f"reg3_n{n}_{b}"))
    elif config_id == 4:
        L = 8 if L is None else L
        e = chimera(L)
        for b in range(1 if batch is None else batch):
            out.append(make(e, 8 * L * L, rng_for(4, b), "pm1", name=f"chimera{L}_pm1_{b}"))
    else:
        raise ValueError(config_id)
    return out


def potts_lattice(L: int, batch: int = 1, Lc: Optional[int] = None, coupling: str = "pm1",
                  seed: int = 5) -> List[Instance]:
    """3-state Potts glasses on an open L x Lc square lattice (Appendix C): J = +-1
    (int32) or J ~ N(0, 1) (float32) per edge, instance b drawn from
    ``default_rng([seed, L, b])``. ``h`` is None (the Potts Hamiltonian has no field)."""
    Lc = L if Lc is None else Lc
    e = square_lattice(L, Lc)
    return [make(e, L * Lc, np.random.default_rng([seed, L, b]), coupling, name=f"potts{L}x{Lc}_{coupling}_{b}")
            for b in range(batch)]


def cubic_lattice(Lx: int, Ly: Optional[int] = None, Lz: Optional[int] = None) -> np.ndarray:
    """Open Lx x Ly x Lz simple cubic lattice (the paper's 3D lattices; Ly, Lz
    default to Lx); spin (x, y, z) = (z Ly + y) Lx + x."""
    Ly = Lx if Ly is None else Ly
    Lz = Lx if Lz is None else Lz
    edges = []
    for z in range(Lz):
        for y in range(Ly):
            for x in range(Lx):
                i = (z * Ly + y) * Lx + x
                if x + 1 < Lx:
                    edges.append((i, i + 1))
                if y + 1 < Ly:
                    edges.append((i, i + Lx))
                if z + 1 < Lz:
                    edges.append((i, i + Lx * Ly))
    return _canon(edges) if edges else np.zeros((0, 2), np.int32)


def cubic_instances(Lx: int, Ly: Optional[int] = None, Lz: Optional[int] = None, batch: int = 1,
                    coupling: str = "pm1", field_std: Optional[float] = None, seed: int = 6) -> List[Instance]:
    """Ising instances on an open cubic lattice; instance b drawn from
    ``default_rng([seed, Lx, Ly, Lz, b])``."""
    Ly = Lx if Ly is None else Ly
    Lz = Lx if Lz is None else Lz
    e = cubic_lattice(Lx, Ly, Lz)
    n = Lx * Ly * Lz
    return [make(e, n, np.random.default_rng([seed, Lx, Ly, Lz, b]), coupling, field_std=field_std,
                 name=f"cubic{Lx}x{Ly}x{Lz}_{coupling}_{b}") for b in range(batch)]


def planted(edges: np.ndarray, n: int, rng: np.random.Generator, coupling: str = "pm1"):
    """Mattis (planted) instance J_ij = tau_i tau_j |J0_ij|, h = 0.

    Its ground states are exactly +-tau when the graph is connected and every
    |J0| > 0. Returns (instance, tau) with tau in {+1, -1}^n.
    """
    tau = (2 * rng.integers(0, 2, size=n) - 1).astype(np.int64)
    m = edges.shape[0]
    if coupling == "pm1":
        mag = np.ones(m, np.int64)
        J = (tau[edges[:, 0]] * tau[edges[:, 1]] * mag).astype(np.int32)
    else:
        mag = np.abs(rng.standard_normal(m)) + 0.1
        J = (tau[edges[:, 0]] * tau[edges[:, 1]] * mag).astype(np.float32)
    return Instance(n=n, edges=edges, J=J, h=None, name="planted"), tau.astype(np.int8)


def gauge(inst: Instance, tau: np.ndarray) -> Instance:
    """Gauge transform J'_ij = tau_i tau_j J_ij, h'_i = tau_i h_i (tau in {+1,-1}^n)."""
    t = np.asarray(tau).astype(np.int64)
    J = (inst.J.astype(np.float64) * t[inst.edges[:, 0]] * t[inst.edges[:, 1]]).astype(inst.J.dtype)
    h = None if inst.h is None else (inst.h.astype(np.float64) * t).astype(inst.h.dtype)
    return Instance(n=inst.n, edges=inst.edges, J=J, h=h, name=inst.name + "_gauged")

"""Chimera plans, executed by a host emulation of the kernels' algorithm.

The relabel passes run through the pass emulator (the encoded program the
kernels read); the row chain is computed here from its definition (the best
horizontal-chain energy given the row's vertical groups) by a dynamic
program over the cells. Energies must match the oracle's elimination exactly
(integer couplings) or to float64 rounding (Gaussian couplings and fields),
and the configuration rebuilt row by row (last row first) must attain E*.
"""
import numpy as np
import pytest

import kernel_emulator as K
from oracle import spinglass as O
from paper_2008_06888_amd import binding as B
from paper_2008_06888_amd import instances as I


def sg(v, bit):
    return 1.0 - 2.0 * ((np.asarray(v) >> bit) & 1)


class Couplers:
    """Edges of a chimera instance by role (written independently of the planner)."""

    def __init__(self, rows, cols, edges, J, h):
        self.rows, self.cols = rows, cols
        self.n = 8 * rows * cols
        self.J = np.asarray(J, np.float64)
        self.h = np.zeros(self.n) if h is None else np.asarray(h, np.float64)
        self.intra, self.vert, self.horz = {}, {}, {}
        for e, (a, b) in enumerate(np.asarray(edges)):
            ca, cb, ka, kb = a // 8, b // 8, a % 8, b % 8
            r, c = divmod(ca, cols)
            if ca == cb:
                self.intra[(r, c, ka, kb - 4)] = e
            elif kb == ka and ka < 4:
                self.vert[(r, c, ka)] = e
            else:
                self.horz[(r, c, ka - 4)] = e

    def spin(self, r, c, k):
        return 8 * (r * self.cols + c) + k

    def K(self, r, c):
        """K[w, h]: cell (r, c), vertical group w, horizontal group h (negated energy)."""
        w = np.arange(16)[:, None]
        hh = np.arange(16)[None, :]
        out = np.zeros((16, 16))
        for k in range(4):
            out += sg(w, k) * self.h[self.spin(r, c, k)]
            out += sg(hh, k) * self.h[self.spin(r, c, 4 + k)]
            for l in range(4):
                e = self.intra.get((r, c, k, l))
                if e is not None:
                    out += self.J[e] * sg(w, k) * sg(hh, l)
        return out

    def L(self, r, c):
        a = np.arange(16)[:, None]
        b = np.arange(16)[None, :]
        out = np.zeros((16, 16))
        for l in range(4):
            e = self.horz.get((r, c, l))
            if e is not None:
                out += self.J[e] * sg(a, l) * sg(b, l)
        return out

    def chain(self, r):
        """g(W) for every row state W (index bit 4c + k = v_k of cell c)."""
        W = np.arange(1 << (4 * self.cols))
        D = self.K(r, 0)[W & 15]                                  # [entries, h_0]
        for c in range(1, self.cols):
            best = (D[:, :, None] + self.L(r, c - 1)[None]).max(axis=1)
            D = self.K(r, c)[(W >> (4 * c)) & 15] + best
        return D.max(axis=1)

    def viterbi(self, r, W):
        """Best horizontal groups of row r given its vertical groups W."""
        Ds, bps = [self.K(r, 0)[W & 15]], []
        for c in range(1, self.cols):
            cand = Ds[-1][:, None] + self.L(r, c - 1)
            bps.append(cand.argmax(axis=0))
            Ds.append(self.K(r, c)[(W >> (4 * c)) & 15] + cand.max(axis=0))
        hs = [int(np.argmax(Ds[-1]))]
        for c in range(self.cols - 1, 0, -1):
            hs.append(int(bps[c - 1][hs[-1]]))
        return hs[::-1]

    def bonus(self, r, Wnext):
        """Vertical couplers of rows r -> r + 1 for every row-r state, the next row fixed."""
        V = np.arange(1 << (4 * self.cols))
        out = np.zeros(len(V))
        for c in range(self.cols):
            for k in range(4):
                e = self.vert.get((r, c, k))
                if e is not None:
                    s = 4 * c + k
                    out += self.J[e] * sg(V, s) * sg(Wnext, s)
        return out


def emulate(rows, cols, edges, J, h, tile_bits=0, z2=False):
    n = 8 * rows * cols
    plan = B.Plan(n, edges, chimera=(rows, cols), has_field=h is not None, tile_bits=tile_bits, z2=z2)
    prog = K.load_program(plan)
    cp = Couplers(rows, cols, edges, J, h)
    w = 4 * cols
    assert plan.info()["width"] == w
    assert prog["final_pos"] == list(range(w))
    after = prog["chain_after"]
    assert sorted(r for r in after if r >= 0) == list(range(1, rows))

    def hook(q, state):
        if after[q] >= 0:
            state += cp.chain(after[q])

    x0 = cp.chain(0)
    if z2:
        # half state: only the stored entries (top bit 0) are kept; the chain
        # is even under flipping every spin, so adding it everywhere is the
        # same on them
        x0 = np.where(np.arange(1 << w) < (1 << (w - 1)), x0, np.nan)
    states = K.forward(prog, w, cp.J, cp.h, x0=x0, after_pass=hook, z2=z2)
    # the state after each row: x0, then the output of each row's last pass
    row_state = [x0] + [states[q + 1] for q in range(len(after)) if after[q] >= 0]
    if z2:
        # every entry read at its stored address, as the kernels do
        idx = np.array([K.z2_addr(i, w) for i in range(1 << w)])
        assert not np.any(np.isnan(np.stack([r[: 1 << (w - 1)] for r in row_state])))
        row_state = [r[idx] for r in row_state]
    final = row_state[-1]
    E = -final.max()
    Ws = [0] * rows
    Ws[-1] = int(np.argmax(final))
    for r in range(rows - 1, 0, -1):
        Ws[r - 1] = int(np.argmax(row_state[r - 1] + cp.bonus(r - 1, Ws[r])))
    sigma = np.zeros(n, np.int8)
    for r in range(rows):
        hs = cp.viterbi(r, Ws[r])
        for c in range(cols):
            for k in range(4):
                sigma[cp.spin(r, c, k)] = 1 - 2 * ((Ws[r] >> (4 * c + k)) & 1)
                sigma[cp.spin(r, c, 4 + k)] = 1 - 2 * ((hs[c] >> k) & 1)
    return E, sigma, plan


@pytest.mark.parametrize("rows,cols,tb", [(1, 1, 0), (1, 2, 0), (2, 1, 0), (2, 2, 0), (3, 2, 0), (2, 3, 0),
                                          (3, 3, 0), (3, 3, 8), (2, 4, 0), (2, 4, 9), (3, 4, 10)])
def test_chimera_pm1_matches_oracle(rows, cols, tb):
    rng = np.random.default_rng([71, rows, cols])
    e = I.chimera(rows, cols)
    J = I.pm1(len(e), rng)
    E, sigma, _ = emulate(rows, cols, e, J, None, tb)
    ref = O.eliminate(8 * rows * cols, e, J, None)
    assert E == ref["energy"]
    assert O.energy(8 * rows * cols, e, J, None, sigma) == E


@pytest.mark.parametrize("rows,cols", [(1, 2), (2, 2), (2, 3)])
def test_chimera_gauss_fields_matches_oracle(rows, cols):
    rng = np.random.default_rng([72, rows, cols])
    e = I.chimera(rows, cols)
    x = I.make(e, 8 * rows * cols, rng, "gauss", field_std=0.3)
    E, sigma, _ = emulate(rows, cols, e, x.J, x.h)
    ref = O.eliminate(8 * rows * cols, e, x.J, x.h)
    assert abs(E - ref["energy"]) < 1e-9
    assert np.array_equal(sigma, ref["sigma"])


def test_chimera_brute_force_one_by_two():
    """16 spins: the emulated chain and passes against all 2^16 configurations."""
    rng = np.random.default_rng(73)
    e = I.chimera(1, 2)
    J = I.pm1(len(e), rng)
    E, sigma, _ = emulate(1, 2, e, J, None)
    bf = O.brute_force(16, e, J, None)
    assert E == bf["energy"] and O.energy(16, e, J, None, sigma) == E


def test_chimera_missing_couplers():
    """A subgraph of the chimera graph (missing couplers, as on a real device)."""
    rng = np.random.default_rng(74)
    e = I.chimera(3, 3)
    keep = rng.random(len(e)) > 0.2
    e2 = e[keep]
    J = I.pm1(len(e2), rng)
    E, sigma, _ = emulate(3, 3, e2, J, None)
    ref = O.eliminate(72, e2, J, None)
    assert E == ref["energy"] and O.energy(72, e2, J, None, sigma) == E


def test_chimera_plan_rejects_other_graphs():
    with pytest.raises(B.TTError):
        B.Plan(32, I.square_lattice(4) * 2, chimera=(2, 2))
    with pytest.raises(B.TTError):
        B.Plan(32, I.chimera(2, 2), chimera=(2, 3))      # wrong spin count
    with pytest.raises(B.TTError):
        B.Plan(8 * 9, I.chimera(1, 9), chimera=(1, 9))   # 2^36 state


def test_chimera_full_size_plan_shape():
    """8 x 8 cells: 32-slot state, four relabel passes per row, chains after each row."""
    e = I.chimera(8)
    plan = B.Plan(512, e, chimera=(8, 8))
    info = plan.info()
    assert info["width"] == 32 and info["n_passes"] == 7 * 4
    after = np.frombuffer(plan.program(6), dtype=np.int32)
    assert list(after[after >= 0]) == list(range(1, 8))
    passes = K.load_program(plan)["passes"]
    for P in passes:   # six low index bits shared by every pair of neighbouring tiles
        assert P.t == 14 and P.n_ld >= 6 and P.n_st >= 6


@pytest.mark.parametrize("rows,cols,tb", [(2, 2, 0), (3, 2, 0), (2, 3, 0), (3, 3, 8), (2, 4, 9), (3, 4, 10)])
def test_chimera_half_state_matches_oracle(rows, cols, tb):
    """Half-state chimera plans: passes on the stored half (every stored entry
    written), the row chain on stored entries, the row walk reading every
    entry at its stored address: E* and a ground state of the oracle's."""
    rng = np.random.default_rng([73, rows, cols])
    e = I.chimera(rows, cols)
    J = I.pm1(len(e), rng)
    E, sigma, _ = emulate(rows, cols, e, J, None, tb, z2=True)
    ref = O.eliminate(8 * rows * cols, e, J, None)
    assert E == ref["energy"]
    assert O.energy(8 * rows * cols, e, J, None, sigma) == E

"""Half-state plans (z2, h = 0) on the host emulation of the pass kernels:
with only the tiles whose z2_skip bit is 0 run and every read and write at
the stored address (the complement when the top address bit is 1), every
stored entry of every pass output is written (once, or twice with the same
value), and the energy and the walked-back ground state match the oracle and
the full-state run. CPU only: checks the tile pairing of the encoded program
before any GPU run."""
import numpy as np
import pytest

import kernel_emulator as K
from oracle import spinglass as O
from paper_2008_06888_amd import binding as B
from paper_2008_06888_amd import instances as I


def _run(plan, n, J, z2):
    prog = K.load_program(plan)
    info = plan.info()
    _, fs = plan.ops()
    Jf = J.astype(np.float64)
    zero = np.zeros(n)
    states = K.forward(prog, info["width"], Jf, zero, z2=z2)
    mx, sigma = K.backward(prog, states, len(fs), fs, n, Jf, zero, z2=z2)
    return -mx, sigma


@pytest.mark.parametrize("L,tb", [(4, 7), (6, 7), (8, 7), (9, 8), (10, 7)])
def test_square_lattices(L, tb):
    n = L * L
    e = I.square_lattice(L)
    x = I.make(e, n, np.random.default_rng([61, L]), "gauss")
    plan = B.Plan(n, e, order=list(range(n)), tile_bits=tb, z2=True)
    E, sig = _run(plan, n, x.J, True)
    E0, _ = _run(plan, n, x.J, False)
    ref = O.eliminate(n, e, x.J, None)
    assert abs(E - ref["energy"]) < 1e-9 and E == E0
    assert abs(O.energy(n, e, x.J, None, sig) - ref["energy"]) < 1e-9
    assert np.array_equal(sig, ref["sigma"]) or np.array_equal(sig, -ref["sigma"])


@pytest.mark.parametrize("n,seed", [(14, 0), (20, 1), (26, 2), (32, 3)])
def test_greedy_random_regular(n, seed):
    rng = np.random.default_rng([62, seed])
    e = I.random_regular(n, 3, rng)
    J = I.pm1(len(e), rng)
    plan = B.Plan(n, e, seed=seed, tile_bits=7, z2=True)
    E, sig = _run(plan, n, J, True)
    ref = O.eliminate(n, e, J, None, traceback=False)
    assert E == ref["energy"]
    assert O.energy(n, e, J, None, sig) == ref["energy"]


@pytest.mark.parametrize("case", ["path", "ring", "complete", "two_parts"])
def test_small_graphs(case):
    if case == "path":
        n, e = 9, I.path(9)
    elif case == "ring":
        n, e = 11, I.ring(11)
    elif case == "complete":
        n, e = 8, I.complete(8)
    else:
        n, e = 14, np.concatenate([I.ring(7), I.ring(7) + 7]).astype(np.int32)
    J = I.pm1(len(e), np.random.default_rng([63, n]))
    plan = B.Plan(n, e, seed=1, tile_bits=7, z2=True)
    E, sig = _run(plan, n, J, True)
    ref = O.brute_force(n, e, J, None)
    assert E == ref["energy"] and O.energy(n, e, J, None, sig) == ref["energy"]


def test_z2_needs_a_plan_without_fields():
    with pytest.raises(B.TTError):
        B.Plan(16, I.square_lattice(4), order=list(range(16)), has_field=True, z2=True)
    with pytest.raises(B.TTError):
        B.Plan(32, I.chimera(2, 2), chimera=(2, 2), has_field=True, z2=True)
    with pytest.raises(B.TTError):
        B.Plan(16, I.square_lattice(4), order=list(range(16)), z2=True, n_fixed=2)
    with pytest.raises(B.TTError):
        B.Plan(16, I.square_lattice(4), order=list(range(16)), q=3, z2=True)


@pytest.mark.parametrize("L,tb", [(8, 7), (12, 9), (16, 12)])
def test_half_state_work_counts(L, tb):
    """Plan info of a half-state plan counts the entries its passes visit: a
    pass whose encoded z2_skip is set visits half of its state, the others all
    of it, and the final maximum half of the final state."""
    n = L * L
    e = I.square_lattice(L)
    full = B.Plan(n, e, order=list(range(n)), tile_bits=tb).info()
    half_plan = B.Plan(n, e, order=list(range(n)), tile_bits=tb, z2=True)
    half = half_plan.info()
    passes = K.load_program(half_plan)["passes"]
    frac = [0.5 if P.z2_skip >= 0 else 1.0 for P in passes]
    assert half["entry_updates"] == sum(2.0 * f * 2.0 ** P.w_max for f, P in zip(frac, passes))
    assert half["reduce_ops"] == full["reduce_ops"] / 2
    assert full["terms"] / 2 <= half["terms"] <= full["terms"]
    if all(f == 0.5 for f in frac):
        assert half["terms"] == full["terms"] / 2 and half["elementwise"] == full["elementwise"] / 2


def _split_addresses(w, base, lanes, ks):
    """The buffer addressing of half-state tiles: with lm, km the lane and k
    bit sets and fm the other address bits below w, an entry whose top bit is
    set is read at (base ^ fm) | (lane ^ lm) | (k ^ km). Returns None where
    the top bit is a lane bit (the kernels then address entry by entry)."""
    lm = 0
    for x in lanes:
        lm |= x
    km = 0
    for x in ks:
        km |= x
    assert lm & km == 0 and base & (lm | km) == 0
    full = (1 << w) - 1
    fm = full & ~(lm | km)
    top = w - 1
    if w == 0 or (lm >> top) & 1:
        return None
    out = {}
    for ln in lanes:
        for k in ks:
            a = base | ln | k
            flip = (base >> top) & 1 or (k >> top) & 1
            out[a] = ((base ^ fm) | (ln ^ lm) | (k ^ km)) if flip else a
    return out


@pytest.mark.parametrize("L,tb", [(12, 10), (12, 11), (14, 12), (16, 12), (16, 14)])
def test_half_state_buffer_addressing(L, tb):
    """Every load and store address the pass kernels form on the fast path of
    a half-state plan equals the stored address of its entry."""
    n = L * L
    plan = B.Plan(n, I.square_lattice(L), order=list(range(n)), tile_bits=tb, z2=True)
    prog = K.load_program(plan)
    checked = 0
    for P in prog["passes"]:
        t, tpb = P.t, P.tb
        fin = [P.fin[k] for k in range(P.n_free)]
        fout = [P.fout[k] for k in range(P.n_free)]
        run = [tid for tid in range(1 << P.n_free) if P.z2_skip < 0 or not (tid >> P.z2_skip) & 1]
        for side in ("ld", "st"):
            ns = t if side == "ld" else P.n_st
            nb = min(ns, tpb)
            nk = 1 << (ns - nb)
            if nk != 16:
                continue
            bad = list(getattr(P, side + "_bad"))[:nb]
            had = list(getattr(P, side + "_had"))[:16]
            lanes = [sum(bad[q] for q in range(nb) if (u >> q) & 1) for u in range(1 << nb)]
            w = P.in_w if side == "ld" else P.out_w
            pos = fin if side == "ld" else fout
            for tid in run[:8]:
                if side == "st" and any(p == 255 and (tid >> k) & 1 for k, p in enumerate(pos)):
                    continue   # a duplicate tile: nothing stored
                base = sum(1 << p for k, p in enumerate(pos) if p != 255 and (tid >> k) & 1)
                got = _split_addresses(w, base, lanes, had)
                if got is None:
                    continue
                for a, s in got.items():
                    assert s == K.z2_addr(a, w)
                checked += 1
    assert checked > 0

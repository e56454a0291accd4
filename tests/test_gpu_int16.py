"""GPU parity of the int16 path (TT_I16: int16 couplings and fields, the
state held as int16 and worked on as packed 16-bit integers, k_pass16):
energies, ground states and gradients against the oracle (stored values for
the 64 headline lattices) and bit for bit against the int32 path (the same
plan, tie rules and walk), over tile sizes, greedy plans with integer fields,
the concurrent-parts path, graph replays, the unfused final maximum, sliced
plans and the autotuner; the exact-range guard."""
import json
import os
import sys

import numpy as np
import pytest

from oracle import spinglass as O
from paper_2008_06888_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2008_06888_amd import binding as B  # noqa: E402

DEV = "cuda:0"
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "parity_large.json")))


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x, dt):
    return torch.tensor(np.ascontiguousarray(x).astype(dt), device=DEV)


def both(plan, J32, h32=None, tie=0):
    """(E, sigma, dJ, dh) on the int32 and the int16 path, as numpy."""
    out = []
    for dt in (np.int32, np.int16):
        J = dev(J32, dt)
        h = dev(h32, dt) if h32 is not None else None
        if tie:
            r = B.backward_tie(plan, J, h, tie=tie)
        else:
            r = B.backward(plan, J, h)
        out.append([None if x is None else x.cpu().numpy() for x in r])
    return out


def assert_same(a, b):
    for x, y in zip(a, b):
        if x is None:
            assert y is None
        else:
            assert np.array_equal(x, y)


def test_square4_brute_force():
    insts = I.config_instances(0, batch=4, L=4)
    e = insts[0].edges
    plan = B.Plan(16, e, order=list(range(16)))
    J = np.stack([x.J for x in insts])
    r32, r16 = both(plan, J)
    assert_same(r32, r16)
    for b, x in enumerate(insts):
        bf = O.brute_force(16, e, x.J, None)
        assert r16[0][b] == bf["energy"] and O.energy(16, e, x.J, None, r16[1][b]) == bf["energy"]


def test_headline_pm1_b64_against_stored_oracle():
    insts = I.config_instances(0, batch=64, L=16)
    gold = GOLD["square16_pm1_b64"]["cases"]
    n = 256
    plan = B.Plan(n, insts[0].edges, order=list(range(n)), tile_bits=12)
    say("int16 headline b64 tile 12")
    J = np.stack([x.J for x in insts])
    r32, r16 = both(plan, J)                  # 64 x 2^16 entries: the concurrent-parts path
    assert_same(r32, r16)
    E16 = B.contract(plan, dev(J, np.int16)).cpu().numpy()
    assert np.array_equal(E16, r16[0])
    for b, x in enumerate(insts):
        assert r16[0][b] == gold[str(b)]["energy"], b
        assert O.energy(n, x.edges, x.J, None, r16[1][b]) == gold[str(b)]["energy"], b


@pytest.mark.parametrize("tile", [7, 9, 11, 12, 13, 14])
def test_tiles_with_integer_fields(tile):
    L = 12
    e = I.square_lattice(L)
    rng = np.random.default_rng([16, tile])
    J = (2 * rng.integers(0, 2, (3, len(e))) - 1).astype(np.int32) * rng.integers(1, 4, (3, len(e))).astype(np.int32)
    h = rng.integers(-2, 3, (3, L * L)).astype(np.int32)
    plan = B.Plan(L * L, e, order=list(range(L * L)), has_field=True, tile_bits=tile)
    say("int16 12x12 fields tile", tile, "passes", plan.info()["n_passes"])
    r32, r16 = both(plan, J, h)
    assert_same(r32, r16)
    for b in range(3):
        ref = O.eliminate(L * L, e, J[b], h[b], counts=None)
        assert r16[0][b] == ref["energy"], b
        assert O.energy(L * L, e, J[b], h[b], r16[1][b]) == ref["energy"], b


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_greedy_plans_random_regular(seed):
    n = 60
    rng = np.random.default_rng([17, seed])
    e = I.random_regular(n, 3, rng)
    J = np.stack([I.pm1(len(e), rng) for _ in range(4)])
    h = rng.integers(-1, 2, (4, n)).astype(np.int32)
    plan = B.Plan(n, e, seed=seed, has_field=True)
    say("int16 reg3 n=60 seed", seed, "width", plan.info()["width"])
    for tie in (0, 1, 12345):
        r32, r16 = both(plan, J, h, tie=tie)
        assert_same(r32, r16)
    for b in range(4):
        ref = O.eliminate(n, e, J[b], h[b])
        assert r16[0][b] == ref["energy"] and O.energy(n, e, J[b], h[b], r16[1][b]) == ref["energy"], b


def test_graph_replays_match_eager():
    insts = I.config_instances(0, batch=4, L=10)
    e = insts[0].edges
    plan = B.Plan(100, e, order=list(range(100)))
    J = dev(np.stack([x.J for x in insts]), np.int16)
    first = [x.cpu().numpy() for x in B.backward(plan, J)[:3]]
    for rep in range(4):               # the second call is captured, later ones replay the graph
        again = [x.cpu().numpy() for x in B.backward(plan, J)[:3]]
        assert_same(first, again)
        torch.cuda.synchronize()


def test_unfused_final_maximum():
    """26 x 26 at tile 12: the last pass has 2^14 tiles per instance, so the
    final maximum runs as its own reduction over the int16 state."""
    L = 26
    x = I.config_instances(0, batch=1, L=L)[0]
    plan = B.Plan(L * L, x.edges, order=list(range(L * L)), tile_bits=12)
    say("int16 26x26 width", plan.info()["width"])
    E32 = B.contract(plan, dev(x.J[None], np.int32)).cpu().numpy()
    E16 = B.contract(plan, dev(x.J[None], np.int16)).cpu().numpy()
    assert np.array_equal(E32, E16)


def test_sliced_plan():
    insts = I.cubic_instances(4, batch=3)
    e = insts[0].edges
    plan = B.Plan(64, e, seed=0, n_fixed=3)
    J = np.stack([x.J for x in insts])
    r32, r16 = both(plan, J)
    assert_same(r32, r16)
    for b, x in enumerate(insts):
        assert r16[0][b] == O.eliminate(64, e, x.J, None, traceback=False)["energy"]


def test_autotune_int16():
    insts = I.config_instances(0, batch=8, L=12)
    plan = B.Plan(144, insts[0].edges, order=list(range(144)))
    J = dev(np.stack([x.J for x in insts]), np.int16)
    ref = B.backward(plan, J)[0].cpu().numpy()
    bits, ms = B.autotune(plan, J, config=True)
    say("int16 autotune", bits, ms)
    assert 7 <= bits <= 14
    assert np.array_equal(B.backward(plan, J)[0].cpu().numpy(), ref)


def test_range_guard():
    e = I.square_lattice(8)
    plan = B.Plan(64, e, order=list(range(64)))
    J = torch.full((1, len(e)), 100, dtype=torch.int16, device=DEV)   # sum |J| = 11200 >= 2^13
    with pytest.raises(B.TTError) as ei:
        B.contract(plan, J)
    assert ei.value.code == B.TT_E_RANGE
    J = torch.full((1, len(e)), 70, dtype=torch.int16, device=DEV)    # 7840 < 2^13: exact
    E = B.contract(plan, J).cpu().numpy()[0]
    assert E == -70 * len(e)


@pytest.mark.parametrize("rows,cols,tb", [(1, 3, 0), (2, 2, 0), (3, 3, 8), (3, 4, 9), (4, 4, 0)])
def test_chimera_int16(rows, cols, tb):
    """Chimera plans (relabel passes, row chains, row-by-row argmax) with the
    int16 state: bit for bit the int32 path, energies those of the oracle,
    integer fields included."""
    n = 8 * rows * cols
    e = I.chimera(rows, cols)
    rng = np.random.default_rng([18, rows, cols])
    J = np.stack([I.pm1(len(e), rng) for _ in range(3)])
    h = rng.integers(-1, 2, (3, n)).astype(np.int32)
    for fields in (False, True):
        plan = B.Plan(n, e, chimera=(rows, cols), tile_bits=tb, has_field=fields)
        say("int16 chimera", rows, cols, "fields", fields)
        r32, r16 = both(plan, J, h if fields else None)
        assert_same(r32, r16)
        for b in range(3):
            hb = h[b] if fields else None
            ref = O.eliminate(n, e, J[b], hb, traceback=False)
            assert r16[0][b] == ref["energy"] and O.energy(n, e, J[b], hb, r16[1][b]) == ref["energy"], b


def test_chimera8_int16_full_size():
    """8 x 8 cells (2^32-entry state): the planted instance's E* = -m and
    sigma = +-tau, and a +-J instance equal to the int32 path."""
    e = I.chimera(8)
    x, tau = I.planted(e, 512, np.random.default_rng(93))
    plan = B.Plan(512, e, chimera=(8, 8))
    say("int16 chimera 8x8 planted")
    E, sig, _, _ = B.backward(plan, dev(x.J[None], np.int16))
    s = sig[0].cpu().numpy()
    assert E[0].item() == -len(e)
    assert np.array_equal(s, tau) or np.array_equal(s, -tau)
    y = I.make(e, 512, I.rng_for(4, 0), "pm1")
    say("int16 chimera 8x8 pm1")
    r32, r16 = both(plan, y.J[None])
    assert_same(r32, r16)
    assert O.energy(512, e, y.J, None, r16[1][0]) == r16[0][0]

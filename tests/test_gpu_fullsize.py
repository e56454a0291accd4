"""GPU parity at the full sizes of the measured workloads, against stored
oracle values (tests/golden/parity_large.json, written by
tests/golden/make_parity_golden.py from the oracle alone).

* 16x16 +-J, batch 64, h = 0 (the solves/s workload): E* and the exact
  degeneracy g of every instance; E(sigma) = E* and E(-sigma) = E* (spin flip
  at h = 0); dE/dJ = -sigma_i sigma_j. Run at the tile size the autotuner picks
  and on the two-stream split path the timed call takes.
* 16x16 Gaussian J and h, batch 64: E* within 1e-5 N of the float64 oracle and
  the unique ground state, for all 64 instances, at tile 2^12 and at the
  autotuned tile.
* 16 uneven random 3-regular graphs (n = 100 .. 220) in one call: oracle E* and
  ground state (up to the global flip) where the oracle reaches; E(sigma) = E*,
  dE/dJ = -sigma sigma and gauge invariance of E* for all of them.
"""
import json
import os
import sys
import hashlib

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


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), device=DEV)


def digest(inst):
    h = hashlib.sha256(np.ascontiguousarray(inst.J).tobytes())
    if inst.h is not None:
        h.update(np.ascontiguousarray(inst.h).tobytes())
    return h.hexdigest()[:16]


def sigma_of(s):
    return np.array([-1 if c == "1" else 1 for c in s], np.int8)


def tol(n):
    return 1e-5 * n


@pytest.fixture(scope="module")
def pm1_b64():
    insts = I.config_instances(0, batch=64, L=16)
    gold = GOLD["square16_pm1_b64"]["cases"]
    for b, x in enumerate(insts):
        assert digest(x) == gold[str(b)]["digest"], "generator changed: rerun make_parity_golden.py"
    return insts, gold


@pytest.mark.parametrize("tile", ["autotuned", 12])
def test_square16_pm1_b64_energy_config_count(pm1_b64, tile):
    insts, gold = pm1_b64
    n = 256
    J = dev(np.stack([x.J for x in insts]))
    plan = B.Plan(n, insts[0].edges, order=list(range(n)), tile_bits=0 if tile == "autotuned" else tile)
    if tile == "autotuned":
        bits, _ = B.autotune(plan, J, config=True)
        say("square16 pm1 b64 autotuned tile", bits)
    else:
        say("square16 pm1 b64 tile", tile)
    E, sig, dJ, _ = B.backward(plan, J)                 # 64 x 2^16 entries: the split path
    Ef = B.contract(plan, J)
    E, sig, dJ, Ef = E.cpu().numpy(), sig.cpu().numpy(), dJ.cpu().numpy(), Ef.cpu().numpy()
    assert np.array_equal(E, Ef)
    for b, x in enumerate(insts):
        g = gold[str(b)]
        assert E[b] == g["energy"], b
        assert O.energy(n, x.edges, x.J, None, sig[b]) == g["energy"], b
        assert O.energy(n, x.edges, x.J, None, -sig[b]) == g["energy"], b
        ref_dJ, _ = O.ground_state_gradient(x.edges, sig[b])
        assert np.array_equal(dJ[b], ref_dJ.astype(np.float32)), b
    cplan = B.Plan(n, insts[0].edges, order=list(range(n)))
    say("square16 pm1 b64 count")
    Ec, _, cnt = B.count(cplan, J)
    for b in range(64):
        assert Ec[b] == gold[str(b)]["energy"] and cnt[b] == int(gold[str(b)]["count"]), b
        assert cnt[b] % 2 == 0


@pytest.mark.parametrize("tile", [12, "autotuned"])
def test_square16_gauss_b64_all_instances(tile):
    insts = I.config_instances(1)
    gold = GOLD["square16_gauss_b64"]["cases"]
    n = 256
    plan = B.Plan(n, insts[0].edges, order=list(range(n)), has_field=True,
                  tile_bits=0 if tile == "autotuned" else tile)
    J, h = dev(np.stack([x.J for x in insts])), dev(np.stack([x.h for x in insts]))
    if tile == "autotuned":
        bits, _ = B.autotune(plan, J, h, config=True)
        say("square16 gauss b64 autotuned tile", bits)
    else:
        say("square16 gauss b64 tile", tile)
    E, sig, dJ, dh = B.backward(plan, J, h)
    E, sig, dJ, dh = E.cpu().numpy(), sig.cpu().numpy(), dJ.cpu().numpy(), dh.cpu().numpy()
    worst = 0.0
    for b, x in enumerate(insts):
        g = gold[str(b)]
        assert digest(x) == g["digest"]
        worst = max(worst, abs(E[b] - g["energy"]))
        assert abs(E[b] - g["energy"]) <= tol(n), b
        ref = sigma_of(g["sigma"])
        assert np.array_equal(sig[b], ref), b
        gJ, gh = O.ground_state_gradient(x.edges, ref)
        assert np.array_equal(dJ[b], gJ.astype(np.float32)) and np.array_equal(dh[b], gh.astype(np.float32)), b
    say("max |E - E_oracle| =", worst)


def test_reg3_uneven16_fullsize():
    insts = I.config_instances(3)
    gold = GOLD["reg3_uneven16"]["cases"]
    say("reg3 uneven 16: plans")
    plans = [B.Plan(x.n, x.edges, seed=i) for i, x in enumerate(insts)]
    Js = [dev(x.J) for x in insts]
    say("reg3 uneven 16: autotune")
    for p, j in zip(plans, Js):
        B.autotune(p, j[None], config=True)
    say("reg3 uneven 16: one call")
    E, sig, dJ = B.contract_uneven(plans, Js)
    E = E.cpu().numpy()
    checked = 0
    for i, x in enumerate(insts):
        g = gold[str(i)]
        assert digest(x) == g["digest"]
        s = sig[i].cpu().numpy()
        Es = O.energy(x.n, x.edges, x.J, None, s)
        assert abs(Es - E[i]) <= tol(x.n), i
        gJ, _ = O.ground_state_gradient(x.edges, s)
        assert np.array_equal(dJ[i].cpu().numpy(), gJ.astype(np.float32)), i
        if "energy" in g:
            checked += 1
            assert abs(E[i] - g["energy"]) <= tol(x.n), i
            ref = sigma_of(g["sigma"])
            assert np.array_equal(s, ref) or np.array_equal(s, -ref), i
    assert checked >= 8
    # gauge invariance of E* for every instance (per-instance calls on gauged couplings)
    say("reg3 uneven 16: gauge")
    for i, x in enumerate(insts):
        tau = (2 * np.random.default_rng([40, i]).integers(0, 2, x.n) - 1).astype(np.int8)
        y = I.gauge(x, tau)
        Eg = B.contract(plans[i], dev(y.J[None])).cpu().numpy()[0]
        assert abs(Eg - E[i]) <= tol(x.n), i


def test_split_batch_varying_widths_matches_single_calls():
    """A greedy plan on a random graph changes the state width from pass to
    pass; a batch large enough to run as two concurrent parts must give every
    instance the result of its own call (the parts' state regions stay disjoint)."""
    rng = np.random.default_rng([41, 0])
    n = 100
    e = I.random_regular(n, 3, rng)
    insts = [I.make(e, n, np.random.default_rng([41, 1, b]), "gauss") for b in range(64)]
    plan = B.Plan(n, e, seed=3)
    info = plan.info()
    assert (64 << info["width"]) >= (1 << 20), "must take the split path"
    say("split regression reg3 n=100 batch 64 width", info["width"])
    J = dev(np.stack([x.J for x in insts]))
    E = B.contract(plan, J).cpu().numpy()
    Eb, sig, _, _ = B.backward(plan, J)
    Eb, sig = Eb.cpu().numpy(), sig.cpu().numpy()
    assert np.array_equal(E, Eb)
    for b, x in enumerate(insts):
        E1 = B.contract(plan, J[b:b + 1].contiguous()).cpu().numpy()[0]
        assert E1 == E[b], b
    for b in (0, 31, 32, 63):
        x = insts[b]
        ref = O.eliminate(n, e, x.J, None)
        assert abs(E[b] - ref["energy"]) <= tol(n), b
        assert np.array_equal(sig[b], ref["sigma"]) or np.array_equal(sig[b], -ref["sigma"]), b

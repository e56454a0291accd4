"""GPU parity of sliced plans (tt_plan_create_sliced): s fixed spins, the
2^s reduced instances contracted as batches of the reduced plan, the minimum
over slices (energy), the first minimising slice walked back (ground state),
and the sum of the counts of the minimising slices (degeneracy, Eq. (4)).

Checked against the oracle on the whole graph (energies, ground states,
degeneracies), stored oracle values for 5^3, the unsliced HIP path on the
6 x 6 x 6 lattice, and a planted instance whose ground state is known.
"""
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
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "parity_cubic.json")))


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), device=DEV)


def int_fields(n, seed):
    return np.random.default_rng([77, n, seed]).integers(-1, 2, n).astype(np.int32)


@pytest.mark.parametrize("n_fixed,fixed", [(1, None), (3, None), (5, None), (3, [0, 27, 63]), (2, [9, 10])])
def test_sliced_gauss_fields_against_oracle(n_fixed, fixed):
    """8 x 8 square lattice, J ~ N(0, 1), h ~ N(0, 0.1^2): E*, sigma (unique),
    dE/dJ and dE/dh against the oracle on the whole graph."""
    insts = I.config_instances(1, batch=5, L=8)
    n, e = 64, insts[0].edges
    p = B.Plan(n, e, has_field=True, seed=3, n_fixed=n_fixed, fixed=fixed)
    say("sliced gauss 8x8", n_fixed, fixed, "->", p.fixed().tolist(), "width", p.info()["width"])
    J = dev(np.stack([x.J for x in insts]))
    h = dev(np.stack([x.h for x in insts]))
    Ec = B.contract(p, J, h).cpu().numpy()
    E, sig, dJ, dh = B.backward(p, J, h)
    E, sig, dJ, dh = E.cpu().numpy(), sig.cpu().numpy(), dJ.cpu().numpy(), dh.cpu().numpy()
    for b, x in enumerate(insts):
        ref = O.eliminate(n, e, x.J, x.h)
        assert abs(Ec[b] - ref["energy"]) <= 1e-5 * n and abs(E[b] - ref["energy"]) <= 1e-5 * n, b
        assert np.array_equal(sig[b], ref["sigma"]), b
        gJ, gh = O.ground_state_gradient(e, sig[b])
        assert np.array_equal(dJ[b], gJ.astype(np.float32)) and np.array_equal(dh[b], gh.astype(np.float32))


def test_sliced_gauss_without_fields():
    """No fields: every bond to a fixed spin is still a field of the reduced
    graph; sigma is one of the two ground states sigma, -sigma."""
    insts = I.config_instances(3, batch=3, L=40)
    for x in insts:
        p = B.Plan(x.n, x.edges, seed=1, n_fixed=4)
        say("sliced reg3 n=40", p.fixed().tolist())
        E, sig, _, _ = B.backward(p, dev(x.J[None]))
        ref = O.eliminate(x.n, x.edges, x.J, None)
        s = sig.cpu().numpy()[0]
        assert abs(E.cpu().numpy()[0] - ref["energy"]) <= 1e-5 * x.n
        assert np.array_equal(s, ref["sigma"]) or np.array_equal(s, -ref["sigma"])


@pytest.mark.parametrize("with_h", [False, True])
@pytest.mark.parametrize("n_fixed", [2, 4])
def test_sliced_count_against_oracle(n_fixed, with_h):
    """4 x 4 x 4 cubic lattice, J = +-1 (and integer fields in {-1, 0, 1}):
    E* and the exact degeneracy, and a ground state of the backward walk."""
    insts = I.cubic_instances(4, batch=3)
    n, e = 64, insts[0].edges
    p = B.Plan(n, e, seed=0, has_field=with_h, n_fixed=n_fixed)
    say("sliced count 4^3", n_fixed, with_h, p.fixed().tolist())
    J = dev(np.stack([x.J for x in insts]))
    hs = [int_fields(n, b) for b in range(3)] if with_h else None
    h = dev(np.stack(hs)) if with_h else None
    Ec, _, g = B.count(p, J, h)
    E, sig, _, _ = B.backward(p, J, h)
    E, sig = E.cpu().numpy(), sig.cpu().numpy()
    for b, x in enumerate(insts):
        hb = hs[b] if with_h else None
        ref = O.eliminate(n, e, x.J, hb, counts="exact", traceback=False)
        assert Ec[b] == ref["energy"] and g[b] == ref["count"], b
        assert E[b] == ref["energy"] and O.energy(n, e, x.J, hb, sig[b]) == ref["energy"], b


def test_sliced_cubic5_stored_oracle_values():
    insts = I.cubic_instances(5, batch=4)
    gold = GOLD["cubic5_pm1"]["cases"]
    p = B.Plan(125, insts[0].edges, seed=0, n_fixed=3)
    say("sliced cubic5 width", p.info()["width"], p.fixed().tolist())
    J = dev(np.stack([x.J for x in insts]))
    Ec, _, g = B.count(p, J)
    E = B.contract(p, J).cpu().numpy()
    for b in range(4):
        gb = gold[str(b)]
        assert E[b] == gb["energy"] and Ec[b] == gb["energy"] and g[b] == int(gb["count"]), b


def test_sliced_calls_chunked_under_a_budget():
    """max_bytes admits a few reduced instances per call only: the slices run
    in chunks, with the same results as one call."""
    insts = I.cubic_instances(4, batch=3)
    n, e = 64, insts[0].edges
    free = B.Plan(n, e, seed=0, n_fixed=3)
    w = free.info()["width"]
    tight = B.Plan(n, e, seed=0, n_fixed=3, fixed=free.fixed(), max_bytes=64 << w)
    say("sliced chunks width", w, "budget", 64 << w)
    J = dev(np.stack([x.J for x in insts]))
    assert np.array_equal(B.contract(tight, J).cpu().numpy(), B.contract(free, J).cpu().numpy())
    Et, st, _, _ = B.backward(tight, J)
    Ef, sf, _, _ = B.backward(free, J)
    assert np.array_equal(Et.cpu().numpy(), Ef.cpu().numpy()) and np.array_equal(st.cpu().numpy(), sf.cpu().numpy())
    ct, ft = B.count(tight, J), B.count(free, J)
    assert np.array_equal(ct[0], ft[0]) and ct[2] == ft[2]
    for b, x in enumerate(insts):
        ref = O.eliminate(n, e, x.J, None, counts="exact", traceback=False)
        assert ct[0][b] == ref["energy"] and ct[2][b] == ref["count"]


def test_cubic6_sliced_full_size():
    """6 x 6 x 6, four fixed spins (reduced width <= 28 instead of 30): the
    planted instance's known E* and ground state; on a +-1 instance the same
    E* and g as the unsliced plan, and E(sigma) = E*."""
    e = I.cubic_lattice(6)
    p = B.Plan(216, e, seed=0, n_fixed=4)
    info = p.info()
    assert info["width"] <= 28
    say("cubic6 sliced width", info["width"], "fixed", p.fixed().tolist())
    x, tau = I.planted(e, 216, np.random.default_rng([6, 216]))
    E, sig, _, _ = B.backward(p, dev(x.J[None]))
    assert E.cpu().numpy()[0] == -len(e)
    s = sig.cpu().numpy()[0]
    assert np.array_equal(s, tau) or np.array_equal(s, -tau)
    y = I.cubic_instances(6)[0]
    J = dev(y.J[None])
    say("cubic6 sliced pm1 count")
    Es, _, gs, exs = B.count_with_flags(p, J)
    whole = B.Plan(216, e, seed=0)
    say("cubic6 unsliced pm1 count")
    Ew, _, gw, exw = B.count_with_flags(whole, J)
    assert Es[0] == Ew[0] and gs[0] == gw[0] and exs[0] and exw[0]
    E2, sig2, _, _ = B.backward(p, J)
    assert E2.cpu().numpy()[0] == Ew[0]
    assert O.energy(216, e, y.J, None, sig2.cpu().numpy()[0]) == Ew[0]

"""GPU parity of chimera plans (row relabel passes + row chain kernel).

Small graphs: energies and counts against the oracle's exact elimination,
configurations attain E* (unique ground states of Gaussian instances with
fields compared spin by spin). Full size (8 x 8 cells, 512 spins, a 2^32-entry
state): a planted instance with closed-form E* = -m and g = 2, and for a
random +-J instance the properties that hold at any size: E(sigma) = E*, the
forward energy equals the counting energy, g is even (spin-flip symmetry at
h = 0) and a gauge transform leaves E* and g unchanged.
"""
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


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), device=DEV)


@pytest.mark.parametrize("rows,cols,tb", [(1, 1, 0), (1, 3, 0), (2, 1, 0), (2, 2, 0), (3, 3, 0), (3, 3, 8),
                                          (2, 4, 0), (3, 4, 9), (4, 4, 10)])
def test_chimera_pm1_energy_sigma_count(rows, cols, tb):
    n = 8 * rows * cols
    e = I.chimera(rows, cols)
    insts = [I.make(e, n, I.rng_for(90, b), "pm1") for b in range(3 if rows * cols < 16 else 1)]
    say("chimera pm1", rows, cols, "tile_bits", tb)
    plan = B.Plan(n, e, chimera=(rows, cols), tile_bits=tb)
    J = dev(np.stack([x.J for x in insts]))
    Ef = B.contract(plan, J.float().contiguous()).cpu().numpy()
    E2, sig, dJ, _ = B.backward(plan, J)
    Ec, res, g = B.count(plan, J)
    sig = sig.cpu().numpy()
    dJ = dJ.cpu().numpy()
    for b, x in enumerate(insts):
        ref = O.eliminate(n, e, x.J, None, counts="exact")
        assert Ef[b] == ref["energy"] and E2[b].item() == ref["energy"] and Ec[b] == ref["energy"]
        assert g[b] == ref["count"]
        assert O.energy(n, e, x.J, None, sig[b]) == ref["energy"]
        assert np.array_equal(dJ[b], -(sig[b][e[:, 0]].astype(np.float32) * sig[b][e[:, 1]]))


@pytest.mark.parametrize("rows,cols", [(2, 2), (2, 3), (3, 4)])
def test_chimera_gauss_fields(rows, cols):
    n = 8 * rows * cols
    e = I.chimera(rows, cols)
    insts = [I.make(e, n, I.rng_for(91, b), "gauss", field_std=0.3) for b in range(4)]
    say("chimera gauss+h", rows, cols)
    plan = B.Plan(n, e, chimera=(rows, cols), has_field=True)
    J = dev(np.stack([x.J for x in insts]))
    h = dev(np.stack([x.h for x in insts]))
    E, sig, dJ, dh = B.backward(plan, J, h)
    E = E.cpu().numpy()
    sig = sig.cpu().numpy()
    for b, x in enumerate(insts):
        ref = O.eliminate(n, e, x.J, x.h)
        assert abs(E[b] - ref["energy"]) <= 1e-5 * n
        assert np.array_equal(sig[b], ref["sigma"])
        assert np.array_equal(dh[b].cpu().numpy(), -sig[b].astype(np.float32))


def test_chimera_missing_couplers():
    rng = np.random.default_rng(92)
    e = I.chimera(3, 3)
    e2 = e[rng.random(len(e)) > 0.25]
    J = I.pm1(len(e2), rng)
    say("chimera 3x3 with missing couplers")
    plan = B.Plan(72, e2, chimera=(3, 3))
    E, sig, _, _ = B.backward(plan, dev(J[None]))
    Ec, _, g = B.count(plan, dev(J[None]))
    ref = O.eliminate(72, e2, J, None, counts="exact")
    assert E[0].item() == ref["energy"] and Ec[0] == ref["energy"] and g[0] == ref["count"]
    assert O.energy(72, e2, J, None, sig[0].cpu().numpy()) == ref["energy"]


def test_chimera_full_size_planted():
    """8 x 8 cells: the Mattis instance has E* = -m and exactly the two ground states +-tau."""
    e = I.chimera(8)
    x, tau = I.planted(e, 512, np.random.default_rng(93))
    say("chimera 8x8 planted: backward")
    plan = B.Plan(512, e, chimera=(8, 8))
    E, sig, _, _ = B.backward(plan, dev(x.J[None]))
    sig = sig[0].cpu().numpy()
    assert E[0].item() == -len(e)
    assert np.array_equal(sig, tau) or np.array_equal(sig, -tau)
    plan.close()
    say("chimera 8x8 planted: count")
    plan = B.Plan(512, e, chimera=(8, 8))
    Ec, _, g = B.count(plan, dev(x.J[None]))
    plan.close()
    assert Ec[0] == -len(e) and g[0] == 2


def test_chimera_full_size_random_properties():
    x = I.config_instances(4)[0]
    e = x.edges
    tau = (2 * np.random.default_rng(94).integers(0, 2, 512) - 1).astype(np.int8)
    xg = I.gauge(x, tau)
    say("chimera 8x8 pm1: backward")
    plan = B.Plan(512, e, chimera=(8, 8))
    E, sig, _, _ = B.backward(plan, dev(x.J[None]))
    Ef = B.contract(plan, dev(x.J[None]).float().contiguous()).cpu().numpy()
    E = E[0].item()
    assert Ef[0] == E
    assert O.energy(512, e, x.J, None, sig[0].cpu().numpy()) == E
    plan.close()
    say("chimera 8x8 pm1: count and gauge")
    plan = B.Plan(512, e, chimera=(8, 8))
    Ec, res, g = B.count(plan, dev(x.J[None]))
    Eg, resg, gg = B.count(plan, dev(xg.J[None]))
    plan.close()
    assert Ec[0] == E and Eg[0] == E
    assert g[0] == gg[0] and np.array_equal(res, resg)
    assert g[0] % 2 == 0 and g[0] >= 2

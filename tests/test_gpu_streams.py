"""GPU tests of calls in flight on two streams at once: two plans of the same
graph and configuration, each on its own stream, take consecutive batches, so
one batch's walk overlaps the next batch's passes. Every call owns its
plan's device state, so each result must equal that of the same batch solved
alone, bit for bit."""
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


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("z2", [False, True])
def test_two_streams_alternating_batches(z2):
    L, batch, calls = 16, 64, 6
    n = L * L
    insts = I.config_instances(0, batch=batch, L=L)
    rng = np.random.default_rng([71, int(z2)])
    # a different gauge of the couplings per call (J_ij s_i s_j with random
    # s): every batch its own input, same ground-state energies
    gauges = [rng.choice(np.array([-1, 1], np.int32), size=(batch, n)) for _ in range(calls)]
    e = np.asarray(insts[0].edges)
    Js = [torch.tensor(np.stack([x.J for x in insts]) * g[:, e[:, 0]] * g[:, e[:, 1]], device="cuda:0")
          for g in gauges]
    say("two streams, 16x16 pm1 batch 64, half state" if z2 else "two streams, 16x16 pm1 batch 64")
    ref_plan = B.Plan(n, insts[0].edges, order=list(range(n)), tile_bits=12, parts=1, z2=z2)
    ref = [[t.cpu().numpy() for t in B.backward(ref_plan, J)[:3]] for J in Js]
    plans = [B.Plan(n, insts[0].edges, order=list(range(n)), tile_bits=12, parts=1, z2=z2) for _ in range(2)]
    # two consecutive streams of torch's pool: they take different hardware
    # queues, so the calls really overlap
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    outs = []
    for i, J in enumerate(Js):
        with torch.cuda.stream(streams[i & 1]):
            outs.append(B.backward(plans[i & 1], J)[:3])
    torch.cuda.synchronize()
    for i in range(calls):
        got = [t.cpu().numpy() for t in outs[i]]
        for a, b in zip(ref[i], got):
            assert np.array_equal(a, b), f"call {i}"
    # the energies are those of the oracle (gauge-invariant)
    for k in (0, 31, 63):
        o = O.eliminate(n, insts[k].edges, insts[k].J, None, order=list(range(n)), traceback=False)
        assert all(outs[i][0][k].item() == o["energy"] for i in range(calls))

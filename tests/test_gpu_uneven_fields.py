"""GPU test of the uneven batch with fields (tt_contract_uneven_fields):
instances on different graphs, some with fields and some without, in one
call; E*, sigma, dE/dJ and dE/dh against the oracle's unique ground states and
against one tt_backward call per instance."""
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


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), device=DEV)


def test_uneven_batch_with_and_without_fields():
    rng = np.random.default_rng([60, 0])
    insts = []
    for k, n in enumerate((18, 24, 30, 36, 22, 40)):
        e = I.random_regular(n, 3, rng)
        insts.append(I.make(e, n, np.random.default_rng([60, 1, k]), "gauss", field_std=0.3 if k % 2 == 0 else None))
    plans = [B.Plan(x.n, x.edges, seed=k, has_field=x.h is not None) for k, x in enumerate(insts)]
    Js = [dev(x.J) for x in insts]
    hs = [dev(x.h) if x.h is not None else None for x in insts]
    E, sig, dJ, dh = B.contract_uneven_fields(plans, Js, hs)
    E = E.cpu().numpy()
    for k, x in enumerate(insts):
        ref = O.eliminate(x.n, x.edges, x.J, x.h)
        s = sig[k].cpu().numpy()
        assert abs(E[k] - ref["energy"]) <= 1e-5 * x.n, k
        if x.h is not None:
            assert np.array_equal(s, ref["sigma"]), k
            assert np.array_equal(dh[k].cpu().numpy(), -s.astype(np.float32)), k
        else:
            assert np.array_equal(s, ref["sigma"]) or np.array_equal(s, -ref["sigma"]), k
            assert dh[k] is None
        assert np.array_equal(dJ[k].cpu().numpy(), O.ground_state_gradient(x.edges, s)[0].astype(np.float32)), k
        E1, s1, _, _ = B.backward(plans[k], Js[k][None], hs[k][None] if hs[k] is not None else None)
        assert E1.cpu().numpy()[0] == E[k] and np.array_equal(s1.cpu().numpy()[0], s), k


def test_uneven_fields_checks():
    e = I.square_lattice(4)
    p = B.Plan(16, e, has_field=True, order=list(range(16)))
    J = dev(np.ones(len(e), np.float32))
    with pytest.raises(ValueError):
        B.contract_uneven_fields([p], [J], [None])
    h = dev(np.zeros(16, np.float32))
    h[3] = float("nan")
    with pytest.raises(B.TTError) as ei:
        B.contract_uneven_fields([p], [J], [h])
    assert ei.value.code == B.TT_E_INVAL

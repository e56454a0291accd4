"""GPU parity of the dense tropical matrix product (tt_tgemm) against the oracle.

Bit-exact: the float32 product equals the float64 oracle rounded to float32
(every sum the inputs produce is exact in float64, see oracle/tropical.py).
Shapes span several 128 x 128 output tiles and 16-deep k tiles with ragged
tails, the 1 x 1 x 1 case, and batches.
"""
import sys

import numpy as np
import pytest

from oracle import tropical as T

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2008_06888_amd import binding as B  # noqa: E402

DEV = "cuda:0"


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def operands(rng, shape_a, shape_b):
    A = rng.normal(size=shape_a).astype(np.float32)
    Bm = rng.normal(size=shape_b).astype(np.float32)
    return A, Bm


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (7, 5, 3), (128, 128, 16), (130, 257, 33), (256, 128, 512),
                                   (300, 17, 1000), (1, 1000, 77)])
def test_tgemm_matches_oracle(M, N, K):
    say("tgemm", M, N, K)
    rng = np.random.default_rng([M, N, K])
    A, Bm = operands(rng, (M, K), (K, N))
    C = B.tgemm(torch.tensor(A, device=DEV), torch.tensor(Bm, device=DEV)).cpu().numpy()
    ref = T.maxplus_matmul(A, Bm).astype(np.float32)
    assert C.shape == (M, N)
    assert np.array_equal(C, ref)


def test_tgemm_batched():
    say("tgemm batched 5 x (140, 90, 70)")
    rng = np.random.default_rng(7)
    A, Bm = operands(rng, (5, 140, 70), (5, 70, 90))
    C = B.tgemm(torch.tensor(A, device=DEV), torch.tensor(Bm, device=DEV)).cpu().numpy()
    assert np.array_equal(C, T.maxplus_matmul(A, Bm).astype(np.float32))


def test_tgemm_integer_valued_and_ties():
    """Integer couplings (the +-J case): many equal candidates per entry."""
    say("tgemm integer 200 x 200 x 64")
    rng = np.random.default_rng(11)
    A = rng.integers(-3, 4, size=(200, 64)).astype(np.float32)
    Bm = rng.integers(-3, 4, size=(64, 200)).astype(np.float32)
    C = B.tgemm(torch.tensor(A, device=DEV), torch.tensor(Bm, device=DEV)).cpu().numpy()
    assert np.array_equal(C, T.maxplus_matmul(A, Bm).astype(np.float32))


def test_tgemm_empty_k_gives_minus_infinity():
    """K = 0: the empty maximum is the semiring zero (-inf)."""
    say("tgemm K=0")
    A = torch.empty(3, 0, device=DEV)
    Bm = torch.empty(0, 4, device=DEV)
    C = B.tgemm(A, Bm).cpu().numpy()
    assert C.shape == (3, 4) and np.all(np.isneginf(C))

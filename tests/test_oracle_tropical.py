"""Pins of the tropical-product oracle: explicit loops, the semiring's
identity element, distributivity over max, associativity, scalar offsets,
and the float32 rounding argument."""
import numpy as np

from oracle import tropical as T


def test_matches_explicit_loops():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((7, 5)).astype(np.float32)
    B = rng.standard_normal((5, 9)).astype(np.float32)
    assert np.array_equal(T.maxplus_matmul(A, B), T.maxplus_matmul_loops(A, B))


def test_tropical_identity():
    rng = np.random.default_rng(1)
    B = rng.standard_normal((6, 4))
    I = np.full((6, 6), -np.inf)
    np.fill_diagonal(I, 0.0)          # 0 is the multiplicative identity, -inf the zero (Eq. 2)
    assert np.array_equal(T.maxplus_matmul(I, B), B)


def test_offsets_associativity_distributivity():
    rng = np.random.default_rng(2)
    A = rng.integers(-9, 9, (4, 5)).astype(np.float64)
    B = rng.integers(-9, 9, (5, 6)).astype(np.float64)
    C = rng.integers(-9, 9, (6, 3)).astype(np.float64)
    B2 = rng.integers(-9, 9, (5, 6)).astype(np.float64)
    assert np.array_equal(T.maxplus_matmul(A + 3, B), T.maxplus_matmul(A, B) + 3)
    assert np.array_equal(T.maxplus_matmul(T.maxplus_matmul(A, B), C), T.maxplus_matmul(A, T.maxplus_matmul(B, C)))
    assert np.array_equal(T.maxplus_matmul(A, np.maximum(B, B2)),
                          np.maximum(T.maxplus_matmul(A, B), T.maxplus_matmul(A, B2)))


def test_float32_rounding_commutes_with_max():
    rng = np.random.default_rng(3)
    A = (rng.standard_normal((33, 70)) * 100).astype(np.float32)
    B = (rng.standard_normal((70, 17)) * 100).astype(np.float32)
    ref32 = T.maxplus_matmul(A, B).astype(np.float32)
    direct = (A[:, :, None] + B[None, :, :]).max(axis=1)      # float32 sums
    assert np.array_equal(ref32, direct)

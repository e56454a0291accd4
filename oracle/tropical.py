"""CPU oracle for the dense tropical (max-plus) matrix product.

TEST INFRASTRUCTURE ONLY (see spinglass.py for the usage rule).

C[i, j] = max_k (A[i, k] + B[k, j])  -- the tropical product of Eq. (2)
written out as a matrix product (the "generic BLAS" over max and + of
Sec. III). Computed in float64 from the given (float32) inputs. When the
exponents of two addends differ by at most 29 (true of every input the
tests draw), their sum is exact in float64; max is exact and rounding is
monotonic, so it commutes with max, and rounding the result to float32
gives the float32 product bit for bit.
"""
import numpy as np


def maxplus_matmul(A, B, chunk: int = 64):
    """Tropical product of A [M, K] and B [K, N] (or batches [b, M, K], [b, K, N])."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if A.ndim == 3:
        return np.stack([maxplus_matmul(a, b, chunk) for a, b in zip(A, B)])
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    C = np.full((M, N), -np.inf)
    for k0 in range(0, K, chunk):
        blk = A[:, k0:k0 + chunk, None] + B[None, k0:k0 + chunk, :]   # [M, kc, N]
        C = np.maximum(C, blk.max(axis=1))
    return C


def maxplus_matmul_loops(A, B):
    """The same product by three explicit loops (small inputs only)."""
    M, K = len(A), len(A[0])
    N = len(B[0])
    C = [[-np.inf] * N for _ in range(M)]
    for i in range(M):
        for j in range(N):
            best = -np.inf
            for k in range(K):
                v = float(A[i][k]) + float(B[k][j])
                if v > best:
                    best = v
            C[i][j] = best
    return np.array(C)

// HIP kernel (gfx950) of the dense tropical matrix product
//   C[i, j] = max_k (A[i, k] + B[k, j])
// (Eq. (2) as a matrix product; the paper's "generic BLAS" over max and +).
// It is the contraction of two large tensors over a run of shared labels,
// reshaped as a (batched) matrix product.
//
// Max-plus has no MFMA form, so the product runs on the VALU: each thread
// keeps an 8x8 register tile of C; per pair of k it issues 128 adds and 64
// three-input maxima (max(c, a0 + b0, a1 + b1)), i.e. 1.5 VALU instructions
// per term. Operand tiles (128 x 16 of A, transposed, and 16 x 128 of B) are
// staged in LDS, double-buffered, with the next tile's global loads in flight
// during the current tile's arithmetic.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace tt {

constexpr int TG_T = 256;          // threads (16 x 16)
constexpr int TG_BM = 128, TG_BN = 128, TG_BK = 16;

__global__ __launch_bounds__(TG_T, 2) void k_tgemm(int64_t M, int64_t N, int64_t K, const float* __restrict__ A,
                                                int64_t lda, int64_t sA, const float* __restrict__ B, int64_t ldb,
                                                int64_t sB, float* __restrict__ C, int64_t ldc, int64_t sC) {
  __shared__ float As[2][TG_BK][TG_BM];
  __shared__ float Bs[2][TG_BK][TG_BN];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int64_t bz = blockIdx.z;
  const int64_t m0 = (int64_t)blockIdx.y * TG_BM, n0 = (int64_t)blockIdx.x * TG_BN;
  A += bz * sA;
  B += bz * sB;
  C += bz * sC;
  // global -> register staging: A rows (tid / 2), 8 k's; B row (tid / 16), 8 columns
  const int ar = tid >> 1, ak = (tid & 1) * 8;
  const int bk = tid >> 4, bc = (tid & 15) * 8;
  float ra[8], rb[8];
  auto load_tile = [&](int64_t k0) {
    const int64_t gr = m0 + ar;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t gk = k0 + ak + q;
      ra[q] = (gr < M && gk < K) ? A[gr * lda + gk] : -INFINITY;
    }
    const int64_t gk = k0 + bk;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int64_t gc = n0 + bc + q;
      rb[q] = (gk < K && gc < N) ? B[gk * ldb + gc] : -INFINITY;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 8; ++q) As[buf][ak + q][ar] = ra[q];
#pragma unroll
    for (int q = 0; q < 8; ++q) Bs[buf][bk][bc + q] = rb[q];
  };
  float c[8][8];
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) c[i][j] = -INFINITY;
  const int64_t nk = (K + TG_BK - 1) / TG_BK;
  load_tile(0);
  store_tile(0);
  __syncthreads();
  for (int64_t t = 0; t < nk; ++t) {
    const int buf = (int)(t & 1);
    if (t + 1 < nk) load_tile((t + 1) * TG_BK);   // in flight during the arithmetic below
#pragma unroll 2
    for (int kk = 0; kk < TG_BK; kk += 2) {
      float a0[8], b0[8], a1[8], b1[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        a0[i] = As[buf][kk][ty * 8 + i];
        a1[i] = As[buf][kk + 1][ty * 8 + i];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        b0[j] = Bs[buf][kk][tx * 8 + j];
        b1[j] = Bs[buf][kk + 1][tx * 8 + j];
      }
#pragma unroll
      for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) c[i][j] = fmaxf(c[i][j], fmaxf(a0[i] + b0[j], a1[i] + b1[j]));
    }
    if (t + 1 < nk) {
      store_tile(buf ^ 1);
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int64_t gr = m0 + ty * 8 + i;
    if (gr >= M) continue;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int64_t gc = n0 + tx * 8 + j;
      if (gc < N) C[gr * ldc + gc] = c[i][j];
    }
  }
}

hipError_t launch_tgemm(int batch, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda, int64_t sA,
                        const float* B, int64_t ldb, int64_t sB, float* C, int64_t ldc, int64_t sC,
                        hipStream_t stream) {
  const int64_t gx = (N + TG_BN - 1) / TG_BN, gy = (M + TG_BM - 1) / TG_BM;
  if (gx >= (1ll << 31) || gy >= 65536 || batch >= 65536) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(k_tgemm, dim3((uint32_t)gx, (uint32_t)gy, (uint32_t)batch), dim3(TG_T), 0, stream, M, N, K, A,
                     lda, sA, B, ldb, sB, C, ldc, sC);
  return hipGetLastError();
}

}  // namespace tt

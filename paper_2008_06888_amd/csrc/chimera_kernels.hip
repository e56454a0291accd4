// HIP kernels (gfx950) of the chimera row step (Sec. V, chimera graph).
//
// The sweep state holds the vertical group of four spins of every cell of
// the current row (slot 4 c + k = index bit 4 c + k at every row boundary).
// After the vertical couplers have relabelled the previous row's groups into
// this row's (ordinary GATE passes), each entry W = (w_0 .. w_{C-1}) of the
// state gains the best energy of the row's horizontal chain given W:
//
//   g(W) = max over h_0 .. h_{C-1} of
//          sum_c K_c(w_c, h_c) + sum_c L_c(h_c, h_{c+1}),
//
// K_c the 16 x 16 intra-cell matrix of cell c (with the fields of its
// spins), L_c the 16 x 16 matrix of the horizontal couplers between cells c
// and c + 1 (the black and blue tensors of the paper's chimera network).
// A workgroup covers 2^16 consecutive entries: index bits 0..7 (cells 0, 1)
// vary per entry, bits 8..15 (cells 2, 3) per group of 256 entries, and the
// higher cells are fixed per workgroup. The chain is cut at the link from
// cell 1 to cell 2:
//
//   g(W) = max_{h_2} S(w_0 w_1, h_2) + B_2(w_2 w_3, h_2),
//
// S the chain over cells 0, 1 (with the link to h_2) and B_2 the chain over
// cells 2 .. C-1 (maximised from the far end inwards). Both tables live in
// LDS; each entry then costs one 16-way maximum. With counting, every table
// carries the number of maximising horizontal configurations (Eq. (4)) and
// the state's residues are multiplied by the entry's count.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"
#include "device_mem.hpp"

namespace tt {

constexpr int CH_T = 1024;

__device__ __constant__ uint64_t c_ch_p[3] = {(1ull << 61) - 1, (1ull << 61) - 31, (1ull << 61) - 45};
__device__ __constant__ uint64_t c_ch_c[3] = {1, 31, 45};

// a * b mod p, p = 2^61 - c, a < p, b < 2^34: a b = q 2^61 + r0 with
// q < 2^34, and 2^61 = c (mod p), so a b = q c + r0 < 2p (mod p).
__device__ __forceinline__ uint64_t mulmod_small(uint64_t a, uint64_t b, int r) {
  const uint64_t lo = a * b, hi = __umul64hi(a, b);
  const uint64_t q = (hi << 3) | (lo >> 61);
  const uint64_t s = (lo & ((1ull << 61) - 1)) + q * c_ch_c[r];
  return s >= c_ch_p[r] ? s - c_ch_p[r] : s;
}

__device__ __forceinline__ float sgn4(int v, int bit) { return ((v >> bit) & 1) ? -1.f : 1.f; }

template <typename IT>
__device__ __forceinline__ float coup(cptr<IT> J, int e) {
  return e >= 0 ? (float)J[e] : 0.f;
}

// max with the number of maximisers
__device__ __forceinline__ void vc_acc(float& m, uint32_t& n, float v, uint32_t c) {
  if (v > m) {
    m = v;
    n = c;
  } else if (v == m) {
    n += c;
  }
}

// K[c][16 w + h]: cell c with vertical group w and horizontal group h;
// L[c][16 a + b]: horizontal couplers of cell c (group a) and cell c + 1 (group b).
template <typename IT>
__device__ void chain_tables(cptr<ChimeraRow> R, int cols, cptr<IT> J, cptr<IT> h, float (*K)[256],
                             float (*L)[256]) {
  for (int j = threadIdx.x; j < cols * 256; j += blockDim.x) {
    const int c = j >> 8, wv = (j >> 4) & 15, hv = j & 15;
    float s = 0.f;
    for (int k = 0; k < 4; ++k)
      for (int l = 0; l < 4; ++l) {
        const float Jv = coup(J, R->intra[c][4 * k + l]);
        s += (((wv >> k) ^ (hv >> l)) & 1) ? -Jv : Jv;
      }
    if (h) {
      for (int k = 0; k < 4; ++k) s += sgn4(wv, k) * (float)h[R->vspin[c][k]];
      for (int l = 0; l < 4; ++l) s += sgn4(hv, l) * (float)h[R->hspin[c][l]];
    }
    K[c][j & 255] = s;
  }
  for (int j = threadIdx.x; j < (cols - 1) * 256; j += blockDim.x) {
    const int c = j >> 8, a = (j >> 4) & 15, b = j & 15;
    float s = 0.f;
    for (int l = 0; l < 4; ++l) {
      const float Jv = coup(J, R->horz[c][l]);
      s += (((a ^ b) >> l) & 1) ? -Jv : Jv;
    }
    L[c][j & 255] = s;
  }
}

// SV: the state's entries (float32; int16 with int16 couplings, whose chain
// values are integers well inside int16 by the input check).
template <typename IT, bool COUNT, typename SV = float>
__global__ __launch_bounds__(CH_T) void k_chain(const ChainItem* __restrict__ item) {
  const auto& I = *as_const(item);
  __shared__ float K[8][256], L[8][256];
  __shared__ float S[256][17];
  __shared__ __align__(16) float B2[256][16];
  __shared__ float B3[256], A0[256], F[2][16];
  constexpr int NC = COUNT ? 256 : 1;
  __shared__ uint32_t Sc[NC][17], B2c[NC][16], B3c[NC], A0c[NC], Fc[2][16];

  const int64_t inst = (int64_t)(blockIdx.x >> I.log2_blocks);
  const uint64_t blk = blockIdx.x & ((1u << I.log2_blocks) - 1u);
  const cptr<IT> J = as_const(static_cast<const IT*>(I.J)) + inst * I.jst;
  const cptr<IT> h = I.h ? as_const(static_cast<const IT*>(I.h)) + inst * I.hst : nullptr;
  const int cols = I.cols, tid = threadIdx.x;
  chain_tables<IT>(as_const(I.row), cols, J, h, K, L);
  __syncthreads();
  // A0[16 w0 + h1] = max over h0 of K_0(w0, h0) + L_0(h0, h1)
  if (cols >= 2 && tid < 256) {
    const int w0 = tid >> 4, h1 = tid & 15;
    float m = -INFINITY;
    uint32_t n = 0;
    for (int h0 = 0; h0 < 16; ++h0) vc_acc(m, n, K[0][16 * w0 + h0] + L[0][16 * h0 + h1], 1u);
    A0[tid] = m;
    if (COUNT) A0c[tid] = n;
  }
  __syncthreads();
  // S[w0 + 16 w1][h2] = max over h0, h1 of the chain over cells 0, 1 (+ link to h2)
  const int lh2 = cols >= 3 ? 4 : 0;
  for (int j = tid; j < (256 << lh2); j += CH_T) {
    const int idx = j >> lh2, h2 = j & ((1 << lh2) - 1);
    const int w0 = idx & 15, w1 = idx >> 4;
    float m = -INFINITY;
    uint32_t n = 0;
    if (cols == 1) {
      if (w1 == 0)
        for (int h0 = 0; h0 < 16; ++h0) vc_acc(m, n, K[0][16 * w0 + h0], 1u);
    } else {
      for (int h1 = 0; h1 < 16; ++h1) {
        float v = A0[16 * w0 + h1] + K[1][16 * w1 + h1];
        if (cols >= 3) v += L[1][16 * h1 + h2];
        vc_acc(m, n, v, COUNT ? A0c[16 * w0 + h1] : 0u);
      }
    }
    S[idx][h2] = m;
    if (COUNT) Sc[idx][h2] = n;
  }
  // cells 4 .. cols-1 are fixed per workgroup: fold them from the far end
  int fb = 0;
  for (int c = cols - 1; c >= 4; --c) {
    if (tid < 16) {
      const int wc = (int)((blk >> (4 * c - 16)) & 15u);
      float m;
      uint32_t n;
      if (c == cols - 1) {
        m = 0.f;
        n = 1;
      } else {
        m = -INFINITY;
        n = 0;
        for (int hp = 0; hp < 16; ++hp) vc_acc(m, n, L[c][16 * tid + hp] + F[fb][hp], COUNT ? Fc[fb][hp] : 0u);
      }
      F[fb ^ 1][tid] = K[c][16 * wc + tid] + m;
      if (COUNT) Fc[fb ^ 1][tid] = n;
    }
    __syncthreads();
    fb ^= 1;
  }
  // B3[16 w3 + h3] = K_3(w3, h3) + max over h4 of L_3(h3, h4) + F(h4)
  if (cols >= 4 && tid < 256) {
    const int w3 = tid >> 4, h3 = tid & 15;
    float m = 0.f;
    uint32_t n = 1;
    if (cols >= 5) {
      m = -INFINITY;
      n = 0;
      for (int h4 = 0; h4 < 16; ++h4) vc_acc(m, n, L[3][16 * h3 + h4] + F[fb][h4], COUNT ? Fc[fb][h4] : 0u);
    }
    B3[tid] = K[3][16 * w3 + h3] + m;
    if (COUNT) B3c[tid] = n;
  }
  __syncthreads();
  // B2[w2 + 16 w3][h2] = K_2(w2, h2) + max over h3 of L_2(h2, h3) + B3(w3, h3)
  if (cols >= 3) {
    for (int j = tid; j < 4096; j += CH_T) {
      const int mid = j >> 4, h2 = j & 15, w2 = mid & 15, w3 = mid >> 4;
      float m = 0.f;
      uint32_t n = 1;
      if (cols >= 4) {
        m = -INFINITY;
        n = 0;
        for (int h3 = 0; h3 < 16; ++h3)
          vc_acc(m, n, L[2][16 * h2 + h3] + B3[16 * w3 + h3], COUNT ? B3c[16 * w3 + h3] : 0u);
      }
      B2[mid][h2] = K[2][16 * w2 + h2] + m;
      if (COUNT) B2c[mid][h2] = n;
    }
  }
  __syncthreads();

  const int lb = I.w < 16 ? I.w : 16;
  const uint32_t E = 1u << lb;
  const int64_t off = inst * I.sst + (int64_t)(blk << 16);
  const gptr<SV> x = as_global(reinterpret_cast<SV*>(I.x)) + off;
  const int np = I.nres;   // residue planes: three primes, and modulo 2^64 when there are four
  const gptr<uint64_t> nres = COUNT ? as_global(I.n) + inst * np * I.sst + (int64_t)(blk << 16) : nullptr;
  const bool init = I.init != 0;
  const int64_t sst = I.sst;
  auto update = [&](uint32_t e, float g, uint64_t gc) {
    // non-temporal stores: the next launch reads the state from memory
    __builtin_nontemporal_store((SV)(init ? g : (float)x[e] + g), &x[e]);
    if (COUNT) {
      for (int r = 0; r < 3; ++r) {
        const gptr<uint64_t> pr = nres + (int64_t)r * sst + e;
        __builtin_nontemporal_store(init ? gc : mulmod_small(*pr, gc, r), pr);
      }
      if (np > 3) {
        const gptr<uint64_t> pr = nres + 3 * sst + e;
        __builtin_nontemporal_store(init ? gc : *pr * gc, pr);   // wraps modulo 2^64
      }
    }
  };
  if (cols >= 3) {
    const int inner = tid & 255;
    float sv[16];
    uint32_t sc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      sv[q] = S[inner][q];
      sc[q] = COUNT ? Sc[inner][q] : 0u;
    }
#pragma unroll 4
    for (uint32_t e = tid; e < E; e += CH_T) {
      const int mid = (int)(e >> 8);
      float g = -INFINITY;
      uint64_t gc = 0;
      if (!COUNT) {
#pragma unroll
        for (int q = 0; q < 16; q += 2) g = fmaxf(g, fmaxf(sv[q] + B2[mid][q], sv[q + 1] + B2[mid][q + 1]));
      } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const float v = sv[q] + B2[mid][q];
          const uint64_t c = (uint64_t)sc[q] * B2c[mid][q];
          if (v > g) {
            g = v;
            gc = c;
          } else if (v == g) {
            gc += c;
          }
        }
      }
      update(e, g, gc);
    }
  } else {
    for (uint32_t e = tid; e < E; e += CH_T) update(e, S[e][0], COUNT ? Sc[e][0] : 0u);
  }
}

// Backward finish of a chimera plan: one workgroup per instance.
template <typename IT>
__global__ __launch_bounds__(CH_T) void k_chim_finish(const ChimFinishItem* __restrict__ item) {
  const auto& I = *as_const(item);
  __shared__ int8_t sig[8192];
  __shared__ float D[2][64][16];
  __shared__ uint8_t bp[64][8][16];
  const int64_t inst = blockIdx.x;
  const cptr<IT> J = as_const(static_cast<const IT*>(I.J)) + inst * I.jst;
  const cptr<IT> h = I.h ? as_const(static_cast<const IT*>(I.h)) + inst * I.hst : nullptr;
  const int rows = I.n_rows, cols = I.cols, tid = threadIdx.x;
  const cptr<ChimeraRow> rows_d = as_const(I.rows);
  const cptr<uint64_t> args = as_const(I.args);
  const cptr<int32_t> edges = as_const(I.edges);
  // vertical groups: the selected address of each row
  for (int j = tid; j < rows * cols * 4; j += CH_T) {
    const int r = j / (4 * cols), s = j % (4 * cols);
    const uint64_t a = args[(int64_t)r * I.batch + inst];
    sig[rows_d[r].vspin[s >> 2][s & 3]] = ((a >> s) & 1ull) ? -1 : 1;
  }
  // horizontal groups: Viterbi along each row given its vertical groups;
  // thread (r, hh) holds the best chain value ending in h_c = hh
  const int r = tid >> 4, hh = tid & 15;
  const bool act = r < rows;
  const uint64_t a = act ? args[(int64_t)r * I.batch + inst] : 0ull;
  const cptr<ChimeraRow> R = act ? rows_d + r : rows_d;
  int cur = 0;
  for (int c = 0; c < cols; ++c) {
    if (act) {
      const int wc = (int)((a >> (4 * c)) & 15ull);
      float kv = 0.f;
      for (int k = 0; k < 4; ++k)
        for (int l = 0; l < 4; ++l) {
          const float Jv = coup(J, R->intra[c][4 * k + l]);
          kv += (((wc >> k) ^ (hh >> l)) & 1) ? -Jv : Jv;
        }
      if (h) {
        for (int k = 0; k < 4; ++k) kv += sgn4(wc, k) * (float)h[R->vspin[c][k]];
        for (int l = 0; l < 4; ++l) kv += sgn4(hh, l) * (float)h[R->hspin[c][l]];
      }
      float best = 0.f;
      int arg = 0;
      if (c > 0) {
        best = -INFINITY;
        for (int hp = 0; hp < 16; ++hp) {
          float lv = 0.f;
          for (int l = 0; l < 4; ++l) {
            const float Jv = coup(J, R->horz[c - 1][l]);
            lv += (((hp ^ hh) >> l) & 1) ? -Jv : Jv;
          }
          const float v = D[cur][r][hp] + lv;
          if (v > best) {
            best = v;
            arg = hp;
          }
        }
      }
      D[cur ^ 1][r][hh] = best + kv;
      bp[r][c][hh] = (uint8_t)arg;
    }
    __syncthreads();
    cur ^= 1;
  }
  if (act && hh == 0) {
    int hb = 0;
    float bv = D[cur][r][0];
    for (int hp = 1; hp < 16; ++hp)
      if (D[cur][r][hp] > bv) {
        bv = D[cur][r][hp];
        hb = hp;
      }
    for (int c = cols - 1; c >= 0; --c) {
      for (int l = 0; l < 4; ++l) sig[R->hspin[c][l]] = ((hb >> l) & 1) ? -1 : 1;
      if (c > 0) hb = bp[r][c][hb];
    }
  }
  __syncthreads();
  const gptr<int8_t> sigma = as_global(I.sigma);
  const gptr<float> dh = as_global(I.dh), dJ = as_global(I.dJ);
  for (int j = tid; j < I.n; j += CH_T) {
    sigma[inst * I.n + j] = sig[j];
    if (dh) dh[inst * I.n + j] = -(float)sig[j];
  }
  if (dJ)
    for (int64_t e = tid; e < I.m; e += CH_T) {
      const int u = edges[2 * e], v = edges[2 * e + 1];
      dJ[inst * I.m + e] = -(float)(sig[u] * sig[v]);
    }
}

hipError_t launch_chain(const ChainItem* item, int64_t n_blocks, int dtype, bool count, hipStream_t stream) {
  if (n_blocks >= (1ll << 31)) return hipErrorInvalidConfiguration;
  if (count)
    hipLaunchKernelGGL((k_chain<int32_t, true>), dim3((uint32_t)n_blocks), dim3(CH_T), 0, stream, item);
  else if (dtype == 2)
    hipLaunchKernelGGL((k_chain<int16_t, false, int16_t>), dim3((uint32_t)n_blocks), dim3(CH_T), 0, stream, item);
  else if (dtype == 0)
    hipLaunchKernelGGL((k_chain<float, false>), dim3((uint32_t)n_blocks), dim3(CH_T), 0, stream, item);
  else
    hipLaunchKernelGGL((k_chain<int32_t, false>), dim3((uint32_t)n_blocks), dim3(CH_T), 0, stream, item);
  return hipGetLastError();
}

hipError_t launch_chim_finish(const ChimFinishItem* item, int batch, int dtype, hipStream_t stream) {
  if (dtype == 2)
    hipLaunchKernelGGL(k_chim_finish<int16_t>, dim3(batch), dim3(CH_T), 0, stream, item);
  else if (dtype == 0)
    hipLaunchKernelGGL(k_chim_finish<float>, dim3(batch), dim3(CH_T), 0, stream, item);
  else
    hipLaunchKernelGGL(k_chim_finish<int32_t>, dim3(batch), dim3(CH_T), 0, stream, item);
  return hipGetLastError();
}

}  // namespace tt

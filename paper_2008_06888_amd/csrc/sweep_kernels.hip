// HIP kernels (gfx950) of the tropical sweep, energy path: passes, final
// reduction and the argmax-routing backward walk.
//
// A pass applies a run of operations (see plan.hpp) to the state tensor.
// Each workgroup owns one tile: the 2^t entries that share the values of
// every non-resident slot. The tile is read from HBM into LDS (coalesced in
// the order of the input layout), worked on in stages, and written back in
// the order of the output layout, so the bit order of the state changes from
// pass to pass at no extra cost and every load and store streams whole
// cache lines. In a stage each thread holds 16 entries spanning up to four
// gate bits in registers and applies every operation of the stage to them.
//
// Arithmetic is the max-plus semiring of Eq. (2): the tropical product is a
// float add, the tropical sum a float max. Bond entries follow Sec. II: the
// bond matrix is [[J, -J], [-J, J]] with index 0 <-> sigma = +1, so the
// state holds negative energies and its final maximum is -E*.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"
#include "device_mem.hpp"
#include "plan.hpp"

namespace tt {

constexpr int NT = 1024;   // threads per workgroup (energy pass, backward)
constexpr int NTR = 256;   // threads per workgroup (final reduction)


template <typename IT>
__device__ __forceinline__ float ldv(cptr<IT> p, int64_t k) {
  return (float)p[k];
}

// LDS position of tile entry i: the low five bits are XORed with the next
// five, which spreads the strided accesses of a stage over the 32 banks.
__device__ __forceinline__ uint32_t swz(uint32_t i) { return i ^ ((i >> 5) & 31u); }

// Value (0/1) of an encoded slot for an entry with tile index i.
__device__ __forceinline__ uint32_t ebit(uint8_t enc, uint32_t i, uint64_t base_slots) {
  return enc < SLOT_FIXED ? ((i >> enc) & 1u) : (uint32_t)((base_slots >> (enc - SLOT_FIXED)) & 1ull);
}

// Workgroup -> (instance, tile). With `xcd_group` the tiles of one instance
// run on one XCD (workgroups are dispatched round-robin over the 8 XCDs), so
// the pass-to-pass exchange of an instance stays in that XCD's L2.
__device__ __forceinline__ bool wg_to_tile(uint64_t b, int log2_tiles, int batch, int xcd_group, int64_t* inst,
                                           uint64_t* tile) {
  if (xcd_group) {
    const uint64_t xcd = b & 7ull, k = b >> 3;
    *inst = (int64_t)(((k >> log2_tiles) << 3) | xcd);
    *tile = k & ((1ull << log2_tiles) - 1ull);
  } else {
    *inst = (int64_t)(b >> log2_tiles);
    *tile = b & ((1ull << log2_tiles) - 1ull);
  }
  return *inst < batch;
}



// A lane value the compiler may not re-derive (keeps a pre-shifted LDS
// address part from being folded back into a shift after the XOR).
__device__ __forceinline__ uint32_t opaque(uint32_t x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Half-state plans: entry base | lane | k of a tile (three disjoint sets of
// address bits) is stored at itself, or, when its top address bit (w - 1)
// is set, at its complement (base ^ fm) | (lane ^ lm) | (k ^ km), where fm
// holds every address bit below w outside lm | km. When the top bit is a
// lane bit the choice differs across lanes (ok = false: the per-entry path);
// otherwise it is made per tile (the top bit in the base) or per k, both
// wave-uniform, so the buffer accesses keep their scalar parts.
struct Z2Fast {
  bool ok;
  bool tile_flip;
  int top;
  uint64_t fm, lm, km;
};

__device__ __forceinline__ Z2Fast z2_fast(int w, uint64_t base, uint64_t lm, uint64_t km) {
  Z2Fast z;
  z.top = w > 0 ? w - 1 : 0;
  z.lm = lm;
  z.km = km;
  z.fm = (w > 0 ? (~0ull >> (64 - w)) : 0ull) & ~(lm | km);
  z.ok = w > 0 && ((lm >> z.top) & 1ull) == 0;
  // base is the same in every lane: made a scalar so the selections below are too
  z.tile_flip = w > 0 && __builtin_amdgcn_readfirstlane((int)((base >> z.top) & 1ull)) != 0;
  return z;
}

__device__ __forceinline__ bool z2_flip(const Z2Fast& z, uint64_t hk) { return z.tile_flip || ((hk >> z.top) & 1ull); }

// Cache-policy operand of the raw buffer intrinsics: non-temporal.
constexpr int AUX_NT = 2;

// Raw buffer resource over `records` bytes from p (with 0 records every
// access is out of range: loads return zero and touch no memory). Callers
// keep every offset (lane part plus scalar part, disjoint bits) below
// BUF_MAX_ENTRIES floats, i.e. below 2^31 bytes, inside the records.
constexpr uint64_t BUF_MAX_ENTRIES = 1ull << 29;
template <typename P>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(P p, int records = 0x7fffffff) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)(uintptr_t)p, 0, records, 0x00020000);
}

// Value (0/1) of tile bit w of an entry index.
__device__ __forceinline__ uint32_t tbit(uint32_t ix, uint32_t w) { return __builtin_amdgcn_ubfe(ix, w, 1); }


// (value, lowest 64-bit index) maximum of a wave by DPP lane moves, in lane
// 63: quad swaps, half-row and row mirrors, then the broadcasts of lanes 15
// and 31 across rows.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void best64_step(float& v, uint64_t& i) {
  const float ov =
      __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)i, (int)(uint32_t)i, CTRL, ROW_MASK, 0xF, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(i >> 32), (int)(uint32_t)(i >> 32), CTRL, ROW_MASK, 0xF, false);
  const uint64_t oi = ((uint64_t)hi << 32) | lo;
  if (ov > v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}

__device__ __forceinline__ void wave_best64_dpp(float& v, uint64_t& i) {
  best64_step<0xB1, 0xF>(v, i);    // quad_perm [1,0,3,2]
  best64_step<0x4E, 0xF>(v, i);    // quad_perm [2,3,0,1]
  best64_step<0x141, 0xF>(v, i);   // row_half_mirror
  best64_step<0x140, 0xF>(v, i);   // row_mirror
  best64_step<0x142, 0xA>(v, i);   // row_bcast:15 into rows 1 and 3
  best64_step<0x143, 0xC>(v, i);   // row_bcast:31 into rows 2 and 3
}

template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t or_dpp(uint32_t x) {
  return x | (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xF, false);
}

// OR over the whole wave by DPP lane moves (as for the maxima above), made
// uniform from lane 63.
__device__ __forceinline__ uint64_t wave_or_dpp(uint64_t v) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = or_dpp<0xB1, 0xF>(lo);
  hi = or_dpp<0xB1, 0xF>(hi);
  lo = or_dpp<0x4E, 0xF>(lo);
  hi = or_dpp<0x4E, 0xF>(hi);
  lo = or_dpp<0x141, 0xF>(lo);
  hi = or_dpp<0x141, 0xF>(hi);
  lo = or_dpp<0x140, 0xF>(lo);
  hi = or_dpp<0x140, 0xF>(hi);
  lo = or_dpp<0x142, 0xA>(lo);
  hi = or_dpp<0x142, 0xA>(hi);
  lo = or_dpp<0x143, 0xC>(lo);
  hi = or_dpp<0x143, 0xC>(hi);
  lo = (uint32_t)__builtin_amdgcn_readlane((int)lo, 63);
  hi = (uint32_t)__builtin_amdgcn_readlane((int)hi, 63);
  return ((uint64_t)hi << 32) | lo;
}

// The pass's ops resolved for this instance and tile, one op per lane (lane
// o holds op o of the pass; a pass has at most 64): GATE keeps 2J and the
// four constants J +- cst +- J_first; STAR keeps cst; up to three further
// resident partners follow. Every wave resolves the ops itself, in
// registers, while its tile loads are in flight.
struct OpLanes {
  float J2, p0, m0, p1, m1;
  // kind | lidx << 4 | wf << 8 | sbit << 16 | wl << 24 | sl << 27 | nx << 30
  // (wf: first resident partner bit, 255 none; sbit: STAR spin's tile bit,
  // 255 fixed slot with its sign folded; wl / sl: their stage-bit indices,
  // 4 if not a stage bit; nx: further partners)
  uint32_t pk;
  float x0, x1, x2;   // further partners' couplings (STAR: with the spin's sign)
  uint32_t xwl;       // partner k: tile bit at 7k, stage-bit index at 7k + 4
};

// An op's record and the couplings and field it reads, loaded as soon as the
// pass is known (they do not depend on the tile).
struct OpIn {
  FOp f;
  float hv, Je, Jt[STAR_TERMS];
};

// Zero words: what an op reads in place of a coupling or field it does not
// have, so that every lane loads unconditionally (no branch, no early wait).
__device__ const int32_t g_zero_words[4] = {0, 0, 0, 0};

// The couplings and field an op record refers to.
template <typename IT>
__device__ __forceinline__ void load_op_values(OpIn& x, cptr<IT> Jrow, cptr<IT> hrow) {
  const cptr<IT> zero = as_const(reinterpret_cast<const IT*>(g_zero_words));
  const bool hf = x.f.hspin >= 0, ge = x.f.kind == FK_GATE;
  x.hv = ldv(hf ? hrow : zero, hf ? x.f.hspin : 0);
  x.Je = ldv(ge ? Jrow : zero, ge ? x.f.edge : 0);
#pragma unroll
  for (int k = 0; k < STAR_TERMS; ++k) x.Jt[k] = ldv(k < x.f.nt ? Jrow : zero, k < x.f.nt ? x.f.te[k] : 0);
}

// The op resolved for the tile whose fixed slots hold the bits bs.
__device__ __forceinline__ OpLanes resolve_lane(const OpIn& x, uint64_t bs) {
  const FOp& op = x.f;
  OpLanes r{0.f, 0.f, 0.f, 0.f, 0.f, 0u, 0.f, 0.f, 0.f, 0u};
  float cst = x.hv;
  const uint32_t kind = op.kind, lidx = op.lidx;
  const int nt = op.nt;
#pragma unroll
  for (int k = 0; k < STAR_TERMS; ++k) {
    const uint8_t w = op.w[k];
    if (k < nt && w >= SLOT_FIXED) cst += ((bs >> (w - SLOT_FIXED)) & 1ull) ? -x.Jt[k] : x.Jt[k];
  }
  uint32_t nx = 0, sbit = 255, sl = 4, wf = 255, wl = 4;
  float sg = 1.f;
  const float J = x.Je;
  if (kind == FK_STAR) {
    if (op.bit >= SLOT_FIXED) {
      if ((bs >> (op.bit - SLOT_FIXED)) & 1ull) sg = -1.f;
    } else {
      sbit = op.bit;
      sl = lidx;
    }
    r.p0 = sg * cst;
  } else if (kind == FK_GATE) {
    r.J2 = J + J;
    r.p0 = r.m0 = J + cst;
    r.p1 = r.m1 = J - cst;
  }
  if (kind == FK_STAR || kind == FK_GATE) {
#pragma unroll
    for (int k = 0; k < STAR_TERMS; ++k) {
      const uint8_t w = op.w[k];
      if (k >= nt || w >= SLOT_FIXED) continue;
      const float Jk = x.Jt[k];
      const uint32_t l = op.wl[k] < 4 ? op.wl[k] : 4;
      if (wf == 255) {
        wf = w;
        wl = l;
        if (kind == FK_STAR) {
          r.m0 = sg * Jk;
        } else {
          r.p0 = J + cst + Jk;
          r.m0 = J + cst - Jk;
          r.p1 = J - cst - Jk;
          r.m1 = J - cst + Jk;
        }
      } else {
        const float xj = kind == FK_STAR ? sg * Jk : Jk;
        if (nx == 0) r.x0 = xj;
        else if (nx == 1) r.x1 = xj;
        else r.x2 = xj;
        r.xwl |= ((uint32_t)w | (l << 4)) << (7 * nx);
        ++nx;
      }
    }
  }
  r.pk = kind | (lidx << 4) | (wf << 8) | (sbit << 16) | (wl << 24) | (sl << 27) | (nx << 30);
  return r;
}

// The fields of an op that every lane shares, made wave-uniform: they live in
// scalar registers, so the dispatch on the op's kind and bits is a scalar
// branch and its coefficients are scalar operands.
struct UOp {
  float J2, p0, m0, p1, m1;
  uint32_t kind, lidx, wf, nx, sbit, wl, sl;
};

// Further resident partners of an op (rare), also wave-uniform.
struct XOp {
  float xJ[3];
  uint32_t xwl;
};

__device__ __forceinline__ float rl_f(float x, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), k));
}

__device__ __forceinline__ UOp op_at(const OpLanes& R, int k) {
  UOp u;
  u.J2 = rl_f(R.J2, k);
  u.p0 = rl_f(R.p0, k);
  u.m0 = rl_f(R.m0, k);
  u.p1 = rl_f(R.p1, k);
  u.m1 = rl_f(R.m1, k);
  const uint32_t pk = (uint32_t)__builtin_amdgcn_readlane((int)R.pk, k);
  u.kind = pk & 15u;
  u.lidx = (pk >> 4) & 15u;
  u.wf = (pk >> 8) & 255u;
  u.sbit = (pk >> 16) & 255u;
  u.wl = (pk >> 24) & 7u;
  u.sl = (pk >> 27) & 7u;
  u.nx = pk >> 30;
  return u;
}

__device__ __forceinline__ XOp xop_at(const OpLanes& R, int k) {
  XOp x;
  x.xJ[0] = rl_f(R.x0, k);
  x.xJ[1] = rl_f(R.x1, k);
  x.xJ[2] = rl_f(R.x2, k);
  x.xwl = (uint32_t)__builtin_amdgcn_readlane((int)R.xwl, k);
  return x;
}

// Bit (0/1) of register entry J (a compile-time index) for a slot that is
// stage bit l (< 4) or the non-stage tile bit w (from the group base gb).
template <int J>
__device__ __forceinline__ uint32_t rbit(uint32_t l, uint32_t w, uint32_t gb) {
  return l < 4 ? ((uint32_t)J >> l) & 1u : tbit(gb, w);
}

// Extra star terms of a gate (rare: more than one resident partner).
template <int L>
__device__ __forceinline__ void gate_extra(float (&e0)[8], float (&e1)[8], const XOp& x, uint32_t nx, uint32_t gb) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const uint32_t w = (x.xwl >> (7 * k)) & 15u, l = (x.xwl >> (7 * k + 4)) & 7u;
    const float Jk = (uint32_t)k < nx ? x.xJ[k] : 0.f;
#define TT_EXTRA(P)                                                            \
  {                                                                           \
    constexpr int j0 = ((P >> L) << (L + 1)) | (P & ((1 << L) - 1));         \
    const float sk = rbit<j0>(l, w, gb) ? -Jk : Jk;                            \
    e0[P] += sk;                                                              \
    e1[P] -= sk;                                                              \
  }
    TT_EXTRA(0) TT_EXTRA(1) TT_EXTRA(2) TT_EXTRA(3) TT_EXTRA(4) TT_EXTRA(5) TT_EXTRA(6) TT_EXTRA(7)
#undef TT_EXTRA
  }
}

// Every op of a stage reads the 16 register entries from one array and writes
// all 16 to the other (the stage alternates between two arrays), so no op
// needs register copies to put its results back in place.
//
// One relabelling gate on stage bit L, with the star of the entering spin,
// sw = h + sum_k J_k sigma(partner_k):
//   new[0] = max(a0 + J, a1 - J) + sw = max(a0, a1 - 2J) + (J + sw)
//   new[1] = max(a0 - J, a1 + J) - sw = max(a0 - 2J, a1) + (J - sw).
// The core of a gate pair, max(a0, a1 - J2) + e, with J2 and e scalar
// operands; written as one asm unit per output so that the compiler cannot
// merge the variants below into one body that first copies every pair's
// constant to a vector register.
__device__ __forceinline__ float gate_out_s(float a_keep, float a_move, float J2, float e) {
  float r;
  asm("v_subrev_f32 %0, %3, %2\n\tv_max_f32 %0, %1, %0\n\tv_add_f32 %0, %4, %0"
      : "=&v"(r)
      : "v"(a_keep), "v"(a_move), "s"(J2), "s"(e));
  return r;
}

// W < 4: the first partner is stage bit W, so its sign per pair is known at
// compile time (scalar constants); W == 4: the partner is constant over the
// group (or absent). A gate with further partners (rare) takes gate_x.
template <int L, int W>
__device__ __forceinline__ void gate_l(const float (&a)[16], float (&o)[16], uint32_t gb, const UOp& u) {
  const float J2 = u.J2;
  if constexpr (W == 4) {
    const bool b = u.wf != 255 && tbit(gb, u.wf);
    const float c0 = b ? u.m0 : u.p0, c1 = b ? u.m1 : u.p1;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int j0 = ((p >> L) << (L + 1)) | (p & ((1 << L) - 1));
      const int j1 = j0 | (1 << L);
      o[j0] = fmaxf(a[j0], a[j1] - J2) + c0;
      o[j1] = fmaxf(a[j0] - J2, a[j1]) + c1;
    }
  } else {
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int j0 = ((p >> L) << (L + 1)) | (p & ((1 << L) - 1));
      const int j1 = j0 | (1 << L);
      const bool b = (j0 >> W) & 1;
      o[j0] = gate_out_s(a[j0], a[j1], J2, b ? u.m0 : u.p0);
      o[j1] = gate_out_s(a[j1], a[j0], J2, b ? u.m1 : u.p1);
    }
  }
}

template <int L>
__device__ __forceinline__ void gate_lw(const float (&a)[16], float (&o)[16], uint32_t gb, const UOp& u) {
  switch (u.wl) {
    case 0: gate_l<L, 0>(a, o, gb, u); break;
    case 1: gate_l<L, 1>(a, o, gb, u); break;
    case 2: gate_l<L, 2>(a, o, gb, u); break;
    case 3: gate_l<L, 3>(a, o, gb, u); break;
    default: gate_l<L, 4>(a, o, gb, u); break;
  }
}

template <int L>
__device__ __forceinline__ void gate_x(const float (&a)[16], float (&o)[16], uint32_t gb, const UOp& u,
                                       const XOp& x) {
  const float J2 = u.J2;
  float e0[8], e1[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    e0[p] = u.p0;
    e1[p] = u.p1;
  }
  if (u.wf != 255) {
#define TT_FIRST(P)                                                            \
  {                                                                           \
    constexpr int j0 = ((P >> L) << (L + 1)) | (P & ((1 << L) - 1));         \
    if (rbit<j0>(u.wl, u.wf, gb)) {                                           \
      e0[P] = u.m0;                                                           \
      e1[P] = u.m1;                                                           \
    }                                                                         \
  }
    TT_FIRST(0) TT_FIRST(1) TT_FIRST(2) TT_FIRST(3) TT_FIRST(4) TT_FIRST(5) TT_FIRST(6) TT_FIRST(7)
#undef TT_FIRST
  }
  gate_extra<L>(e0, e1, x, u.nx, gb);
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const int j0 = ((p >> L) << (L + 1)) | (p & ((1 << L) - 1));
    const int j1 = j0 | (1 << L);
    o[j0] = fmaxf(a[j0], a[j1] - J2) + e0[p];
    o[j1] = fmaxf(a[j0] - J2, a[j1]) + e1[p];
  }
}

template <int L>
__device__ __forceinline__ void cut_l(const float (&a)[16], float (&o)[16]) {
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const int j0 = ((p >> L) << (L + 1)) | (p & ((1 << L) - 1));
    const int j1 = j0 | (1 << L);
    const float m = fmaxf(a[j0], a[j1]);
    o[j0] = m;
    o[j1] = m;
  }
}

// Signed coupling of further partner K for register entry J.
template <int J, int K>
__device__ __forceinline__ float xterm(const XOp& x, uint32_t gb) {
  const uint32_t xw = (x.xwl >> (7 * K)) & 15u, xl = (x.xwl >> (7 * K + 4)) & 7u;
  return rbit<J>(xl, xw, gb) ? -x.xJ[K] : x.xJ[K];
}

// Star of a spin that entered without a gate: x += sigma(spin) * sw.
__device__ __forceinline__ void star16(const float (&a)[16], float (&o)[16], uint32_t gb, const UOp& u,
                                       const XOp& x) {
  const uint32_t wl = u.wl, wf = u.wf, sl = u.sl, sbit = u.sbit;
#define TT_STAR(J)                                                              \
  {                                                                            \
    float sw = u.p0;                                                           \
    if (wf != 255) sw += rbit<J>(wl, wf, gb) ? -u.m0 : u.m0;                   \
    if (u.nx > 0) sw += xterm<J, 0>(x, gb);                                     \
    if (u.nx > 1) sw += xterm<J, 1>(x, gb);                                     \
    if (u.nx > 2) sw += xterm<J, 2>(x, gb);                                     \
    o[J] = a[J] + ((sbit != 255 && rbit<J>(sl, sbit, gb)) ? -sw : sw);         \
  }
  TT_STAR(0) TT_STAR(1) TT_STAR(2) TT_STAR(3) TT_STAR(4) TT_STAR(5) TT_STAR(6) TT_STAR(7)
  TT_STAR(8) TT_STAR(9) TT_STAR(10) TT_STAR(11) TT_STAR(12) TT_STAR(13) TT_STAR(14) TT_STAR(15)
#undef TT_STAR
}

// A star with at most one resident partner, specialised on where the
// spin's and the partner's bits are: SL / WL a stage bit (< 4, its sign per
// register entry known at compile time) or 4 (constant over the group: a
// non-stage tile bit, a fixed slot or no partner; sneg / pm carry the
// spin's sign and the signed partner term per thread). The same sums as
// star16, one add per entry.
template <int SL, int WL>
__device__ __forceinline__ void star_sw(const float (&a)[16], float (&o)[16], const UOp& u, bool sneg, float pm) {
  if constexpr (SL < 4 && WL < 4) {
    const float v0 = u.p0 + u.m0, v1 = u.p0 - u.m0;   // partner bit 0 / 1
#pragma unroll
    for (int J = 0; J < 16; ++J) {
      const float sw = ((J >> WL) & 1) ? v1 : v0;
      o[J] = ((J >> SL) & 1) ? a[J] - sw : a[J] + sw;
    }
  } else if constexpr (SL < 4) {
    const float sw = u.p0 + pm;
#pragma unroll
    for (int J = 0; J < 16; ++J) o[J] = ((J >> SL) & 1) ? a[J] - sw : a[J] + sw;
  } else if constexpr (WL < 4) {
    const float v0 = u.p0 + u.m0, v1 = u.p0 - u.m0;
    const float c0 = sneg ? -v0 : v0, c1 = sneg ? -v1 : v1;
#pragma unroll
    for (int J = 0; J < 16; ++J) o[J] = a[J] + (((J >> WL) & 1) ? c1 : c0);
  } else {
    const float sw = u.p0 + pm;
    const float c = sneg ? -sw : sw;
#pragma unroll
    for (int J = 0; J < 16; ++J) o[J] = a[J] + c;
  }
}

__device__ __forceinline__ void star_fast(const float (&a)[16], float (&o)[16], uint32_t gb, const UOp& u) {
  const bool sneg = u.sl == 4 && u.sbit != 255 && tbit(gb, u.sbit);
  const float pm = (u.wl == 4 && u.wf != 255) ? (tbit(gb, u.wf) ? -u.m0 : u.m0) : 0.f;
#define TT_SW(S, W) \
  case S * 5 + W: star_sw<S, W>(a, o, u, sneg, pm); break;
  switch (u.sl * 5 + u.wl) {
    TT_SW(0, 1) TT_SW(0, 2) TT_SW(0, 3) TT_SW(0, 4)
    TT_SW(1, 0) TT_SW(1, 2) TT_SW(1, 3) TT_SW(1, 4)
    TT_SW(2, 0) TT_SW(2, 1) TT_SW(2, 3) TT_SW(2, 4)
    TT_SW(3, 0) TT_SW(3, 1) TT_SW(3, 2) TT_SW(3, 4)
    TT_SW(4, 0) TT_SW(4, 1) TT_SW(4, 2) TT_SW(4, 3)
    default: star_sw<4, 4>(a, o, u, sneg, pm); break;
  }
#undef TT_SW
}

// One op of a stage: reads a, writes every entry of o.
__device__ __forceinline__ void apply_op(const float (&a)[16], float (&o)[16], uint32_t gb, const OpLanes& R,
                                         int k) {
  const UOp u = op_at(R, k);
  if (u.kind == FK_STAR) {
    if (u.nx == 0) {
      star_fast(a, o, gb, u);
    } else {
      const XOp x = xop_at(R, k);
      star16(a, o, gb, u, x);
    }
  } else if (u.kind == FK_CUT) {
    switch (u.lidx) {
      case 0: cut_l<0>(a, o); break;
      case 1: cut_l<1>(a, o); break;
      case 2: cut_l<2>(a, o); break;
      default: cut_l<3>(a, o); break;
    }
  } else if (u.nx) {
    const XOp x = xop_at(R, k);
    switch (u.lidx) {
      case 0: gate_x<0>(a, o, gb, u, x); break;
      case 1: gate_x<1>(a, o, gb, u, x); break;
      case 2: gate_x<2>(a, o, gb, u, x); break;
      default: gate_x<3>(a, o, gb, u, x); break;
    }
  } else {
    switch (u.lidx) {
      case 0: gate_lw<0>(a, o, gb, u); break;
      case 1: gate_lw<1>(a, o, gb, u); break;
      case 2: gate_lw<2>(a, o, gb, u); break;
      default: gate_lw<3>(a, o, gb, u); break;
    }
  }
}

// Z2: the launch holds half-state items (their code is compiled out of the
// full-state instantiation).
template <typename IT, bool Z2>
// Six waves per SIMD: the register budget that fits without spilling
// vector registers, for more tile bytes in flight on the memory-bound passes
// of large states (2^32-entry chimera passes 5% faster than at five waves).
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(6))) void k_pass(const PassItem* __restrict__ items,
                                                                                   int n_items) {
  // LDS holds the tile only (2^t floats, dynamic, so it starts at address
  // 0). The byte address of a tile entry is the XOR of a lane's part and a
  // scalar part (the swizzle is linear over GF(2) and the two parts have
  // disjoint bits): one VALU op per access.
  const int64_t wg = blockIdx.x;
  int it = 0;
  const cptr<PassItem> citems = as_const(items);
  while (it + 1 < n_items && wg >= citems[it + 1].wg_begin) ++it;
  const auto& I = citems[it];
  const auto& P = *as_const(I.P);
  const cptr<DevStage> stages = as_const(I.stages);
  const cptr<FOp> fops = as_const(I.fops);
  int64_t inst;
  uint64_t ktile;
  // half-state plans run the tiles with fixed slot z2_skip at 0 only
  const bool z2 = Z2 && I.z2 != 0;
  const int zskip = z2 ? P.z2_skip : -1;
  const int run_bits = P.n_free - (zskip >= 0 ? 1 : 0);
  if (!wg_to_tile((uint64_t)(wg - I.wg_begin), run_bits, I.batch, I.xcd_group, &inst, &ktile)) return;
  const uint64_t tid_bits = z2_tile(ktile, zskip);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const cptr<IT> Jrow = as_const(static_cast<const IT*>(I.J)) + inst * I.jst;
  const cptr<IT> hrow = I.h ? as_const(static_cast<const IT*>(I.h)) + inst * I.hst : nullptr;
  // Set-up in two rounds of loads: first the per-lane tables of the fixed
  // slots and the op records (lane o of every wave takes op o), then the
  // tile itself together with the couplings the ops refer to.
  // Both reads are unconditional (clamped indices: the encoder leaves a
  // record past the last pass's ops), so no wait is forced before the tile's
  // addresses are known.
  const int n_ops = P.n_ops;
  const int li = lane < 48 ? lane : 47;
  const uint32_t fi = P.fin[li], fo = P.fout[li], fr = P.fre[li];
  OpIn opin;
  opin.f = ldc(fops + P.op_begin + (lane < n_ops ? lane : 0));
  const int t = P.t;
  const int tb = P.tb;              // this tile uses threads 0 .. 2^tb - 1
  const uint32_t size = 1u << t;
  // fixed (non-resident) slots of this tile, in slot space and in both
  // layouts: lane k of every wave takes tile-id bit k (n_free <= 48), then
  // an OR across the wave; no serial loop over dependent loads
  uint64_t bs = 0, in_base = 0, out_base = 0, dropped = 0;
  {
    if (lane < P.n_free) {
      const uint64_t b = (tid_bits >> lane) & 1ull;
      bs = b << fr;
      in_base = fi != NO_POS ? b << fi : 0ull;
      out_base = fo != NO_POS ? b << fo : 0ull;
      dropped = fo == NO_POS ? b : 0ull;
    }
    bs = wave_or_dpp(bs);
    in_base = wave_or_dpp(in_base);
    out_base = wave_or_dpp(out_base);
    dropped = wave_or_dpp(dropped);
  }
  const bool stored = dropped == 0;   // only the copy with dropped slots at 0 is kept
  const cptr<float> in = as_const(I.in) + inst * I.in_st;     // read-only in this pass (in != out)
  const gptr<float> out = as_global(I.out) + inst * I.out_st;
  // load: enumeration index u = tid + 2^tb k; bit q of u -> tile bit / address
  // bit. The tile's global loads are issued first and stay in flight while
  // the pass's ops are resolved; then they are written to LDS.
  const int nb_ld = t < tb ? t : tb;
  const bool loader = tid < (1 << nb_ld);
  const int nk_ld = 1 << (t - nb_ld);
  uint32_t ti_ld = 0;
  float vals[16];
  bool fast_ld = false;
  cptr<float> src;
  uint64_t ad_lo_ld, had_ld[16];
  const bool init = P.init != 0;   // first pass: the state starts at zero, nothing is read
  {
    // the pass's tables are read unconditionally, so their scalar loads
    // issue together instead of one dependent round trip per element
    uint32_t bti[10];
    uint64_t bad[10], had[16];
#pragma unroll
    for (int q = 0; q < 10; ++q) {   // tb <= 10
      bti[q] = P.ld_bti[q];
      bad[q] = P.ld_bad[q];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) had[k] = P.ld_had[k];
    uint64_t ad_lo = 0, all = 0;
#pragma unroll
    for (int q = 0; q < 10; ++q) {
      const uint32_t m = (q < nb_ld) ? (uint32_t)0 - (((uint32_t)tid >> q) & 1u) : 0u;
      ti_ld |= bti[q] & m;
      ad_lo |= bad[q] & (uint64_t)(int64_t)(int32_t)m;
      if (q < nb_ld) all |= bad[q];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) all |= had[k];
    src = in + in_base;
    // the ops' couplings first: they depend only on the op records, and a
    // wait for them below then leaves the tile's loads in flight
    load_op_values<IT>(opin, Jrow, hrow);
    __builtin_amdgcn_sched_barrier(0);   // keep them issued before the tile's loads
    // When every offset in the tile fits the buffer range and each thread takes 16
    // entries (t = tb + 4: every thread of the workgroup loads), the tile
    // is read by buffer loads with the lane's offset in a VGPR and each k's
    // in an SGPR, no per-load address arithmetic. The loads are issued
    // without a branch: otherwise (and in the first pass, whose state
    // starts at zero) the resource has no records and they return zeros
    // without touching memory.
    fast_ld = !init && nk_ld == 16 && all < BUF_MAX_ENTRIES;
    Z2Fast zf{};
    if (z2) {
      uint64_t lm = 0, km = 0;
#pragma unroll
      for (int q = 0; q < 10; ++q)
        if (q < nb_ld) lm |= bad[q];
#pragma unroll
      for (int k = 0; k < 16; ++k) km |= had[k];
      zf = z2_fast(P.in_w, in_base, lm, km);
      fast_ld = fast_ld && zf.ok;
    }
    const __amdgpu_buffer_rsrc_t rs = raw_rsrc(src, fast_ld ? 0x7fffffff : 0);
    const uint32_t off = (uint32_t)ad_lo << 2;
    if (z2) {
      // stored addresses: the complemented entries through a second buffer
      const __amdgpu_buffer_rsrc_t rs2 = raw_rsrc(in + (in_base ^ zf.fm), fast_ld ? 0x7fffffff : 0);
      const uint32_t off2 = (uint32_t)(ad_lo ^ zf.lm) << 2;
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const bool f = z2_flip(zf, had[k]);
        vals[k] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                                f ? rs2 : rs, (int)(f ? off2 : off),
                                                (int)((f ? had[k] ^ zf.km : had[k]) << 2), AUX_NT));
      }
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k)
        vals[k] =
            __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, (int)(had[k] << 2), AUX_NT));
    }
    ad_lo_ld = ad_lo;
#pragma unroll
    for (int k = 0; k < 16; ++k) had_ld[k] = had[k];
  }
  // the ops resolved for this tile (the signs of its fixed slots) while the
  // tile's loads are in flight
  // (every lane resolves a valid record; lanes beyond the pass's ops are
  // never read)
  const OpLanes R = resolve_lane(opin, bs);
  if (loader && !init && !fast_ld) {
    // the general load (64-bit addresses, fewer than 16 entries per thread,
    // or stored addresses of a half-state plan), after the resolve so that
    // its branch does not hold back the loads above
    if (z2) {
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < nk_ld) vals[k] = in[z2_addr(in_base | ad_lo_ld | had_ld[k], P.in_w)];
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < nk_ld) vals[k] = src[ad_lo_ld | had_ld[k]];
    }
  }
  if (loader) {
    uint32_t hs[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) hs[k] = swz(P.ld_hti[k]) << 2;
    const uint32_t ls = opaque(swz(ti_ld) << 2);
    if (nk_ld == 16) {
#pragma unroll
      for (int k = 0; k < 16; ++k) lds_at(ls ^ hs[k]) = vals[k];
    } else {
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < nk_ld) lds_at(ls ^ hs[k]) = vals[k];
    }
  }
  __syncthreads();
  const int n_stages = P.n_stages;
  const uint32_t groups = size >> 4;   // 16 entries each; 1 <= groups <= 2^tb
  // one group per thread. With fewer than 64 groups (t < 10) the first wave
  // does them all, its lanes repeating groups: lanes of one wave read before
  // any of them writes and write the same values, and every lane stays
  // active, so op words can be read from any lane. With 64 or more, whole
  // waves beyond the groups (a launch with more threads than this tile uses)
  // sit the stages out.
  const bool active = (uint32_t)tid < (groups > 64u ? groups : 64u);
  const uint32_t g = (uint32_t)tid & (groups - 1);
  for (int s = 0; s < n_stages; ++s) {
    if (active) {
      const cptr<DevStage> ST = stages + P.stage_begin + s;
      const int ob = ST->op_begin - P.op_begin, oe = ST->op_end - P.op_begin;
      uint32_t so[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) so[j] = ST->soff[j] << 2;
      const uint32_t gb = (uint32_t)ST->g_lo[g & 31u] | (uint32_t)ST->g_hi[g >> 5];
      const uint32_t sg = opaque(((uint32_t)ST->sg_lo[g & 31u] ^ (uint32_t)ST->sg_hi[g >> 5]) << 2);
      float va[16], vb[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) va[j] = lds_at(sg ^ so[j]);
      // ops in pairs: va -> vb -> va; an odd last op copies its result back
      for (int o = ob; o < oe; o += 2) {
        apply_op(va, vb, gb, R, o);
        if (o + 1 < oe) {
          apply_op(vb, va, gb, R, o + 1);
        } else {
#pragma unroll
          for (int j = 0; j < 16; ++j) va[j] = vb[j];
        }
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) lds_at(sg ^ so[j]) = va[j];
    }
    __syncthreads();
  }
  const int64_t red_at = I.red_base + (inst << run_bits) + (int64_t)ktile;
  if (!stored) {
    // a duplicate tile (a dropped slot at 1): nothing to store or rank
    if (I.red_v && tid == 0) {
      as_global(I.red_v)[red_at] = -INFINITY;
      as_global(I.red_i)[red_at] = ~0ull;
    }
    return;
  }
  // store, enumerating the tile in the order of the output layout
  {
    const int ns = P.n_st;
    uint32_t bti[10], hs[16];
    uint64_t bad[10], had[16];
#pragma unroll
    for (int q = 0; q < 10; ++q) {   // tb <= 10
      bti[q] = P.st_bti[q];
      bad[q] = P.st_bad[q];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      hs[k] = swz(P.st_hti[k]) << 2;
      had[k] = P.st_had[k];
    }
    uint32_t ti_lo = 0;
    uint64_t ad_lo = 0, all = 0;
    const int nb = ns < tb ? ns : tb;
#pragma unroll
    for (int q = 0; q < 10; ++q) {
      const uint32_t m = (q < nb) ? (uint32_t)0 - (((uint32_t)tid >> q) & 1u) : 0u;
      ti_lo |= bti[q] & m;
      ad_lo |= bad[q] & (uint64_t)(int64_t)(int32_t)m;
      if (q < nb) all |= bad[q];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) all |= had[k];
    const gptr<float> dst = out + out_base;
    if (I.red_v) {
      // fused final reduction: the tile's maximum over the entries it would
      // store, ties to the lowest output address (as a scan of the stored
      // state would give); the state itself is not stored
      float bv = -INFINITY;
      uint64_t bi = ~0ull;
      if (tid < (1 << nb)) {
        const int nk = 1 << (ns - nb);
        const uint32_t ls = opaque(swz(ti_lo) << 2);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          if (k < nk) {
            const float v = lds_at(ls ^ hs[k]);
            const uint64_t a = z2 ? z2_addr(out_base | ad_lo | had[k], P.out_w) : (out_base | ad_lo | had[k]);
            if (v > bv || (v == bv && a < bi)) {
              bv = v;
              bi = a;
            }
          }
        }
      }
      wave_best64_dpp(bv, bi);
      __syncthreads();   // every tile read is done: LDS is reused below
      const int wv = tid >> 6;
      if ((tid & 63) == 63) {
        lds_at(16 * wv) = bv;
        lds_at(16 * wv + 4) = __uint_as_float((uint32_t)bi);
        lds_at(16 * wv + 8) = __uint_as_float((uint32_t)(bi >> 32));
      }
      __syncthreads();
      if (tid < 64) {
        const int nw = (int)(blockDim.x >> 6);
        bv = -INFINITY;
        bi = ~0ull;
        if (tid < nw) {
          bv = lds_at(16 * tid);
          bi = ((uint64_t)__float_as_uint(lds_at(16 * tid + 8)) << 32) | __float_as_uint(lds_at(16 * tid + 4));
        }
        wave_best64_dpp(bv, bi);
        if (tid == 63) {
          as_global(I.red_v)[red_at] = bv;
          as_global(I.red_i)[red_at] = bi;
        }
      }
      return;
    }
    if (tid < (1 << nb)) {
      const int nk = 1 << (ns - nb);
      const uint32_t ls = opaque(swz(ti_lo) << 2);
      float vals[16];
      bool fast = nk == 16 && all < BUF_MAX_ENTRIES;
      Z2Fast zf{};
      if (z2) {
        // half-state plan: every output at its stored address (the mirror
        // outputs of the tile's complement included)
        uint64_t lm = 0, km = 0;
#pragma unroll
        for (int q = 0; q < 10; ++q)
          if (q < nb) lm |= bad[q];
#pragma unroll
        for (int k = 0; k < 16; ++k) km |= had[k];
        zf = z2_fast(P.out_w, out_base, lm, km);
        fast = fast && zf.ok;
      }
      if (fast) {
#pragma unroll
        for (int k = 0; k < 16; ++k) vals[k] = lds_at(ls ^ hs[k]);
        const __amdgpu_buffer_rsrc_t rs = raw_rsrc(dst);
        const uint32_t off = (uint32_t)ad_lo << 2;
        // non-temporal: the next pass reads the state from memory on any XCD,
        // so it is not kept dirty in this XCD's L2 (which the end of the
        // launch would otherwise write back)
        if (z2) {
          const __amdgpu_buffer_rsrc_t rs2 = raw_rsrc(out + (out_base ^ zf.fm));
          const uint32_t off2 = (uint32_t)(ad_lo ^ zf.lm) << 2;
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            const bool f = z2_flip(zf, had[k]);
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, vals[k]), f ? rs2 : rs,
                                                  (int)(f ? off2 : off), (int)((f ? had[k] ^ zf.km : had[k]) << 2),
                                                  AUX_NT);
          }
        } else {
#pragma unroll
          for (int k = 0; k < 16; ++k)
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, vals[k]), rs, (int)off,
                                                  (int)(had[k] << 2), AUX_NT);
        }
      } else if (z2) {
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (k < nk) vals[k] = lds_at(ls ^ hs[k]);
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (k < nk) __builtin_nontemporal_store(vals[k], &out[z2_addr(out_base | ad_lo | had[k], P.out_w)]);
      } else {
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (k < nk) vals[k] = lds_at(ls ^ hs[k]);
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (k < nk) __builtin_nontemporal_store(vals[k], &dst[ad_lo | had[k]]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 16-bit pass: the program of k_pass for integer couplings given as int16,
// with the state held as int16 in HBM and LDS (half the bytes) and each
// group of 16 register entries packed two to a register (entry j in register
// j & 7, half j >> 3), so every add and max of a stage handles two entries
// per instruction (packed 16-bit integer arithmetic). With NG = 2 each thread
// owns two groups of the tile (half the threads of k_pass), so the decoding
// of every op (scalar work) and the set-up are shared by 32 entries. Exact:
// with S = sum |J| + sum |h| < 2^13 every state value lies in [-S, S] and
// every intermediate (a - 2J, a maximum before its star term) in [-3S, 3S].
// ---------------------------------------------------------------------------

typedef short s2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ s2v pmax(s2v a, s2v b) { return __builtin_elementwise_max(a, b); }
__device__ __forceinline__ s2v pswap(s2v a) { return __builtin_shufflevector(a, a, 1, 0); }
__device__ __forceinline__ s2v plo2(s2v a) { return __builtin_shufflevector(a, a, 0, 0); }
__device__ __forceinline__ s2v phi2(s2v a) { return __builtin_shufflevector(a, a, 1, 1); }
__device__ __forceinline__ s2v pcat_lo(s2v a, s2v b) { return __builtin_shufflevector(a, b, 0, 2); }
__device__ __forceinline__ s2v pcat_hi(s2v a, s2v b) { return __builtin_shufflevector(a, b, 1, 3); }
__device__ __forceinline__ s2v as_s2(uint32_t x) { return __builtin_bit_cast(s2v, x); }
__device__ __forceinline__ uint32_t as_u32(s2v x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ s2v pk(int lo, int hi) { return s2v{(short)lo, (short)hi}; }

// The ops of a pass resolved as 16-bit integers, one op per lane (the float
// resolution converted exactly: every value is an integer of the state's range).
struct OpLanes16 {
  int32_t j2;          // 2J
  uint32_t pm0, pm1;   // (p0, m0), (p1, m1) as int16 pairs
  uint32_t pk;         // as OpLanes
  int32_t x0, x1, x2;  // further partners' couplings
  uint32_t xwl;
};

__device__ __forceinline__ OpLanes16 lanes16(const OpLanes& r) {
  OpLanes16 o;
  o.j2 = (int32_t)r.J2;
  o.pm0 = as_u32(pk((int)r.p0, (int)r.m0));
  o.pm1 = as_u32(pk((int)r.p1, (int)r.m1));
  o.pk = r.pk;
  o.x0 = (int32_t)r.x0;
  o.x1 = (int32_t)r.x1;
  o.x2 = (int32_t)r.x2;
  o.xwl = r.xwl;
  return o;
}

// Wave-uniform fields of op k (scalar registers).
struct UOp16 {
  s2v jj;        // (2J, 2J)
  s2v pm0, pm1;  // (p0, m0), (p1, m1)
  uint32_t kind, lidx, wf, nx, sbit, wl, sl;
};

struct XOp16 {
  int32_t xJ[3];
  uint32_t xwl;
};

__device__ __forceinline__ UOp16 op16_at(const OpLanes16& R, int k) {
  UOp16 u;
  const int j2 = __builtin_amdgcn_readlane(R.j2, k);
  u.jj = pk(j2, j2);
  u.pm0 = as_s2((uint32_t)__builtin_amdgcn_readlane((int)R.pm0, k));
  u.pm1 = as_s2((uint32_t)__builtin_amdgcn_readlane((int)R.pm1, k));
  const uint32_t pkd = (uint32_t)__builtin_amdgcn_readlane((int)R.pk, k);
  u.kind = pkd & 15u;
  u.lidx = (pkd >> 4) & 15u;
  u.wf = (pkd >> 8) & 255u;
  u.sbit = (pkd >> 16) & 255u;
  u.wl = (pkd >> 24) & 7u;
  u.sl = (pkd >> 27) & 7u;
  u.nx = pkd >> 30;
  return u;
}

__device__ __forceinline__ XOp16 xop16_at(const OpLanes16& R, int k) {
  XOp16 x;
  x.xJ[0] = __builtin_amdgcn_readlane(R.x0, k);
  x.xJ[1] = __builtin_amdgcn_readlane(R.x1, k);
  x.xJ[2] = __builtin_amdgcn_readlane(R.x2, k);
  x.xwl = (uint32_t)__builtin_amdgcn_readlane((int)R.xwl, k);
  return x;
}

// Gate on stage bit L < 3 (register pairs d0, d1 = d0 | 2^L, both halves at
// once) or L == 3 (the two halves of each register), for each of the NG
// groups. W: the first partner is stage bit W (< 4, its value per entry
// known here) or constant over a group's entries (4: bit wf of the group
// base, or no partner).
template <int L, int W, int NG>
__device__ __forceinline__ void gate16(const s2v (&a)[NG][8], s2v (&o)[NG][8], const uint32_t (&gb)[NG],
                                       const UOp16& u) {
  const s2v jj = u.jj;
#pragma unroll
  for (int gi = 0; gi < NG; ++gi) {
    const bool bt = W == 4 && u.wf != 255 && tbit(gb[gi], u.wf);
    if constexpr (L < 3) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int d0 = ((p >> L) << (L + 1)) | (p & ((1 << L) - 1));
        const int d1 = d0 | (1 << L);
        s2v c0, c1;
        if constexpr (W < 3) {
          const bool b = (d0 >> W) & 1;
          c0 = b ? phi2(u.pm0) : plo2(u.pm0);
          c1 = b ? phi2(u.pm1) : plo2(u.pm1);
        } else if constexpr (W == 3) {
          c0 = u.pm0;   // low half: partner +1 (p), high half: partner -1 (m)
          c1 = u.pm1;
        } else {
          c0 = bt ? phi2(u.pm0) : plo2(u.pm0);
          c1 = bt ? phi2(u.pm1) : plo2(u.pm1);
        }
        o[gi][d0] = pmax(a[gi][d0], a[gi][d1] - jj) + c0;
        o[gi][d1] = pmax(a[gi][d0] - jj, a[gi][d1]) + c1;
      }
    } else {
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        s2v c;
        if constexpr (W < 3) {
          const bool b = (d >> W) & 1;
          c = b ? pcat_hi(u.pm0, u.pm1) : pcat_lo(u.pm0, u.pm1);
        } else {
          c = bt ? pcat_hi(u.pm0, u.pm1) : pcat_lo(u.pm0, u.pm1);
        }
        o[gi][d] = pmax(a[gi][d], pswap(a[gi][d]) - jj) + c;
      }
    }
  }
}

template <int L, int NG>
__device__ __forceinline__ void gate16_w(const s2v (&a)[NG][8], s2v (&o)[NG][8], const uint32_t (&gb)[NG],
                                         const UOp16& u) {
  if constexpr (L == 3) {
    switch (u.wl) {
      case 0: gate16<3, 0, NG>(a, o, gb, u); break;
      case 1: gate16<3, 1, NG>(a, o, gb, u); break;
      case 2: gate16<3, 2, NG>(a, o, gb, u); break;
      default: gate16<3, 4, NG>(a, o, gb, u); break;   // (a partner on the gate's own bit cannot occur)
    }
  } else {
    switch (u.wl) {
      case 0: gate16<L, 0, NG>(a, o, gb, u); break;
      case 1: gate16<L, 1, NG>(a, o, gb, u); break;
      case 2: gate16<L, 2, NG>(a, o, gb, u); break;
      case 3: gate16<L, 3, NG>(a, o, gb, u); break;
      default: gate16<L, 4, NG>(a, o, gb, u); break;
    }
  }
}

// Bit (0/1) of register entry j (compile-time after unrolling) for a slot
// that is stage bit l (< 4) or non-stage tile bit w.
__device__ __forceinline__ uint32_t rbit16(int j, uint32_t l, uint32_t w, uint32_t gb) {
  return l < 4 ? ((uint32_t)j >> l) & 1u : tbit(gb, w);
}

// The value added to output entry j of a gate on stage bit L with further
// resident partners (rare): as gate_x of the float pass, per entry.
template <int L>
__device__ __forceinline__ int gate_const16(int j, const UOp16& u, const XOp16& x, uint32_t gb) {
  const int j0 = j & ~(1 << L);
  const bool upper = (j >> L) & 1;
  const bool bf = u.wf != 255 && rbit16(j0, u.wl, u.wf, gb);
  const s2v pm = upper ? u.pm1 : u.pm0;
  int c = bf ? pm.y : pm.x;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if ((uint32_t)k >= u.nx) break;
    const uint32_t w = (x.xwl >> (7 * k)) & 15u, l = (x.xwl >> (7 * k + 4)) & 7u;
    const int sk = rbit16(j0, l, w, gb) ? -x.xJ[k] : x.xJ[k];
    c += upper ? -sk : sk;
  }
  return c;
}

template <int L, int NG>
__device__ __forceinline__ void gate16_x(const s2v (&a)[NG][8], s2v (&o)[NG][8], const uint32_t (&gb)[NG],
                                         const UOp16& u, const XOp16& x) {
  const s2v jj = u.jj;
#pragma unroll
  for (int gi = 0; gi < NG; ++gi) {
    if constexpr (L < 3) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int d0 = ((p >> L) << (L + 1)) | (p & ((1 << L) - 1));
        const int d1 = d0 | (1 << L);
        const s2v c0 = pk(gate_const16<L>(d0, u, x, gb[gi]), gate_const16<L>(d0 + 8, u, x, gb[gi]));
        const s2v c1 = pk(gate_const16<L>(d1, u, x, gb[gi]), gate_const16<L>(d1 + 8, u, x, gb[gi]));
        o[gi][d0] = pmax(a[gi][d0], a[gi][d1] - jj) + c0;
        o[gi][d1] = pmax(a[gi][d0] - jj, a[gi][d1]) + c1;
      }
    } else {
#pragma unroll
      for (int d = 0; d < 8; ++d) {
        const s2v c = pk(gate_const16<3>(d, u, x, gb[gi]), gate_const16<3>(d + 8, u, x, gb[gi]));
        o[gi][d] = pmax(a[gi][d], pswap(a[gi][d]) - jj) + c;
      }
    }
  }
}

template <int L, int NG>
__device__ __forceinline__ void cut16(const s2v (&a)[NG][8], s2v (&o)[NG][8]) {
#pragma unroll
  for (int gi = 0; gi < NG; ++gi) {
    if constexpr (L < 3) {
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        const int d0 = ((p >> L) << (L + 1)) | (p & ((1 << L) - 1));
        const int d1 = d0 | (1 << L);
        const s2v m = pmax(a[gi][d0], a[gi][d1]);
        o[gi][d0] = m;
        o[gi][d1] = m;
      }
    } else {
#pragma unroll
      for (int d = 0; d < 8; ++d) o[gi][d] = pmax(a[gi][d], pswap(a[gi][d]));
    }
  }
}

// Star of a spin that entered without a gate: x += sigma(spin) * sw with
// sw = p0 + sigma(first partner) m0 + further partners (per entry).
__device__ __forceinline__ int star_val16(int j, const UOp16& u, const XOp16& x, uint32_t gb) {
  int sw = u.pm0.x;
  if (u.wf != 255) sw += rbit16(j, u.wl, u.wf, gb) ? -(int)u.pm0.y : (int)u.pm0.y;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if ((uint32_t)k >= u.nx) break;
    const uint32_t w = (x.xwl >> (7 * k)) & 15u, l = (x.xwl >> (7 * k + 4)) & 7u;
    sw += rbit16(j, l, w, gb) ? -x.xJ[k] : x.xJ[k];
  }
  return (u.sbit != 255 && rbit16(j, u.sl, u.sbit, gb)) ? -sw : sw;
}

template <int NG>
__device__ __forceinline__ void star16p(const s2v (&a)[NG][8], s2v (&o)[NG][8], const uint32_t (&gb)[NG],
                                        const UOp16& u, const XOp16& x) {
#pragma unroll
  for (int gi = 0; gi < NG; ++gi)
#pragma unroll
    for (int d = 0; d < 8; ++d) o[gi][d] = a[gi][d] + pk(star_val16(d, u, x, gb[gi]), star_val16(d + 8, u, x, gb[gi]));
}

// One op of a stage on the thread's NG groups: decoded once, applied to all.
template <int NG>
__device__ __forceinline__ void apply_op16(const s2v (&a)[NG][8], s2v (&o)[NG][8], const uint32_t (&gb)[NG],
                                           const OpLanes16& R, int k) {
  const UOp16 u = op16_at(R, k);
  if (u.kind == FK_STAR) {
    XOp16 x{{0, 0, 0}, 0u};
    if (u.nx) x = xop16_at(R, k);
    star16p<NG>(a, o, gb, u, x);
  } else if (u.kind == FK_CUT) {
    switch (u.lidx) {
      case 0: cut16<0, NG>(a, o); break;
      case 1: cut16<1, NG>(a, o); break;
      case 2: cut16<2, NG>(a, o); break;
      default: cut16<3, NG>(a, o); break;
    }
  } else if (u.nx) {
    const XOp16 x = xop16_at(R, k);
    switch (u.lidx) {
      case 0: gate16_x<0, NG>(a, o, gb, u, x); break;
      case 1: gate16_x<1, NG>(a, o, gb, u, x); break;
      case 2: gate16_x<2, NG>(a, o, gb, u, x); break;
      default: gate16_x<3, NG>(a, o, gb, u, x); break;
    }
  } else {
    switch (u.lidx) {
      case 0: gate16_w<0, NG>(a, o, gb, u); break;
      case 1: gate16_w<1, NG>(a, o, gb, u); break;
      case 2: gate16_w<2, NG>(a, o, gb, u); break;
      default: gate16_w<3, NG>(a, o, gb, u); break;
    }
  }
}

// The tile index and address (low enumeration bits) of enumeration index u
// from the pass's per-bit tables, bits q < nb.
__device__ __forceinline__ void enum_lo(const uint32_t (&bti)[10], const uint64_t (&bad)[10], uint32_t u, int nb,
                                        uint32_t* ti, uint64_t* ad) {
  uint32_t t = 0;
  uint64_t a = 0;
#pragma unroll
  for (int q = 0; q < 10; ++q) {
    const uint32_t m = (q < nb) ? (uint32_t)0 - ((u >> q) & 1u) : 0u;
    t |= bti[q] & m;
    a |= bad[q] & (uint64_t)(int64_t)(int32_t)m;
  }
  *ti = t;
  *ad = a;
}

// NG = 1: one group per thread, 2^tb threads (as k_pass). NG = 2: two groups
// per thread, 2^(tb-1) threads (tb >= 7); thread i then takes enumeration
// indices i and i + 2^(tb-1) of the loads and stores and groups i and
// i + 2^(tb-1) of every stage.
// (NG = 2 keeps two groups' registers: four waves per SIMD, within 128 VGPRs)
// Z2 as in k_pass.
template <int NG, bool Z2>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NG == 2 ? 4 : 6))) void k_pass16(
    const PassItem* __restrict__ items, int n_items) {
  // LDS holds the tile as int16 (2^t entries, dynamic, from address 0);
  // entry i sits at byte 2 swz(i).
  const int64_t wg = blockIdx.x;
  int it = 0;
  const cptr<PassItem> citems = as_const(items);
  while (it + 1 < n_items && wg >= citems[it + 1].wg_begin) ++it;
  const auto& I = citems[it];
  const auto& P = *as_const(I.P);
  const cptr<DevStage> stages = as_const(I.stages);
  const cptr<FOp> fops = as_const(I.fops);
  int64_t inst;
  uint64_t ktile;
  // half-state plans run the tiles with fixed slot z2_skip at 0 only
  const bool z2 = Z2 && I.z2 != 0;
  const int zskip = z2 ? P.z2_skip : -1;
  const int run_bits = P.n_free - (zskip >= 0 ? 1 : 0);
  if (!wg_to_tile((uint64_t)(wg - I.wg_begin), run_bits, I.batch, I.xcd_group, &inst, &ktile)) return;
  const uint64_t tid_bits = z2_tile(ktile, zskip);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const cptr<int16_t> Jrow = as_const(static_cast<const int16_t*>(I.J)) + inst * I.jst;
  const cptr<int16_t> hrow = I.h ? as_const(static_cast<const int16_t*>(I.h)) + inst * I.hst : nullptr;
  const int n_ops = P.n_ops;
  const int li = lane < 48 ? lane : 47;
  const uint32_t fi = P.fin[li], fo = P.fout[li], fr = P.fre[li];
  OpIn opin;
  opin.f = ldc(fops + P.op_begin + (lane < n_ops ? lane : 0));
  const int t = P.t;
  const int tb = P.tb;
  const uint32_t size = 1u << t;
  const uint32_t half = NG == 2 ? 1u << (tb - 1) : 0u;   // the second enumeration index / group of a thread
  uint64_t bs = 0, in_base = 0, out_base = 0, dropped = 0;
  {
    if (lane < P.n_free) {
      const uint64_t b = (tid_bits >> lane) & 1ull;
      bs = b << fr;
      in_base = fi != NO_POS ? b << fi : 0ull;
      out_base = fo != NO_POS ? b << fo : 0ull;
      dropped = fo == NO_POS ? b : 0ull;
    }
    bs = wave_or_dpp(bs);
    in_base = wave_or_dpp(in_base);
    out_base = wave_or_dpp(out_base);
    dropped = wave_or_dpp(dropped);
  }
  const bool stored = dropped == 0;
  const int16_t* in16 = reinterpret_cast<const int16_t*>(I.in) + inst * I.in_st;
  int16_t* out16 = reinterpret_cast<int16_t*>(I.out) + inst * I.out_st;
  const int nb_ld = t < tb ? t : tb;
  const int nk_ld = 1 << (t - nb_ld);
  bool loader[NG];
  uint32_t ti_ld[NG];
  uint64_t ad_ld[NG];
  int16_t vals[NG][16];
  bool fast_ld = false;
  const int16_t* src = in16 + in_base;
  uint64_t had_ld[16];
  const bool init = P.init != 0;
  {
    uint32_t bti[10];
    uint64_t bad[10], had[16];
#pragma unroll
    for (int q = 0; q < 10; ++q) {
      bti[q] = P.ld_bti[q];
      bad[q] = P.ld_bad[q];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) had[k] = P.ld_had[k];
    uint64_t all = 0;
#pragma unroll
    for (int q = 0; q < 10; ++q)
      if (q < nb_ld) all |= bad[q];
#pragma unroll
    for (int k = 0; k < 16; ++k) all |= had[k];
#pragma unroll
    for (int h = 0; h < NG; ++h) {
      const uint32_t u = (uint32_t)tid + (h ? half : 0u);
      loader[h] = u < (1u << nb_ld);
      enum_lo(bti, bad, u, nb_ld, &ti_ld[h], &ad_ld[h]);
    }
    load_op_values<int16_t>(opin, Jrow, hrow);
    __builtin_amdgcn_sched_barrier(0);
    // the buffer covers the instance's input state from this tile's base
    // (records in bytes): every entry the tile reads lies inside it
    fast_ld = !init && nk_ld == 16 && all < BUF_MAX_ENTRIES;
    Z2Fast zf{};
    if (z2) {
      uint64_t lm = 0, km = 0;
#pragma unroll
      for (int q = 0; q < 10; ++q)
        if (q < nb_ld) lm |= bad[q];
#pragma unroll
      for (int k = 0; k < 16; ++k) km |= had[k];
      zf = z2_fast(P.in_w, in_base, lm, km);
      fast_ld = fast_ld && zf.ok;
    }
    const uint64_t rec = ((uint64_t)I.in_st - in_base) * 2ull;
    const __amdgpu_buffer_rsrc_t rs =
        raw_rsrc(src, fast_ld ? (int)(rec < 0x7fffffffull ? rec : 0x7fffffffull) : 0);
    if (z2) {
      // stored addresses: the complemented entries through a second buffer
      const uint64_t base2 = in_base ^ zf.fm;
      const uint64_t rec2 = ((uint64_t)I.in_st - base2) * 2ull;
      const __amdgpu_buffer_rsrc_t rs2 =
          raw_rsrc(in16 + base2, fast_ld ? (int)(rec2 < 0x7fffffffull ? rec2 : 0x7fffffffull) : 0);
#pragma unroll
      for (int h = 0; h < NG; ++h) {
        const uint32_t off = (uint32_t)ad_ld[h] << 1, off2 = (uint32_t)(ad_ld[h] ^ zf.lm) << 1;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const bool f = z2_flip(zf, had[k]);
          vals[h][k] = (int16_t)__builtin_amdgcn_raw_buffer_load_b16(
              f ? rs2 : rs, (int)(f ? off2 : off), (int)((f ? had[k] ^ zf.km : had[k]) << 1), AUX_NT);
        }
      }
    } else {
#pragma unroll
      for (int h = 0; h < NG; ++h) {
        const uint32_t off = (uint32_t)ad_ld[h] << 1;
#pragma unroll
        for (int k = 0; k < 16; ++k)
          vals[h][k] = (int16_t)__builtin_amdgcn_raw_buffer_load_b16(rs, (int)off, (int)(had[k] << 1), AUX_NT);
      }
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) had_ld[k] = had[k];
  }
  const OpLanes16 R = lanes16(resolve_lane(opin, bs));
  if (!init && !fast_ld) {
#pragma unroll
    for (int h = 0; h < NG; ++h)
      if (loader[h]) {
        if (z2) {   // stored addresses of a half-state plan
#pragma unroll
          for (int k = 0; k < 16; ++k)
            if (k < nk_ld) vals[h][k] = in16[z2_addr(in_base | ad_ld[h] | had_ld[k], P.in_w)];
        } else {
#pragma unroll
          for (int k = 0; k < 16; ++k)
            if (k < nk_ld) vals[h][k] = src[ad_ld[h] | had_ld[k]];
        }
      }
  }
  {
    uint32_t hs[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) hs[k] = swz(P.ld_hti[k]) << 1;
#pragma unroll
    for (int h = 0; h < NG; ++h) {
      if (!loader[h]) continue;
      const uint32_t ls = opaque(swz(ti_ld[h]) << 1);
      if (nk_ld == 16) {
#pragma unroll
        for (int k = 0; k < 16; ++k) lds16_at(ls ^ hs[k]) = vals[h][k];
      } else {
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (k < nk_ld) lds16_at(ls ^ hs[k]) = vals[h][k];
      }
    }
  }
  __syncthreads();
  const int n_stages = P.n_stages;
  const uint32_t groups = size >> 4;
  // NG = 1 as k_pass: one group per thread (with fewer than 64 groups the
  // first wave repeats groups); NG = 2: groups tid and tid + half, all active
  const bool active = NG == 2 || (uint32_t)tid < (groups > 64u ? groups : 64u);
  uint32_t g[NG];
#pragma unroll
  for (int h = 0; h < NG; ++h) g[h] = NG == 2 ? (uint32_t)tid + (h ? half : 0u) : ((uint32_t)tid & (groups - 1));
  for (int s = 0; s < n_stages; ++s) {
    if (active) {
      const cptr<DevStage> ST = stages + P.stage_begin + s;
      const int ob = ST->op_begin - P.op_begin, oe = ST->op_end - P.op_begin;
      uint32_t so[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) so[j] = ST->soff[j] << 1;
      uint32_t gb[NG], sg[NG];
#pragma unroll
      for (int h = 0; h < NG; ++h) {
        gb[h] = (uint32_t)ST->g_lo[g[h] & 31u] | (uint32_t)ST->g_hi[g[h] >> 5];
        sg[h] = opaque(((uint32_t)ST->sg_lo[g[h] & 31u] ^ (uint32_t)ST->sg_hi[g[h] >> 5]) << 1);
      }
      s2v va[NG][8], vb[NG][8];
#pragma unroll
      for (int h = 0; h < NG; ++h)
#pragma unroll
        for (int d = 0; d < 8; ++d) va[h][d] = s2v{lds16_at(sg[h] ^ so[d]), lds16_at(sg[h] ^ so[d + 8])};
      for (int o = ob; o < oe; o += 2) {
        apply_op16<NG>(va, vb, gb, R, o);
        if (o + 1 < oe) {
          apply_op16<NG>(vb, va, gb, R, o + 1);
        } else {
#pragma unroll
          for (int h = 0; h < NG; ++h)
#pragma unroll
            for (int d = 0; d < 8; ++d) va[h][d] = vb[h][d];
        }
      }
#pragma unroll
      for (int h = 0; h < NG; ++h)
#pragma unroll
        for (int d = 0; d < 8; ++d) {
          lds16_at(sg[h] ^ so[d]) = va[h][d].x;
          lds16_at(sg[h] ^ so[d + 8]) = va[h][d].y;
        }
    }
    __syncthreads();
  }
  const int64_t red_at = I.red_base + (inst << run_bits) + (int64_t)ktile;
  if (!stored) {
    if (I.red_v && tid == 0) {
      as_global(I.red_v)[red_at] = -INFINITY;
      as_global(I.red_i)[red_at] = ~0ull;
    }
    return;
  }
  {
    const int ns = P.n_st;
    uint32_t bti[10], hs[16];
    uint64_t bad[10], had[16];
#pragma unroll
    for (int q = 0; q < 10; ++q) {
      bti[q] = P.st_bti[q];
      bad[q] = P.st_bad[q];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      hs[k] = swz(P.st_hti[k]) << 1;
      had[k] = P.st_had[k];
    }
    const int nb = ns < tb ? ns : tb;
    const int nk = 1 << (ns - nb);
    uint64_t all = 0;
#pragma unroll
    for (int q = 0; q < 10; ++q)
      if (q < nb) all |= bad[q];
#pragma unroll
    for (int k = 0; k < 16; ++k) all |= had[k];
    bool storer[NG];
    uint32_t ti_st[NG];
    uint64_t ad_st[NG];
#pragma unroll
    for (int h = 0; h < NG; ++h) {
      const uint32_t u = (uint32_t)tid + (h ? half : 0u);
      storer[h] = u < (1u << nb);
      enum_lo(bti, bad, u, nb, &ti_st[h], &ad_st[h]);
    }
    int16_t* dst = out16 + out_base;
    if (I.red_v) {
      // fused final reduction (as k_pass): the tile's maximum and its lowest
      // output address, as a float partial
      float bv = -INFINITY;
      uint64_t bi = ~0ull;
#pragma unroll
      for (int h = 0; h < NG; ++h) {
        if (!storer[h]) continue;
        const uint32_t ls = opaque(swz(ti_st[h]) << 1);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          if (k < nk) {
            const float v = (float)lds16_at(ls ^ hs[k]);
            const uint64_t a = z2 ? z2_addr(out_base | ad_st[h] | had[k], P.out_w) : (out_base | ad_st[h] | had[k]);
            if (v > bv || (v == bv && a < bi)) {
              bv = v;
              bi = a;
            }
          }
        }
      }
      wave_best64_dpp(bv, bi);
      __syncthreads();
      const int wv = tid >> 6;
      if ((tid & 63) == 63) {
        lds_at(16 * wv) = bv;
        lds_at(16 * wv + 4) = __uint_as_float((uint32_t)bi);
        lds_at(16 * wv + 8) = __uint_as_float((uint32_t)(bi >> 32));
      }
      __syncthreads();
      if (tid < 64) {
        const int nw = (int)(blockDim.x >> 6);
        bv = -INFINITY;
        bi = ~0ull;
        if (tid < nw) {
          bv = lds_at(16 * tid);
          bi = ((uint64_t)__float_as_uint(lds_at(16 * tid + 8)) << 32) | __float_as_uint(lds_at(16 * tid + 4));
        }
        wave_best64_dpp(bv, bi);
        if (tid == 63) {
          as_global(I.red_v)[red_at] = bv;
          as_global(I.red_i)[red_at] = bi;
        }
      }
      return;
    }
    bool fast_st = nk == 16 && all < BUF_MAX_ENTRIES;
    Z2Fast zf{};
    if (z2) {
      uint64_t lm = 0, km = 0;
#pragma unroll
      for (int q = 0; q < 10; ++q)
        if (q < nb) lm |= bad[q];
#pragma unroll
      for (int k = 0; k < 16; ++k) km |= had[k];
      zf = z2_fast(P.out_w, out_base, lm, km);
      fast_st = fast_st && zf.ok;
    }
    const uint64_t rec = ((uint64_t)I.out_st - out_base) * 2ull;
    const __amdgpu_buffer_rsrc_t rs = raw_rsrc(dst, (int)(rec < 0x7fffffffull ? rec : 0x7fffffffull));
    const uint64_t base2 = out_base ^ zf.fm;
    const uint64_t rec2 = ((uint64_t)I.out_st - base2) * 2ull;
    const __amdgpu_buffer_rsrc_t rs2 = raw_rsrc(out16 + base2, (int)(rec2 < 0x7fffffffull ? rec2 : 0x7fffffffull));
#pragma unroll
    for (int h = 0; h < NG; ++h) {
      if (!storer[h]) continue;
      const uint32_t ls = opaque(swz(ti_st[h]) << 1);
      int16_t sv[16];
      if (fast_st) {
#pragma unroll
        for (int k = 0; k < 16; ++k) sv[k] = lds16_at(ls ^ hs[k]);
        const uint32_t off = (uint32_t)ad_st[h] << 1;
        if (z2) {   // stored addresses, the complemented ones through the second buffer
          const uint32_t off2 = (uint32_t)(ad_st[h] ^ zf.lm) << 1;
#pragma unroll
          for (int k = 0; k < 16; ++k) {
            const bool f = z2_flip(zf, had[k]);
            __builtin_amdgcn_raw_buffer_store_b16((uint16_t)sv[k], f ? rs2 : rs, (int)(f ? off2 : off),
                                                  (int)((f ? had[k] ^ zf.km : had[k]) << 1), AUX_NT);
          }
        } else {
#pragma unroll
          for (int k = 0; k < 16; ++k)
            __builtin_amdgcn_raw_buffer_store_b16((uint16_t)sv[k], rs, (int)off, (int)(had[k] << 1), AUX_NT);
        }
      } else {
#pragma unroll
        for (int k = 0; k < 16; ++k)
          if (k < nk) sv[k] = lds16_at(ls ^ hs[k]);
        if (z2) {   // every output at its stored address (the mirror outputs included)
#pragma unroll
          for (int k = 0; k < 16; ++k)
            if (k < nk) __builtin_nontemporal_store(sv[k], &out16[z2_addr(out_base | ad_st[h] | had[k], P.out_w)]);
        } else {
#pragma unroll
          for (int k = 0; k < 16; ++k)
            if (k < nk) __builtin_nontemporal_store(sv[k], &dst[ad_st[h] | had[k]]);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// final reduction: max over the state and its lowest address (Sec. II: the
// contraction with the product state (0, 0)^n of App. A)
// ---------------------------------------------------------------------------

struct VI {
  float v;
  uint64_t i;
};

__device__ __forceinline__ VI vi_best(VI a, VI b) {
  if (b.v > a.v || (b.v == a.v && b.i < a.i)) return b;
  return a;
}

template <int THREADS>
__device__ VI block_best(VI x) {
  __shared__ float sv[THREADS / 64];
  __shared__ uint64_t si[THREADS / 64];
  for (int off = 32; off > 0; off >>= 1) {
    VI y;
    y.v = __shfl_xor(x.v, off, 64);
    y.i = __shfl_xor(x.i, off, 64);
    x = vi_best(x, y);
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) {
    sv[w] = x.v;
    si[w] = x.i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < THREADS / 64; ++k) x = vi_best(x, VI{sv[k], si[k]});
    sv[0] = x.v;
    si[0] = x.i;
  }
  __syncthreads();
  VI r{sv[0], si[0]};
  __syncthreads();
  return r;
}

// Four consecutive state entries as floats.
__device__ __forceinline__ float4 ld4(cptr<float> s, uint64_t i) { return ldc((cptr<float4>)(s + i)); }
__device__ __forceinline__ float4 ld4(cptr<int16_t> s, uint64_t i) {
  const uint2 w = ldc((cptr<uint2>)(s + i));
  return float4{(float)(int16_t)(w.x & 0xffffu), (float)(int16_t)(w.x >> 16), (float)(int16_t)(w.y & 0xffffu),
                (float)(int16_t)(w.y >> 16)};
}

template <typename SV>
__global__ __launch_bounds__(NTR) void k_reduce_stage1(const RedItem* __restrict__ items, int n_items,
                                                       float* __restrict__ pv, uint64_t* __restrict__ pi) {
  __shared__ float bt[5][256];   // bonus of each index byte (chimera row walk)
  const int64_t wg = blockIdx.x;
  int it = 0;
  const cptr<RedItem> citems = as_const(items);
  while (it + 1 < n_items && wg >= citems[it + 1].chunk_begin) ++it;
  const auto& I = citems[it];
  const uint64_t chunk = (uint64_t)(wg - I.chunk_begin);
  const uint64_t len = 1ull << (I.w - I.log2_chunks);
  const uint64_t base = chunk * len;
  const cptr<SV> s = as_const(reinterpret_cast<const SV*>(I.st));
  const bool bonus = I.bedge != nullptr;
  if (bonus) {
    const uint64_t ref = *as_const(I.bref);
    const cptr<int32_t> bedge = as_const(I.bedge);
    for (int j = threadIdx.x; j < 5 * 256; j += NTR) {
      const int b = j >> 8, v = j & 255;
      float t = 0.f;
      for (int q = 0; q < 8; ++q) {
        const int sl = 8 * b + q;
        if (sl >= I.w) break;
        const int e = bedge[sl];
        if (e < 0) continue;
        const float Jv = I.bdtype == 0   ? as_const(static_cast<const float*>(I.bJ))[e]
                         : I.bdtype == 2 ? (float)as_const(static_cast<const int16_t*>(I.bJ))[e]
                                         : (float)as_const(static_cast<const int32_t*>(I.bJ))[e];
        t += (((ref >> sl) ^ (uint64_t)(v >> q)) & 1ull) ? -Jv : Jv;
      }
      bt[b][v] = t;
    }
    __syncthreads();
  }
  VI best{-INFINITY, ~0ull};
  // half-state plan: four consecutive entries of the upper half (top bit set;
  // with w >= 3 they share it) are stored reversed at the complement addresses
  const uint64_t wmask = I.w > 0 ? (~0ull >> (64 - I.w)) : 0ull;
  if (len >= 4) {
    // four consecutive entries per load; ties keep the smaller address
#pragma unroll 4
    for (uint64_t k = threadIdx.x; k < len / 4; k += NTR) {
      const uint64_t i0 = base + 4 * k;
      float4 v;
      if (I.z2 && ((i0 >> (I.w - 1)) & 1ull)) {
        const float4 r = ld4(s, wmask ^ (i0 + 3));   // entries i0 + 3 .. i0, in that order
        v = float4{r.w, r.z, r.y, r.x};
      } else {
        v = ld4(s, i0);
      }
      float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
      if (bonus) {
        const float hi = bt[1][(i0 >> 8) & 255] + bt[2][(i0 >> 16) & 255] + bt[3][(i0 >> 24) & 255] +
                         bt[4][(i0 >> 32) & 255];
        const uint32_t lo = (uint32_t)(i0 & 255);
        a0 = bt[0][lo] + hi;
        a1 = bt[0][lo + 1] + hi;
        a2 = bt[0][lo + 2] + hi;
        a3 = bt[0][lo + 3] + hi;
      }
      best = vi_best(best, VI{v.x + a0, i0});
      best = vi_best(best, VI{v.y + a1, i0 + 1});
      best = vi_best(best, VI{v.z + a2, i0 + 2});
      best = vi_best(best, VI{v.w + a3, i0 + 3});
    }
  } else {
    for (uint64_t k = threadIdx.x; k < len; k += NTR) {
      const uint64_t idx = base + k;
      float a = 0.f;
      if (bonus)
        a = bt[0][idx & 255] + bt[1][(idx >> 8) & 255] + bt[2][(idx >> 16) & 255] + bt[3][(idx >> 24) & 255] +
            bt[4][(idx >> 32) & 255];
      best = vi_best(best, VI{(float)s[I.z2 ? z2_addr(idx, I.w) : idx] + a, idx});
    }
  }
  best = block_best<NTR>(best);
  if (threadIdx.x == 0) {
    pv[wg] = best.v;
    pi[wg] = best.i;
  }
}

__global__ __launch_bounds__(NTR) void k_reduce_stage2(const RedItem* __restrict__ items,
                                                       const float* __restrict__ pv,
                                                       const uint64_t* __restrict__ pi) {
  const auto& I = as_const(items)[blockIdx.x];
  const int64_t nc = 1ll << I.log2_chunks;
  VI best{-INFINITY, ~0ull};
  for (int64_t k = threadIdx.x; k < nc; k += NTR) best = vi_best(best, VI{pv[I.chunk_begin + k], pi[I.chunk_begin + k]});
  best = block_best<NTR>(best);
  if (threadIdx.x == 0) {
    if (I.energy) *as_global(I.energy) = -(double)best.v;
    if (I.arg) *as_global(I.arg) = best.i;
  }
}

// ---------------------------------------------------------------------------
// backward: argmax routing (Sec. IV: cache intermediates, backtrack; the
// reverse-mode derivative of E* with respect to the tensor elements picks the
// maximising entries). One workgroup per instance walks the passes in
// reverse. Given the selected entry t of a pass's output, the spins the pass
// eliminated (at most 16) are the only unknowns: the workgroup scores every
// joint assignment a of them as x_in(a, t) + (terms of the pass that touch an
// eliminated spin) and keeps the first maximiser. That is the value the pass
// maximised over, so the chain of choices is a ground state.
// ---------------------------------------------------------------------------

constexpr int MAX_SPINS = 8192;

struct LTerm {      // a backward term with its coefficient resolved
  float c;
  uint8_t a, b, pad0, pad1;
};

__device__ __forceinline__ float term_sigma(uint8_t op, uint32_t a, uint64_t t) {
  const uint32_t b = op < 64 ? ((a >> op) & 1u) : (uint32_t)((t >> (op - 64)) & 1ull);
  return b ? -1.f : 1.f;
}

__device__ __forceinline__ float lterm_val(const LTerm& tm, uint32_t a, uint64_t t) {
  float s = term_sigma(tm.a, a, t);
  if (tm.b != 255) s *= term_sigma(tm.b, a, t);
  return tm.c * s;
}

// Wave reductions over DPP lane moves (no LDS traffic). The row steps pair
// lanes within a row of 16 (quad swaps, then half-row and row mirrors); the
// broadcasts of lanes 15 and 31 then combine the four rows, so lane 63 ends
// with the result of the whole wave.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void best_step(float& v, uint32_t& i) {
  const float ov =
      __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, ROW_MASK, 0xF, false));
  const uint32_t oi = (uint32_t)__builtin_amdgcn_update_dpp((int)i, (int)i, CTRL, ROW_MASK, 0xF, false);
  if (ov > v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}

// (value, lowest index) maximum of the wave, in lane 63.
__device__ __forceinline__ void wave_best_dpp(float& v, uint32_t& i) {
  best_step<0xB1, 0xF>(v, i);    // quad_perm [1,0,3,2]
  best_step<0x4E, 0xF>(v, i);    // quad_perm [2,3,0,1]
  best_step<0x141, 0xF>(v, i);   // row_half_mirror
  best_step<0x140, 0xF>(v, i);   // row_mirror
  best_step<0x142, 0xA>(v, i);   // row_bcast:15 into rows 1 and 3
  best_step<0x143, 0xC>(v, i);   // row_bcast:31 into rows 2 and 3
}

template <int CTRL>
__device__ __forceinline__ uint32_t or_step(uint32_t x) {
  return x | (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, CTRL, 0xF, 0xF, false);
}

// OR over the 16 lanes of each row, in every lane of the row.
__device__ __forceinline__ uint64_t row_or_dpp(uint64_t x) {
  uint32_t lo = (uint32_t)x, hi = (uint32_t)(x >> 32);
  lo = or_step<0xB1>(lo);
  hi = or_step<0xB1>(hi);
  lo = or_step<0x4E>(lo);
  hi = or_step<0x4E>(hi);
  lo = or_step<0x141>(lo);
  hi = or_step<0x141>(hi);
  lo = or_step<0x140>(lo);
  hi = or_step<0x140>(hi);
  return ((uint64_t)hi << 32) | lo;
}

// Per-pass backward data held in LDS for a chunk of passes.
struct LPass {
  uint64_t surv;
  int32_t n_cand, n_lo, n_hi, n_cross;
  int32_t in_w, init, cand_off, term_off;   // offsets inside the chunk
};


__device__ __forceinline__ uint64_t readlane64(uint64_t x, int k) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, k);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), k);
  return ((uint64_t)hi << 32) | lo;
}

// Address tables of a pass (they depend only on the pass, not on the
// selected entry): entry x of the low / high table is the OR of the input
// address bits of the candidates set in x, over candidate bits 0..7 / 8..15.
// Called by 512 threads, x_tid = 0..511.
__device__ __forceinline__ void bwd_address_tables(const LPass& Q, const uint64_t* lcad, uint64_t* tlo, uint64_t* thi,
                                                   int x_tid) {
  const int nc = Q.n_cand;
  const int nlo = nc < 8 ? nc : 8, nhi = nc - nlo;
  const int hi = x_tid >= 256;
  const uint32_t x = hi ? (uint32_t)(x_tid - 256) : (uint32_t)x_tid;
  if (nc == 0 || x >= (1u << (hi ? nhi : nlo))) return;
  const uint64_t* cad = lcad + Q.cand_off;
  const int kb = hi ? 8 : 0, ke = hi ? nc : nlo;
  uint64_t ad = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (kb + k < ke && ((x >> k) & 1u)) ad |= cad[kb + k];
  (hi ? thi : tlo)[x] = ad;
}

// The input address of a pass's surviving slots under the selected output
// entry t: lane c takes slot c, then an OR across the wave (a whole wave
// calls it, lane = 0..63); the result is the same in every lane.
__device__ __forceinline__ uint64_t bwd_surviving_base(const LPass& Q, const uint8_t* ipos, uint64_t t, int lane) {
  uint64_t b = 0;
  if (lane < Q.in_w && ((Q.surv >> lane) & 1ull) && ((t >> lane) & 1ull)) b = 1ull << ipos[lane];
  return wave_or_dpp(b);
}

// A 64-bit lane value the compiler may not re-derive (so that it cannot
// turn a load whose offset it could prove uniform into a separate scalar
// path).
__device__ __forceinline__ uint64_t opaque64(uint64_t x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Where a pass's candidates read their input entries: the checkpoint at the
// surviving-slot address (or the zero word in the first pass, whose input is
// all zero) and the two address tables.
template <typename SV>
struct BwdSrc {
  bool have;
  cptr<SV> src;   // the pass's input state (float32, or int16 for int16 couplings)
  const uint64_t* AL;
  const uint64_t* AH;
  uint32_t na;
  uint64_t base;  // input address of the surviving slots
  int zw;         // half-state plan: the input width (stored addresses), else 0
};

__device__ __forceinline__ bool have_src_of(const LPass& P) { return !P.init; }

// Loads of the input entries of candidates a0 + j NT, j < W. The loads are
// unconditional (a branch around each would make every one wait for the one
// before) and nothing here uses their values, so they stay in flight until
// the scoring: a candidate beyond the last reads a valid word instead
// (offset 0; the scoring skips it), and in the first pass every candidate
// reads the zero word.
template <int W, typename SV>
__device__ __forceinline__ void bwd_issue(float (&val)[8], const BwdSrc<SV>& S, uint32_t a0) {
#pragma unroll
  for (int j = 0; j < W; ++j) {
    const uint32_t a = a0 + (uint32_t)j * NT;
    const uint64_t off = S.AL[a & 255u] | S.AH[(a >> 8) & 255u];
    const uint64_t ad = S.base | ((S.have && a < S.na) ? off : 0ull);
    val[j] = (float)S.src[opaque64(S.zw ? z2_addr(ad, S.zw) : ad)];
  }
}

// The terms of a pass that are not in the two tables (they touch a low and a
// high candidate bit) and the selected output entry t.
struct BwdTerms {
  const LTerm* T;
  int cross_b, nterm;
  uint64_t t;
  uint32_t na;
  uint32_t m;   // tie key of candidate a: a ^ m (m = 0: the first maximiser)
};

// Tie mask of pass p for the walk's tie rule (< na): 0 keeps the first
// maximiser of every choice (the paper's default max), 1 the last, any other
// value a pseudo-random rule per pass (a 32-bit mix of the value and p).
__device__ __forceinline__ uint32_t tie_mask(uint64_t tie, int p, uint32_t na) {
  if (tie == 0) return 0u;
  if (tie == 1) return na - 1u;
  uint64_t z = tie + 0x9E3779B97F4A7C15ull * (uint64_t)(p + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (uint32_t)z & (na - 1u);
}

// Scores candidates a0 + j NT, j < W (input entry + table terms + cross
// terms) into the thread's best (value, lowest tie key a ^ m).
template <int W>
__device__ __forceinline__ void bwd_score(float (&val)[8], const BwdTerms& X, const float* lut_lo, const float* lut_hi,
                                          uint32_t a0, float& bv, uint32_t& bi) {
#pragma unroll
  for (int j = 0; j < W; ++j) {
    const uint32_t a = (a0 + (uint32_t)j * NT) & (X.na - 1u);
    val[j] += lut_lo[a & 255u] + lut_hi[a >> 8];
  }
  for (int k = X.cross_b; k < X.nterm; ++k) {
    const LTerm tk = X.T[k];
#pragma unroll
    for (int j = 0; j < W; ++j) val[j] += lterm_val(tk, a0 + (uint32_t)j * NT, X.t);
  }
#pragma unroll
  for (int j = 0; j < W; ++j) {
    const uint32_t a = a0 + (uint32_t)j * NT;
    const uint32_t key = a ^ X.m;
    if (a < X.na && (val[j] > bv || (val[j] == bv && key < bi))) {
      bv = val[j];
      bi = key;
    }
  }
}

template <typename IT, typename SV = float>
__global__ __launch_bounds__(NT) void k_backward(const BwdItem* __restrict__ items) {
  __shared__ int8_t s_sh[MAX_SPINS];
  __shared__ float lut_lo[256], lut_hi[256];
  __shared__ uint64_t ad_lo[2][256], ad_hi[2][256];   // by pass parity
  __shared__ uint64_t sh_t, sh_final;   // the first selected entry, the final address
  __shared__ LTerm lt[BCH_TERMS];
  __shared__ BCand lc[BCH_CANDS];
  __shared__ LPass lp[BCH_PASSES];
  __shared__ uint8_t lpos[BCH_PASSES][64];
  __shared__ uint64_t lcad[BCH_CANDS];   // input address bit of each candidate (0: none)
  __shared__ float part_v[2][NT / 64];   // by pass parity
  __shared__ uint32_t part_i[2][NT / 64];
  __shared__ uint64_t part_a[NT / 64];
  const auto& I = as_const(items)[blockIdx.x];
  const int tid = threadIdx.x;
  const cptr<IT> Jrow = as_const(static_cast<const IT*>(I.J));
  const cptr<IT> hrow = as_const(static_cast<const IT*>(I.h));
  const cptr<DevPass2> passes = as_const(I.passes);
  const cptr<uint8_t> final_pos = as_const(I.final_pos);
  const cptr<int32_t> final_slot_spin = as_const(I.final_slot_spin);
  const cptr<BChunk> chunks = as_const(I.chunks);
  const cptr<BCand> cands = as_const(I.cands);
  const cptr<BTerm> terms = as_const(I.terms);
  const cptr<int32_t> edges = as_const(I.edges);
  const cptr<const float*> ckpt = as_const(I.ckpt);
  const int final_w = I.final_w, n = I.n;
  const int64_t m = I.m;
  const int seg_lo = I.seg_lo, seg_hi = I.seg_hi;
  const bool seg_top = seg_hi == I.n_passes - 1;   // the walk starts at the final state
  const bool seg_end = seg_lo == 0;                // the walk ends here: gradients out
  if (seg_top) {
    for (int v = tid; v < n; v += NT) s_sh[v] = 0;
  } else {
    const cptr<int8_t> sg = as_const(static_cast<const int8_t*>(I.sigma));
    for (int v = tid; v < n; v += NT) s_sh[v] = sg[v] < 0 ? 1 : 0;
  }
  if (seg_top && I.red_v) {
    // the final maximum over the last pass's per-tile partials: the largest
    // value, ties to the lowest address
    float bv = -INFINITY;
    uint64_t bi = ~0ull;
    const cptr<float> rv = as_const(I.red_v);
    const cptr<uint64_t> ri = as_const(I.red_i);
    for (int64_t k = tid; k < I.red_n; k += NT) {
      const float v = rv[k];
      const uint64_t a = ri[k];
      if (v > bv || (v == bv && a < bi)) {
        bv = v;
        bi = a;
      }
    }
    wave_best64_dpp(bv, bi);
    if ((tid & 63) == 63) {
      part_v[0][tid >> 6] = bv;
      part_a[tid >> 6] = bi;
    }
    __syncthreads();
    if (tid < 64) {
      bv = tid < NT / 64 ? part_v[0][tid] : -INFINITY;
      bi = tid < NT / 64 ? part_a[tid] : ~0ull;
      wave_best64_dpp(bv, bi);
      if (tid == 63) {
        sh_final = bi;   // the selected final address
        if (I.energy) *as_global(I.energy) = -(double)bv;
      }
    }
  }
  __syncthreads();
  if (!seg_top) {
    if (tid == 0) sh_t = *as_const(static_cast<const uint64_t*>(I.carry));
  } else if (tid < 64) {
    // final state: address -> slot index; spins still in a slot take its bit
    const uint64_t addr = I.red_v ? sh_final : *as_const(I.final_addr);
    uint64_t tb = 0;
    if (tid < final_w) {
      const uint64_t b = (addr >> final_pos[tid]) & 1ull;
      tb = b << tid;
      const int sp = final_slot_spin[tid];
      if (sp >= 0) s_sh[sp] = (int8_t)b;
    }
    tb = wave_or_dpp(tb);
    if (tid == 0) sh_t = tb;
  }
  __syncthreads();
  // the selected output entry of the pass being walked and the input address
  // of its surviving slots: wave-uniform, and every wave follows the choices
  // itself (no exchange through LDS)
  uint64_t t_cur = sh_t, base_cur = 0;
  const int lane = tid & 63;
  for (int ci = 0; ci < I.n_chunks; ++ci) {
    const BChunk CH = ldc(chunks + ci);
    if (CH.p_lo > seg_hi || CH.p_hi < seg_lo) continue;   // outside the segment (uniform)
    // the passes of the chunk inside the segment
    const int top = CH.p_hi < seg_hi ? CH.p_hi : seg_hi, bot = CH.p_lo > seg_lo ? CH.p_lo : seg_lo;
    // stage the chunk: pass fields and layouts, candidates, terms (coefficients resolved)
    for (int q = tid; q <= CH.p_hi - CH.p_lo; q += NT) {
      const cptr<DevPass2> P = passes + CH.p_lo + q;
      LPass x;
      x.surv = P->surv_mask;
      x.n_cand = P->n_cand;
      x.n_lo = P->n_lo;
      x.n_hi = P->n_hi;
      x.n_cross = P->n_cross;
      x.in_w = P->in_w;
      x.init = P->init;
      x.cand_off = P->cand_begin - CH.cand_begin;
      x.term_off = P->term_begin - CH.term_begin;
      lp[q] = x;
    }
    for (int k = tid; k < (CH.p_hi - CH.p_lo + 1) * 64; k += NT)
      lpos[k >> 6][k & 63] = passes[CH.p_lo + (k >> 6)].in_pos[k & 63];
    for (int k = tid; k < CH.n_cand; k += NT) lc[k] = ldc(cands + CH.cand_begin + k);
    for (int k = tid; k < CH.n_term; k += NT) {
      const BTerm b = ldc(terms + CH.term_begin + k);
      LTerm x;
      x.c = b.is_field ? ldv(hrow, b.coef) : ldv(Jrow, b.coef);
      x.a = b.a;
      x.b = b.b;
      x.pad0 = x.pad1 = 0;
      lt[k] = x;
    }
    __syncthreads();
    {
      // the input address bit of each candidate's starting slot: thread
      // 16 q + k takes candidate k of the chunk's pass q (<= 16 per pass)
      const int q = tid >> 4, k = tid & 15;
      if (q <= CH.p_hi - CH.p_lo && k < lp[q].n_cand) {
        const int ss = lc[lp[q].cand_off + k].start_slot;
        lcad[lp[q].cand_off + k] = (ss >= 0 && lpos[q][ss] != NO_POS) ? 1ull << lpos[q][ss] : 0ull;
      }
    }
    __syncthreads();
    // the chunk's last pass walked here: its address tables, and the address
    // of its surviving slots under the selected output entry
    bwd_address_tables(lp[top - CH.p_lo], lcad, ad_lo[top & 1], ad_hi[top & 1], tid);
    base_cur = bwd_surviving_base(lp[top - CH.p_lo], lpos[top - CH.p_lo], t_cur, lane);
    __syncthreads();
    for (int p = top; p >= bot; --p) {
      const LPass& P = lp[p - CH.p_lo];
      const int nc = P.n_cand;
      const uint64_t surv = P.surv;
      const uint64_t t = t_cur;
      const bool has_next = p > bot;
      if (nc == 0) {
        t_cur = t & surv;
        if (has_next) {
          base_cur = bwd_surviving_base(lp[p - 1 - CH.p_lo], lpos[p - 1 - CH.p_lo], t_cur, lane);
          if (tid >= 512)
            bwd_address_tables(lp[p - 1 - CH.p_lo], lcad, ad_lo[(p - 1) & 1], ad_hi[(p - 1) & 1], tid - 512);
        }
        __syncthreads();
        continue;
      }
      const BCand* C = lc + P.cand_off;
      const LTerm* T = lt + P.term_off;
      const int n_lo = P.n_lo, n_hi = P.n_hi;
      const int nterm = n_lo + n_hi + P.n_cross;
      const int nlo = nc < 8 ? nc : 8, nhi = nc - nlo;
      const uint32_t na = 1u << nc;
      // the candidates' entries of the pass's input, in batches of 8 per
      // thread (with NT = 1024 and at most 2^16 candidates, at most eight
      // batches); their addresses come from tables built during the pass
      // before, so the first batch's loads are issued here, without a
      // branch, and stay in flight while the term tables are built. Only
      // the W = 1, 2, 4 or 8 of them that cover the candidates are scored.
      const bool hv = have_src_of(P);
      const BwdSrc<SV> S{hv, hv ? as_const(reinterpret_cast<const SV*>(ckpt[p]))
                                : as_const(reinterpret_cast<const SV*>(g_zero_words)),
                         ad_lo[p & 1], ad_hi[p & 1], na, hv ? base_cur : 0ull, (hv && I.z2) ? P.in_w : 0};
      const int wsel = na <= (uint32_t)NT ? 1 : na <= 2u * NT ? 2 : na <= 4u * NT ? 4 : 8;
      const uint32_t nb = (na + 8u * NT - 1u) / (8u * NT);
      float val[8];
      bwd_issue<8>(val, S, (uint32_t)tid);
      // tables of the terms over the low / high halves of the candidate
      // bits (threads 0..511); the next pass's address tables (threads
      // 512..1023)
      if (tid < 512) {
        const int hi = tid >= 256;
        const uint32_t x = hi ? (uint32_t)(tid - 256) : (uint32_t)tid;
        if (x < (1u << (hi ? nhi : nlo))) {
          const uint32_t full = hi ? (x << 8) : x;
          float acc = 0.f;
          const int tb = hi ? n_lo : 0, te = hi ? n_lo + n_hi : n_lo;
          // terms four at a time: their LDS reads issue together
          for (int k0 = tb; k0 < te; k0 += 4) {
            LTerm tt[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) tt[j] = T[k0 + j < te ? k0 + j : te - 1];
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (k0 + j < te) acc += lterm_val(tt[j], full, t);
          }
          if (hi)
            lut_hi[x] = acc;
          else
            lut_lo[x] = acc;
        }
      } else if (has_next) {
        bwd_address_tables(lp[p - 1 - CH.p_lo], lcad, ad_lo[(p - 1) & 1], ad_hi[(p - 1) & 1], tid - 512);
      }
      __syncthreads();
      const int cross_b = n_lo + n_hi;
      float bv = -INFINITY;
      uint32_t bi = ~0u;
      const uint32_t tm = tie_mask(I.tie, p, na);
      const BwdTerms TT{T, cross_b, nterm, t, na, tm};
      switch (wsel) {
        case 1: bwd_score<1>(val, TT, lut_lo, lut_hi, (uint32_t)tid, bv, bi); break;
        case 2: bwd_score<2>(val, TT, lut_lo, lut_hi, (uint32_t)tid, bv, bi); break;
        case 4: bwd_score<4>(val, TT, lut_lo, lut_hi, (uint32_t)tid, bv, bi); break;
        default:
          for (uint32_t bt = 0; bt < nb; ++bt) {
            const uint32_t a0 = (uint32_t)tid + bt * 8u * NT;
            if (bt > 0) bwd_issue<8>(val, S, a0);
            bwd_score<8>(val, TT, lut_lo, lut_hi, a0, bv, bi);
          }
          break;
      }
      // the best (value, lowest index) of the workgroup: each wave's, then
      // every wave ranks the wave results and follows the choice (wave 0
      // records the spins)
      wave_best_dpp(bv, bi);
      float* pv = part_v[p & 1];
      uint32_t* pi = part_i[p & 1];
      if (lane == 63) {
        pv[tid >> 6] = bv;
        pi[tid >> 6] = bi;
      }
      __syncthreads();
      bv = lane < NT / 64 ? pv[lane] : -INFINITY;
      bi = lane < NT / 64 ? pi[lane] : ~0u;
      wave_best_dpp(bv, bi);
      const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)bi, 63) ^ tm;
      uint64_t b = 0;
      if (lane < nc) {   // nc <= 16: the first row of lanes
        const uint32_t bit = (a >> lane) & 1u;
        if (tid < 64) s_sh[C[lane].spin] = (int8_t)bit;
        if (C[lane].start_slot >= 0) b = (uint64_t)bit << C[lane].start_slot;
      }
      b = row_or_dpp(b);
      t_cur = (t & surv) | readlane64(b, 0);
      if (has_next) base_cur = bwd_surviving_base(lp[p - 1 - CH.p_lo], lpos[p - 1 - CH.p_lo], t_cur, lane);
    }
    __syncthreads();   // the chunk's LDS data is replaced next
  }
  const gptr<int8_t> sigma = as_global(I.sigma);
  const gptr<float> dh = as_global(I.dh), dJ = as_global(I.dJ);
  if (!seg_end) {
    // a later segment continues the walk: the spins chosen so far and the
    // selected entry of the pass below this segment
    for (int v = tid; v < n; v += NT) sigma[v] = (int8_t)(s_sh[v] ? -1 : 1);
    if (tid == 0) *as_global(I.carry) = t_cur;
    return;
  }
  for (int v = tid; v < n; v += NT) {
    sigma[v] = (int8_t)(s_sh[v] ? -1 : 1);
    if (dh) dh[v] = s_sh[v] ? 1.f : -1.f;           // -sigma_v
  }
  if (dJ) {
    for (int64_t e = tid; e < m; e += NT) {
      const int a = edges[2 * e], c = edges[2 * e + 1];
      dJ[e] = (s_sh[a] ^ s_sh[c]) ? 1.f : -1.f;   // -sigma_a sigma_c
    }
  }
}

// ---------------------------------------------------------------------------
// host launch wrappers (kernels are launched from this translation unit)
// ---------------------------------------------------------------------------

// Raises the dynamic LDS limit of a kernel once (static tables come on top);
// slot: which of the pass kernels (0 .. 7).
template <typename K>
static hipError_t allow_lds(K kernel, int slot, size_t bytes) {
  static int done[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (done[slot]) return hipSuccess;
  // the pass kernel addresses LDS from 0: it must have no static LDS
  hipFuncAttributes fa;
  hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kernel));
  if (e != hipSuccess) return e;
  if (fa.sharedSizeBytes != 0) return hipErrorInvalidConfiguration;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)bytes);
  if (e == hipSuccess) done[slot] = 1;
  return e;
}

hipError_t launch_pass(const PassItem* items, int n_items, int64_t n_wg, int threads, size_t lds, int dtype,
                       hipStream_t stream, hipEvent_t t0, hipEvent_t t1, int ng, bool z2) {
  if (n_wg >= (1ll << 31) || threads < 64 || threads > NT || lds > 65536) return hipErrorInvalidConfiguration;
  const dim3 grid((uint32_t)n_wg), block(threads);
  // int16: two groups per thread when the host launches half the threads of
  // a tile (ng == 2), else one; z2: the launch holds half-state items
  using Kern = void (*)(const PassItem*, int);
  Kern kern;
  int slot;
  if (dtype == 2) {
    kern = ng == 2 ? (z2 ? k_pass16<2, true> : k_pass16<2, false>) : (z2 ? k_pass16<1, true> : k_pass16<1, false>);
    slot = ng == 2 ? 2 : 3;
  } else if (dtype == 0) {
    kern = z2 ? k_pass<float, true> : k_pass<float, false>;
    slot = 0;
  } else {
    kern = z2 ? k_pass<int32_t, true> : k_pass<int32_t, false>;
    slot = 1;
  }
  hipError_t e = allow_lds(kern, 2 * slot + (z2 ? 1 : 0), PASS_LDS_MAX);
  if (e != hipSuccess) return e;
  if (t0 || t1)
    hipExtLaunchKernelGGL(kern, grid, block, (uint32_t)lds, stream, t0, t1, 0u, items, n_items);
  else
    hipLaunchKernelGGL(kern, grid, block, lds, stream, items, n_items);
  return hipGetLastError();
}

int reduce_log2_chunks(int w) {
  // chunks of at least 2^12 entries, at most 2^10 chunks per instance
  int c = w - 12;
  if (c < 0) c = 0;
  if (c > 10) c = 10;
  return c;
}

hipError_t launch_reduce(const RedItem* items, int n_items, int64_t n_chunks, float* pv, uint64_t* pi,
                         hipStream_t stream, bool partials_ready, bool state16) {
  if (!partials_ready) {
    if (state16)
      hipLaunchKernelGGL(k_reduce_stage1<int16_t>, dim3((uint32_t)n_chunks), dim3(NTR), 0, stream, items, n_items,
                         pv, pi);
    else
      hipLaunchKernelGGL(k_reduce_stage1<float>, dim3((uint32_t)n_chunks), dim3(NTR), 0, stream, items, n_items,
                         pv, pi);
  }
  hipLaunchKernelGGL(k_reduce_stage2, dim3((uint32_t)n_items), dim3(NTR), 0, stream, items, pv, pi);
  return hipGetLastError();
}

hipError_t launch_backward(const BwdItem* items, int n_items, int dtype, hipStream_t stream) {
  if (dtype == 2)
    hipLaunchKernelGGL((k_backward<int16_t, int16_t>), dim3(n_items), dim3(NT), 0, stream, items);
  else if (dtype == 0)
    hipLaunchKernelGGL(k_backward<float>, dim3(n_items), dim3(NT), 0, stream, items);
  else
    hipLaunchKernelGGL(k_backward<int32_t>, dim3(n_items), dim3(NT), 0, stream, items);
  return hipGetLastError();
}

}  // namespace tt

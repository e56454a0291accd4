// 3-state Potts glasses (the paper's Appendix C): descriptors shared by the
// host encoder and the HIP kernels.
//
// H(s) = sum over edges of J_ij M[s_i][s_j], s in {0, 1, 2}, M = 1 on the
// diagonal and -1/2 off it. The state holds negative doubled energies, so the
// bond tensor is T[a][b] = -J (2 if a = b else -1) = (a = b ? -2J : J): integer
// couplings give integer entries, exact in float32 below 2^24.
//
// The sweep is the Ising one with three labels per slot: the state over the
// live spins is a 3^W table, slot s being the base-3 digit of weight 3^s (a
// fixed layout: passes read and write the same entries, so they run in
// place). Ops: GATE (relabel: new[b] = max_a x[a] + T[a][b]), CUT (max over
// the slot's three labels, the slot becomes free: constant along its digit),
// DIAG (x += T[d_a][d_b]); INTRO is a no-op (it enters a free slot).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "plan.hpp"

namespace tt {

constexpr int POTTS_MAX_W = 20;     // 3^20 entries (14 GB of float32) per instance at most
constexpr int POTTS_MAX_T = 4;      // tile digits a thread holds in registers (3^4 entries)
constexpr int POTTS_COUNT_T = 3;    // ... on the counting path (entries carry residues)
constexpr int POTTS_MAX_OPS = 48;   // ops per pass

struct PottsOp {
  uint8_t kind;    // OP_GATE, OP_CUT, OP_DIAG
  uint8_t a, b;    // tile digits of the slot(s)
  uint8_t pad;
  int32_t edge;    // coupling (GATE, DIAG)
};

// One pass = one launch: every thread owns the 3^t entries that share one
// assignment of the non-tile digits, applies the pass's ops to them in
// registers, and writes them back in place.
struct PottsPass {
  int32_t t, n_nt, n_ops, init;     // init: the state starts at zero (no read)
  int32_t low, pad;                 // low: the tile digits are slots 0 .. t-1 (see the kernels)
  int64_t threads;                  // 3^(W - t) threads per instance
  int64_t tile_st[POTTS_MAX_T];     // entry stride (3^slot) of tile digit r
  int64_t nt_st[POTTS_MAX_W];       // entry strides of the non-tile digits, lowest slot first
  PottsOp ops[POTTS_MAX_OPS];
};

// Final maximum (and count) over the entries whose free slots hold label 0:
// the combinations of the live digits.
struct PottsReduce {
  int32_t n_live, contig;           // contig: the live digits are slots 0 .. n_live-1
  int64_t combos;                   // 3^n_live
  int64_t st[POTTS_MAX_W];          // entry strides of the live digits, lowest slot first
};

struct PottsProgram {
  int32_t width = 0, t = 0;
  std::vector<PottsPass> passes;
  PottsReduce red;
  double terms = 0, elementwise = 0;   // algorithmic work per instance at the live width
};

// Encodes the plan's sweep ops for tiles of t digits; returns "" or an error.
std::string encode_potts(const Plan& p, int t, PottsProgram& out);

}  // namespace tt

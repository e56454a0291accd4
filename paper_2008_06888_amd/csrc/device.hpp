// Device-side descriptors shared by the kernels and the host launcher.
#pragma once
#include <cstdint>

namespace tt {

// One operation of a pass, in tile coordinates. Slot operands are encoded as
// a tile bit (0..31) when the slot is resident in the tile, or as
// SLOT_FIXED + slot when it is one of the tile's fixed index bits.
constexpr uint8_t SLOT_FIXED = 64;

struct DevOp {
  uint8_t kind;   // OpKind
  uint8_t a;      // first slot operand
  uint8_t b;      // second slot operand (DIAG)
  uint8_t dec;    // decision row (GATE / CUT / GATE4) within the pass
  int32_t param;  // edge (GATE / DIAG), spin (FIELD), group matrix (GATE4)
  uint8_t g4[4];  // GATE4: the four tile bits
};

struct DevPass {
  int32_t in_w, out_w, w_max, t;
  int32_t op_begin, n_ops, n_dec, init;
  int32_t n_free, reg, merge_src, pad;
  uint8_t R[16];     // tile bit -> slot
  uint8_t fre[48];   // slots below w_max outside the tile, ascending (tile id bits)
};

// Spins eliminated / entering at an op (for the backward walk).
struct DevSpin {
  int32_t old_spin, new_spin;
  int32_t old4[4];
};

// Group matrix of a GATE4 op: [t_old][t_new] = sum_k J[edge_k] sigma(old bit) sigma(new bit).
struct DevGroup {
  int32_t edges[16];
  uint8_t old_bit[16];
  uint8_t new_bit[16];
  int32_t n_edges, pad;
};

}  // namespace tt

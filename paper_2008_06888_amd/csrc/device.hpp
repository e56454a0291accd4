// Device-side descriptors shared by the kernels and the host launcher.
#pragma once
#include <cstdint>

#include "plan.hpp"

namespace tt {

// Slot operands are encoded as a tile bit (0..31) when the slot is resident
// in the tile, or as SLOT_FIXED + slot when it is one of the tile's fixed
// index bits.
constexpr uint8_t SLOT_FIXED = 64;
constexpr uint8_t NO_POS = 0xFF;

// ---- counting path (one LDS sweep per operation, identity bit order) ----
struct DevOp {
  uint8_t kind;   // OpKind
  uint8_t a;      // first slot operand
  uint8_t b;      // second slot operand (DIAG)
  uint8_t dec;
  int32_t param;  // edge (GATE / DIAG), spin (FIELD)
  uint8_t g4[4];
};

struct DevPass {
  int32_t in_w, out_w, w_max, t;
  int32_t op_begin, n_ops, n_dec, init;
  int32_t n_free, reg, merge_src;
  int32_t z2_skip;   // half-state plans: tile-id bit of the lowest fixed slot below out_w (-1: none)
  uint8_t R[16];     // tile bit -> slot
  uint8_t fre[48];   // slots below w_max outside the tile, ascending (tile id bits)
};

// ---- energy path ----
// Fused operation: a relabelling gate (or cut) on one tile bit, followed by
// the "star" of diagonal terms of the spin that enters: the field h and the
// bonds to spins already in the state, all linear in sigma(new spin).
enum FKind : uint8_t { FK_GATE = 1, FK_CUT = 2, FK_STAR = 3 };
constexpr int STAR_TERMS = 4;

struct FOp {
  uint8_t kind;
  uint8_t bit;     // GATE/CUT: tile bit; STAR: encoded slot of the spin
  uint8_t lidx;    // GATE/CUT: index of `bit` among the stage bits
  uint8_t nt;      // star terms used
  int32_t edge;    // GATE: bond edge
  int32_t hspin;   // star field: spin, -1 none
  uint8_t w[STAR_TERMS];    // star partners (encoded slots)
  int32_t te[STAR_TERMS];   // star edges
  uint8_t wl[STAR_TERMS];   // partner's index among the stage bits (255: not a stage bit)
};
// (STAR: lidx is the index of `bit` among the stage bits, 4 if it is not one.)

// A stage: up to four gate bits applied in registers, each thread owning
// groups of 16 entries that span the stage bits.
struct DevStage {
  uint8_t sb[4];     // stage tile bits
  uint8_t nns;       // non-stage tile bits (t - 4)
  uint8_t ns[15];    // non-stage tile bits, ascending
  int32_t op_begin, op_end;
  int32_t pad[2];
  uint16_t g_lo[32]; // group index (low / high 5 bits) -> its non-stage tile bits
  uint16_t g_hi[32];
  uint16_t sg_lo[32]; // the same, LDS-swizzled (the swizzle is linear over GF(2))
  uint16_t sg_hi[32];
  uint32_t soff[16];  // swizzled LDS offset of register entry j (stage bits of j)
};

struct DevPass2 {
  int32_t in_w, out_w, w_max, t;
  int32_t stage_begin, n_stages, init, n_free;
  int32_t cand_begin, n_cand, term_begin, n_lo, n_hi, n_cross;
  uint64_t surv_mask;    // slots (< in_w) whose spin is not eliminated in the pass
  uint8_t R[16];         // tile bit -> slot
  uint8_t fre[48];       // slots below w_max outside the tile (tile id bits, ascending)
  uint8_t in_pos[64];    // slot -> input address bit (NO_POS if none)
  uint8_t out_pos[64];   // slot -> output address bit (NO_POS if none)
  uint8_t ld_order[16];  // tile bits with an input position, ascending by position
  uint8_t st_order[16];  // tile bits with an output position, ascending by position
  int32_t n_ld, n_st;
  // bit q of the load (store) enumeration index -> tile-index bit, address bit
  uint32_t ld_bti[16], st_bti[16];
  uint64_t ld_bad[16], st_bad[16];
  // the same maps for the index bits from tb up (k = u >> tb), all 16 combinations
  uint32_t ld_hti[16], st_hti[16];
  uint64_t ld_had[16], st_had[16];
  int32_t tb;            // log2 of the threads a tile uses (max(6, t - 4), at most 10)
  int32_t z2_skip;       // half-state plans: tile-id bit k (fixed slot fre[k], one with an
                         // output position) whose tiles at 1 are not run, -1 if none
  uint8_t fin[48];       // fre[k] -> input address bit (NO_POS if none)
  uint8_t fout[48];      // fre[k] -> output address bit (NO_POS if none)
  int32_t op_begin, n_ops;   // the pass's fused ops (all its stages)
};

// Fused ops of one pass: the pass kernel resolves them one per lane of a
// wave (the planner keeps passes within this).
constexpr int MAX_PASS_OPS = 64;

// Dynamic LDS of a pass launch: the tile of 2^t floats.
inline size_t pass_lds_bytes(int t) { return sizeof(float) << t; }
constexpr size_t PASS_LDS_MAX = sizeof(float) << 14;

// Backward walk: a spin eliminated in a pass (candidate bit k) and the slot it
// held when the pass started (-1 if it entered during the pass).
struct BCand {
  int32_t spin;
  int32_t start_slot;
};

// A run of consecutive passes whose backward data fits in LDS at once.
struct BChunk {
  int32_t p_lo, p_hi;          // passes p_lo..p_hi (inclusive)
  int32_t cand_begin, n_cand;  // their candidates (contiguous)
  int32_t term_begin, n_term;  // their terms (contiguous)
};
constexpr int BCH_PASSES = 64, BCH_CANDS = 1024, BCH_TERMS = 2048;

// A term of the pass's energy that involves an eliminated spin:
// coef * sigma(a) [* sigma(b)], operands = candidate k (< 64) or 64 + slot of
// the selected output index; b = 255 for a field term.
struct BTerm {
  int32_t coef;     // edge (bond) or spin (field)
  uint8_t is_field;
  uint8_t a, b, pad;
};

// ---- launch tables ----
// One item of a pass launch: one pass of one plan over `batch` instances.
struct PassItem {
  const DevPass2* P;
  const DevStage* stages;
  const FOp* fops;
  const void* J;         // row of the item's first instance
  const void* h;         // (NULL without fields)
  int64_t jst, hst;      // row strides between instances
  const float* in;       // input state of the first instance
  float* out;
  int64_t in_st, out_st; // state strides between instances (2^in_w, 2^out_w)
  int64_t wg_begin;      // first workgroup of the item in the launch
  int32_t batch, xcd_group;
  // Last pass of a plan whose final state only feeds the final maximum: each
  // tile writes its maximum and first address (in the output layout) to
  // red_v / red_i[red_base + instance * 2^n_free + tile] instead of storing
  // the state (NULL: store).
  float* red_v;
  uint64_t* red_i;
  int64_t red_base;
  // Half-state plan (h = 0): entries whose top address bit is 1 are read and
  // written at the complement address; the tiles with fixed slot
  // P.z2_skip at 1 are not run (their outputs are the complements of the
  // others'), and red_base indexes the run tiles only.
  int32_t z2, pad_z2;
};

// Final reduction of one instance's state (2^w entries): maximum and its
// first address. With `bedge` set, entry a scores x[a] + sum over slots s of
// J[bedge[s]] sigma(a_s) sigma(ref_s), ref = *bref (a chimera row's vertical
// couplers to the already selected next row).
struct RedItem {
  const float* st;
  int64_t chunk_begin;   // first partial of the instance
  double* energy;        // may be NULL
  uint64_t* arg;         // may be NULL
  int32_t w, log2_chunks;
  const void* bJ;        // couplings of the instance (bonus), or NULL
  const int32_t* bedge;  // [w] edge per slot, -1 = none
  const uint64_t* bref;  // selected address of the next row
  int32_t bdtype;        // dtype of bJ: 0 float32, 1 int32, 2 int16
  int32_t z2;            // half-state plan: entries of the w-bit state read at their stored address
};

// Chimera row chain (see ChimeraRow): adds (init: writes) to every entry of
// one row's state the maximum over the row's horizontal groups; with `n` set
// (counting) multiplies the residues by the number of maximisers.
struct ChainItem {
  const ChimeraRow* row;
  const void* J;         // couplings / fields of the first instance
  const void* h;         // (NULL without fields)
  int64_t jst, hst;
  float* x;              // state of the first instance
  uint64_t* n;           // residue planes (counting), else NULL
  int64_t sst;           // entries per instance (2^w)
  int32_t w, cols, batch, init, log2_blocks, dtype;
  int32_t nres, pad;     // counting: residue planes (3, or 4 with the modulo-2^64 guard)
};

// Chimera backward finish: spins of every row from the selected addresses,
// horizontal groups by a Viterbi walk along each row, then sigma, dE/dJ, dE/dh.
struct ChimFinishItem {
  const ChimeraRow* rows;
  const int32_t* edges;
  const uint64_t* args;  // [rows][batch] selected address per row
  const void* J;
  const void* h;
  int64_t jst, hst, m;
  int8_t* sigma;
  float* dJ;
  float* dh;
  int32_t n, n_rows, cols, batch, dtype, pad;
};

// Input check of a call (k_check_inputs): one item per group of instances
// that share row strides; instance b of the item gets status[first + b].
struct CheckItem {
  const void* J;         // first instance's couplings
  const void* h;         // first instance's fields, or NULL
  int64_t m, n;          // couplings / fields per instance
  int64_t jst, hst;      // row strides between instances (elements)
  int64_t first;         // status index of the item's first instance
  int64_t limit;         // integer inputs: sum |J| + sum |h| must stay below this
  int32_t batch, dtype;  // dtype 0 = float32, 2 = int16, else int32
};
constexpr int CHECK_ITEMS = 32;   // items per launch (passed by value)
struct CheckArgs {
  CheckItem it[CHECK_ITEMS];
  int32_t n, pad;
};
constexpr uint32_t CHK_NONFINITE = 1u;   // a coupling or field is inf or NaN
constexpr uint32_t CHK_RANGE = 2u;       // sum |J| + sum |h| >= limit

// Backward walk of one instance.
struct BwdItem {
  const DevPass2* passes;
  const BChunk* chunks;
  int32_t n_chunks, pad2;
  const BCand* cands;
  const BTerm* terms;
  const void* J;
  const void* h;
  const float* const* ckpt;   // per-pass input states of this instance
  const uint64_t* final_addr;
  const uint8_t* final_pos;
  const int32_t* final_slot_spin;
  const int32_t* edges;
  int8_t* sigma;
  float* dJ;
  float* dh;
  int64_t m;
  int32_t n_passes, final_w, n, pad;
  // With red_v set, the selected final address is not read from final_addr:
  // the kernel ranks the instance's red_n partials of the final maximum
  // itself (ties to the lowest address) and writes -max to energy.
  const float* red_v;
  const uint64_t* red_i;
  int64_t red_n;
  double* energy;
  // Segment of the walk (checkpoint recomputation): passes seg_lo..seg_hi.
  // A segment that does not end the walk (seg_hi below the last pass) starts
  // from the selected entry in *carry and the spins already chosen, read back
  // from sigma; one that does not reach pass 0 writes its chosen spins to
  // sigma and the next selected entry to *carry instead of the gradients.
  // The whole walk is the single segment 0..n_passes-1.
  int32_t seg_lo, seg_hi;
  uint64_t* carry;
  // Tie rule of every choice of the walk: 0 the first maximiser, 1 the last,
  // other values a pseudo-random order per pass (the final state's own
  // maximum keeps the lowest address).
  uint64_t tie;
  // Half-state plan: checkpoint entries whose top address bit is 1 are read
  // at the complement address.
  int32_t z2, pad_z2;
};

}  // namespace tt

// Host-side plan IR of the tropical contraction.
//
// The tensor network of Sec. II (bond tensors on edges, field vectors, copy
// tensors = shared spin labels) is contracted as a sweep, the way Sec. V casts
// the square lattice as a tropical circuit acting on a 2^L state: one dense
// state tensor over the "live" spins absorbs leaf tensors one at a time.
// Each live spin occupies a slot = one bit of the state index (index bit 0 of
// a slot <-> sigma = +1). Operations on the state x[s]:
//
//   INTRO  slot      a new spin enters a free slot (free slots hold values that
//                    are constant along their bit, so this is a no-op: the
//                    start symbol (0, 0) of App. A)
//   FIELD  slot, i   x += h_i sigma(slot)                  (field gate, App. A)
//   DIAG   a, b, e   x += J_e sigma(a) sigma(b)            (two-site gate, App. A)
//   GATE   slot, e   x'[.., t, ..] = max_s x[.., s, ..] + J_e sigma(s) sigma(t):
//                    the bond matrix [[J,-J],[-J,J]] applied as a single-site
//                    gate; the old spin is eliminated and the new spin takes
//                    its slot (App. A, horizontal coupling gate)
//   CUT    slot      x'[.., t, ..] = max_s x[.., s, ..]: eliminate a spin whose
//                    bonds are all absorbed (App. A, cut gate)
//   GATE4  4 slots   a 16x16 tropical matrix between two groups of four spins
//                    (Sec. V, chimera): the four old spins are eliminated and
//                    four new spins take their slots
//   MERGE  reg       x += y elementwise with a second state y over the same
//                    spins in the same slots
//
// At the end the maximum over the remaining state is -E* (Sec. II).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace tt {

enum OpKind : uint8_t {
  OP_INTRO = 0,
  OP_GATE = 1,
  OP_CUT = 2,
  OP_DIAG = 3,
  OP_FIELD = 4,
  OP_GATE4 = 5,
  OP_MERGE = 6,
};

struct SweepOp {
  uint8_t kind = 0;
  int8_t reg = 0;          // state register the op acts on
  int16_t slot_a = -1;     // GATE/CUT/INTRO/FIELD slot; DIAG first slot; GATE4 first slot
  int16_t slot_b = -1;     // DIAG second slot
  int16_t slots4[4] = {-1, -1, -1, -1};  // GATE4 slots (group order)
  int32_t param = -1;      // GATE/DIAG: edge; FIELD: spin; GATE4: group-matrix id; MERGE: source register
  int32_t old_spin = -1;   // spin eliminated (GATE/CUT)
  int32_t new_spin = -1;   // spin entering (GATE/INTRO)
  int32_t old4[4] = {-1, -1, -1, -1};
  int32_t new4[4] = {-1, -1, -1, -1};
  int32_t live = 0;        // live spins after the op (algorithmic state size = 2^live)
  int32_t w_before = 0;    // physical width (highest used slot + 1) before / after
  int32_t w_after = 0;
};

// One pass = a run of ops executed by one kernel launch; every op that mixes
// entries along a slot (GATE, CUT, GATE4) has its slot among the t resident
// tile bits R, so a workgroup applies the whole run to its tile on chip.
struct Pass {
  int32_t op_begin = 0, op_end = 0;
  int32_t in_w = 0, out_w = 0, w_max = 0, t = 0;
  bool init = false;       // starts from the all-zero state
  int32_t reg = 0;         // state register of the pass
  int32_t merge_src = -1;  // register merged by an OP_MERGE inside the pass
  std::vector<int> R;      // tile bit -> slot (ascending)
  int32_t n_dec = 0;       // ops that record an argmax decision
};

// Group matrices of GATE4 ops: entry [t_old][t_new] = sum over the listed
// edges of J_e sigma(old bit) sigma(new bit).
struct GroupMatrix {
  int32_t edges[16];       // edge index, -1 = none
  uint8_t old_bit[16];     // bit of the old-group index for edge k
  uint8_t new_bit[16];     // bit of the new-group index for edge k
  int32_t n_edges = 0;
};

// Chimera graph of rows x cols K_{4,4} unit cells (Sec. V): spin
// 8 (r cols + c) + k of cell (r, c); k < 4 the group coupled vertically,
// k >= 4 the group coupled horizontally. The sweep state holds the vertical
// group of every cell of the current row (slot 4 c + k, 16^cols entries).
// Per row, one-to-one vertical couplers relabel the previous row's group into
// the current one (GATE ops); then the row's horizontal chain (the intra-cell
// 16 x 16 matrices and the horizontal couplers, with the horizontal groups
// maximised out) is added to every entry as a function of the whole state
// index ("chain" step, a kernel of its own between passes).
struct ChimeraRow {
  int32_t intra[8][16];   // edge of (v_k, h_l), index 4 k + l; -1 = no coupler
  int32_t horz[8][4];     // edge of h_l of cell c and h_l of cell c + 1; -1 = none
  int32_t vspin[8][4];    // spin of v_k of cell c
  int32_t hspin[8][4];    // spin of h_l of cell c
};

struct ChimeraInfo {
  int32_t rows = 0, cols = 0;
  std::vector<ChimeraRow> row;        // per row
  std::vector<int32_t> vert;          // [rows][cols][4] edge to the cell below, -1 = none
  std::vector<int32_t> row_end_op;    // op index after the last op of row r (row 0: 0)
};

struct Plan {
  int32_t n = 0;
  int64_t m = 0;
  std::vector<int32_t> edges;       // [m][2]
  bool has_field = false;
  std::vector<int32_t> order;
  std::vector<SweepOp> ops;
  std::vector<GroupMatrix> groups;
  int32_t width = 0;                // max physical width
  int32_t final_w = 0;
  std::vector<int32_t> final_slot_spin;   // slot -> spin after the last op, -1 free
  int32_t n_regs = 1;               // state registers (chimera plans use two)
  int32_t final_reg = 0;
  int32_t tile_bits = 14, count_tile_bits = 12;
  int32_t max_dec = 16;
  std::vector<Pass> passes;          // energy / backward path
  std::vector<Pass> count_passes;    // count path
  double terms = 0;                  // contraction terms per instance (one add + one max)
  double elementwise = 0;            // elementwise ops per instance (absorbs, cuts, final maximum)
  double reduce_ops = 0;             // of which the final maximum
  int64_t max_bytes = 0;
  int32_t parts = 2;                 // concurrent parts of a large same-graph batch (1 or 2)
  bool parts_auto = true;            // parts left to the library (the autotuner may choose 1)
  std::vector<int32_t> breaks;       // op indices where a pass must begin
  bool is_chimera = false;
  ChimeraInfo chim;
  void* dev = nullptr;               // device-side cache (owned, see capi)
  void* host_prog = nullptr;         // host encoding of the energy passes (owned, see capi)
  int32_t q = 2;                     // labels per spin: 2 (Ising) or 3 (Potts glass, App. C)
  bool z2 = false;                   // energy path keeps half of every state (h = 0 symmetry)
  void* potts = nullptr;             // 3-label programs and device cache (owned, see capi)
  void* slice = nullptr;             // sliced plan: fixed spins and the reduced plan (owned, see capi)
  uint64_t serial = 0;               // unique over the process lifetime (never reused)
};

// Builds ops from a spin order; returns "" or an error message.
std::string build_sweep_ops(Plan& p);
// Max-plus work per instance of the plan's ops at their live widths, each op's
// entries scaled by op_scale[k] (null: 1) and the final maximum by
// final_scale.
void sweep_work(const Plan& p, const double* op_scale, double final_scale, double* terms, double* elementwise,
                double* reduce_ops);
// Greedy order search with restarts.
std::vector<int32_t> greedy_order(int32_t n, const std::vector<int32_t>& edges, uint64_t seed,
                                  int trials);
// Chimera row-by-row plan (see ChimeraInfo); returns "" or an error.
std::string build_chimera_ops(Plan& p, int rows, int cols);
// Splits ops into passes of at most `t` resident bits and `max_dec` gated
// slots; `separable` adds the conditions of the one-argmax backward walk.
// `low` lowest slots are kept resident in every tile (identity bit order).
// `reserve` tile bits stay free for slots shared with the next pass (when
// the state is at least that much wider than the tile).
std::vector<Pass> partition_passes(const Plan& p, int t, int max_dec, bool separable, int low, int reserve = 0);

}  // namespace tt

// Host encoding of a sweep plan for 3-state labels (Potts glasses, App. C):
// ops are grouped into passes whose touched slots fit in the t tile digits a
// thread holds in registers.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>

#include "potts.hpp"

namespace tt {

namespace {

int64_t pow3(int k) {
  int64_t r = 1;
  while (k-- > 0) r *= 3;
  return r;
}

// Tile digits: the touched slots, padded (when fewer than t) with the highest
// untouched slots, so that the lowest slots stay non-tile digits, which vary
// fastest across threads (consecutive threads read consecutive entries).
// When every touched slot is below t the tile is slots 0 .. t-1 instead: a
// thread's entries are then one run and a workgroup's one contiguous block,
// which the kernel stages through LDS ("low" passes).
void finish_pass(const std::set<int>& touched, int W, int t, PottsPass& P) {
  std::vector<int> tile(touched.begin(), touched.end());
  const bool low = !touched.empty() && *touched.rbegin() < t;
  if (low) {
    tile.clear();
    for (int s = 0; s < t; ++s) tile.push_back(s);
  }
  for (int s = W - 1; s >= 0 && (int)tile.size() < t; --s)
    if (!touched.count(s)) tile.push_back(s);
  std::sort(tile.begin(), tile.end());
  P.low = low ? 1 : 0;
  P.t = t;
  for (int r = 0; r < t; ++r) P.tile_st[r] = pow3(tile[r]);
  P.n_nt = 0;
  for (int s = 0; s < W; ++s)
    if (!std::binary_search(tile.begin(), tile.end(), s)) P.nt_st[P.n_nt++] = pow3(s);
  P.threads = pow3(W - t);
  for (int o = 0; o < P.n_ops; ++o) {
    PottsOp& op = P.ops[o];
    op.a = (uint8_t)(std::lower_bound(tile.begin(), tile.end(), (int)op.a) - tile.begin());
    if (op.kind == OP_DIAG) op.b = (uint8_t)(std::lower_bound(tile.begin(), tile.end(), (int)op.b) - tile.begin());
  }
}

}  // namespace

std::string encode_potts(const Plan& p, int t, PottsProgram& out) {
  const int W = p.width;
  if (W < 1) return "empty plan";
  if (W > POTTS_MAX_W) return "state of 3^" + std::to_string(W) + " entries per instance is beyond the 3^20 limit";
  if (p.has_field) return "the Potts Hamiltonian has no field term";
  if (t < 2) return "tiles need at least two digits (a diagonal term touches two slots)";
  t = std::min(t, W);
  out.width = W;
  out.t = t;
  out.passes.clear();
  PottsPass cur;
  std::memset(&cur, 0, sizeof(cur));
  cur.init = 1;
  std::set<int> touched;
  auto flush = [&](bool force) {
    if (cur.n_ops == 0 && !force) return;
    finish_pass(touched, W, t, cur);
    out.passes.push_back(cur);
    std::memset(&cur, 0, sizeof(cur));
    touched.clear();
  };
  for (const SweepOp& op : p.ops) {
    if (op.kind == OP_INTRO) continue;          // a free slot is constant along its digit
    if (op.kind != OP_GATE && op.kind != OP_CUT && op.kind != OP_DIAG) return "unsupported op for 3-state labels";
    std::set<int> need = touched;
    need.insert(op.slot_a);
    if (op.kind == OP_DIAG) need.insert(op.slot_b);
    if ((int)need.size() > t || cur.n_ops == POTTS_MAX_OPS) {
      flush(false);
      need.clear();
      need.insert(op.slot_a);
      if (op.kind == OP_DIAG) need.insert(op.slot_b);
    }
    touched = need;
    PottsOp& d = cur.ops[cur.n_ops++];
    d.kind = op.kind;
    d.a = (uint8_t)op.slot_a;          // slot for now, tile digit after finish_pass
    d.b = (uint8_t)(op.kind == OP_DIAG ? op.slot_b : 0);
    d.edge = op.kind == OP_CUT ? -1 : op.param;
  }
  flush(out.passes.empty());            // at least one pass: it writes the zero state
  // final reduction over the live digits
  std::memset(&out.red, 0, sizeof(out.red));
  for (int s = 0; s < W; ++s) {
    const bool live = s < (int)p.final_slot_spin.size() && p.final_slot_spin[s] >= 0;
    if (live) out.red.st[out.red.n_live++] = pow3(s);
  }
  out.red.combos = pow3(out.red.n_live);
  out.red.contig = 1;
  for (int r = 0; r < out.red.n_live; ++r)
    if (out.red.st[r] != pow3(r)) out.red.contig = 0;
  // algorithmic work at the live width (base 3): a GATE is a contraction with
  // K = 3 (three terms per output entry), a DIAG one add per entry, a CUT two
  // maxima per output entry, the final maximum one per entry
  double terms = 0, elem = 0;
  int live_now = 0;
  for (const SweepOp& op : p.ops) {
    if (op.kind == OP_INTRO) live_now += 1;
    const double sz = std::pow(3.0, live_now);
    if (op.kind == OP_GATE) terms += 3 * sz;
    if (op.kind == OP_DIAG) elem += sz;
    if (op.kind == OP_CUT) {
      elem += 2 * sz / 3;
      live_now -= 1;
    }
  }
  out.terms = terms;
  out.elementwise = elem + std::pow(3.0, live_now);
  return "";
}

}  // namespace tt

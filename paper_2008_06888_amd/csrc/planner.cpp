// Host planner: spin order -> sweep ops -> passes.
//
// The contraction order question of Sec. III (cost exponential in the width of
// the largest intermediate) is answered here by a linear order of spins: the
// state tensor absorbs the spins one by one; its size is 2^(live spins), where
// a spin is live from its first absorbed bond until its last. The greedy
// search picks, at every step, the spin whose absorption leaves the fewest
// live spins (randomised ties, restarts), in the spirit of the greedy
// heuristics the paper cites for general graphs.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <queue>
#include <random>
#include <set>

#include "plan.hpp"

namespace tt {

namespace {

constexpr int MAX_OPS_PER_PASS = 64;   // the energy kernel resolves a pass's ops one per lane of a wave

struct Adj {
  std::vector<std::vector<std::pair<int, int>>> nb;  // (neighbour, edge)
  Adj(int n, const std::vector<int32_t>& e) : nb(n) {
    const size_t m = e.size() / 2;
    for (size_t k = 0; k < m; ++k) {
      nb[e[2 * k]].push_back({e[2 * k + 1], (int)k});
      nb[e[2 * k + 1]].push_back({e[2 * k], (int)k});
    }
  }
};

int lowest_free(std::vector<int>& slot_spin) {
  for (size_t s = 0; s < slot_spin.size(); ++s)
    if (slot_spin[s] < 0) return (int)s;
  slot_spin.push_back(-1);
  return (int)slot_spin.size() - 1;
}

int phys_width(const std::vector<int>& slot_spin) {
  int w = 0;
  for (size_t s = 0; s < slot_spin.size(); ++s)
    if (slot_spin[s] >= 0) w = (int)s + 1;
  return w;
}

}  // namespace

std::string build_sweep_ops(Plan& p) {
  const int n = p.n;
  Adj adj(n, p.edges);
  std::vector<int> pos(n, -1);
  for (int i = 0; i < n; ++i) {
    const int v = p.order[i];
    if (v < 0 || v >= n || pos[v] >= 0) return "order is not a permutation of the spins";
    pos[v] = i;
  }
  std::vector<char> processed(n, 0);
  std::vector<int> remaining(n, 0);   // bonds of a spin not yet absorbed
  for (int v = 0; v < n; ++v) remaining[v] = (int)adj.nb[v].size();
  std::vector<int> slot_of(n, -1);
  std::vector<int> slot_spin;          // slot -> spin (-1 free)
  std::vector<char> edge_done(p.m, 0);
  int live = 0;
  p.ops.clear();
  auto push = [&](SweepOp op) {
    op.w_after = phys_width(slot_spin);
    op.live = live;
    p.ops.push_back(op);
  };
  std::vector<int> completed;         // live spins with every bond absorbed (eliminated lazily)
  auto cut = [&](int x) {
    SweepOp c;
    c.w_before = phys_width(slot_spin);
    c.kind = OP_CUT;
    c.slot_a = (int16_t)slot_of[x];
    c.old_spin = x;
    slot_spin[slot_of[x]] = -1;
    slot_of[x] = -1;
    live -= 1;
    completed.erase(std::find(completed.begin(), completed.end(), x));
    push(c);
  };
  for (int step = 0; step < n; ++step) {
    const int v = p.order[step];
    // relabel candidate: a live spin whose only unabsorbed bond joins it to v;
    // the oldest such spin is preferred (the vertical bond of a lattice sweep)
    int rel_u = -1, rel_e = -1;
    for (auto [u, e] : adj.nb[v]) {
      if (processed[u] && slot_of[u] >= 0 && remaining[u] == 1 && !edge_done[e]) {
        if (rel_u < 0 || pos[u] < pos[rel_u]) {
          rel_u = u;
          rel_e = e;
        }
      }
    }
    SweepOp op;
    if (rel_u >= 0) {
      op.w_before = phys_width(slot_spin);
      const int s = slot_of[rel_u];
      op.kind = OP_GATE;
      op.slot_a = (int16_t)s;
      op.param = rel_e;
      op.old_spin = rel_u;
      op.new_spin = v;
      edge_done[rel_e] = 1;
      remaining[rel_u] -= 1;
      remaining[v] -= 1;
      slot_of[rel_u] = -1;
      slot_of[v] = s;
      slot_spin[s] = v;
      push(op);
    } else {
      // a free slot, else the slot of a completed spin, else a new slot
      int s = -1;
      for (size_t q = 0; q < slot_spin.size(); ++q)
        if (slot_spin[q] < 0) {
          s = (int)q;
          break;
        }
      if (s < 0 && !completed.empty()) {
        int best = completed[0];
        for (int x : completed)
          if (slot_of[x] < slot_of[best]) best = x;
        s = slot_of[best];
        cut(best);
      }
      if (s < 0) s = lowest_free(slot_spin);
      op.w_before = phys_width(slot_spin);
      op.kind = OP_INTRO;
      op.slot_a = (int16_t)s;
      op.new_spin = v;
      slot_of[v] = s;
      slot_spin[s] = v;
      live += 1;
      push(op);
    }
    processed[v] = 1;
    // bonds between v and live spins become two-site diagonal gates
    for (auto [w, e] : adj.nb[v]) {
      if (edge_done[e] || !processed[w] || slot_of[w] < 0) continue;
      SweepOp d;
      d.w_before = phys_width(slot_spin);
      d.kind = OP_DIAG;
      d.slot_a = (int16_t)slot_of[v];
      d.slot_b = (int16_t)slot_of[w];
      d.param = e;
      edge_done[e] = 1;
      remaining[v] -= 1;
      remaining[w] -= 1;
      push(d);
    }
    if (p.has_field) {
      SweepOp f;
      f.w_before = phys_width(slot_spin);
      f.kind = OP_FIELD;
      f.slot_a = (int16_t)slot_of[v];
      f.param = v;
      push(f);
    }
    for (auto [w, e] : adj.nb[v]) {
      (void)e;
      if (slot_of[w] >= 0 && remaining[w] == 0 &&
          std::find(completed.begin(), completed.end(), w) == completed.end())
        completed.push_back(w);
    }
    if (slot_of[v] >= 0 && remaining[v] == 0 &&
        std::find(completed.begin(), completed.end(), v) == completed.end())
      completed.push_back(v);
    if (step == n - 1) break;   // the final reduction eliminates what is left
    // completed spins in the highest slots are eliminated at once (the state shrinks)
    for (;;) {
      const int w = phys_width(slot_spin);
      if (w == 0) break;
      const int x = slot_spin[w - 1];
      if (x < 0 || remaining[x] != 0) break;
      cut(x);
    }
  }
  for (int v = 0; v < n; ++v)
    if (remaining[v] != 0) return "internal: unabsorbed bond";
  p.width = 0;
  for (auto& op : p.ops) p.width = std::max(p.width, std::max(op.w_before, op.w_after));
  p.final_w = p.ops.empty() ? 0 : p.ops.back().w_after;
  p.final_slot_spin.assign(p.final_w, -1);
  for (int s = 0; s < p.final_w && s < (int)slot_spin.size(); ++s) p.final_slot_spin[s] = slot_spin[s];
  sweep_work(p, nullptr, 1.0, &p.terms, &p.elementwise, &p.reduce_ops);
  return "";
}

void sweep_work(const Plan& p, const double* op_scale, double final_scale, double* terms, double* elementwise,
                double* reduce_ops) {
  // algorithmic work, at the live (not the physical) width: a GATE is a
  // contraction with K = 2, i.e. two terms (add + max) per output entry; a
  // DIAG or FIELD is an elementwise tropical product (one add per entry), a
  // CUT an elementwise maximum of the two halves (one max per output entry),
  // and the final maximum one max per entry of the last state
  double t = 0, elem = 0;
  int live_now = 0;
  for (size_t k = 0; k < p.ops.size(); ++k) {
    const SweepOp& op = p.ops[k];
    if (op.kind == OP_INTRO) live_now += 1;
    const double sz = std::ldexp(1.0, live_now) * (op_scale ? op_scale[k] : 1.0);
    if (op.kind == OP_GATE) t += 2 * sz;
    if (op.kind == OP_DIAG || op.kind == OP_FIELD) elem += sz;
    if (op.kind == OP_CUT) {
      elem += sz / 2;
      live_now -= 1;
    }
  }
  *reduce_ops = std::ldexp(1.0, live_now) * final_scale;   // final reduction
  *terms = t;
  *elementwise = elem + *reduce_ops;
}

std::vector<int32_t> greedy_order(int32_t n, const std::vector<int32_t>& edges, uint64_t seed,
                                  int trials) {
  Adj adj(n, edges);
  std::mt19937_64 rng(seed * 0x9E3779B97F4A7C15ull + 12345);
  std::vector<int32_t> best;
  double best_key1 = 1e300, best_key2 = 1e300;
  for (int t = 0; t < std::max(1, trials); ++t) {
    std::vector<char> processed(n, 0);
    std::vector<int> rem(n);
    for (int v = 0; v < n; ++v) rem[v] = (int)adj.nb[v].size();
    std::vector<int32_t> order;
    order.reserve(n);
    std::set<int> frontier;   // unprocessed spins adjacent to processed ones
    int live = 0, peak = 0;
    double cost = 0;
    std::vector<double> noise(n);
    for (int step = 0; step < n; ++step) {
      for (int v = 0; v < n; ++v) noise[v] = std::uniform_real_distribution<double>(0, 1)(rng);
      int pick = -1;
      long key_best[3] = {0, 0, 0};
      double nz_best = 2;
      auto consider = [&](int v) {
        int unproc = 0, closing = 0;
        bool rel = false;
        for (auto [w, e] : adj.nb[v]) {
          (void)e;
          if (processed[w]) {
            if (rem[w] == 1) {
              closing += 1;
              rel = true;
            }
          } else {
            unproc += 1;
          }
        }
        const long pk = live + (rel ? 0 : 1);
        const long nl = live + (unproc > 0 ? 1 : 0) - closing;
        const long key[3] = {std::max(pk, nl), nl, -(long)(adj.nb[v].size() - unproc)};
        bool better = pick < 0;
        if (!better) {
          for (int k = 0; k < 3; ++k) {
            if (key[k] != key_best[k]) {
              better = key[k] < key_best[k];
              goto decided;
            }
          }
          better = noise[v] < nz_best;
        decided:;
        }
        if (better) {
          pick = v;
          std::memcpy(key_best, key, sizeof(key));
          nz_best = noise[v];
        }
      };
      if (step == 0) {
        pick = (int)(rng() % (uint64_t)n);
      } else if (!frontier.empty()) {
        for (int v : frontier) consider(v);
      } else {
        for (int v = 0; v < n; ++v)
          if (!processed[v]) consider(v);
      }
      const int v = pick;
      int unproc = 0;
      bool rel = false;
      const int live_before = live;
      for (auto [w, e] : adj.nb[v]) {
        (void)e;
        if (processed[w] && rem[w] == 1) rel = true;
      }
      for (auto [w, e] : adj.nb[v]) {
        (void)e;
        if (processed[w]) {
          rem[w] -= 1;
          rem[v] -= 1;
          if (rem[w] == 0) live -= 1;
        } else {
          unproc += 1;
          frontier.insert(w);
        }
      }
      processed[v] = 1;
      frontier.erase(v);
      if (unproc > 0) live += 1;
      // peak: an absorption without a relabel briefly holds one more spin
      peak = std::max(peak, std::max(live_before + (rel ? 0 : 1), live));
      cost += std::ldexp(1.0, live);
      order.push_back(v);
    }
    if (peak < best_key1 || (peak == best_key1 && cost < best_key2)) {
      best_key1 = peak;
      best_key2 = cost;
      best = order;
    }
  }
  return best;
}

std::vector<Pass> partition_passes(const Plan& p, int t, int max_dec, bool separable, int low, int reserve) {
  // separable: every pass can be walked back by one argmax over its gated
  // slots (see the backward kernel): no slot gated twice, no gate on a slot
  // that a diagonal term or an INTRO already touched in the same pass.
  std::vector<Pass> out;
  const int n_ops = (int)p.ops.size();
  const int LOW = low;   // lowest slots always resident (consecutive entries per load)
  std::vector<char> brk(n_ops + 1, 0);
  for (int b : p.breaks)
    if (b >= 0 && b <= n_ops) brk[b] = 1;
  int i = 0;
  while (i < n_ops) {
    const int start = i;
    const int reg = p.ops[i].reg;
    std::set<int> need, touched, intro;
    int wmax = p.ops[i].w_before;
    int ndec = 0;
    int merge_src = -1;
    while (i < n_ops) {
      const SweepOp& op = p.ops[i];
      if (op.reg != reg || (i > start && brk[i])) break;
      std::set<int> need2 = need;
      int ndec2 = ndec;
      bool sep_ok = true;
      if (op.kind == OP_GATE || op.kind == OP_CUT) {
        sep_ok = !need.count(op.slot_a) && !touched.count(op.slot_a) && !intro.count(op.slot_a);
        need2.insert(op.slot_a);
        ndec2 += 1;
      } else if (op.kind == OP_GATE4) {
        for (int k = 0; k < 4; ++k) {
          sep_ok = sep_ok && !need.count(op.slots4[k]) && !touched.count(op.slots4[k]) && !intro.count(op.slots4[k]);
          need2.insert(op.slots4[k]);
        }
        ndec2 += 1;
      }
      if (op.kind == OP_MERGE && merge_src >= 0 && merge_src != op.param) break;
      const int wmax2 = std::max(wmax, std::max(op.w_before, op.w_after));
      std::set<int> with_low = need2;
      for (int s = 0; s < std::min(LOW, wmax2); ++s) with_low.insert(s);
      // keep `reserve` tile bits for slots shared with the next pass when at
      // least that many slots lie outside the tile (else the neighbours'
      // tiles overlap anyway): consecutive tiles then share the low address
      // bits and both the store and the next load stream whole runs
      const int rsv = (wmax2 - t >= reserve) ? reserve : 0;
      bool ok = (wmax2 <= t) || ((int)with_low.size() + rsv <= t);
      ok = ok && ndec2 <= max_dec && (!separable || sep_ok) && (i - start) < MAX_OPS_PER_PASS;
      if (!ok && i > start) break;
      need.swap(need2);
      ndec = ndec2;
      wmax = wmax2;
      if (op.kind == OP_DIAG) {
        touched.insert(op.slot_a);
        touched.insert(op.slot_b);
      } else if (op.kind == OP_FIELD) {
        touched.insert(op.slot_a);
      } else if (op.kind == OP_INTRO) {
        intro.insert(op.slot_a);
      }
      if (op.kind == OP_MERGE) merge_src = op.param;
      ++i;
    }
    Pass ps;
    ps.op_begin = start;
    ps.op_end = i;
    ps.reg = reg;
    ps.merge_src = merge_src;
    ps.in_w = p.ops[start].w_before;
    ps.out_w = p.ops[i - 1].w_after;
    ps.w_max = wmax;
    ps.n_dec = ndec;
    // a register's first pass starts from zeros
    ps.init = true;
    for (const Pass& q : out)
      if (q.reg == reg) ps.init = false;
    if (wmax <= t) {
      ps.t = wmax;
      for (int s = 0; s < wmax; ++s) ps.R.push_back(s);
    } else {
      ps.t = t;
      std::set<int> R = need;
      for (int s = 0; s < std::min(LOW, wmax); ++s) R.insert(s);
      for (int s = 0; (int)R.size() < t && s < wmax; ++s) R.insert(s);
      ps.R.assign(R.begin(), R.end());
    }
    out.push_back(ps);
  }
  return out;
}

std::string build_chimera_ops(Plan& p, int rows, int cols) {
  if (rows < 1 || cols < 1 || rows > 64) return "chimera plans need 1 <= rows <= 64 and cols >= 1";
  if (cols > 8) return "chimera plans hold at most 8 cells per row (a 2^32-entry state)";
  if ((int64_t)p.n != 8ll * rows * cols) return "chimera plan: n_spins must be 8 * rows * cols";
  ChimeraInfo& ch = p.chim;
  ch.rows = rows;
  ch.cols = cols;
  ch.row.assign(rows, ChimeraRow());
  for (ChimeraRow& R : ch.row) {
    std::memset(&R, 0xff, sizeof(R));   // -1 everywhere
  }
  ch.vert.assign((size_t)rows * cols * 4, -1);
  auto id = [&](int r, int c, int k) { return 8 * (r * cols + c) + k; };
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < cols; ++c)
      for (int k = 0; k < 4; ++k) {
        ch.row[r].vspin[c][k] = id(r, c, k);
        ch.row[r].hspin[c][k] = id(r, c, 4 + k);
      }
  // classify every edge as an intra-cell, vertical or horizontal coupler
  for (int64_t e = 0; e < p.m; ++e) {
    const int a = p.edges[2 * e], b = p.edges[2 * e + 1];
    const int ca = a / 8, cb = b / 8, ka = a % 8, kb = b % 8;
    const int ra = ca / cols, ma = ca % cols, rb = cb / cols, mb = cb % cols;
    int32_t* slot = nullptr;
    if (ca == cb && ka < 4 && kb >= 4) {
      slot = &ch.row[ra].intra[ma][4 * ka + (kb - 4)];
    } else if (ka == kb && ka < 4 && mb == ma && rb == ra + 1) {
      slot = &ch.vert[((size_t)ra * cols + ma) * 4 + ka];
    } else if (ka == kb && ka >= 4 && rb == ra && mb == ma + 1) {
      slot = &ch.row[ra].horz[ma][ka - 4];
    }
    if (!slot) return "edge (" + std::to_string(a) + ", " + std::to_string(b) + ") is not a chimera coupler";
    *slot = (int32_t)e;
  }
  // ops: per row r >= 1, relabel the vertical group of every cell (one-to-one
  // couplers; a missing coupler eliminates the old spin and frees the slot)
  const int w = 4 * cols;
  p.ops.clear();
  p.order.clear();
  ch.row_end_op.assign(rows, 0);
  for (int r = 0; r < rows; ++r) {
    for (int c = 0; c < cols; ++c)
      for (int k = 0; k < 8; ++k) p.order.push_back(id(r, c, k));
    if (r > 0) {
      for (int c = 0; c < cols; ++c)
        for (int k = 0; k < 4; ++k) {
          const int slot = 4 * c + k;
          const int e = ch.vert[((size_t)(r - 1) * cols + c) * 4 + k];
          SweepOp op;
          op.slot_a = (int16_t)slot;
          op.old_spin = id(r - 1, c, k);
          op.live = w;
          op.w_before = op.w_after = w;
          if (e >= 0) {
            op.kind = OP_GATE;
            op.param = e;
            op.new_spin = id(r, c, k);
            p.ops.push_back(op);
          } else {
            op.kind = OP_CUT;
            p.ops.push_back(op);
            SweepOp in;
            in.kind = OP_INTRO;
            in.slot_a = (int16_t)slot;
            in.new_spin = id(r, c, k);
            in.live = w;
            in.w_before = in.w_after = w;
            p.ops.push_back(in);
          }
        }
    }
    ch.row_end_op[r] = (int32_t)p.ops.size();
  }
  p.breaks.assign(ch.row_end_op.begin(), ch.row_end_op.end());
  p.is_chimera = true;
  p.width = w;
  p.final_w = w;
  p.final_slot_spin.assign(w, -1);
  for (int c = 0; c < cols; ++c)
    for (int k = 0; k < 4; ++k) p.final_slot_spin[4 * c + k] = id(rows - 1, c, k);
  // algorithmic work: two terms per entry for every vertical relabel (K = 2),
  // sixteen per entry for the chain of every row (a 16-way maximum over the
  // split chain), and the final maximum (one max per entry, elementwise)
  const double W = std::ldexp(1.0, w);
  p.reduce_ops = W;
  p.terms = (double)(rows - 1) * 4 * cols * 2.0 * W + (double)rows * 16.0 * W;
  p.elementwise = W;
  return "";
}

}  // namespace tt

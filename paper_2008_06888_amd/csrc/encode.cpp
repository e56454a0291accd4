// Host encoding of the energy passes (see sweep_kernels.hip):
//  * tiles: the resident slots R of each pass (its gate slots, then slots
//    the neighbouring passes gate, so consecutive tiles overlap);
//  * layouts: the bit order of the state between passes; the lowest address
//    bits go to slots resident in both neighbouring tiles, so every load and
//    store streams runs of consecutive entries;
//  * fused ops: each gate carries the diagonal terms of the spin it brings
//    in; stages of at most four gate bits for the register kernel;
//  * backward tables: the spins each pass eliminates and every energy term
//    of the pass that touches one of them.
#include <algorithm>
#include <cstring>
#include <map>
#include <set>

#include "encode.hpp"

namespace tt {

namespace {

constexpr int LOW_BITS = 6;   // 64 consecutive floats per run

// LDS swizzle of a tile index (must match the kernel's swz()).
uint32_t swz(uint32_t i) { return i ^ ((i >> 5) & 31u); }

std::vector<int> gate_slots(const Plan& p, const Pass& ps) {
  std::vector<int> g;
  for (int o = ps.op_begin; o < ps.op_end; ++o) {
    const SweepOp& op = p.ops[o];
    if ((op.kind == OP_GATE || op.kind == OP_CUT) && std::find(g.begin(), g.end(), op.slot_a) == g.end())
      g.push_back(op.slot_a);
  }
  return g;
}

}  // namespace

std::string encode_energy(const Plan& p, const std::vector<Pass>& passes, EnergyProgram& out) {
  out = EnergyProgram();
  const int np = (int)passes.size();
  const int tmax = p.tile_bits;
  if (np == 0) {   // nothing to sweep (a one-row chimera plan): identity layout
    for (int s = 0; s < p.final_w; ++s) out.final_pos.push_back((uint8_t)s);
    return "";
  }
  // slot -> spin before every op (replay of the op list)
  std::vector<std::vector<int>> slot_spin_at(p.ops.size() + 1);
  {
    std::vector<int> cur;
    if (p.is_chimera) {   // the sweep starts from row 0's vertical groups
      cur.assign(p.width, -1);
      for (int c = 0; c < p.chim.cols; ++c)
        for (int k = 0; k < 4; ++k) cur[4 * c + k] = p.chim.row[0].vspin[c][k];
    }
    for (size_t o = 0; o < p.ops.size(); ++o) {
      slot_spin_at[o] = cur;
      const SweepOp& op = p.ops[o];
      if (op.kind == OP_INTRO || op.kind == OP_GATE) {
        if ((int)cur.size() <= op.slot_a) cur.resize(op.slot_a + 1, -1);
        cur[op.slot_a] = op.new_spin;
      } else if (op.kind == OP_CUT) {
        if ((int)cur.size() <= op.slot_a) cur.resize(op.slot_a + 1, -1);
        cur[op.slot_a] = -1;
      }
    }
    slot_spin_at[p.ops.size()] = cur;
  }
  // resident slots per pass
  std::vector<std::vector<int>> G(np), R(np);
  for (int q = 0; q < np; ++q) G[q] = gate_slots(p, passes[q]);
  for (int q = 0; q < np; ++q) {
    const Pass& ps = passes[q];
    std::vector<int> r;
    if (ps.w_max <= tmax) {
      for (int s = 0; s < ps.w_max; ++s) r.push_back(s);
    } else {
      r = G[q];
      if ((int)r.size() > tmax) return "internal: pass gates more slots than the tile holds";
      auto add = [&](int s) {
        if ((int)r.size() < tmax && s < ps.w_max && std::find(r.begin(), r.end(), s) == r.end()) r.push_back(s);
      };
      if (q + 1 < np)
        for (int s : G[q + 1]) add(s);
      else if (p.is_chimera)   // the final state is stored in slot order
        for (int s = 0; s < LOW_BITS; ++s) add(s);
      if (q > 0)
        for (int s : G[q - 1]) add(s);
      for (int s = 0; s < ps.w_max; ++s) add(s);
    }
    // at least four resident bits (a register group spans four): pad with
    // slots beyond the state, which have no address and are never stored
    for (int s = ps.w_max; (int)r.size() < 4; ++s) r.push_back(s);
    std::sort(r.begin(), r.end());
    R[q] = r;
  }
  // layouts at the pass boundaries: pos[b][slot], b = 0..np; a chimera
  // plan's row boundaries keep slot order (its chain step reads slot s at
  // index bit s)
  auto row_boundary = [&](int b) {
    if (!p.is_chimera) return false;
    if (b == 0 || b == np) return true;
    const int e = passes[b - 1].op_end;
    return std::find(p.chim.row_end_op.begin(), p.chim.row_end_op.end(), e) != p.chim.row_end_op.end();
  };
  std::vector<std::vector<int>> pos(np + 1);
  for (int b = 0; b <= np; ++b) {
    const int w = b < np ? passes[b].in_w : passes[np - 1].out_w;
    std::vector<int> low;
    if (b > 0 && !row_boundary(b)) {
      for (int s : R[b - 1]) {
        if (s >= w) continue;
        if (b < np && std::find(R[b].begin(), R[b].end(), s) == R[b].end()) continue;
        if ((int)low.size() < LOW_BITS) low.push_back(s);
      }
    }
    // above the shared bits: the rest of the next tile (so a tile loads one
    // contiguous block), then the rest of the previous tile (so a tile's
    // stores stay inside a region of 2^(t + 8) entries), then slot order;
    // both keep the pages a workgroup touches few
    std::vector<int> ps(w, -1);
    int k = 0;
    for (int s : low) ps[s] = k++;
    if (!row_boundary(b)) {
      if (b < np)
        for (int s : R[b])
          if (s < w && ps[s] < 0) ps[s] = k++;
      if (b > 0)
        for (int s : R[b - 1])
          if (s < w && ps[s] < 0) ps[s] = k++;
    }
    for (int s = 0; s < w; ++s)
      if (ps[s] < 0) ps[s] = k++;
    pos[b] = ps;
  }
  out.final_pos.assign(pos[np].begin(), pos[np].end());
  for (int q = 0; q < np; ++q) {
    const Pass& ps = passes[q];
    DevPass2 d;
    std::memset(&d, 0, sizeof(d));
    d.in_w = ps.in_w;
    d.out_w = ps.out_w;
    d.w_max = ps.w_max;
    d.t = (int)R[q].size();
    d.init = ps.init ? 1 : 0;
    if (d.t > 16) return "internal: tile too large";
    int tbit[80];
    for (int s = 0; s < 80; ++s) tbit[s] = -1;
    for (int k = 0; k < d.t; ++k) {
      d.R[k] = (uint8_t)R[q][k];
      tbit[R[q][k]] = k;
    }
    int nf = 0;
    for (int s = 0; s < ps.w_max; ++s) {
      if (tbit[s] >= 0) continue;
      if (nf >= 48) return "state wider than the index supports";
      d.fre[nf++] = (uint8_t)s;
    }
    d.n_free = nf;
    std::memset(d.in_pos, NO_POS, sizeof(d.in_pos));
    std::memset(d.out_pos, NO_POS, sizeof(d.out_pos));
    for (int s = 0; s < ps.in_w; ++s) d.in_pos[s] = (uint8_t)pos[q][s];
    for (int s = 0; s < ps.out_w; ++s) d.out_pos[s] = (uint8_t)pos[q + 1][s];
    for (int k = 0; k < nf; ++k) {
      d.fin[k] = d.in_pos[d.fre[k]];
      d.fout[k] = d.out_pos[d.fre[k]];
    }
    // threads per tile: 16 entries each, one wave at least, 1024 at most
    d.tb = std::min(10, std::max(6, d.t - 4));
    // half-state plans pair each tile with its complement: the lowest tile-id
    // bit whose fixed slot has an output position separates the pairs
    d.z2_skip = -1;
    for (int k = 0; k < d.n_free; ++k)
      if (d.fout[k] != NO_POS) {
        d.z2_skip = k;
        break;
      }
    // enumeration orders of the load and the store
    std::vector<int> ld, st, ld_rest, st_rest;
    for (int k = 0; k < d.t; ++k) {
      const int s = R[q][k];
      (s < ps.in_w ? ld : ld_rest).push_back(k);
      (s < ps.out_w ? st : st_rest).push_back(k);
    }
    std::sort(ld.begin(), ld.end(), [&](int a, int b) { return d.in_pos[R[q][a]] < d.in_pos[R[q][b]]; });
    std::sort(st.begin(), st.end(), [&](int a, int b) { return d.out_pos[R[q][a]] < d.out_pos[R[q][b]]; });
    d.n_ld = (int)ld.size();
    d.n_st = (int)st.size();
    ld.insert(ld.end(), ld_rest.begin(), ld_rest.end());
    st.insert(st.end(), st_rest.begin(), st_rest.end());
    for (int k = 0; k < d.t; ++k) {
      d.ld_order[k] = (uint8_t)ld[k];
      d.st_order[k] = (uint8_t)st[k];
      d.ld_bti[k] = 1u << ld[k];
      d.st_bti[k] = 1u << st[k];
      d.ld_bad[k] = k < d.n_ld ? (1ull << d.in_pos[R[q][ld[k]]]) : 0ull;
      d.st_bad[k] = k < d.n_st ? (1ull << d.out_pos[R[q][st[k]]]) : 0ull;
    }
    for (int kk = 0; kk < 16; ++kk) {
      uint32_t lt = 0, stt = 0;
      uint64_t la = 0, sa = 0;
      for (int b = 0; b < 4; ++b) {
        if (!((kk >> b) & 1)) continue;
        if (d.tb + b < d.t) {
          lt |= d.ld_bti[d.tb + b];
          la |= d.ld_bad[d.tb + b];
        }
        if (d.tb + b < d.n_st) {
          stt |= d.st_bti[d.tb + b];
          sa |= d.st_bad[d.tb + b];
        }
      }
      d.ld_hti[kk] = lt;
      d.ld_had[kk] = la;
      d.st_hti[kk] = stt;
      d.st_had[kk] = sa;
    }
    auto enc = [&](int slot) -> uint8_t {
      return tbit[slot] >= 0 ? (uint8_t)tbit[slot] : (uint8_t)(SLOT_FIXED + slot);
    };
    // fused ops
    std::vector<FOp> f;
    for (int o = ps.op_begin; o < ps.op_end;) {
      const SweepOp& op = p.ops[o];
      FOp x;
      std::memset(&x, 0, sizeof(x));
      x.hspin = -1;
      if (op.kind == OP_CUT) {
        x.kind = FK_CUT;
        x.bit = (uint8_t)tbit[op.slot_a];
        f.push_back(x);
        ++o;
        continue;
      }
      int slot;
      if (op.kind == OP_GATE) {
        x.kind = FK_GATE;
        x.bit = (uint8_t)tbit[op.slot_a];
        x.edge = op.param;
        slot = op.slot_a;
        ++o;
      } else if (op.kind == OP_INTRO) {
        x.kind = FK_STAR;
        x.bit = enc(op.slot_a);
        slot = op.slot_a;
        ++o;
      } else {   // a diagonal term not following its spin's entry: a star of its own
        x.kind = FK_STAR;
        x.bit = enc(op.slot_a);
        slot = op.slot_a;
      }
      // the diagonal terms of the spin in `slot` that follow
      bool any = x.kind != FK_STAR;
      while (o < ps.op_end) {
        const SweepOp& d2 = p.ops[o];
        if (d2.slot_a != slot || (d2.kind != OP_DIAG && d2.kind != OP_FIELD)) break;
        if (d2.kind == OP_FIELD) {
          if (x.hspin >= 0) break;
          x.hspin = d2.param;
        } else {
          if (x.nt == STAR_TERMS) {
            f.push_back(x);
            std::memset(&x, 0, sizeof(x));
            x.kind = FK_STAR;
            x.bit = enc(slot);
            x.hspin = -1;
          }
          x.w[x.nt] = enc(d2.slot_b);
          x.te[x.nt] = d2.param;
          x.nt += 1;
        }
        any = true;
        ++o;
      }
      if (any) f.push_back(x);
    }
    // stages of at most four distinct gate bits
    d.stage_begin = (int)out.stages.size();
    size_t b0 = 0;
    while (b0 < f.size()) {
      std::vector<int> S;
      size_t e = b0;
      for (; e < f.size(); ++e) {
        if (f[e].kind == FK_STAR) continue;
        const int b = f[e].bit;
        if (std::find(S.begin(), S.end(), b) != S.end()) continue;
        if ((int)S.size() == 4) break;
        S.push_back(b);
      }
      for (int k = d.t - 1; (int)S.size() < 4 && k >= 0; --k)
        if (std::find(S.begin(), S.end(), k) == S.end()) S.push_back(k);
      DevStage st2;
      std::memset(&st2, 0, sizeof(st2));
      for (int l = 0; l < 4; ++l) st2.sb[l] = (uint8_t)S[l];
      int nns = 0;
      for (int k = 0; k < d.t; ++k)
        if (std::find(S.begin(), S.end(), k) == S.end()) st2.ns[nns++] = (uint8_t)k;
      st2.nns = (uint8_t)nns;
      for (int x = 0; x < 32; ++x) {
        uint16_t lo = 0, hi = 0;
        for (int q = 0; q < 5; ++q) {
          if ((x >> q) & 1) {
            if (q < nns) lo |= (uint16_t)(1u << st2.ns[q]);
            if (q + 5 < nns) hi |= (uint16_t)(1u << st2.ns[q + 5]);
          }
        }
        st2.g_lo[x] = lo;
        st2.g_hi[x] = hi;
        st2.sg_lo[x] = (uint16_t)swz(lo);
        st2.sg_hi[x] = (uint16_t)swz(hi);
      }
      for (int j = 0; j < 16; ++j) {
        uint32_t sj = 0;
        for (int l = 0; l < 4; ++l)
          if ((j >> l) & 1) sj |= 1u << S[l];
        st2.soff[j] = swz(sj);
      }
      st2.op_begin = (int)out.fops.size();
      for (size_t k = b0; k < e; ++k) {
        FOp x = f[k];
        x.lidx = (uint8_t)(std::find(S.begin(), S.end(), (int)x.bit) - S.begin());   // 4 if absent
        for (int q = 0; q < STAR_TERMS; ++q) {
          x.wl[q] = 255;
          if (q < x.nt && x.w[q] < SLOT_FIXED) {
            auto it = std::find(S.begin(), S.end(), (int)x.w[q]);
            if (it != S.end()) x.wl[q] = (uint8_t)(it - S.begin());
          }
        }
        out.fops.push_back(x);
      }
      st2.op_end = (int)out.fops.size();
      out.stages.push_back(st2);
      b0 = e;
    }
    d.n_stages = (int)out.stages.size() - d.stage_begin;
    d.op_begin = d.n_stages ? out.stages[d.stage_begin].op_begin : (int)out.fops.size();
    d.n_ops = d.n_stages ? out.stages.back().op_end - d.op_begin : 0;
    if (d.n_ops > MAX_PASS_OPS) return "a pass holds more ops than the pass kernel resolves (one per lane)";
    // backward tables
    const std::vector<int>& start = slot_spin_at[ps.op_begin];
    const std::vector<int>& end = slot_spin_at[ps.op_end];
    std::map<int, int> cand;      // spin -> candidate index
    std::map<int, int> end_slot;  // spin -> slot at the end of the pass
    for (size_t s = 0; s < end.size(); ++s)
      if (end[s] >= 0) end_slot[end[s]] = (int)s;
    d.cand_begin = (int)out.cands.size();
    for (int o = ps.op_begin; o < ps.op_end; ++o) {
      const SweepOp& op = p.ops[o];
      if (op.kind != OP_GATE && op.kind != OP_CUT) continue;
      const int k = (int)cand.size();
      cand[op.old_spin] = k;
      BCand c;
      c.spin = op.old_spin;
      c.start_slot = -1;
      for (size_t s = 0; s < start.size(); ++s)
        if (start[s] == op.old_spin) c.start_slot = (int)s;
      out.cands.push_back(c);
    }
    d.n_cand = (int)cand.size();
    if (d.n_cand > 16) return "internal: too many eliminations in one pass";
    out.max_cand = std::max(out.max_cand, d.n_cand);
    uint64_t surv = 0;
    for (int s = 0; s < ps.in_w && s < (int)start.size(); ++s)
      if (start[s] >= 0 && !cand.count(start[s])) surv |= 1ull << s;
    d.surv_mask = surv;
    std::vector<BTerm> lo, hi, cross;
    auto operand = [&](int spin, bool* is_cand, int* k) -> uint8_t {
      auto it = cand.find(spin);
      if (it != cand.end()) {
        *is_cand = true;
        *k = it->second;
        return (uint8_t)it->second;
      }
      *is_cand = false;
      *k = -1;
      return (uint8_t)(64 + end_slot.at(spin));
    };
    for (int o = ps.op_begin; o < ps.op_end; ++o) {
      const SweepOp& op = p.ops[o];
      const std::vector<int>& cur = slot_spin_at[o];
      int sa = -1, sb = -1, coef = -1;
      uint8_t field = 0;
      if (op.kind == OP_GATE) {
        sa = op.old_spin;
        sb = op.new_spin;
        coef = op.param;
      } else if (op.kind == OP_DIAG) {
        sa = cur[op.slot_a];
        sb = cur[op.slot_b];
        coef = op.param;
      } else if (op.kind == OP_FIELD) {
        sa = cur[op.slot_a];
        coef = op.param;
        field = 1;
      } else {
        continue;
      }
      bool ca = false, cb = false;
      int ka = -1, kb = -1;
      BTerm tm;
      tm.coef = coef;
      tm.is_field = field;
      tm.pad = 0;
      tm.a = operand(sa, &ca, &ka);
      tm.b = 255;
      if (sb >= 0) tm.b = operand(sb, &cb, &kb);
      if (!ca && !cb) continue;   // constant given the selected output entry
      const bool any_lo = (ca && ka < 8) || (cb && kb < 8);
      const bool any_hi = (ca && ka >= 8) || (cb && kb >= 8);
      (any_lo && any_hi ? cross : (any_hi ? hi : lo)).push_back(tm);
    }
    if (lo.size() + hi.size() + cross.size() > 1024) return "too many energy terms in one pass";
    d.term_begin = (int)out.terms.size();
    d.n_lo = (int)lo.size();
    d.n_hi = (int)hi.size();
    d.n_cross = (int)cross.size();
    out.terms.insert(out.terms.end(), lo.begin(), lo.end());
    out.terms.insert(out.terms.end(), hi.begin(), hi.end());
    out.terms.insert(out.terms.end(), cross.begin(), cross.end());
    out.passes.push_back(d);
  }
  // backward chunks, from the last pass down
  for (int hi = np - 1; hi >= 0;) {
    int lo = hi, nc = 0, nt = 0;
    while (lo >= 0) {
      const DevPass2& d = out.passes[lo];
      const int c = d.n_cand, t = d.n_lo + d.n_hi + d.n_cross;
      if (hi - lo + 1 > BCH_PASSES || nc + c > BCH_CANDS || nt + t > BCH_TERMS) break;
      nc += c;
      nt += t;
      --lo;
    }
    ++lo;
    if (lo > hi) return "internal: a pass's backward data exceeds the LDS chunk";
    BChunk ch;
    ch.p_lo = lo;
    ch.p_hi = hi;
    ch.cand_begin = out.passes[lo].cand_begin;
    ch.n_cand = nc;
    ch.term_begin = out.passes[lo].term_begin;
    ch.n_term = nt;
    out.chunks.push_back(ch);
    hi = lo - 1;
  }
  // a record past the last pass's ops: every lane of the pass kernel reads a
  // valid record (lanes beyond a pass's ops read one and ignore it)
  FOp pad;
  std::memset(&pad, 0, sizeof(pad));
  pad.hspin = -1;
  out.fops.push_back(pad);
  return "";
}

}  // namespace tt

// C-ABI entry points of libtt.so (declared in include/tt.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "../../include/tt.h"
#include "device.hpp"
#include "encode.hpp"
#include "launch.hpp"
#include "plan.hpp"

using namespace tt;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      return fail(TT_E_DEVICE, "%s failed: %s (%d)", #expr, hipGetErrorString(_e), (int)_e); \
  } while (0)

// ----------------------------------------------------------------------------
// kernel timing (tt_prof_*)
// ----------------------------------------------------------------------------
struct ProfRec {
  std::string name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
std::vector<hipEvent_t> g_event_pool;
std::map<std::string, std::pair<double, int64_t>> g_prof_acc;

hipEvent_t pool_get() {
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct ProfScope {
  hipStream_t s;
  const char* name;
  hipEvent_t a = nullptr, b = nullptr;
  bool on;
  ProfScope(hipStream_t s_, const char* n) : s(s_), name(n), on(g_prof_on) {
    if (!on) return;
    a = pool_get();
    b = pool_get();
    on = a && b && hipEventRecord(a, s) == hipSuccess;
  }
  ~ProfScope() {
    if (!on) return;
    if (hipEventRecord(b, s) != hipSuccess) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_pending.push_back({name, a, b});
  }
};

void prof_drain() {
  std::lock_guard<std::mutex> g(g_prof_mu);
  for (auto& r : g_prof_pending) {
    float ms = 0;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) ms = 0;
    auto& acc = g_prof_acc[r.name];
    acc.first += ms;
    acc.second += 1;
    g_event_pool.push_back(r.a);
    g_event_pool.push_back(r.b);
  }
  g_prof_pending.clear();
}

// ----------------------------------------------------------------------------
// device-side cache of a plan
// ----------------------------------------------------------------------------
struct Encoded {
  std::vector<DevPass> passes;
  std::vector<DevOp> ops;
  int max_t = 0, max_dec = 0;
};

struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  int ensure(size_t bytes) {
    if (bytes <= cap) return 0;
    if (p) {
      (void)hipFree(p);
      p = nullptr;
      cap = 0;
    }
    hipError_t e = hipMalloc(&p, bytes == 0 ? 1 : bytes);
    if (e != hipSuccess) return fail(TT_E_DEVICE, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    cap = bytes;
    return 0;
  }
};

struct DevCache {
  int device = -1;
  EnergyProgram ep;
  Encoded cen;
  DevBuf d_passes, d_stages, d_fops, d_cands, d_terms, d_final_pos, d_final_slot, d_edges;
  DevBuf d_cops;
  DevBuf state, ckpt, ckpt_ptrs, part_v, part_i, arg;
  DevBuf cx, cn, cpart;
  std::vector<float*> h_ckpt_ptrs, uploaded_ckpt_ptrs;
};

int encode(const Plan& p, const std::vector<Pass>& passes, Encoded& en) {
  en.passes.clear();
  en.ops.clear();
  en.max_t = 0;
  en.max_dec = 0;
  for (const Pass& ps : passes) {
    DevPass d;
    std::memset(&d, 0, sizeof(d));
    d.in_w = ps.in_w;
    d.out_w = ps.out_w;
    d.w_max = ps.w_max;
    d.t = ps.t;
    d.op_begin = (int32_t)en.ops.size();
    d.n_ops = ps.op_end - ps.op_begin;
    d.n_dec = ps.n_dec;
    d.init = ps.init ? 1 : 0;
    d.reg = ps.reg;
    d.merge_src = ps.merge_src;
    if (ps.t > 16 || (int)ps.R.size() != ps.t) return fail(TT_E_INVAL, "internal: bad tile");
    int tbit[64];
    for (int s = 0; s < 64; ++s) tbit[s] = -1;
    for (int k = 0; k < ps.t; ++k) {
      d.R[k] = (uint8_t)ps.R[k];
      tbit[ps.R[k]] = k;
    }
    int nf = 0;
    for (int s = 0; s < ps.w_max; ++s) {
      if (tbit[s] >= 0) continue;
      if (nf >= 48) return fail(TT_E_TOOBIG, "state wider than 64 bits");
      d.fre[nf++] = (uint8_t)s;
    }
    d.n_free = nf;
    if (ps.w_max > 60) return fail(TT_E_TOOBIG, "state width %d exceeds the 60-bit index", ps.w_max);
    auto enc = [&](int slot) -> uint8_t {
      if (slot < 0) return 0;
      return tbit[slot] >= 0 ? (uint8_t)tbit[slot] : (uint8_t)(SLOT_FIXED + slot);
    };
    int dec = 0;
    for (int o = ps.op_begin; o < ps.op_end; ++o) {
      const SweepOp& op = p.ops[o];
      DevOp x;
      std::memset(&x, 0, sizeof(x));
      x.kind = op.kind;
      x.a = enc(op.slot_a);
      x.b = enc(op.slot_b);
      x.param = op.param;
      if (op.kind == OP_GATE || op.kind == OP_CUT || op.kind == OP_GATE4) {
        if (op.kind != OP_GATE4 && tbit[op.slot_a] < 0) return fail(TT_E_INVAL, "internal: gate slot not resident");
        x.dec = (uint8_t)dec++;
      }
      if (op.kind == OP_GATE4)
        for (int k = 0; k < 4; ++k) {
          if (tbit[op.slots4[k]] < 0) return fail(TT_E_INVAL, "internal: group slot not resident");
          x.g4[k] = (uint8_t)tbit[op.slots4[k]];
        }
      en.ops.push_back(x);
    }
    en.max_t = std::max(en.max_t, ps.t);
    en.max_dec = std::max(en.max_dec, ps.n_dec);
    en.passes.push_back(d);
  }
  return 0;
}

template <typename T>
int upload(DevBuf& b, const std::vector<T>& v) {
  const size_t bytes = v.size() * sizeof(T);
  if (int r = b.ensure(bytes)) return r;
  if (bytes) HIP_TRY(hipMemcpy(b.p, v.data(), bytes, hipMemcpyHostToDevice));
  return 0;
}

int ensure_device(Plan& p, DevCache*& dc) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  dc = static_cast<DevCache*>(p.dev);
  if (dc && dc->device == dev) return 0;
  if (dc) {
    delete dc;
    p.dev = nullptr;
  }
  dc = new (std::nothrow) DevCache();
  if (!dc) return fail(TT_E_NOMEM, "out of host memory");
  p.dev = dc;
  dc->device = dev;
  {
    const std::string err = encode_energy(p, p.passes, dc->ep);
    if (!err.empty()) return fail(TT_E_INVAL, "%s", err.c_str());
  }
  if (int r = encode(p, p.count_passes, dc->cen)) return r;
  if (int r = upload(dc->d_passes, dc->ep.passes)) return r;
  if (int r = upload(dc->d_stages, dc->ep.stages)) return r;
  if (int r = upload(dc->d_fops, dc->ep.fops)) return r;
  if (int r = upload(dc->d_cands, dc->ep.cands)) return r;
  if (int r = upload(dc->d_terms, dc->ep.terms)) return r;
  if (int r = upload(dc->d_final_pos, dc->ep.final_pos)) return r;
  if (int r = upload(dc->d_final_slot, p.final_slot_spin)) return r;
  if (int r = upload(dc->d_edges, p.edges)) return r;
  if (int r = upload(dc->d_cops, dc->cen.ops)) return r;
  return 0;
}

int64_t budget_bytes(const Plan& p) {
  if (p.max_bytes > 0) return p.max_bytes;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return INT64_MAX;
  return (int64_t)(fr / 8 * 7);
}

int check_common(tt_plan* plan, int32_t batch, int32_t dtype, const void* J, const void* h) {
  if (!plan) return fail(TT_E_INVAL, "null plan");
  const Plan& p = *reinterpret_cast<Plan*>(plan);
  if (batch < 1) return fail(TT_E_INVAL, "batch must be >= 1");
  if (dtype != TT_F32 && dtype != TT_I32) return fail(TT_E_DTYPE, "unknown dtype %d", dtype);
  if (p.m > 0 && !J) return fail(TT_E_INVAL, "null J");
  if (p.has_field && !h) return fail(TT_E_INVAL, "plan has fields but h is NULL");
  if (!p.has_field && h) return fail(TT_E_INVAL, "plan has no fields but h is given");
  return 0;
}

// A count pass may overwrite its input when every tile reads exactly the
// entries it writes: no width change (or no read at all).
bool in_place_ok(const DevPass& P) { return P.init || (P.in_w == P.w_max && P.out_w == P.w_max); }

// Runs the energy passes. Every pass writes a buffer other than its input
// (the bit order changes between passes); keep_all gives every pass a fresh
// buffer so that each pass input stays available for the backward walk.
int run_forward(Plan& p, DevCache* dc, int32_t batch, int32_t dtype, const void* J, const void* h,
                bool keep_all, hipStream_t s, float** final_state) {
  const int64_t sst = (int64_t)1 << p.width;
  const size_t per = (size_t)batch * (size_t)sst * sizeof(float);
  const int np = (int)dc->ep.passes.size();
  if (np == 0) return fail(TT_E_INVAL, "empty plan");
  const size_t nbuf = keep_all ? (size_t)np + 1 : 2;
  const int64_t need = (int64_t)(per * nbuf);
  DevBuf& buf = keep_all ? dc->ckpt : dc->state;
  if (need > (int64_t)buf.cap && need > budget_bytes(p) + (int64_t)buf.cap)
    return fail(TT_E_TOOBIG, "plan needs %lld bytes of device state (budget %lld)", (long long)need,
                (long long)budget_bytes(p));
  if (int r = buf.ensure(per * nbuf)) return r;
  char* base = static_cast<char*>(buf.p);
  auto bufp = [&](size_t k) { return reinterpret_cast<float*>(base + per * k); };
  const int64_t jst = p.m, hst = p.n;
  int cur = 0;
  if (keep_all) dc->h_ckpt_ptrs.assign(np, nullptr);
  for (int q = 0; q < np; ++q) {
    const DevPass2& P = dc->ep.passes[q];
    const int src = keep_all ? q : cur;
    const int dst = keep_all ? q + 1 : (cur ^ 1);
    if (keep_all) dc->h_ckpt_ptrs[q] = P.init ? nullptr : bufp(src);
    ProfScope ps(s, "sweep_pass");
    HIP_TRY(launch_pass(P, static_cast<const DevPass2*>(dc->d_passes.p) + q, static_cast<const DevStage*>(dc->d_stages.p),
                        static_cast<const FOp*>(dc->d_fops.p), dtype, J, h, jst, hst, bufp(src), bufp(dst), sst, batch,
                        s));
    cur = dst;
  }
  *final_state = bufp(keep_all ? np : cur);
  return 0;
}

int run_reduce(Plan& p, DevCache* dc, int32_t batch, const float* st, double* energy, uint64_t* arg,
               hipStream_t s) {
  const int lc = reduce_log2_chunks(p.final_w);
  const size_t nparts = (size_t)batch << lc;
  if (int r = dc->part_v.ensure(nparts * sizeof(float))) return r;
  if (int r = dc->part_i.ensure(nparts * sizeof(uint64_t))) return r;
  ProfScope ps(s, "final_reduce");
  HIP_TRY(launch_reduce(st, (int64_t)1 << p.width, p.final_w, batch, static_cast<float*>(dc->part_v.p),
                        static_cast<uint64_t*>(dc->part_i.p), energy, arg, s));
  return 0;
}

}  // namespace

// ============================================================================
// C-ABI
// ============================================================================
extern "C" {

const char* tt_last_error(void) { return g_err.c_str(); }

int tt_plan_create(int32_t n_spins, int64_t n_edges, const int32_t* edges, const tt_plan_opts* opts,
                   tt_plan** out) {
  try {
    if (!out) return fail(TT_E_INVAL, "null output pointer");
    *out = nullptr;
    if (n_spins < 1 || n_spins > 8192) return fail(TT_E_INVAL, "n_spins must be in [1, 8192]");
    if (n_edges < 0 || (n_edges > 0 && !edges)) return fail(TT_E_INVAL, "bad edge list");
    tt_plan_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    std::set<std::pair<int, int>> seen;
    for (int64_t k = 0; k < n_edges; ++k) {
      const int a = edges[2 * k], b = edges[2 * k + 1];
      if (a < 0 || b >= n_spins || a >= b) return fail(TT_E_INVAL, "edge %lld = (%d, %d) needs 0 <= i < j < n", (long long)k, a, b);
      if (!seen.insert({a, b}).second) return fail(TT_E_INVAL, "duplicate edge (%d, %d)", a, b);
    }
    std::unique_ptr<Plan> p(new Plan());
    p->n = n_spins;
    p->m = n_edges;
    p->edges.assign(edges, edges + 2 * n_edges);
    p->has_field = o.has_field != 0;
    p->tile_bits = o.tile_bits > 0 ? o.tile_bits : 14;
    p->count_tile_bits = o.count_tile_bits > 0 ? o.count_tile_bits : 12;
    if (p->tile_bits < 7 || p->tile_bits > 14) return fail(TT_E_INVAL, "tile_bits must be in [7, 14]");
    if (p->count_tile_bits < 7 || p->count_tile_bits > 12) return fail(TT_E_INVAL, "count_tile_bits must be in [7, 12]");
    p->max_bytes = o.max_bytes;
    std::string err;
    if (o.kind == TT_ORDER_GIVEN) {
      if (!o.order) return fail(TT_E_INVAL, "TT_ORDER_GIVEN needs opts.order");
      p->order.assign(o.order, o.order + n_spins);
      err = build_sweep_ops(*p);
    } else if (o.kind == TT_ORDER_GREEDY) {
      p->order = greedy_order(n_spins, p->edges, o.seed, o.trials > 0 ? o.trials : 32);
      err = build_sweep_ops(*p);
    } else if (o.kind == TT_ORDER_CHIMERA) {
      err = build_chimera_ops(*p, o.chimera_rows, o.chimera_cols);
    } else {
      return fail(TT_E_INVAL, "unknown order kind %d", o.kind);
    }
    if (!err.empty()) return fail(TT_E_INVAL, "%s", err.c_str());
    if (p->width > 40) return fail(TT_E_TOOBIG, "plan width %d exceeds 40 bits", p->width);
    p->max_dec = 16;
    p->passes = partition_passes(*p, p->tile_bits, p->max_dec, false, 0);
    p->count_passes = partition_passes(*p, p->count_tile_bits, 1 << 20, false, 6);
    *out = reinterpret_cast<tt_plan*>(p.release());
    return TT_OK;
  } catch (const std::bad_alloc&) {
    return fail(TT_E_NOMEM, "out of host memory");
  } catch (...) {
    return fail(TT_E_INVAL, "planner failed");
  }
}

int tt_plan_info(const tt_plan* plan, tt_plan_stats* out) {
  if (!plan || !out) return fail(TT_E_INVAL, "null argument");
  const Plan& p = *reinterpret_cast<const Plan*>(plan);
  std::memset(out, 0, sizeof(*out));
  out->n_spins = p.n;
  out->n_edges = p.m;
  out->width = p.width;
  out->n_ops = (int32_t)p.ops.size();
  out->n_passes = (int32_t)p.passes.size();
  out->n_count_passes = (int32_t)p.count_passes.size();
  out->terms = p.terms;
  out->reduce_terms = p.reduce_terms;
  double upd = 0;
  for (const Pass& ps : p.passes) upd += 2.0 * std::ldexp(1.0, ps.w_max);
  out->entry_updates = upd;
  return TT_OK;
}

int tt_plan_order(const tt_plan* plan, int32_t* order_out) {
  if (!plan || !order_out) return fail(TT_E_INVAL, "null argument");
  const Plan& p = *reinterpret_cast<const Plan*>(plan);
  std::copy(p.order.begin(), p.order.end(), order_out);
  return TT_OK;
}

int tt_plan_ops(const tt_plan* plan, int32_t* out, int64_t cap, int32_t* final_slot_spin, int32_t* final_width) {
  if (!plan) return fail(TT_E_INVAL, "null plan");
  const Plan& p = *reinterpret_cast<const Plan*>(plan);
  const int64_t n = (int64_t)p.ops.size();
  for (int64_t k = 0; k < n && k < cap && out; ++k) {
    const SweepOp& o = p.ops[k];
    int32_t* r = out + 8 * k;
    r[0] = o.kind;
    r[1] = o.slot_a;
    r[2] = o.slot_b;
    r[3] = o.param;
    r[4] = o.old_spin;
    r[5] = o.new_spin;
    r[6] = o.w_before;
    r[7] = o.w_after;
  }
  if (final_width) *final_width = p.final_w;
  if (final_slot_spin) std::copy(p.final_slot_spin.begin(), p.final_slot_spin.end(), final_slot_spin);
  return (int)n;
}

int64_t tt_plan_program(const tt_plan* plan, int32_t which, void* out, int64_t cap) {
  if (!plan) return fail(TT_E_INVAL, "null plan");
  const Plan& p = *reinterpret_cast<const Plan*>(plan);
  EnergyProgram ep;
  const std::string err = encode_energy(p, p.passes, ep);
  if (!err.empty()) return fail(TT_E_INVAL, "%s", err.c_str());
  const void* src = nullptr;
  int64_t bytes = 0;
  switch (which) {
    case 0: src = ep.passes.data(); bytes = (int64_t)(ep.passes.size() * sizeof(DevPass2)); break;
    case 1: src = ep.stages.data(); bytes = (int64_t)(ep.stages.size() * sizeof(DevStage)); break;
    case 2: src = ep.fops.data(); bytes = (int64_t)(ep.fops.size() * sizeof(FOp)); break;
    case 3: src = ep.cands.data(); bytes = (int64_t)(ep.cands.size() * sizeof(BCand)); break;
    case 4: src = ep.terms.data(); bytes = (int64_t)(ep.terms.size() * sizeof(BTerm)); break;
    case 5: src = ep.final_pos.data(); bytes = (int64_t)ep.final_pos.size(); break;
    default: return fail(TT_E_INVAL, "unknown program part %d", which);
  }
  if (out && bytes) std::memcpy(out, src, (size_t)std::min(bytes, cap));
  return bytes;
}

void tt_plan_destroy(tt_plan* plan) {
  if (!plan) return;
  Plan* p = reinterpret_cast<Plan*>(plan);
  delete static_cast<DevCache*>(p->dev);
  delete p;
}

int tt_contract(tt_plan* plan, int32_t batch, int32_t dtype, const void* J, const void* h, double* energy,
                void* stream) {
  try {
    if (int r = check_common(plan, batch, dtype, J, h)) return r;
    if (!energy) return fail(TT_E_INVAL, "null energy");
    Plan& p = *reinterpret_cast<Plan*>(plan);
    DevCache* dc = nullptr;
    if (int r = ensure_device(p, dc)) return r;
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* fin = nullptr;
    if (int r = run_forward(p, dc, batch, dtype, J, h, false, s, &fin)) return r;
    return run_reduce(p, dc, batch, fin, energy, nullptr, s);
  } catch (...) {
    return fail(TT_E_INVAL, "unexpected failure");
  }
}

int tt_backward(tt_plan* plan, int32_t batch, int32_t dtype, const void* J, const void* h, double* energy,
                int8_t* sigma, float* dJ, float* dh, void* stream) {
  try {
    if (int r = check_common(plan, batch, dtype, J, h)) return r;
    if (!sigma) return fail(TT_E_INVAL, "null sigma");
    Plan& p = *reinterpret_cast<Plan*>(plan);
    if (p.n_regs != 1) return fail(TT_E_INVAL, "backward over multi-register plans is not supported");
    if (p.n > 8192) return fail(TT_E_INVAL, "too many spins for the backward walk");
    DevCache* dc = nullptr;
    if (int r = ensure_device(p, dc)) return r;
    hipStream_t s = static_cast<hipStream_t>(stream);
    float* fin = nullptr;
    if (int r = run_forward(p, dc, batch, dtype, J, h, true, s, &fin)) return r;
    if (int r = dc->arg.ensure((size_t)batch * sizeof(uint64_t))) return r;
    uint64_t* arg = static_cast<uint64_t*>(dc->arg.p);
    if (int r = run_reduce(p, dc, batch, fin, energy, arg, s)) return r;
    const int np = (int)dc->ep.passes.size();
    if (dc->h_ckpt_ptrs != dc->uploaded_ckpt_ptrs || dc->ckpt_ptrs.cap < np * sizeof(float*)) {
      if (int r = dc->ckpt_ptrs.ensure(np * sizeof(float*))) return r;
      HIP_TRY(hipStreamSynchronize(s));
      HIP_TRY(hipMemcpy(dc->ckpt_ptrs.p, dc->h_ckpt_ptrs.data(), np * sizeof(float*), hipMemcpyHostToDevice));
      dc->uploaded_ckpt_ptrs = dc->h_ckpt_ptrs;
    }
    {
      ProfScope ps(s, "sweep_backward");
      HIP_TRY(launch_backward(static_cast<const DevPass2*>(dc->d_passes.p), np,
                              static_cast<const BCand*>(dc->d_cands.p), static_cast<const BTerm*>(dc->d_terms.p),
                              dtype, J, h, p.m, p.n, static_cast<const float* const*>(dc->ckpt_ptrs.p),
                              (int64_t)1 << p.width, arg, static_cast<const uint8_t*>(dc->d_final_pos.p),
                              static_cast<const int32_t*>(dc->d_final_slot.p), p.final_w,
                              static_cast<const int32_t*>(dc->d_edges.p), p.n, p.m, sigma, dJ, dh, batch, s));
    }
    return TT_OK;
  } catch (...) {
    return fail(TT_E_INVAL, "unexpected failure");
  }
}

int tt_count_moduli(uint64_t moduli_out[3]) {
  if (!moduli_out) return fail(TT_E_INVAL, "null argument");
  moduli_out[0] = (1ull << 61) - 1;
  moduli_out[1] = (1ull << 61) - 31;
  moduli_out[2] = (1ull << 61) - 45;
  return TT_OK;
}

int tt_count(tt_plan* plan, int32_t batch, const int32_t* J, const int32_t* h, int64_t* energy, uint64_t* residues,
             void* stream) {
  try {
    if (int r = check_common(plan, batch, TT_I32, J, h)) return r;
    if (!energy || !residues) return fail(TT_E_INVAL, "null output");
    Plan& p = *reinterpret_cast<Plan*>(plan);
    if (p.n_regs != 1) return fail(TT_E_INVAL, "counting over multi-register plans is not supported");
    hipStream_t s = static_cast<hipStream_t>(stream);
    // exactness guard: every state value lies in [-S, S], S = sum|J| + sum|h|,
    // which float32 holds exactly below 2^24
    {
      std::vector<int32_t> hj((size_t)batch * p.m), hh(p.has_field ? (size_t)batch * p.n : 0);
      if (p.m) HIP_TRY(hipMemcpyAsync(hj.data(), J, hj.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      if (!hh.empty()) HIP_TRY(hipMemcpyAsync(hh.data(), h, hh.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      for (int b = 0; b < batch; ++b) {
        int64_t S = 0;
        for (int64_t e = 0; e < p.m; ++e) S += std::llabs((long long)hj[(size_t)b * p.m + e]);
        if (!hh.empty())
          for (int v = 0; v < p.n; ++v) S += std::llabs((long long)hh[(size_t)b * p.n + v]);
        if (S >= (1ll << 24)) return fail(TT_E_RANGE, "instance %d: sum|J|+sum|h| = %lld needs more than 24 bits", b, (long long)S);
      }
    }
    DevCache* dc = nullptr;
    if (int r = ensure_device(p, dc)) return r;
    const int64_t sst = (int64_t)1 << p.width;
    const size_t xper = (size_t)batch * sst * sizeof(float);
    const size_t nper = (size_t)batch * sst * 3 * sizeof(uint64_t);
    bool all_in_place = true;
    for (const DevPass& P : dc->cen.passes) all_in_place = all_in_place && in_place_ok(P);
    const int nb2 = all_in_place ? 1 : 2;
    const int64_t need = (int64_t)(nb2 * (xper + nper));
    if (need > (int64_t)(dc->cx.cap + dc->cn.cap) && need > budget_bytes(p) + (int64_t)(dc->cx.cap + dc->cn.cap))
      return fail(TT_E_TOOBIG, "count path needs %lld bytes of device state (budget %lld)", (long long)need,
                  (long long)budget_bytes(p));
    if (int r = dc->cx.ensure(nb2 * xper)) return r;
    if (int r = dc->cn.ensure(nb2 * nper)) return r;
    float* xb[2] = {static_cast<float*>(dc->cx.p),
                    reinterpret_cast<float*>(static_cast<char*>(dc->cx.p) + (nb2 - 1) * xper)};
    uint64_t* nb[2] = {static_cast<uint64_t*>(dc->cn.p),
                       reinterpret_cast<uint64_t*>(static_cast<char*>(dc->cn.p) + (nb2 - 1) * nper)};
    int cur = 0;
    for (const DevPass& P : dc->cen.passes) {
      ProfScope ps(s, "count_pass");
      const int dst = in_place_ok(P) ? cur : (cur ^ 1);
      HIP_TRY(launch_count_pass(P, static_cast<const DevOp*>(dc->d_cops.p), J, h, p.m, p.n, xb[cur], nb[cur],
                                xb[dst], nb[dst], sst, batch, s));
      cur = dst;
    }
    const int lc = count_reduce_log2_chunks(p.final_w);
    const size_t nparts = (size_t)batch << lc;
    const size_t bytes = nparts * sizeof(float) + nparts * 3 * sizeof(uint64_t) + (size_t)batch * 4 * sizeof(uint64_t) + 64;
    if (int r = dc->cpart.ensure(bytes)) return r;
    char* c = static_cast<char*>(dc->cpart.p);
    uint64_t* pn = reinterpret_cast<uint64_t*>(c);
    uint64_t* res = pn + nparts * 3;
    int64_t* en = reinterpret_cast<int64_t*>(res + (size_t)batch * 3);
    float* pv = reinterpret_cast<float*>(en + batch);
    {
      ProfScope ps(s, "count_reduce");
      uint64_t free_mask = 0;
      for (int c = 0; c < p.final_w; ++c)
        if (p.final_slot_spin[c] < 0) free_mask |= 1ull << c;
      HIP_TRY(launch_count_reduce(xb[cur], nb[cur], sst, p.final_w, free_mask, batch, pv, pn, en, res, s));
    }
    HIP_TRY(hipMemcpyAsync(energy, en, (size_t)batch * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(residues, res, (size_t)batch * 3 * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return TT_OK;
  } catch (...) {
    return fail(TT_E_INVAL, "unexpected failure");
  }
}

int tt_count_to_decimal(const uint64_t residues[3], char* buf, size_t len) {
  if (!residues || !buf || len == 0) return fail(TT_E_INVAL, "null argument");
  typedef unsigned __int128 u128;
  uint64_t P[3];
  tt_count_moduli(P);
  for (int r = 0; r < 3; ++r)
    if (residues[r] >= P[r]) return fail(TT_E_INVAL, "residue %d out of range", r);
  auto mulmod = [](uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); };
  auto powmod = [&](uint64_t a, uint64_t e, uint64_t m) {
    uint64_t r = 1 % m;
    a %= m;
    while (e) {
      if (e & 1) r = mulmod(r, a, m);
      a = mulmod(a, a, m);
      e >>= 1;
    }
    return r;
  };
  // Garner: g = a0 + a1 P0 + a2 P0 P1 with 0 <= a_r < P_r
  const uint64_t a0 = residues[0];
  const uint64_t inv01 = powmod(P[0] % P[1], P[1] - 2, P[1]);
  const uint64_t a1 = mulmod((residues[1] + P[1] - a0 % P[1]) % P[1], inv01, P[1]);
  const uint64_t p01 = mulmod(P[0] % P[2], P[1] % P[2], P[2]);
  const uint64_t partial = (a0 % P[2] + mulmod(a1 % P[2], P[0] % P[2], P[2])) % P[2];
  const uint64_t inv012 = powmod(p01, P[2] - 2, P[2]);
  const uint64_t a2 = mulmod((residues[2] + P[2] - partial) % P[2], inv012, P[2]);
  // big integer in 32-bit limbs, little endian
  std::vector<uint32_t> x(8, 0);
  auto add_small = [&](std::vector<uint32_t>& v, uint64_t a) {
    uint64_t carry = a;
    for (size_t k = 0; k < v.size() && carry; ++k) {
      const uint64_t s = (uint64_t)v[k] + (carry & 0xffffffffull);
      v[k] = (uint32_t)s;
      carry = (carry >> 32) + (s >> 32);
    }
  };
  auto mul_small = [&](std::vector<uint32_t>& v, uint64_t a) {
    // v *= a with a < 2^64 in two 32-bit halves
    std::vector<uint32_t> out(v.size(), 0);
    const uint64_t h[2] = {a & 0xffffffffull, a >> 32};
    for (int part = 0; part < 2; ++part) {
      uint64_t carry = 0;
      for (size_t k = 0; k + part < v.size(); ++k) {
        const uint64_t s = (uint64_t)v[k] * h[part] + out[k + part] + carry;
        out[k + part] = (uint32_t)s;
        carry = s >> 32;
      }
    }
    v.swap(out);
  };
  // g = a0 + P0 (a1 + P1 a2)
  add_small(x, a2);
  mul_small(x, P[1]);
  add_small(x, a1);
  mul_small(x, P[0]);
  add_small(x, a0);
  std::string digits;
  bool zero = false;
  while (!zero) {
    uint64_t rem = 0;
    zero = true;
    for (size_t k = x.size(); k-- > 0;) {
      const uint64_t cur = (rem << 32) | x[k];
      x[k] = (uint32_t)(cur / 10);
      rem = cur % 10;
      if (x[k]) zero = false;
    }
    digits.push_back((char)('0' + rem));
  }
  std::reverse(digits.begin(), digits.end());
  if (digits.size() + 1 > len) return fail(TT_E_INVAL, "buffer too small (%zu digits)", digits.size());
  std::memcpy(buf, digits.c_str(), digits.size() + 1);
  return TT_OK;
}

int tt_contract_uneven(int32_t n_inst, tt_plan* const* plans, int32_t dtype, const void* J, const int64_t* j_off,
                       double* energy, int8_t* sigma, const int64_t* s_off, float* dJ, void* stream) {
  if (n_inst < 1 || !plans || !j_off || !energy) return fail(TT_E_INVAL, "bad uneven-batch arguments");
  if (sigma && !s_off) return fail(TT_E_INVAL, "sigma needs s_off");
  const size_t esz = dtype == TT_F32 ? sizeof(float) : sizeof(int32_t);
  for (int i = 0; i < n_inst; ++i) {
    const void* Ji = static_cast<const char*>(J) + (size_t)j_off[i] * esz;
    int r;
    if (sigma)
      r = tt_backward(plans[i], 1, dtype, Ji, nullptr, energy + i, sigma + s_off[i], dJ ? dJ + j_off[i] : nullptr,
                      nullptr, stream);
    else
      r = tt_contract(plans[i], 1, dtype, Ji, nullptr, energy + i, stream);
    if (r) return r;
  }
  return TT_OK;
}

int tt_prof_enable(int32_t on) {
  g_prof_on = on != 0;
  return TT_OK;
}

int tt_prof_reset(void) {
  prof_drain();
  std::lock_guard<std::mutex> g(g_prof_mu);
  g_prof_acc.clear();
  return TT_OK;
}

int tt_prof_read(const char* name, double* total_ms, int64_t* launches) {
  if (!name || !total_ms || !launches) return fail(TT_E_INVAL, "null argument");
  prof_drain();
  std::lock_guard<std::mutex> g(g_prof_mu);
  auto it = g_prof_acc.find(name);
  *total_ms = it == g_prof_acc.end() ? 0.0 : it->second.first;
  *launches = it == g_prof_acc.end() ? 0 : it->second.second;
  return TT_OK;
}

}  // extern "C"

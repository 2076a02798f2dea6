// Host runtime of libtmc: validation, plans (workspace layout, level schedules,
// device descriptor tables), dispatch to the engines, graphs and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/tmc.h"
#include "fused.h"
#include "tmc_internal.h"
#include "tmc_kernels.h"
#include "tmc_scratch.h"
#include "tmc_logmm.h"
#include "tmc_star.h"

using namespace tmc;

static_assert(kNoallocWorkspaceBytes == TMC_NOALLOC_WORKSPACE_MAX,
              "static workspace size and its ABI constant");

namespace {

thread_local std::string g_err;

tmc_status fail(tmc_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(TMC_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

struct Launch {
  int off = 0, n = 0;
};

// Sets the plan's device for the duration of a call and restores the caller's.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Star-model plan: shape, point grouping and workspace offsets (bytes).
struct StarPlan {
  int S = 0, N = 0, Kt = 0, K = 0, D = 0;
  int P = 1, ngrp = 0, nkb = 0;
  size_t msg = 0, gsum = 0, w = 0, lp = 0, dm = 0, dsp = 0, nsh = 0, wT = 0;
};

constexpr int kKindChain = 0, kKindStar = 1;

}  // namespace

struct tmc_plan {
  int kind = kKindChain;   // chain problem (tmc_plan_create) or star (tmc_star_plan_create)
  StarPlan star;
  int device = 0;
  int prec = TMC_FP32;
  int engine = TMC_ENGINE_PLAIN;
  int flags = 0;
  int n_chains = 0, n_layers = 0, max_depth = 0;
  int64_t entries = 0;
  size_t esz = 4;
  std::vector<ChainDev> chains_h;
  std::vector<LayerDev> layers_h;
  WsLayout ws{};
  // device tables
  ChainDev* chains_d = nullptr;
  LayerDev* layers_d = nullptr;
  Item* items_d = nullptr;
  int* ints_d = nullptr;         // pair ids, slot layers, slot starts, slot D
  int64_t* slot_soff_d = nullptr;
  int64_t* part_off_d = nullptr;    // ds partial rows grouped by s block
  int max_D = 0;
  int* flag_d = nullptr;
  // schedules (offsets into items_d)
  Launch factor;                              // all pairs, factor tiles
  std::vector<Launch> fwd, bwd_vec, bwd_sca;  // per depth step
  std::vector<int> fwd_maxkc;
  std::vector<char> fwd_vec_ws, fwd_vec_caller;   // plain forward: vector loads allowed
  Launch gmu, gtz;
  int n_pairs = 0, pair_ids_off = 0;
  int n_slots = 0, slot_layers_off = 0, slot_start_off = 0, slot_D_off = 0;
  // fused engine
  FusedPlan fused;
  // problems that make one family of entry points unusable (empty = usable)
  std::string gauss_err, logf_err;
  // address of the library's static device workspace on this plan's device (set up at
  // plan creation; null with the reason in scratch_err if it could not be found)
  void* scratch = nullptr;
  std::string scratch_err;
  // graphs
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  bool capturing = false;
  // optional per-launch event timing
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, size_t>> ev_marks;   // (kernel class, index of start event)
  double kc_ms[TMC_KC_COUNT] = {0};
  int64_t kc_n[TMC_KC_COUNT] = {0};
  ~tmc_plan() {
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    for (auto& g : graph)
      if (g) (void)hipGraphExecDestroy(g);
    if (chains_d) (void)hipFree(chains_d);
    if (layers_d) (void)hipFree(layers_d);
    if (items_d) (void)hipFree(items_d);
    if (ints_d) (void)hipFree(ints_d);
    if (slot_soff_d) (void)hipFree(slot_soff_d);
    if (part_off_d) (void)hipFree(part_off_d);
    if (flag_d) (void)hipFree(flag_d);
  }
};

namespace {

struct Range {
  int64_t b, e;
  int who;
};

// Disjointness of [b, e) ranges; returns index pair of an overlap or -1.
bool find_overlap(std::vector<Range>& r, int* a, int* b) {
  std::sort(r.begin(), r.end(), [](const Range& x, const Range& y) {
    return x.b < y.b || (x.b == y.b && x.e < y.e);
  });
  for (size_t i = 1; i < r.size(); ++i)
    if (r[i].b < r[i - 1].e) {
      *a = r[i - 1].who;
      *b = r[i].who;
      return true;
    }
  return false;
}

tmc_status validate(const tmc_problem* pr, int* engine_out, std::string* gauss_err,
                    std::string* logf_err) {
  if (!pr) return fail(TMC_ERR_INVALID_ARG, "problem is NULL");
  if (pr->n_chains < 0 || pr->n_layers < 0)
    return fail(TMC_ERR_INVALID_ARG, "negative n_chains or n_layers");
  if ((pr->n_chains > 0 && !pr->chains) || (pr->n_layers > 0 && !pr->layers))
    return fail(TMC_ERR_INVALID_ARG, "chains or layers array is NULL");
  if (pr->reserved != 0) return fail(TMC_ERR_INVALID_ARG, "reserved field must be 0");
  if (!(pr->exponent == 0.0 || (std::isfinite(pr->exponent) && pr->exponent > 0.0)))
    return fail(TMC_ERR_INVALID_ARG, "exponent must be 0 (meaning 1) or finite and > 0");
  if (pr->precision < TMC_FP64 || pr->precision > TMC_BF16X3)
    return fail(TMC_ERR_INVALID_ARG, "unknown precision %d", pr->precision);
  if (pr->engine < TMC_ENGINE_AUTO || pr->engine > TMC_ENGINE_PLAIN)
    return fail(TMC_ERR_INVALID_ARG, "unknown engine %d", pr->engine);
  if (pr->flags & ~(TMC_FLAG_FORWARD_ONLY | TMC_FLAG_PERSISTENT | TMC_FLAG_PARENT_SCALE))
    return fail(TMC_ERR_INVALID_ARG, "unknown flag bits 0x%x", pr->flags);
  const bool pp = (pr->flags & TMC_FLAG_PARENT_SCALE) != 0;
  int engine = pr->engine;
  if (engine == TMC_ENGINE_AUTO)
    engine = (pr->precision == TMC_FP64 || pp || !kFusedAvailable) ? TMC_ENGINE_PLAIN
                                                                   : TMC_ENGINE_FUSED;
  if (engine == TMC_ENGINE_FUSED && pp)
    return fail(TMC_ERR_UNSUPPORTED, "parent-dependent scales run on the plain engine");
  if (engine == TMC_ENGINE_PLAIN && pr->precision == TMC_BF16X3)
    return fail(TMC_ERR_UNSUPPORTED, "the plain engine has no BF16X3 mode");
  if (engine == TMC_ENGINE_FUSED && pr->precision == TMC_FP64)
    return fail(TMC_ERR_UNSUPPORTED, "the fused engine has no FP64 mode; use the plain engine");
  *engine_out = engine;

  std::vector<int> owner(pr->n_layers, -1);
  for (int c = 0; c < pr->n_chains; ++c) {
    const tmc_chain& ch = pr->chains[c];
    if (ch.n_layers < 1) return fail(TMC_ERR_INVALID_ARG, "chain %d has %d layers", c, ch.n_layers);
    if (ch.first_layer < 0 || (int64_t)ch.first_layer + ch.n_layers > pr->n_layers)
      return fail(TMC_ERR_INVALID_ARG, "chain %d layer range out of bounds", c);
    for (int l = ch.first_layer; l < ch.first_layer + ch.n_layers; ++l) {
      if (owner[l] >= 0)
        return fail(TMC_ERR_INVALID_ARG, "layer %d belongs to chains %d and %d", l, owner[l], c);
      owner[l] = c;
    }
  }
  const bool plain = engine == TMC_ENGINE_PLAIN;
  const int maxK = plain ? kPlainMaxK : kFusedMaxK;
  const int maxD = plain ? kPlainMaxD : kFusedMaxD;
  std::vector<Range> rz, ru, rm, rf, rs;
  bool neg_gauss = false, neg_f = false;
  for (int c = 0; c < pr->n_chains; ++c) {
    const tmc_chain& ch = pr->chains[c];
    for (int q = 0; q < ch.n_layers; ++q) {
      const int l = ch.first_layer + q;
      const tmc_layer& L = pr->layers[l];
      const bool top = q == ch.n_layers - 1;
      if (L.K < 1 || L.K > maxK)
        return fail(TMC_ERR_SHAPE, "layer %d: K=%d outside [1, %d]", l, L.K, maxK);
      if (L.D < 1 || L.D > maxD)
        return fail(TMC_ERR_SHAPE, "layer %d: D=%d outside [1, %d]", l, L.D, maxD);
      if (L.u_off < 0) return fail(TMC_ERR_INVALID_ARG, "layer %d: negative u offset", l);
      ru.push_back({L.u_off, L.u_off + L.K, l});
      if (L.z_off < 0) neg_gauss = true;
      rz.push_back({L.z_off, L.z_off + (int64_t)L.K * L.D, l});
      if (!top) {
        const tmc_layer& U = pr->layers[l + 1];
        if (L.mu_off < 0 || L.s_off < 0) neg_gauss = true;
        if (L.f_off < 0) neg_f = true;
        rm.push_back({L.mu_off, L.mu_off + (int64_t)U.K * L.D, l});
        rf.push_back({L.f_off, L.f_off + (int64_t)L.K * U.K, l});
        rs.push_back({L.s_off, L.s_off + (pp ? (int64_t)U.K : 1) * L.D, l});
      }
    }
  }
  int a, b;
  if (find_overlap(ru, &a, &b)) return fail(TMC_ERR_INVALID_ARG, "u blocks of layers %d and %d overlap", a, b);
  // Gaussian entry points need disjoint z and mu blocks and identical-or-disjoint s
  // blocks; log-factor entry points need disjoint f blocks.  Checked here, reported
  // when the entry point that needs them is called.
  char buf[256];
  gauss_err->clear();
  logf_err->clear();
  if (neg_gauss) *gauss_err = "negative z, mu or s offset";
  else if (find_overlap(rz, &a, &b)) { snprintf(buf, sizeof buf, "z blocks of layers %d and %d overlap", a, b); *gauss_err = buf; }
  else if (find_overlap(rm, &a, &b)) { snprintf(buf, sizeof buf, "mu blocks of layers %d and %d overlap", a, b); *gauss_err = buf; }
  else {
    std::sort(rs.begin(), rs.end(), [](const Range& x, const Range& y) {
      return x.b < y.b || (x.b == y.b && x.e < y.e);
    });
    for (size_t i = 1; i < rs.size(); ++i) {
      // shared-scale blocks may be shared whole (their ds is summed); parent-dependent
      // blocks belong to one layer's parents and may not be shared at all
      const bool same = !pp && rs[i].b == rs[i - 1].b && rs[i].e == rs[i - 1].e;
      if (!same && rs[i].b < rs[i - 1].e) {
        snprintf(buf, sizeof buf, pp ? "s blocks of layers %d and %d overlap"
                                     : "s blocks of layers %d and %d partially overlap",
                 rs[i - 1].who, rs[i].who);
        *gauss_err = buf;
        break;
      }
    }
  }
  if (neg_f) *logf_err = "negative f offset";
  else if (find_overlap(rf, &a, &b)) { snprintf(buf, sizeof buf, "f blocks of layers %d and %d overlap", a, b); *logf_err = buf; }
  return TMC_OK;
}

template <typename T>
T* wsp(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// ---- launch-shape tuning cache ----
// A text file named by TMC_TUNE_CACHE holds lines "<signature> <persist> <grid factor>
// <stages> <wide forward> <wide backward>"; the last line with a plan's signature sets
// its starting launch shape.
void tune_cache_lookup(tmc_plan* P) {
  const char* path = std::getenv("TMC_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  const std::string sig = fused_signature(P->fused, P->layers_h, P->chains_h);
  char line[8192];
  while (std::fgets(line, sizeof line, f)) {
    char key[8000];
    int persist = 0, gf = 1, ns = 2, wf = 1, wb = 0;
    if (std::sscanf(line, "%7999s %d %d %d %d %d", key, &persist, &gf, &ns, &wf, &wb) == 6 &&
        sig == key) {
      P->fused.tune.persist = persist != 0;
      P->fused.tune.grid_factor = std::max(1, std::min(gf, 8));
      P->fused.tune.fwd_ns = ns == 1 ? 1 : 2;
      P->fused.tune.wide_fwd = wf != 0;
      P->fused.tune.wide_bwd = wb != 0;
      P->fused.tuned = true;
    }
  }
  std::fclose(f);
}

void tune_cache_store(const tmc_plan* P) {
  const char* path = std::getenv("TMC_TUNE_CACHE");
  if (!path || !*path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  const FusedTune& t = P->fused.tune;
  std::fprintf(f, "%s %d %d %d %d %d\n", fused_signature(P->fused, P->layers_h, P->chains_h).c_str(),
               t.persist ? 1 : 0, t.grid_factor, t.fwd_ns, t.wide_fwd ? 1 : 0, t.wide_bwd ? 1 : 0);
  std::fclose(f);
}

tmc_status build_plan(tmc_plan* P, const tmc_problem* pr) {
  P->n_chains = pr->n_chains;
  P->n_layers = pr->n_layers;
  P->esz = P->prec == TMC_FP64 ? 8 : 4;
  const size_t esz = P->esz;
  P->layers_h.assign(pr->n_layers, LayerDev{});
  P->chains_h.resize(pr->n_chains);
  int64_t sumK = 0, sum_pairKK = 0, sum_pairKcD = 0, sum_pairD = 0, sum_wmax = 0;
  P->max_depth = 0;
  P->entries = 0;
  for (int c = 0; c < pr->n_chains; ++c) {
    const tmc_chain& ch = pr->chains[c];
    P->chains_h[c] = ChainDev{ch.n_layers, ch.first_layer, ch.first_layer + ch.n_layers - 1, 0};
    P->max_depth = std::max(P->max_depth, ch.n_layers);
    for (int q = 0; q < ch.n_layers; ++q) {
      const int l = ch.first_layer + q;
      const tmc_layer& L = pr->layers[l];
      LayerDev& d = P->layers_h[l];
      const bool top = q == ch.n_layers - 1;
      d.K = L.K;
      d.D = L.D;
      d.chain = c;
      d.depth = q;
      d.kappa = pr->exponent == 0.0 ? 1.0 : pr->exponent;
      d.up = top ? -1 : l + 1;
      d.Kc = top ? 0 : pr->layers[l + 1].K;
      d.z_off = L.z_off;
      d.u_off = L.u_off;
      d.mu_off = top ? 0 : L.mu_off;
      d.s_off = top ? 0 : L.s_off;
      d.f_off = top ? 0 : L.f_off;
      d.u_up_off = top ? 0 : pr->layers[l + 1].u_off;
      d.alpha_off = sumK;
      d.wmax_off = sum_wmax;
      sum_wmax += (L.K + 127) / 128;
      d.p_off = sumK;
      d.rl_off = sumK;
      sumK += L.K;
      if (!top) {
        d.wf_off = sum_pairKK;
        sum_pairKK += align_up((size_t)L.K * d.Kc, 4);
        d.gtz_off = sum_pairKcD;
        sum_pairKcD += (int64_t)d.Kc * L.D;
        d.dsp_parts = P->engine == TMC_ENGINE_FUSED
                          ? (d.Kc + kFusedBwdCols - 1) / kFusedBwdCols +
                                (L.K + kFusedDzRows - 1) / kFusedDzRows
                          : 1;
        d.dsp_off = sum_pairD;
        sum_pairD += (int64_t)L.D * d.dsp_parts;
        P->entries += (int64_t)L.K * d.Kc;
      }
    }
  }
  for (auto& d : P->layers_h)
    if (d.up >= 0) {
      const LayerDev& U = P->layers_h[d.up];
      d.alpha_up_off = U.alpha_off;
      d.p_up_off = U.p_off;
      d.wmax_up_off = U.wmax_off;
      d.nwmax_up = (U.K + 127) / 128;
      d.up_top = U.up < 0 ? 1 : 0;
      d.lnKc = std::log((double)U.K);
    }

  // workspace layout
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o = align_up(o + bytes, 256);
    return r;
  };
  WsLayout& W = P->ws;
  W.alpha = take(sumK * 8);
  W.p = take(sumK * esz);
  W.rl = take(sumK * esz);
  W.pairM = take((size_t)pr->n_layers * 8);
  W.logp = take((size_t)pr->n_chains * 8);
  W.wmax = take((size_t)sum_wmax * 8);
  W.dsp = take(sum_pairD * esz);
  if (P->engine == TMC_ENGINE_PLAIN) {
    W.wf = take(sum_pairKK * esz);
    W.wg = take(sum_pairKK * esz);
    W.gtz = take(sum_pairKcD * esz);
    W.anchor = take(sumK * 8);
  }
  W.total = o;

  // schedules
  std::vector<Item> items;
  auto begin = [&](Launch& L) { L.off = (int)items.size(); };
  auto end = [&](Launch& L) { L.n = (int)items.size() - L.off; };
  const int D1 = P->max_depth - 1;
  P->fwd.assign(std::max(D1, 0), Launch{});
  P->fwd_maxkc.assign(std::max(D1, 0), 0);
  P->fwd_vec_ws.assign(std::max(D1, 0), 1);
  P->fwd_vec_caller.assign(std::max(D1, 0), 1);
  P->bwd_vec.assign(std::max(D1, 0), Launch{});
  P->bwd_sca.assign(std::max(D1, 0), Launch{});
  std::vector<int> pairs;
  for (int l = 0; l < pr->n_layers; ++l)
    if (P->layers_h[l].up >= 0 && P->layers_h[l].K > 0) pairs.push_back(l);
  // only layers that belong to a chain
  {
    std::vector<char> used(pr->n_layers, 0);
    for (auto& c : P->chains_h)
      for (int l = c.first; l <= c.top; ++l) used[l] = 1;
    std::vector<int> pp;
    for (int l : pairs)
      if (used[l]) pp.push_back(l);
    pairs.swap(pp);
  }
  if (P->engine == TMC_ENGINE_PLAIN) {
    begin(P->factor);
    for (int l : pairs) {
      const LayerDev& d = P->layers_h[l];
      const int nt = ((d.K + kPlainFactorRows - 1) / kPlainFactorRows) *
                     ((d.Kc + kPlainFactorCols - 1) / kPlainFactorCols);
      for (int t = 0; t < nt; ++t) items.push_back({l, t});
    }
    end(P->factor);
    for (int t = 0; t < D1; ++t) {
      begin(P->fwd[t]);
      for (int l : pairs) {
        const LayerDev& d = P->layers_h[l];
        const int L = P->chains_h[d.chain].L;
        if (d.depth != L - 2 - t) continue;
        P->fwd_maxkc[t] = std::max(P->fwd_maxkc[t], d.Kc);
        const int VVf = esz == 4 ? 4 : 2;
        if (d.Kc % VVf != 0 || d.wf_off % VVf != 0) P->fwd_vec_ws[t] = 0;
        if (d.Kc % VVf != 0 || d.f_off % VVf != 0) P->fwd_vec_caller[t] = 0;
        for (int r = 0; r < d.K; r += kPlainFwdRowsPerBlock) items.push_back({l, r});
      }
      end(P->fwd[t]);
    }
    const int VV = esz == 4 ? 4 : 2;
    for (int t = 0; t < D1; ++t) {
      for (int pass = 0; pass < 2; ++pass) {
        Launch& Lc = pass == 0 ? P->bwd_vec[t] : P->bwd_sca[t];
        begin(Lc);
        for (int l : pairs) {
          const LayerDev& d = P->layers_h[l];
          if (d.depth != t) continue;
          const bool vec = d.Kc >= 64 * VV && d.Kc % VV == 0 && d.f_off % VV == 0 &&
                           d.wf_off % VV == 0;
          if (vec != (pass == 0)) continue;
          const int step = vec ? 64 * VV : 64;
          for (int j = 0; j < d.Kc; j += step) items.push_back({l, j});
        }
        end(Lc);
      }
    }
    begin(P->gmu);
    for (int l : pairs) {
      const LayerDev& d = P->layers_h[l];
      const int nt = ((d.K + kPlainGemmRows - 1) / kPlainGemmRows) * ((d.D + kPlainGemmD - 1) / kPlainGemmD);
      for (int t = 0; t < nt; ++t) items.push_back({l, t});
    }
    end(P->gmu);
    begin(P->gtz);
    for (int l : pairs) {
      const LayerDev& d = P->layers_h[l];
      const int nt = ((d.Kc + kPlainGemmRows - 1) / kPlainGemmRows) * ((d.D + kPlainGemmD - 1) / kPlainGemmD);
      for (int t = 0; t < nt; ++t) items.push_back({l, t});
    }
    end(P->gtz);
  }

  // integer tables: pair ids, ds slots (layers grouped by identical s block)
  std::vector<int> ints;
  P->n_pairs = (int)pairs.size();
  P->pair_ids_off = 0;
  ints.insert(ints.end(), pairs.begin(), pairs.end());
  std::vector<int> by_s = pairs;
  std::stable_sort(by_s.begin(), by_s.end(), [&](int a, int b) {
    return P->layers_h[a].s_off < P->layers_h[b].s_off;
  });
  std::vector<int> slot_start;
  std::vector<int64_t> slot_soff;
  std::vector<int> slot_D;
  for (size_t i = 0; i < by_s.size(); ++i) {
    if (i == 0 || P->layers_h[by_s[i]].s_off != P->layers_h[by_s[i - 1]].s_off) {
      slot_start.push_back((int)i);
      slot_soff.push_back(P->layers_h[by_s[i]].s_off);
      slot_D.push_back(P->layers_h[by_s[i]].D);
    }
  }
  slot_start.push_back((int)by_s.size());
  P->n_slots = (int)slot_soff.size();
  P->slot_layers_off = (int)ints.size();
  ints.insert(ints.end(), by_s.begin(), by_s.end());
  std::vector<int64_t> part_off;
  std::vector<int> part_start;
  {
    size_t slot = 0;
    for (size_t i = 0; i < by_s.size(); ++i) {
      while (slot < slot_soff.size() && slot_start[slot] == (int)i) {
        part_start.push_back((int)part_off.size());
        ++slot;
      }
      const LayerDev& d = P->layers_h[by_s[i]];
      for (int q = 0; q < d.dsp_parts; ++q) part_off.push_back(d.dsp_off + (int64_t)q * d.D);
    }
    part_start.push_back((int)part_off.size());
  }
  P->max_D = 0;
  for (int dd : slot_D) P->max_D = std::max(P->max_D, dd);
  P->slot_start_off = (int)ints.size();
  ints.insert(ints.end(), part_start.begin(), part_start.end());
  P->slot_D_off = (int)ints.size();
  ints.insert(ints.end(), slot_D.begin(), slot_D.end());

  // fused engine layout and schedules
  if (P->engine == TMC_ENGINE_FUSED) {
    tmc_status st = fused_build(P->fused, P->prec, P->flags, P->layers_h, P->chains_h, pairs,
                                P->ws, o, items, ints);
    if (st != TMC_OK) return fail(st, "fused engine: unsupported layer width");
    tune_cache_lookup(P);
    fused_set_grids(P->fused);
  }

  // upload
  auto upload = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) bytes = 16;
    hipError_t e = hipMalloc(dst, bytes);
    if (e != hipSuccess) return e;
    if (src) return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    return hipSuccess;
  };
  HIP_TRY(upload((void**)&P->chains_d, P->chains_h.empty() ? nullptr : P->chains_h.data(),
                 P->chains_h.size() * sizeof(ChainDev)));
  HIP_TRY(upload((void**)&P->layers_d, P->layers_h.empty() ? nullptr : P->layers_h.data(),
                 P->layers_h.size() * sizeof(LayerDev)));
  HIP_TRY(upload((void**)&P->items_d, items.empty() ? nullptr : items.data(),
                 items.size() * sizeof(Item)));
  HIP_TRY(upload((void**)&P->ints_d, ints.empty() ? nullptr : ints.data(), ints.size() * sizeof(int)));
  HIP_TRY(upload((void**)&P->slot_soff_d, slot_soff.empty() ? nullptr : slot_soff.data(),
                 slot_soff.size() * sizeof(int64_t)));
  HIP_TRY(upload((void**)&P->part_off_d, part_off.empty() ? nullptr : part_off.data(),
                 part_off.size() * sizeof(int64_t)));
  HIP_TRY(hipMalloc((void**)&P->flag_d, sizeof(int)));
  HIP_TRY(hipMemset(P->flag_d, 0, sizeof(int)));
  HIP_TRY(hipDeviceSynchronize());
  return TMC_OK;
}

bool parent_scale(const tmc_plan* P) { return (P->flags & TMC_FLAG_PARENT_SCALE) != 0; }

tmc_status check_exec(tmc_plan* P, void* ws, int kind = kKindChain) {
  if (!P) return fail(TMC_ERR_INVALID_ARG, "plan is NULL");
  if (P->kind != kind)
    return fail(TMC_ERR_INVALID_ARG, P->kind == kKindStar
                                         ? "a star-model plan: use the tmc_star_* entry points"
                                         : "a chain plan: the tmc_star_* entry points need a "
                                           "plan from tmc_star_plan_create");
  if (P->ws.total > 0) {
    if (!ws) return fail(TMC_ERR_WORKSPACE, "workspace is NULL (%zu bytes needed)", P->ws.total);
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
      return fail(TMC_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  }
  return TMC_OK;
}

// Records an event pair around one launch when the plan's timer is on.
struct TimedScope {
  tmc_plan* P;
  hipStream_t st;
  bool on = false;
  TimedScope(tmc_plan* p, int kc, hipStream_t s) : P(p), st(s) {
    if (!P->timing || P->capturing || P->ev_used + 2 > P->ev_pool.size()) return;
    P->ev_marks.push_back({kc, P->ev_used});
    on = hipEventRecord(P->ev_pool[P->ev_used], st) == hipSuccess;
    P->ev_used += 2;
  }
  ~TimedScope() {
    if (on) (void)hipEventRecord(P->ev_pool[P->ev_marks.back().second + 1], st);
  }
};

#define LAUNCH_KC(kc, expr)                                                          \
  do {                                                                               \
    TimedScope ts_(P, kc, st);                                                       \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(TMC_ERR_HIP, "kernel launch %s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)
#define LAUNCH(expr) LAUNCH_KC(TMC_KC_OTHER, expr)

// ---- plain engine ----
template <typename T>
tmc_status plain_fwd(tmc_plan* P, const T* f_caller, const T* z, const T* mu, const T* s,
                     const T* u, double* logp, void* ws, hipStream_t st) {
  const WsLayout& W = P->ws;
  const Item* it = P->items_d;
  const bool caller = f_caller != nullptr;
  T* wf = wsp<T>(ws, W.wf);
  const T* f = caller ? f_caller : wf;
  // stored factors are anchored per row (FP64 anchors in the workspace); a caller's
  // factors are read as given
  double* anchor = caller ? nullptr : wsp<double>(ws, W.anchor);
  if (!caller && P->factor.n > 0)
    LAUNCH_KC(TMC_KC_PLAIN_FACTOR, launch_plain_factor<T>(P->layers_d, it + P->factor.off, P->factor.n, z, mu, s, wf, false,
                                                          anchor, parent_scale(P), st));
  LAUNCH(launch_init_top<T>(P->chains_d, P->n_chains, P->layers_d, u, wsp<double>(ws, W.alpha), st));
  for (size_t t = 0; t < P->fwd.size(); ++t)
    LAUNCH_KC(TMC_KC_PLAIN_LSE_FWD, launch_plain_lse_fwd<T>(P->layers_d, it + P->fwd[t].off, P->fwd[t].n, P->fwd_maxkc[t],
                                   caller ? P->fwd_vec_caller[t] : P->fwd_vec_ws[t], f,
                                   caller, u, wsp<double>(ws, W.alpha), wsp<T>(ws, W.rl),
                                   wsp<double>(ws, W.pairM), anchor, st));
  LAUNCH(launch_finalize(P->chains_d, P->n_chains, P->layers_d, wsp<double>(ws, W.alpha), logp,
                         wsp<double>(ws, W.logp), P->flag_d, st));
  return TMC_OK;
}

template <typename T>
tmc_status plain_bwd(tmc_plan* P, const T* f_caller, const T* z, const T* mu, const T* s,
                     const double* dlogp, void* ws, T* df, T* dz, T* dmu, T* ds, T* du,
                     hipStream_t st) {
  const WsLayout& W = P->ws;
  const Item* it = P->items_d;
  const bool caller = f_caller != nullptr;
  const T* f = caller ? f_caller : wsp<T>(ws, W.wf);
  T* g = caller ? df : wsp<T>(ws, W.wg);
  T* p = wsp<T>(ws, W.p);
  LAUNCH(launch_bwd_init<T>(P->chains_d, P->n_chains, P->layers_d, wsp<double>(ws, W.alpha),
                            wsp<double>(ws, W.logp), dlogp, p, du, dz, st));
  for (size_t t = 0; t < P->bwd_vec.size(); ++t) {
    for (int pass = 0; pass < 2; ++pass) {
      const Launch& L = pass == 0 ? P->bwd_vec[t] : P->bwd_sca[t];
      if (L.n > 0) LAUNCH_KC(TMC_KC_PLAIN_LSE_BWD, launch_plain_lse_bwd<T>(P->layers_d, it + L.off, L.n, pass == 0, f, caller,
                                     wsp<double>(ws, W.alpha), wsp<T>(ws, W.rl),
                                     wsp<double>(ws, W.pairM), dlogp, p, g, caller, caller, du, st));
    }
  }
  if (caller) return TMC_OK;
  if (dz)
    LAUNCH_KC(TMC_KC_PLAIN_GRAD, launch_plain_gmu<T>(P->layers_d, it + P->gmu.off, P->gmu.n, g, z, mu, s, p, dlogp, dz,
                                                     parent_scale(P), st));
  if (parent_scale(P)) {
    // dmu and the per-parent ds of each pair directly (no shared blocks to sum over)
    if (dmu || ds)
      LAUNCH_KC(TMC_KC_PLAIN_GRAD, launch_plain_gtz<T>(P->layers_d, it + P->gtz.off, P->gtz.n, g, z, mu, s, p,
                                                       dlogp, nullptr, dmu, ds, true, st));
    return TMC_OK;
  }
  if (dmu || ds)
    LAUNCH_KC(TMC_KC_PLAIN_GRAD, launch_plain_gtz<T>(P->layers_d, it + P->gtz.off, P->gtz.n, g, z, mu, s, p, dlogp,
                               wsp<T>(ws, W.gtz), dmu, nullptr, false, st));
  if (ds) {
    LAUNCH_KC(TMC_KC_PLAIN_GRAD, launch_pair_dsp<T>(P->layers_d, P->ints_d + P->pair_ids_off, P->n_pairs, z, mu, s, p,
                              wsp<T>(ws, W.gtz), dlogp, wsp<T>(ws, W.dsp), st));
    LAUNCH(launch_ds_reduce<T>(P->part_off_d, P->ints_d + P->slot_start_off, P->slot_soff_d,
                               P->ints_d + P->slot_D_off, P->n_slots, P->max_D, wsp<T>(ws, W.dsp),
                               ds, st));
  }
  return TMC_OK;
}

// ---- fused engine ----
tmc_status fused_fwd_impl(tmc_plan* P, const float* z, const float* mu, const float* s,
                          const float* u, double* logp, void* ws, hipStream_t st) {
  const WsLayout& W = P->ws;
  const FusedPlan& F = P->fused;
  const bool grad = !(P->flags & TMC_FLAG_FORWARD_ONLY);
  FusedFwdPtrs a{P->layers_d, z, mu, s, u, wsp<double>(ws, W.q), wsp<double>(ws, W.alpha),
                 wsp<double>(ws, W.wmax), wsp<float>(ws, W.rl), wsp<float>(ws, W.ev)};
  int* heads = wsp<int>(ws, W.cnt);
  LAUNCH(launch_fused_fwd_init(P->chains_d, P->n_chains, P->layers_d, u, a.alpha, a.wmax, heads,
                               (int)F.pfwd.size(), st));
  auto go = [&](int nkc, int waves, const Item* it, int n, const FusedQueue* q) -> hipError_t {
    return P->prec == TMC_FP32 ? launch_fused_fwd<TMC_FP32>(nkc, waves, grad, F.tune.fwd_ns, a, it, n, q, st)
                               : launch_fused_fwd<TMC_BF16X3>(nkc, waves, grad, F.tune.fwd_ns, a, it, n, q, st);
  };
  if (F.tune.persist) {
    for (auto& g : F.pfwd) {
      FusedQueue q;
      q.chains = P->ints_d + g.off;
      q.n_chains = g.n;
      q.head = heads + g.head;
      q.cd = P->chains_d;
      q.grid = g.grid;
      LAUNCH_KC(TMC_KC_FUSED_FWD, go(g.nkc, 4, P->items_d, g.n, &q));
    }
  } else {
    for (auto& step : F.fwd[F.tune.wide_fwd ? 1 : 0])
      for (auto& g : step) LAUNCH_KC(TMC_KC_FUSED_FWD, go(g.nkc, g.waves, P->items_d + g.off, g.n, nullptr));
  }
  LAUNCH(launch_finalize(P->chains_d, P->n_chains, P->layers_d, a.alpha, logp,
                         wsp<double>(ws, W.logp), P->flag_d, st));
  return TMC_OK;
}

tmc_status fused_bwd_impl(tmc_plan* P, const float* z, const float* mu, const float* s,
                          const double* dlogp, void* ws, float* dz, float* dmu, float* ds,
                          float* du, hipStream_t st) {
  const WsLayout& W = P->ws;
  const FusedPlan& F = P->fused;
  float* dsp = ds ? wsp<float>(ws, W.dsp) : nullptr;
  FusedBwdPtrs a{P->layers_d, z, mu, s, wsp<double>(ws, W.alpha), wsp<double>(ws, W.wmax),
                 wsp<double>(ws, W.q), wsp<float>(ws, W.rl), wsp<float>(ws, W.lam), dlogp,
                 wsp<float>(ws, W.p), dmu, du, dsp, wsp<float>(ws, W.ev), dz, (dz || ds) ? 1 : 0};
  int* heads = wsp<int>(ws, W.cnt);
  LAUNCH(launch_fused_bwd_init(P->chains_d, P->n_chains, P->layers_d, a.alpha,
                               wsp<double>(ws, W.logp), dlogp, a.rl, a.lam, a.p, du, dz,
                               heads + F.pfwd.size(), (int)F.pbwd.size(), st));
  auto go = [&](int nkc, int waves, const Item* it, int n, const FusedQueue* q) -> hipError_t {
    return P->prec == TMC_FP32 ? launch_fused_bwd<TMC_FP32>(nkc, waves, a, it, n, q, st)
                               : launch_fused_bwd<TMC_BF16X3>(nkc, waves, a, it, n, q, st);
  };
  if (F.tune.persist) {
    for (auto& g : F.pbwd) {
      FusedQueue q;
      q.chains = P->ints_d + g.off;
      q.n_chains = g.n;
      q.head = heads + g.head;
      q.cd = P->chains_d;
      q.grid = g.grid;
      LAUNCH_KC(TMC_KC_FUSED_BWD, go(g.nkc, 4, P->items_d, g.n, &q));
    }
  } else {
    for (auto& step : F.bwd[F.tune.wide_bwd ? 1 : 0])
      for (auto& g : step) LAUNCH_KC(TMC_KC_FUSED_BWD, go(g.nkc, g.waves, P->items_d + g.off, g.n, nullptr));
  }
  const FusedLaunch& rows = F.dz[(!F.tune.persist && F.tune.wide_bwd) ? 1 : 0];
  if ((dz || ds) && rows.n > 0)
    LAUNCH(launch_fused_dz(P->layers_d, P->items_d + rows.off, rows.n, z, s, a.p,
                           wsp<float>(ws, W.ev), dlogp, dz, dsp, st));
  if (ds)
    LAUNCH(launch_ds_reduce<float>(P->part_off_d, P->ints_d + P->slot_start_off, P->slot_soff_d,
                                   P->ints_d + P->slot_D_off, P->n_slots, P->max_D, dsp, ds, st));
  return TMC_OK;
}

tmc_status gauss_fwd_impl(tmc_plan* P, const void* z, const void* mu, const void* s,
                          const void* u, double* logp, void* ws, hipStream_t st) {
  if (!P->gauss_err.empty()) return fail(TMC_ERR_INVALID_ARG, "%s", P->gauss_err.c_str());
  if (P->n_chains == 0) return TMC_OK;
  if (!u || !logp || (P->n_pairs > 0 && (!z || !mu || !s)))
    return fail(TMC_ERR_INVALID_ARG, "NULL input or output pointer");
  if (P->engine == TMC_ENGINE_FUSED)
    return fused_fwd_impl(P, (const float*)z, (const float*)mu, (const float*)s, (const float*)u,
                          logp, ws, st);
  if (P->prec == TMC_FP64)
    return plain_fwd<double>(P, nullptr, (const double*)z, (const double*)mu, (const double*)s,
                             (const double*)u, logp, ws, st);
  return plain_fwd<float>(P, nullptr, (const float*)z, (const float*)mu, (const float*)s,
                          (const float*)u, logp, ws, st);
}

tmc_status gauss_bwd_impl(tmc_plan* P, const void* z, const void* mu, const void* s,
                          const void* u, const double* dlogp, void* ws, void* dz, void* dmu,
                          void* ds, void* du, hipStream_t st) {
  if (!P->gauss_err.empty()) return fail(TMC_ERR_INVALID_ARG, "%s", P->gauss_err.c_str());
  if (P->n_chains == 0) return TMC_OK;
  if (!dlogp || (P->n_pairs > 0 && (!z || !mu || !s)))
    return fail(TMC_ERR_INVALID_ARG, "NULL input pointer");
  if (P->engine == TMC_ENGINE_FUSED) {
    if (P->flags & TMC_FLAG_FORWARD_ONLY)
      return fail(TMC_ERR_STATE, "plan was created with TMC_FLAG_FORWARD_ONLY");
    return fused_bwd_impl(P, (const float*)z, (const float*)mu, (const float*)s, dlogp, ws,
                          (float*)dz, (float*)dmu, (float*)ds, (float*)du, st);
  }
  if (P->prec == TMC_FP64)
    return plain_bwd<double>(P, nullptr, (const double*)z, (const double*)mu, (const double*)s,
                             dlogp, ws, nullptr, (double*)dz, (double*)dmu, (double*)ds,
                             (double*)du, st);
  return plain_bwd<float>(P, nullptr, (const float*)z, (const float*)mu, (const float*)s, dlogp,
                          ws, nullptr, (float*)dz, (float*)dmu, (float*)ds, (float*)du, st);
}

// ---- star model ----
template <typename T>
StarArgs<T> star_args(tmc_plan* P, void* ws) {
  const StarPlan& sp = P->star;
  char* base = static_cast<char*>(ws);
  StarArgs<T> a{};
  a.S = sp.S;
  a.N = sp.N;
  a.Kt = sp.Kt;
  a.K = sp.K;
  a.D = sp.D;
  a.P = sp.P;
  a.ngrp = sp.ngrp;
  a.nkb = sp.nkb;
  a.msg = reinterpret_cast<double*>(base + sp.msg);
  a.gsum = reinterpret_cast<double*>(base + sp.gsum);
  a.w = reinterpret_cast<double*>(base + sp.w);
  a.lp = reinterpret_cast<double*>(base + sp.lp);
  a.nsh = reinterpret_cast<T*>(base + sp.nsh);
  a.wT = reinterpret_cast<T*>(base + sp.wT);
  const bool grad = !(P->flags & TMC_FLAG_FORWARD_ONLY);
  a.dm = grad ? reinterpret_cast<double*>(base + sp.dm) : nullptr;
  a.dsp = grad ? reinterpret_cast<double*>(base + sp.dsp) : nullptr;
  a.flag = P->flag_d;
  return a;
}

template <typename T>
tmc_status star_fwd(tmc_plan* P, const T* mth, const T* s, const T* z, const T* u, const T* uth,
                    double* logp, void* ws, hipStream_t st) {
  StarArgs<T> a = star_args<T>(P, ws);
  a.mth = mth;
  a.s = s;
  a.z = z;
  a.u = u;
  a.uth = uth;
  a.logp = logp;
  LAUNCH_KC(TMC_KC_STAR_MSG, launch_star_msg<T>(a, st));
  LAUNCH(launch_star_colsum<T>(a, st));
  LAUNCH(launch_star_logp<T>(a, st));
  return TMC_OK;
}

template <typename T>
tmc_status star_bwd(tmc_plan* P, const T* mth, const T* s, const T* z, const T* u,
                    const double* dlogp, void* ws, T* dmth, T* ds, T* dz, T* du, T* duth,
                    hipStream_t st) {
  StarArgs<T> a = star_args<T>(P, ws);
  a.mth = mth;
  a.s = s;
  a.z = z;
  a.u = u;
  a.dlogp = dlogp;
  a.dmth = dmth;
  a.ds = ds;
  a.dz = dz;
  a.du = du;
  a.duth = duth;
  if (dz || du || ds) LAUNCH_KC(TMC_KC_STAR_BWD, launch_star_bwd_local<T>(a, st));
  if (dmth) LAUNCH_KC(TMC_KC_STAR_BWD, launch_star_bwd_global<T>(a, st));
  if (dmth || ds || duth) LAUNCH(launch_star_reduce<T>(a, st));
  return TMC_OK;
}

tmc_status star_validate(const tmc_star_problem* pr) {
  if (!pr) return fail(TMC_ERR_INVALID_ARG, "problem is NULL");
  if (pr->reserved != 0) return fail(TMC_ERR_INVALID_ARG, "reserved must be 0");
  if (pr->flags & ~TMC_FLAG_FORWARD_ONLY)
    return fail(TMC_ERR_INVALID_ARG, "unknown flags 0x%x for a star problem", pr->flags);
  if (pr->precision == TMC_BF16X3)
    return fail(TMC_ERR_UNSUPPORTED, "star problems run in TMC_FP64 or TMC_FP32");
  if (pr->precision != TMC_FP64 && pr->precision != TMC_FP32)
    return fail(TMC_ERR_INVALID_ARG, "unknown precision %d", pr->precision);
  if (pr->n_instances < 1) return fail(TMC_ERR_INVALID_ARG, "n_instances must be >= 1");
  const int64_t kMaxSamples = (int64_t)65535 * kStarLanes;
  if (pr->N < 1) return fail(TMC_ERR_SHAPE, "N = %d must be >= 1", pr->N);
  if (pr->K < 1 || pr->K > kMaxSamples)
    return fail(TMC_ERR_SHAPE, "K = %d outside [1, %lld]", pr->K, (long long)kMaxSamples);
  if (pr->K_theta < 1 || pr->K_theta > kMaxSamples)
    return fail(TMC_ERR_SHAPE, "K_theta = %d outside [1, %lld]", pr->K_theta, (long long)kMaxSamples);
  if (pr->D < 1 || pr->D > kStarMaxD)
    return fail(TMC_ERR_SHAPE, "D = %d outside [1, %d]", pr->D, kStarMaxD);
  if ((int64_t)pr->n_instances * pr->N > INT32_MAX)
    return fail(TMC_ERR_INVALID_ARG, "n_instances * N exceeds one launch grid");
  if ((int64_t)pr->K_theta * pr->D > (int64_t)65534 * kStarLanes)
    return fail(TMC_ERR_INVALID_ARG, "K_theta * D exceeds one launch grid");
  return TMC_OK;
}

void star_layout(tmc_plan* P, const tmc_star_problem* pr) {
  StarPlan& sp = P->star;
  sp.S = pr->n_instances;
  sp.N = pr->N;
  sp.Kt = pr->K_theta;
  sp.K = pr->K;
  sp.D = pr->D;
  const int64_t nkt = (sp.Kt + kStarLanes - 1) / kStarLanes;
  sp.nkb = (sp.K + kStarLanes - 1) / kStarLanes;
  // points per workgroup: one per wave at least, more while the forward grid would
  // exceed about kStarTargetGroups workgroups
  const int64_t want = (int64_t)sp.S * sp.N * nkt / kStarTargetGroups;
  sp.P = (int)std::max<int64_t>(std::min<int64_t>(sp.N, kStarWaves), std::min<int64_t>(sp.N, want));
  sp.ngrp = (sp.N + sp.P - 1) / sp.P;
  const int64_t S = sp.S;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes, 256);
    return o;
  };
  sp.msg = take((size_t)(S * sp.N * sp.Kt) * 8);
  sp.gsum = take((size_t)(S * sp.ngrp * sp.Kt) * 8);
  sp.w = take((size_t)(S * sp.Kt) * 8);
  sp.lp = take((size_t)S * 8);
  const size_t esz = pr->precision == TMC_FP64 ? 8 : 4;
  sp.nsh = take((size_t)(S * sp.N * sp.Kt) * esz);
  sp.wT = take((size_t)(S * sp.Kt) * esz);
  if (!(P->flags & TMC_FLAG_FORWARD_ONLY)) {
    sp.dm = take((size_t)(S * sp.ngrp * sp.Kt) * sp.D * 8);
    sp.dsp = take((size_t)(S * sp.N * sp.nkb) * sp.D * 8);
  }
  P->ws = WsLayout{};
  P->ws.total = off;
  P->entries = S * sp.N * (int64_t)sp.Kt * sp.K;
  P->max_depth = 2;
  P->max_D = sp.D;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

int tmc_abi_version(void) { return TMC_ABI_VERSION; }

const char* tmc_status_string(tmc_status s) {
  switch (s) {
    case TMC_OK: return "TMC_OK";
    case TMC_ERR_INVALID_ARG: return "TMC_ERR_INVALID_ARG";
    case TMC_ERR_SHAPE: return "TMC_ERR_SHAPE";
    case TMC_ERR_WORKSPACE: return "TMC_ERR_WORKSPACE";
    case TMC_ERR_UNSUPPORTED: return "TMC_ERR_UNSUPPORTED";
    case TMC_ERR_HIP: return "TMC_ERR_HIP";
    case TMC_ERR_NUMERIC: return "TMC_ERR_NUMERIC";
    case TMC_ERR_STATE: return "TMC_ERR_STATE";
  }
  return "TMC_ERR_UNKNOWN";
}

const char* tmc_last_error(void) { return g_err.c_str(); }

tmc_status tmc_plan_create(const tmc_problem* problem, int device, tmc_plan_t* out) {
  try {
    if (!out) return fail(TMC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int engine = 0;
    std::string gerr, ferr;
    tmc_status st = validate(problem, &engine, &gerr, &ferr);
    if (st != TMC_OK) return st;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0)
      return fail(TMC_ERR_HIP, "no HIP device available (%s)", hipGetErrorString(e));
    if (device < 0 || device >= ndev)
      return fail(TMC_ERR_INVALID_ARG, "device %d out of range [0, %d)", device, ndev);
    DeviceGuard g(device);
    if (!g.ok) return fail(TMC_ERR_HIP, "hipSetDevice(%d) failed", device);
    tmc_plan* P = new tmc_plan();
    P->device = device;
    P->prec = problem->precision;
    P->engine = engine;
    P->flags = problem->flags;
    P->gauss_err = gerr;
    P->logf_err = ferr;
    st = build_plan(P, problem);
    if (st != TMC_OK) {
      delete P;
      return st;
    }
    // the static device workspace of tmc_gauss_fwd_noalloc: its address on this device
    // (looked up once per device; a failure disables only that entry point)
    const hipError_t se = scratch_init(device);
    if (se == hipSuccess) P->scratch = scratch_device_ptr(device);
    else P->scratch_err = std::string("hipGetSymbolAddress of the static workspace: ") + hipGetErrorString(se);
    *out = P;
    g_err.clear();
    return TMC_OK;
  } catch (const std::bad_alloc&) {
    return fail(TMC_ERR_INVALID_ARG, "host allocation failed");
  } catch (...) {
    return fail(TMC_ERR_INVALID_ARG, "unexpected host exception");
  }
}

tmc_status tmc_star_plan_create(const tmc_star_problem* problem, int device, tmc_plan_t* out) {
  try {
    if (!out) return fail(TMC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    tmc_status st = star_validate(problem);
    if (st != TMC_OK) return st;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev == 0)
      return fail(TMC_ERR_HIP, "no HIP device available (%s)", hipGetErrorString(e));
    if (device < 0 || device >= ndev)
      return fail(TMC_ERR_INVALID_ARG, "device %d out of range [0, %d)", device, ndev);
    DeviceGuard g(device);
    if (!g.ok) return fail(TMC_ERR_HIP, "hipSetDevice(%d) failed", device);
    tmc_plan* P = new tmc_plan();
    P->kind = kKindStar;
    P->device = device;
    P->prec = problem->precision;
    P->engine = TMC_ENGINE_PLAIN;
    P->flags = problem->flags;
    P->esz = problem->precision == TMC_FP64 ? 8 : 4;
    star_layout(P, problem);
    e = hipMalloc(&P->flag_d, sizeof(int));
    if (e == hipSuccess) e = hipMemset(P->flag_d, 0, sizeof(int));
    if (e != hipSuccess) {
      delete P;
      return fail(TMC_ERR_HIP, "flag allocation: %s", hipGetErrorString(e));
    }
    P->scratch_err = "not available for star-model plans";
    *out = P;
    g_err.clear();
    return TMC_OK;
  } catch (const std::bad_alloc&) {
    return fail(TMC_ERR_INVALID_ARG, "host allocation failed");
  } catch (...) {
    return fail(TMC_ERR_INVALID_ARG, "unexpected host exception");
  }
}

tmc_status tmc_star_gauss_fwd(tmc_plan_t plan, const void* mth, const void* s, const void* z,
                              const void* u, const void* uth, double* logp, void* workspace,
                              void* stream) {
  try {
    tmc_status st = check_exec(plan, workspace, kKindStar);
    if (st != TMC_OK) return st;
    if (!mth || !s || !z || !u || !uth || !logp)
      return fail(TMC_ERR_INVALID_ARG, "NULL input or output pointer");
    DeviceGuard g(plan->device);
    hipStream_t hs = (hipStream_t)stream;
    if (plan->prec == TMC_FP64)
      return star_fwd<double>(plan, (const double*)mth, (const double*)s, (const double*)z,
                              (const double*)u, (const double*)uth, logp, workspace, hs);
    return star_fwd<float>(plan, (const float*)mth, (const float*)s, (const float*)z,
                           (const float*)u, (const float*)uth, logp, workspace, hs);
  } catch (...) {
    return fail(TMC_ERR_INVALID_ARG, "unexpected host exception");
  }
}

tmc_status tmc_star_gauss_bwd(tmc_plan_t plan, const void* mth, const void* s, const void* z,
                              const void* u, const double* dlogp, void* workspace, void* dmth,
                              void* ds, void* dz, void* du, void* duth, void* stream) {
  try {
    tmc_status st = check_exec(plan, workspace, kKindStar);
    if (st != TMC_OK) return st;
    if (plan->flags & TMC_FLAG_FORWARD_ONLY)
      return fail(TMC_ERR_STATE, "plan was created with TMC_FLAG_FORWARD_ONLY");
    if (!mth || !s || !z || !u || !dlogp) return fail(TMC_ERR_INVALID_ARG, "NULL input pointer");
    DeviceGuard g(plan->device);
    hipStream_t hs = (hipStream_t)stream;
    if (plan->prec == TMC_FP64)
      return star_bwd<double>(plan, (const double*)mth, (const double*)s, (const double*)z,
                              (const double*)u, dlogp, workspace, (double*)dmth, (double*)ds,
                              (double*)dz, (double*)du, (double*)duth, hs);
    return star_bwd<float>(plan, (const float*)mth, (const float*)s, (const float*)z,
                           (const float*)u, dlogp, workspace, (float*)dmth, (float*)ds,
                           (float*)dz, (float*)du, (float*)duth, hs);
  } catch (...) {
    return fail(TMC_ERR_INVALID_ARG, "unexpected host exception");
  }
}

namespace {
tmc_status logmm_check(int32_t batch, int32_t M, int32_t K, int32_t N, int32_t precision) {
  if (precision != TMC_FP64 && precision != TMC_FP32 && precision != TMC_BF16X3)
    return fail(TMC_ERR_INVALID_ARG, "unknown precision %d", precision);
  if (batch < 1 || batch > 65535) return fail(TMC_ERR_SHAPE, "batch = %d outside [1, 65535]", batch);
  if (M < 1 || M > 65535) return fail(TMC_ERR_SHAPE, "M = %d outside [1, 65535]", M);
  if (K < 1 || K > (1 << 24)) return fail(TMC_ERR_SHAPE, "K = %d outside [1, 2^24]", K);
  if (N < 1 || N > (1 << 24)) return fail(TMC_ERR_SHAPE, "N = %d outside [1, 2^24]", N);
  return TMC_OK;
}

int32_t logmm_kp(int32_t K) { return (K + 31) / 32 * 32; }

// Shifts, then the prepared operands, in the element size of the mode: 4 bytes (two
// BF16 planes, or FP32) or 8 (FP64).
size_t logmm_ws(int32_t batch, int32_t M, int32_t K, int32_t N, int32_t precision) {
  const size_t kp = (size_t)logmm_kp(K), es = precision == TMC_FP64 ? 8 : 4;
  return align_up((size_t)batch * M * es, 256) + align_up((size_t)batch * N * es, 256) +
         align_up((size_t)batch * M * kp * es, 256) + align_up((size_t)batch * N * kp * es, 256);
}
}  // namespace

tmc_status tmc_logmmexp_workspace_size(int32_t batch, int32_t M, int32_t K, int32_t N,
                                       int32_t precision, size_t* bytes) {
  if (!bytes) return fail(TMC_ERR_INVALID_ARG, "bytes is NULL");
  const tmc_status st = logmm_check(batch, M, K, N, precision);
  if (st != TMC_OK) return st;
  *bytes = logmm_ws(batch, M, K, N, precision);
  return TMC_OK;
}

tmc_status tmc_logmmexp(int32_t batch, int32_t M, int32_t K, int32_t N, int32_t precision,
                        const void* X, const void* Y, void* Z, void* workspace, void* stream) {
  try {
    tmc_status st = logmm_check(batch, M, K, N, precision);
    if (st != TMC_OK) return st;
    if (!X || !Y || !Z) return fail(TMC_ERR_INVALID_ARG, "NULL X, Y or Z");
    if (!workspace) return fail(TMC_ERR_WORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
      return fail(TMC_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    LogmmArgs a{};
    a.B = batch;
    a.M = M;
    a.K = K;
    a.N = N;
    a.Kp = logmm_kp(K);
    const size_t es = precision == TMC_FP64 ? 8 : 4;
    char* w = (char*)workspace;
    void* xs = w;
    w += align_up((size_t)batch * M * es, 256);
    void* ys = w;
    w += align_up((size_t)batch * N * es, 256);
    a.opa = w;
    w += align_up((size_t)batch * M * a.Kp * es, 256);
    a.opb = w;
    if (precision == TMC_FP64) {
      a.Xd = (const double*)X;
      a.Yd = (const double*)Y;
      a.Zd = (double*)Z;
      a.xsd = (double*)xs;
      a.ysd = (double*)ys;
    } else {
      a.X = (const float*)X;
      a.Y = (const float*)Y;
      a.Z = (float*)Z;
      a.xs = (float*)xs;
      a.ys = (float*)ys;
    }
    const hipError_t e = launch_logmm(a, precision, (hipStream_t)stream);
    if (e != hipSuccess) return fail(TMC_ERR_HIP, "log-domain product launch: %s", hipGetErrorString(e));
    return TMC_OK;
  } catch (...) {
    return fail(TMC_ERR_INVALID_ARG, "unexpected host exception");
  }
}

tmc_status tmc_plan_destroy(tmc_plan_t plan) {
  if (!plan) return TMC_OK;
  try {
    DeviceGuard g(plan->device);
    delete plan;
  } catch (...) {
    return fail(TMC_ERR_INVALID_ARG, "unexpected host exception");
  }
  return TMC_OK;
}

tmc_status tmc_plan_workspace_size(tmc_plan_t plan, size_t* bytes) {
  if (!plan || !bytes) return fail(TMC_ERR_INVALID_ARG, "NULL argument");
  *bytes = plan->ws.total;
  return TMC_OK;
}

tmc_status tmc_plan_info_get(tmc_plan_t plan, tmc_plan_info* out) {
  if (!plan || !out) return fail(TMC_ERR_INVALID_ARG, "NULL argument");
  std::memset(out, 0, sizeof(*out));
  out->factor_entries = plan->entries;
  out->workspace_bytes = (int64_t)plan->ws.total;
  out->engine = plan->engine;
  out->precision = plan->prec;
  out->max_depth = plan->max_depth;
  if (plan->engine == TMC_ENGINE_FUSED) fused_info(plan->fused, out);
  return TMC_OK;
}

tmc_status tmc_plan_check(tmc_plan_t plan, void* stream) {
  if (!plan) return fail(TMC_ERR_INVALID_ARG, "plan is NULL");
  try {
    DeviceGuard g(plan->device);
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    int flag = 0;
    HIP_TRY(hipMemcpy(&flag, plan->flag_d, sizeof(int), hipMemcpyDeviceToHost));
    if (flag) {
      HIP_TRY(hipMemset(plan->flag_d, 0, sizeof(int)));
      if (flag & kFlagNonFinite) return fail(TMC_ERR_NUMERIC, "a log P was NaN or +inf");
    }
  } catch (...) {
    return fail(TMC_ERR_INVALID_ARG, "unexpected host exception");
  }
  return TMC_OK;
}

tmc_status tmc_gauss_fwd(tmc_plan_t plan, const void* z, const void* mu, const void* s,
                         const void* u, double* logp, void* workspace, void* stream) {
  try {
    tmc_status st = check_exec(plan, workspace);
    if (st != TMC_OK) return st;
    DeviceGuard g(plan->device);
    return gauss_fwd_impl(plan, z, mu, s, u, logp, workspace, (hipStream_t)stream);
  } catch (...) {
    return fail(TMC_ERR_INVALID_ARG, "unexpected host exception");
  }
}

tmc_status tmc_gauss_bwd(tmc_plan_t plan, const void* z, const void* mu, const void* s,
                         const void* u, const double* dlogp, void* workspace, void* dz,
                         void* dmu, void* ds, void* du, void* stream) {
  try {
    tmc_status st = check_exec(plan, workspace);
    if (st != TMC_OK) return st;
    DeviceGuard g(plan->device);
    return gauss_bwd_impl(plan, z, mu, s, u, dlogp, workspace, dz, dmu, ds, du,
                          (hipStream_t)stream);
  } catch (...) {
    return fail(TMC_ERR_INVALID_ARG, "unexpected host exception");
  }
}

tmc_status tmc_gauss_fwd_noalloc(tmc_plan_t plan, const void* z, const void* mu, const void* s,
                                 const void* u, double* logp, void* stream) {
  try {
    if (!plan) return fail(TMC_ERR_INVALID_ARG, "plan is NULL");
    if (plan->kind != kKindChain) return check_exec(plan, nullptr);
    if (!plan->scratch)
      return fail(TMC_ERR_HIP, "static device workspace unavailable (%s)", plan->scratch_err.c_str());
    if (plan->ws.total > kNoallocWorkspaceBytes)
      return fail(TMC_ERR_WORKSPACE,
                  "plan needs %zu workspace bytes, the allocation-free forward has %zu "
                  "(a forward-only plan needs less)", plan->ws.total, kNoallocWorkspaceBytes);
    DeviceGuard g(plan->device);
    return gauss_fwd_impl(plan, z, mu, s, u, logp, plan->scratch, (hipStream_t)stream);
  } catch (...) {
    return fail(TMC_ERR_INVALID_ARG, "unexpected host exception");
  }
}

tmc_status tmc_gauss_factors(tmc_plan_t plan, const void* z, const void* mu, const void* s,
                             void* f, void* stream) {
  try {
    if (!plan) return fail(TMC_ERR_INVALID_ARG, "plan is NULL");
    if (plan->kind != kKindChain) return check_exec(plan, nullptr);
    if (plan->engine != TMC_ENGINE_PLAIN)
      return fail(TMC_ERR_UNSUPPORTED, "tmc_gauss_factors needs a plain-engine plan");
    if (!plan->gauss_err.empty()) return fail(TMC_ERR_INVALID_ARG, "%s", plan->gauss_err.c_str());
    if (!plan->logf_err.empty()) return fail(TMC_ERR_INVALID_ARG, "%s", plan->logf_err.c_str());
    if (plan->n_pairs == 0) return TMC_OK;
    if (!z || !mu || !s || !f) return fail(TMC_ERR_INVALID_ARG, "NULL pointer");
    DeviceGuard g(plan->device);
    const Item* it = plan->items_d + plan->factor.off;
    hipStream_t st = (hipStream_t)stream;
    tmc_plan* P = plan;
    if (plan->prec == TMC_FP64)
      LAUNCH(launch_plain_factor<double>(plan->layers_d, it, plan->factor.n, (const double*)z,
                                         (const double*)mu, (const double*)s, (double*)f, true, nullptr,
                                         parent_scale(plan), st));
    else
      LAUNCH(launch_plain_factor<float>(plan->layers_d, it, plan->factor.n, (const float*)z,
                                        (const float*)mu, (const float*)s, (float*)f, true, nullptr,
                                        parent_scale(plan), st));
    return TMC_OK;
  } catch (...) {
    return fail(TMC_ERR_INVALID_ARG, "unexpected host exception");
  }
}

tmc_status tmc_logfactor_fwd(tmc_plan_t plan, const void* f, const void* u, double* logp,
                             void* workspace, void* stream) {
  try {
    tmc_status st = check_exec(plan, workspace);
    if (st != TMC_OK) return st;
    if (plan->engine != TMC_ENGINE_PLAIN)
      return fail(TMC_ERR_UNSUPPORTED, "log-factor entry points need a plain-engine plan");
    if (!plan->logf_err.empty()) return fail(TMC_ERR_INVALID_ARG, "%s", plan->logf_err.c_str());
    if (plan->n_chains == 0) return TMC_OK;
    if (!u || !logp || (plan->n_pairs > 0 && !f)) return fail(TMC_ERR_INVALID_ARG, "NULL pointer");
    DeviceGuard g(plan->device);
    hipStream_t s = (hipStream_t)stream;
    if (plan->prec == TMC_FP64)
      return plain_fwd<double>(plan, (const double*)f, nullptr, nullptr, nullptr, (const double*)u,
                               logp, workspace, s);
    return plain_fwd<float>(plan, (const float*)f, nullptr, nullptr, nullptr, (const float*)u, logp,
                            workspace, s);
  } catch (...) {
    return fail(TMC_ERR_INVALID_ARG, "unexpected host exception");
  }
}

tmc_status tmc_logfactor_bwd(tmc_plan_t plan, const void* f, const void* u, const double* dlogp,
                             void* workspace, void* df, void* du, void* stream) {
  (void)u;
  try {
    tmc_status st = check_exec(plan, workspace);
    if (st != TMC_OK) return st;
    if (plan->engine != TMC_ENGINE_PLAIN)
      return fail(TMC_ERR_UNSUPPORTED, "log-factor entry points need a plain-engine plan");
    if (!plan->logf_err.empty()) return fail(TMC_ERR_INVALID_ARG, "%s", plan->logf_err.c_str());
    if (plan->n_chains == 0) return TMC_OK;
    if (!dlogp || (plan->n_pairs > 0 && !f)) return fail(TMC_ERR_INVALID_ARG, "NULL pointer");
    DeviceGuard g(plan->device);
    hipStream_t s = (hipStream_t)stream;
    if (plan->prec == TMC_FP64)
      return plain_bwd<double>(plan, (const double*)f, nullptr, nullptr, nullptr, dlogp, workspace,
                               (double*)df, nullptr, nullptr, nullptr, (double*)du, s);
    return plain_bwd<float>(plan, (const float*)f, nullptr, nullptr, nullptr, dlogp, workspace,
                            (float*)df, nullptr, nullptr, nullptr, (float*)du, s);
  } catch (...) {
    return fail(TMC_ERR_INVALID_ARG, "unexpected host exception");
  }
}

tmc_status tmc_plan_graph_capture_gauss(tmc_plan_t plan, int which, const void* z, const void* mu,
                                        const void* s, const void* u, double* logp,
                                        const double* dlogp, void* workspace, void* dz, void* dmu,
                                        void* ds, void* du, void* stream) {
  try {
    tmc_status st = check_exec(plan, workspace);
    if (st != TMC_OK) return st;
    if (which != 0 && which != 1) return fail(TMC_ERR_INVALID_ARG, "which must be 0 or 1");
    if (!stream) return fail(TMC_ERR_INVALID_ARG, "graph capture needs a non-default stream");
    DeviceGuard g(plan->device);
    hipStream_t hs = (hipStream_t)stream;
    HIP_TRY(hipStreamBeginCapture(hs, hipStreamCaptureModeThreadLocal));
    plan->capturing = true;
    tmc_status rs = which == 0 ? gauss_fwd_impl(plan, z, mu, s, u, logp, workspace, hs)
                               : gauss_bwd_impl(plan, z, mu, s, u, dlogp, workspace, dz, dmu, ds,
                                                du, hs);
    plan->capturing = false;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(hs, &graph);
    if (rs != TMC_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rs;
    }
    if (e != hipSuccess) return fail(TMC_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    if (plan->graph[which]) {
      (void)hipGraphExecDestroy(plan->graph[which]);
      plan->graph[which] = nullptr;
    }
    e = hipGraphInstantiate(&plan->graph[which], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(TMC_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    return TMC_OK;
  } catch (...) {
    return fail(TMC_ERR_INVALID_ARG, "unexpected host exception");
  }
}

tmc_status tmc_plan_graph_launch(tmc_plan_t plan, int which, void* stream) {
  if (!plan) return fail(TMC_ERR_INVALID_ARG, "plan is NULL");
  if (which != 0 && which != 1) return fail(TMC_ERR_INVALID_ARG, "which must be 0 or 1");
  if (!plan->graph[which]) return fail(TMC_ERR_STATE, "no graph captured for which=%d", which);
  DeviceGuard g(plan->device);
  HIP_TRY(hipGraphLaunch(plan->graph[which], (hipStream_t)stream));
  return TMC_OK;
}

tmc_status tmc_plan_autotune(tmc_plan_t plan, const void* z, const void* mu, const void* s,
                             const void* u, const double* dlogp, void* workspace, void* dz,
                             void* dmu, void* ds, void* du, int reps, void* stream) {
  try {
    tmc_status st = check_exec(plan, workspace);
    if (st != TMC_OK) return st;
    if (plan->engine != TMC_ENGINE_FUSED) return TMC_OK;
    if (plan->capturing) return fail(TMC_ERR_STATE, "autotune during graph capture");
    if (reps < 1) return fail(TMC_ERR_INVALID_ARG, "reps must be >= 1");
    if (!plan->gauss_err.empty()) return fail(TMC_ERR_SHAPE, "%s", plan->gauss_err.c_str());
    if (!z || !mu || !s || !u) return fail(TMC_ERR_INVALID_ARG, "z, mu, s and u are required");
    const bool fwd_only = (plan->flags & TMC_FLAG_FORWARD_ONLY) != 0;
    if (!fwd_only && !dlogp) return fail(TMC_ERR_INVALID_ARG, "dlogp is required for a backward");
    DeviceGuard g(plan->device);
    hipStream_t hs = (hipStream_t)stream;
    tmc_plan* P = plan;
    double* logp = wsp<double>(workspace, P->ws.logp);
    const bool was_timing = P->timing;
    P->timing = false;
    // does any per-depth group have an 8-wave form (else the wide flags change nothing)
    bool has_wide = false;
    for (int dir = 0; dir < 2; ++dir)
      for (auto& step : (dir == 0 ? P->fused.fwd[1] : P->fused.bwd[1]))
        for (auto& g : step) has_wide = has_wide || g.waves == 8;
    std::vector<FusedTune> cands;
    for (int persist = 0; persist < 2; ++persist)
      for (int gf = 1; gf <= (persist ? 2 : 1); ++gf)
        for (int ns = 1; ns <= 2; ++ns)
          for (int wide = 0; wide < ((!persist && has_wide) ? 4 : 1); ++wide) {
            if (!fwd_only && ns == 1) continue;   // the gradient forward has one stage width
            FusedTune t;
            t.persist = persist != 0;
            t.grid_factor = gf;
            t.fwd_ns = ns;
            t.wide_fwd = (wide & 1) != 0;
            t.wide_bwd = (wide & 2) != 0;
            cands.push_back(t);
          }
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    auto run = [&]() -> tmc_status {
      tmc_status r = fused_fwd_impl(P, (const float*)z, (const float*)mu, (const float*)s,
                                    (const float*)u, logp, workspace, hs);
      if (r != TMC_OK || fwd_only) return r;
      return fused_bwd_impl(P, (const float*)z, (const float*)mu, (const float*)s, dlogp,
                            workspace, (float*)dz, (float*)dmu, (float*)ds, (float*)du, hs);
    };
    // two rounds over the candidates, each candidate keeping its faster time (a
    // transient disturbance of one measurement then decides nothing)
    std::vector<float> best_ms(cands.size(), -1.0f);
    tmc_status rs = TMC_OK;
    for (size_t k = 0; k < 2 * cands.size() && rs == TMC_OK; ++k) {
      const FusedTune& t = cands[k % cands.size()];
      P->fused.tune = t;
      fused_set_grids(P->fused);
      if ((rs = run()) != TMC_OK) break;   // warm-up
      if (hipEventRecord(e0, hs) != hipSuccess) { rs = fail(TMC_ERR_HIP, "event record"); break; }
      for (int r = 0; r < reps && rs == TMC_OK; ++r) rs = run();
      if (rs != TMC_OK) break;
      if (hipEventRecord(e1, hs) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        rs = fail(TMC_ERR_HIP, "event synchronise");
        break;
      }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      float& b = best_ms[k % cands.size()];
      if (b < 0.0f || ms < b) b = ms;
    }
    FusedTune best_t = P->fused.tune;
    float best = -1.0f;
    for (size_t k = 0; k < cands.size(); ++k)
      if (best_ms[k] >= 0.0f && (best < 0.0f || best_ms[k] < best)) {
        best = best_ms[k];
        best_t = cands[k];
      }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    P->timing = was_timing;
    P->fused.tune = best_t;
    fused_set_grids(P->fused);
    if (rs != TMC_OK) return rs;
    P->fused.tuned = true;
    tune_cache_store(P);
    return tmc_plan_check(plan, stream);
  } catch (...) {
    return fail(TMC_ERR_INVALID_ARG, "unexpected host exception");
  }
}

tmc_status tmc_plan_set_timing(tmc_plan_t plan, int enable) {
  if (!plan) return fail(TMC_ERR_INVALID_ARG, "plan is NULL");
  try {
    DeviceGuard g(plan->device);
    plan->timing = enable != 0;
    plan->ev_used = 0;
    plan->ev_marks.clear();
    for (int k = 0; k < TMC_KC_COUNT; ++k) {
      plan->kc_ms[k] = 0.0;
      plan->kc_n[k] = 0;
    }
    const size_t kPool = 8192;
    while (enable && plan->ev_pool.size() < kPool) {
      hipEvent_t e;
      HIP_TRY(hipEventCreate(&e));
      plan->ev_pool.push_back(e);
    }
    return TMC_OK;
  } catch (...) {
    return fail(TMC_ERR_INVALID_ARG, "unexpected host exception");
  }
}

tmc_status tmc_plan_timing(tmc_plan_t plan, int kc, double* total_ms, int64_t* launches) {
  if (!plan || !total_ms || !launches) return fail(TMC_ERR_INVALID_ARG, "NULL argument");
  if (kc < 0 || kc >= TMC_KC_COUNT) return fail(TMC_ERR_INVALID_ARG, "unknown kernel class %d", kc);
  DeviceGuard g(plan->device);
  for (auto& m : plan->ev_marks) {
    HIP_TRY(hipEventSynchronize(plan->ev_pool[m.second + 1]));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, plan->ev_pool[m.second], plan->ev_pool[m.second + 1]));
    plan->kc_ms[m.first] += ms;
    plan->kc_n[m.first] += 1;
  }
  plan->ev_marks.clear();
  plan->ev_used = 0;
  *total_ms = plan->kc_ms[kc];
  *launches = plan->kc_n[kc];
  return TMC_OK;
}

}  // extern "C"

// Fused engine host side: workspace regions, per-depth schedules grouped by the
// instantiated d-chunk count, the dependency-ordered queues of the persistent launches,
// and the shape signature the launch-shape tuner caches its choices under.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <string>
#include <tuple>

#include "fused.h"
#include "tmc_kernels.h"

namespace tmc {

int nkc_bucket(int D) {
  const int need = (D + 15) / 16;
  for (int b : kNkcBuckets)
    if (b >= need) return b;
  return -1;
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

tmc_status fused_build(FusedPlan& F, int prec, int flags, std::vector<LayerDev>& layers,
                       const std::vector<ChainDev>& chains, const std::vector<int>& pairs,
                       WsLayout& W, size_t& o, std::vector<Item>& items, std::vector<int>& ints) {
  F.prec = prec;
  F.flags = flags;
  F.n_layers = (int)layers.size();
  F.tune.persist = (flags & TMC_FLAG_PERSISTENT) != 0;
  const bool grad = !(flags & TMC_FLAG_FORWARD_ONLY);
  int64_t ev = 0, sumK = 0, sq = 0;
  for (auto& d : layers) sumK += d.K;
  for (int l : pairs) {
    LayerDev& d = layers[l];
    if (nkc_bucket(d.D) < 0) return TMC_ERR_SHAPE;
    d.ev_off = ev;
    d.dz_fused = (d.D % 4 == 0) && (d.z_off % 4 == 0) && (ev % 4 == 0) ? 1 : 0;
    if (grad) ev += (int64_t)d.K * d.D;
    d.q_off = sq;
    sq += d.Kc;
  }
  W.ev = o;
  o = align256(o + (size_t)ev * 4);
  W.lam = o;
  o = align256(o + (size_t)sumK * 4);
  W.q = o;
  o = align256(o + (size_t)sq * 8);

  int max_depth = 0;
  for (auto& c : chains) max_depth = std::max(max_depth, c.L);
  const int steps = std::max(max_depth - 1, 0);

  // level-synchronous schedules: one launch per (depth step, chunk bucket, waves), once
  // with 4-wave workgroups only and once with 8 waves where eligible
  for (int wide = 0; wide < 2; ++wide) {
  F.fwd[wide].assign(steps, {});
  F.bwd[wide].assign(steps, {});
  for (int t = 0; t < steps; ++t) {
    for (int dir = 0; dir < 2; ++dir) {
      std::map<std::pair<int, int>, std::vector<int>> groups;   // (nkc, waves) -> pairs
      for (int l : pairs) {
        const LayerDev& d = layers[l];
        const int L = chains[d.chain].L;
        const bool in_step = dir == 0 ? d.depth == L - 2 - t : d.depth == t;
        if (!in_step) continue;
        // 8 waves (256 rows / columns per workgroup) for wide layers of gradient plans;
        // 4-wave gradient sweeps of the narrow buckets share one launch per step
        const int nkc = nkc_bucket(d.D), n = dir == 0 ? d.K : d.Kc;
        const int waves = (wide && grad && fused_wide_ok(nkc) && n >= kFusedWideMin) ? 8 : 4;
        const bool multi = grad && waves == 4 && nkc <= kFusedMultiMax;
        groups[{multi ? kFusedMulti : nkc, waves}].push_back(l);
      }
      for (auto& kv : groups) {
        FusedLaunch fl;
        fl.nkc = kv.first.first;
        fl.waves = kv.first.second;
        fl.off = (int)items.size();
        const int step_rows = 32 * fl.waves;
        for (int l : kv.second) {
          const LayerDev& d = layers[l];
          const int n = dir == 0 ? d.K : d.Kc;
          for (int x = 0; x < n; x += step_rows) items.push_back({l, x});
        }
        fl.n = (int)items.size() - fl.off;
        (dir == 0 ? F.fwd[wide][t] : F.bwd[wide][t]).push_back(fl);
      }
    }
  }
  }

  // persistent queues: chains grouped by the largest chunk bucket among their pairs,
  // each group's chains ordered by decreasing work (sum of K_l K_{l+1} D_l) so that the
  // longest chains start first
  std::map<int, std::vector<int>> chain_groups;   // nkc -> chains
  std::vector<int> chain_nkc(chains.size(), 0);
  std::vector<double> cost(chains.size(), 0.0);
  for (int l : pairs) {
    const LayerDev& d = layers[l];
    chain_nkc[d.chain] = std::max(chain_nkc[d.chain], nkc_bucket(d.D));
    cost[d.chain] += (double)d.K * d.Kc * d.D;
  }
  for (size_t c = 0; c < chains.size(); ++c)
    if (chain_nkc[c] > 0) chain_groups[chain_nkc[c]].push_back((int)c);
  F.pfwd.clear();
  F.pbwd.clear();
  int heads = 0;
  for (auto& kv : chain_groups) {
    std::vector<int>& cs = kv.second;
    std::stable_sort(cs.begin(), cs.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    PersistGroup g;
    g.nkc = kv.first;
    g.off = (int)ints.size();
    g.n = (int)cs.size();
    ints.insert(ints.end(), cs.begin(), cs.end());
    g.head = heads++;
    F.pfwd.push_back(g);
  }
  for (auto g : F.pfwd) {
    g.head = heads++;
    F.pbwd.push_back(g);
  }
  // queue head counters (forward groups, then backward groups)
  W.cnt = o;
  o = align256(o + (size_t)(heads + 1) * 4);
  W.total = o;

  // row terms: every pair, and (wide schedule) the pairs an 8-wave backward does not cover
  std::vector<char> covered(layers.size(), 0);
  for (auto& step : F.bwd[1])
    for (auto& g : step)
      if (g.waves == 8)
        for (int x = g.off; x < g.off + g.n; ++x)
          if (layers[items[x].layer].dz_fused) {
            // one row partial per workgroup of the pair, within the pair's row partials
            const LayerDev& d = layers[items[x].layer];
            if ((d.Kc + 255) / 256 <= (d.K + kFusedDzRows - 1) / kFusedDzRows) covered[items[x].layer] = 1;
          }
  for (int wide = 0; wide < 2; ++wide) {
    F.dz[wide].off = (int)items.size();
    for (int l : pairs)
      if (!(wide && covered[l]))
        for (int r = 0; r < layers[l].K; r += kFusedDzRows) items.push_back({l, r});
    F.dz[wide].n = (int)items.size() - F.dz[wide].off;
  }
  for (size_t l = 0; l < layers.size(); ++l) layers[l].dz_fused = covered[l];
  F.n_pairs = (int)pairs.size();
  return TMC_OK;
}

// ---- dispatch of the runtime chunk count to the per-bucket launchers ----
#define TMC_NKC_SWITCH(nkc, CALL)                                                          \
  switch (nkc) {                                                                           \
    case 1: return CALL(1); case 2: return CALL(2); case 3: return CALL(3);                 \
    case 4: return CALL(4); case 5: return CALL(5); case 6: return CALL(6);                 \
    case 7: return CALL(7); case 8: return CALL(8); case 12: return CALL(12);               \
    case 16: return CALL(16);                                                              \
    default: break;                                                                        \
  }
static_assert(kNumNkcBuckets == 10 && kNkcBuckets[8] == 12 && kNkcBuckets[9] == 16,
              "the dispatch below lists every chunk bucket");

template <int PREC>
int fused_capacity(int dir, int nkc, bool grad, int ns) {
#define TMC_CALL(N) fused_capacity_n<PREC, N>(dir, grad, ns)
  TMC_NKC_SWITCH(nkc, TMC_CALL)
#undef TMC_CALL
  return 1;
}

template <int PREC>
hipError_t launch_fused_fwd(int nkc, int waves, bool grad, int ns, const FusedFwdPtrs& a,
                            const Item* items, int n, const FusedQueue* q, hipStream_t st) {
  if (nkc == kFusedMulti)
    return (grad && waves == 4 && !q) ? launch_fused_fwd_multi<PREC>(a, items, n, st) : hipErrorInvalidValue;
#define TMC_CALL(N) launch_fused_fwd_n<PREC, N>(waves, grad, ns, a, items, n, q, st)
  TMC_NKC_SWITCH(nkc, TMC_CALL)
#undef TMC_CALL
  return hipErrorInvalidValue;
}

template <int PREC>
hipError_t launch_fused_bwd(int nkc, int waves, const FusedBwdPtrs& a, const Item* items, int n,
                            const FusedQueue* q, hipStream_t st) {
  if (nkc == kFusedMulti)
    return (waves == 4 && !q) ? launch_fused_bwd_multi<PREC>(a, items, n, st) : hipErrorInvalidValue;
#define TMC_CALL(N) launch_fused_bwd_n<PREC, N>(waves, a, items, n, q, st)
  TMC_NKC_SWITCH(nkc, TMC_CALL)
#undef TMC_CALL
  return hipErrorInvalidValue;
}
#undef TMC_NKC_SWITCH

template int fused_capacity<TMC_FP32>(int, int, bool, int);
template int fused_capacity<TMC_BF16X3>(int, int, bool, int);
template hipError_t launch_fused_fwd<TMC_FP32>(int, int, bool, int, const FusedFwdPtrs&,
                                               const Item*, int, const FusedQueue*, hipStream_t);
template hipError_t launch_fused_fwd<TMC_BF16X3>(int, int, bool, int, const FusedFwdPtrs&,
                                                 const Item*, int, const FusedQueue*, hipStream_t);
template hipError_t launch_fused_bwd<TMC_FP32>(int, int, const FusedBwdPtrs&, const Item*, int,
                                               const FusedQueue*, hipStream_t);
template hipError_t launch_fused_bwd<TMC_BF16X3>(int, int, const FusedBwdPtrs&, const Item*, int,
                                                 const FusedQueue*, hipStream_t);

void fused_set_grids(FusedPlan& F) {
  const bool grad = !(F.flags & TMC_FLAG_FORWARD_ONLY);
  for (int dir = 0; dir < 2; ++dir)
    for (auto& g : (dir == 0 ? F.pfwd : F.pbwd)) {
      const int cap = F.prec == TMC_BF16X3 ? fused_capacity<TMC_BF16X3>(dir, g.nkc, grad, F.tune.fwd_ns)
                                           : fused_capacity<TMC_FP32>(dir, g.nkc, grad, F.tune.fwd_ns);
      const int want = cap * std::max(F.tune.grid_factor, 1);
      g.grid = std::max(1, std::min(g.n, want));   // one workgroup per chain at most
    }
}

void fused_info(const FusedPlan& F, tmc_plan_info* out) {
  out->tile_rows = 32;
  out->tile_cols = 32;
  int waves = 4;
  if (!F.tune.persist)
    for (int dir = 0; dir < 2; ++dir)
      if (dir == 0 ? F.tune.wide_fwd : F.tune.wide_bwd)
        for (auto& step : (dir == 0 ? F.fwd[1] : F.bwd[1]))
          for (auto& g : step) waves = std::max(waves, g.waves);
  out->waves_per_group = waves;   // the widest launch of the current launch shape
  out->persistent = F.tune.persist ? 1 : 0;
  out->tuned = F.tuned ? 1 : 0;
  out->wide_fwd = (!F.tune.persist && F.tune.wide_fwd) ? 1 : 0;
  out->wide_bwd = (!F.tune.persist && F.tune.wide_bwd) ? 1 : 0;
}

std::string fused_signature(const FusedPlan& F, const std::vector<LayerDev>& layers,
                            const std::vector<ChainDev>& chains) {
  // precision, flags and the multiset of (K, Kc, D bucket) pair shapes, run-length coded
  std::map<std::tuple<int, int, int>, int> hist;
  for (auto& d : layers)
    if (d.up >= 0) hist[{d.K, d.Kc, nkc_bucket(d.D)}]++;
  std::string s = "p" + std::to_string(F.prec) + "f" + std::to_string(F.flags & ~TMC_FLAG_PERSISTENT) +
                  "c" + std::to_string(chains.size());
  for (auto& kv : hist) {
    char b[64];
    snprintf(b, sizeof b, "_%dx%dx%d:%d", std::get<0>(kv.first), std::get<1>(kv.first),
             std::get<2>(kv.first), kv.second);
    s += b;
  }
  return s;
}

}  // namespace tmc

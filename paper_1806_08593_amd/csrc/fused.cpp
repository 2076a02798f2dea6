// Fused engine host side: workspace regions, per-depth schedules grouped by the
// instantiated d-chunk count, and the forward/backward launch sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>

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
                       WsLayout& W, size_t& o, std::vector<Item>& items) {
  F.prec = prec;
  F.flags = flags;
  const bool grad = !(flags & TMC_FLAG_FORWARD_ONLY);
  int64_t ev = 0, sumK = 0, sq = 0;
  for (auto& d : layers) sumK += d.K;
  for (int l : pairs) {
    LayerDev& d = layers[l];
    if (nkc_bucket(d.D) < 0) return TMC_ERR_SHAPE;
    d.ev_off = ev;
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
  W.total = o;


  int max_depth = 0;
  for (auto& c : chains) max_depth = std::max(max_depth, c.L);
  const int steps = std::max(max_depth - 1, 0);
  F.fwd.assign(steps, {});
  F.bwd.assign(steps, {});
  for (int t = 0; t < steps; ++t) {
    for (int dir = 0; dir < 2; ++dir) {
      std::map<std::pair<int, int>, std::vector<int>> groups;   // (nkc, waves) -> pairs
      for (int l : pairs) {
        const LayerDev& d = layers[l];
        const int L = chains[d.chain].L;
        const bool in_step = dir == 0 ? d.depth == L - 2 - t : d.depth == t;
        if (!in_step) continue;
        const int n = dir == 0 ? d.K : d.Kc;
        const int waves = 4;   // the staged-tile loader assumes 256 threads
        (void)n;
        groups[{nkc_bucket(d.D), waves}].push_back(l);
      }
      for (auto& kv : groups) {
        FusedLaunch fl;
        fl.nkc = kv.first.first;
        fl.waves = kv.first.second;
        fl.off = (int)items.size();
        const int step_rows = dir == 0 ? kFusedFwdRows : kFusedBwdCols;
        for (int l : kv.second) {
          const LayerDev& d = layers[l];
          const int n = dir == 0 ? d.K : d.Kc;
          for (int x = 0; x < n; x += step_rows) items.push_back({l, x});
        }
        fl.n = (int)items.size() - fl.off;
        (dir == 0 ? F.fwd[t] : F.bwd[t]).push_back(fl);
      }
    }
  }
  F.dz.off = (int)items.size();
  for (int l : pairs)
    for (int r = 0; r < layers[l].K; r += kFusedDzRows) items.push_back({l, r});
  F.dz.n = (int)items.size() - F.dz.off;
  F.n_pairs = (int)pairs.size();
  return TMC_OK;
}

void fused_info(const FusedPlan& F, tmc_plan_info* out) {
  out->tile_rows = 32;
  out->tile_cols = 32;
  int w = 0;
  for (auto& st : F.fwd)
    for (auto& g : st) w = std::max(w, g.waves);
  out->waves_per_group = w;
  (void)F;
}

}  // namespace tmc

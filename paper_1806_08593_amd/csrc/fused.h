// Fused engine interface (host side): schedules and launches of the kernels that
// recompute the pairwise factors on MFMA inside the message passes.
#pragma once

#include <vector>

#include "../../include/tmc.h"
#include "tmc_internal.h"

namespace tmc {

constexpr bool kFusedAvailable = true;

// Instantiated numbers of 16-wide d chunks (a layer of width D uses the smallest
// bucket >= ceil(D / 16); padding lanes read zeros).
constexpr int kNkcBuckets[] = {1, 2, 3, 4, 5, 6, 7, 8, 12, 16};
constexpr int kNumNkcBuckets = sizeof(kNkcBuckets) / sizeof(int);

struct FusedLaunch {
  int off = 0, n = 0, nkc = 0, waves = 4;
};

struct FusedPlan {
  int prec = 0, flags = 0;
  std::vector<std::vector<FusedLaunch>> fwd, bwd;   // [depth step][nkc group]
  FusedLaunch dz;                                   // all pairs, 64 rows per item
  int n_pairs = 0;
  int pair_ids_off = 0;                             // into the plan's int table
};

int nkc_bucket(int D);

// Lays out the fused engine's workspace regions (appending at offset `o`), assigns its
// per-layer offsets and appends its work items.  Rows per backward workgroup:
constexpr int kFusedBwdCols = 128;
constexpr int kFusedFwdRows = 128;
constexpr int kFusedDzRows = 64;
tmc_status fused_build(FusedPlan& F, int prec, int flags, std::vector<LayerDev>& layers,
                       const std::vector<ChainDev>& chains, const std::vector<int>& pairs,
                       WsLayout& W, size_t& o, std::vector<Item>& items);
void fused_info(const FusedPlan& F, tmc_plan_info* out);

// kernel launchers (k_fused_*.hip)
template <int PREC>
hipError_t launch_fused_fwd(int nkc, int waves, bool grad, const LayerDev* layers,
                            const Item* items, int n, const float* z, const float* mu,
                            const float* s, const float* u, double* qcol, double* alpha,
                            double* wmax, float* rl, float* ev, hipStream_t st);
template <int PREC>
hipError_t launch_fused_bwd(int nkc, int waves, const LayerDev* layers, const Item* items,
                            int n, const float* z, const float* mu, const float* s,
                            const double* alpha, const double* wmax,
                            const double* qcol, const float* rl, float* lam,
                            const double* dlogp, float* p, float* dmu, float* du, float* dsp,
                            hipStream_t st);
hipError_t launch_fused_dz(const LayerDev* layers, const Item* items, int n, const float* z,
                           const float* s, const float* p, const float* ev, const double* dlogp,
                           float* dz, float* dsp, hipStream_t st);
hipError_t launch_fused_fwd_init(const ChainDev* chains, int n_chains, const LayerDev* layers,
                                 const float* u, double* alpha, double* wmax, hipStream_t st);
hipError_t launch_fused_bwd_init(const ChainDev* chains, int n_chains, const LayerDev* layers,
                                 const double* alpha, const double* logp_ws, const double* dlogp,
                                 const float* rl, float* lam, float* p, float* du, float* dz,
                                 hipStream_t st);


}  // namespace tmc

// Fused engine interface (host side): schedules and launches of the kernels that
// recompute the pairwise factors on MFMA inside the message passes.
#pragma once

#include <string>
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

// A gradient launch of 4-wave workgroups that mixes the chunk buckets 1..kFusedMultiMax
// of one depth step (each workgroup runs its item's bucket; k_fused_multi.hip) has this
// chunk count in its FusedLaunch.
constexpr int kFusedMulti = 0;
constexpr int kFusedMultiMax = 4;

// Chunk counts with an 8-wave kernel (256 rows or columns per workgroup, one workgroup
// per compute unit): the widest ones with a double-buffered stage (d 97..128), whose
// 4-wave kernels already run at two waves per SIMD, so the wider workgroup costs no
// occupancy while it halves each wave's share of the staging.
constexpr bool fused_wide_ok(int nkc) { return nkc == 7 || nkc == 8; }
// Smallest layer width (rows in the forward, columns in the backward) given to 8 waves.
constexpr int kFusedWideMin = 256;

// One persistent launch: the chains ints[off .. off + n) of the plan's int table, most
// expensive first; a workgroup runs all pairs of a chain it takes.  All chains of the
// group use the chunk count nkc (the largest bucket among their pairs).
struct PersistGroup {
  int nkc = 0, off = 0, n = 0;
  int head = 0;       // index of its queue head counter
  int grid = 0;       // workgroups launched
};

// Launch-shape choices (the autotuner picks among them per plan).
struct FusedTune {
  bool persist = false;   // one persistent launch per group instead of one per depth
  int grid_factor = 1;    // persistent grid = min(items, factor x resident capacity)
  int fwd_ns = 2;         // forward-only: staged 32-sample subtiles per LDS stage (1, 2)
  bool wide_fwd = true;   // per-depth gradient forward: 8-wave workgroups where eligible
  bool wide_bwd = false;  // per-depth backward: 8-wave workgroups where eligible
};

struct FusedPlan {
  int prec = 0, flags = 0;
  // per-depth schedules [wide][depth step][(nkc, waves) group]: wide = 0 all 4-wave,
  // wide = 1 with 8-wave groups where eligible
  std::vector<std::vector<FusedLaunch>> fwd[2], bwd[2];
  std::vector<PersistGroup> pfwd, pbwd;             // persistent launches
  // row-term launches (dz and the ds row part), 64 rows per item, [wide]: wide = 0 all
  // pairs, wide = 1 only the pairs whose 8-wave backward does not write them itself
  FusedLaunch dz[2];
  int n_pairs = 0;
  int pair_ids_off = 0;                             // into the plan's int table
  int n_layers = 0;
  FusedTune tune;
  bool tuned = false;
};

int nkc_bucket(int D);

// Lays out the fused engine's workspace regions (appending at offset `o`), assigns its
// per-layer offsets and appends its work items.  Granularity of the per-layer partials
// (alpha maxima per 128 rows, ds column parts per 128 columns; a 256-wide workgroup
// writes two of each) and rows per dz item:
constexpr int kFusedBwdCols = 128;
constexpr int kFusedFwdRows = 128;
constexpr int kFusedDzRows = 64;
tmc_status fused_build(FusedPlan& F, int prec, int flags, std::vector<LayerDev>& layers,
                       const std::vector<ChainDev>& chains, const std::vector<int>& pairs,
                       WsLayout& W, size_t& o, std::vector<Item>& items, std::vector<int>& ints);
// Sets the persistent grids from the device's resident capacity (device must be current).
void fused_set_grids(FusedPlan& F);
void fused_info(const FusedPlan& F, tmc_plan_info* out);
// Signature of the plan's shapes for the tuning cache.
std::string fused_signature(const FusedPlan& F, const std::vector<LayerDev>& layers,
                            const std::vector<ChainDev>& chains);

// kernel arguments of the fused launches
struct FusedFwdPtrs {
  const LayerDev* layers;
  const float *z, *mu, *s, *u;
  double *qcol, *alpha, *wmax;
  float *rl, *ev;
};
struct FusedBwdPtrs {
  const LayerDev* layers;
  const float *z, *mu, *s;
  const double *alpha, *wmax, *qcol;
  const float* rl;
  float* lam;
  const double* dlogp;
  float *p, *dmu, *du, *dsp;
  const float* ev;   // forward's softmax-weighted means (row terms of 8-wave backwards)
  float* dz;
  int rows;          // 1: 8-wave backwards of pairs flagged dz_fused write the row terms
};
struct FusedQueue {
  const int* chains = nullptr;   // chain ids, most expensive first
  int n_chains = 0;
  int* head = nullptr;           // queue head counter (zeroed by the pass's init kernel)
  const ChainDev* cd = nullptr;
  int grid = 0;
};

// kernel launchers of one precision and chunk count (k_fused_bf16.hip, k_fused_f32.hip,
// compiled once per bucket of kNkcBuckets); q == nullptr: one workgroup per item
template <int PREC, int NKC>
int fused_capacity_n(int dir, bool grad, int ns);
template <int PREC, int NKC>
hipError_t launch_fused_fwd_n(int waves, bool grad, int ns, const FusedFwdPtrs& a,
                              const Item* items, int n, const FusedQueue* q, hipStream_t st);
template <int PREC, int NKC>
hipError_t launch_fused_bwd_n(int waves, const FusedBwdPtrs& a, const Item* items, int n,
                              const FusedQueue* q, hipStream_t st);
// the mixed-bucket gradient launches (k_fused_multi.hip)
template <int PREC>
hipError_t launch_fused_fwd_multi(const FusedFwdPtrs& a, const Item* items, int n, hipStream_t st);
template <int PREC>
hipError_t launch_fused_bwd_multi(const FusedBwdPtrs& a, const Item* items, int n, hipStream_t st);
// dispatch over the runtime chunk count (fused.cpp)
template <int PREC>
int fused_capacity(int dir, int nkc, bool grad, int ns);
template <int PREC>
hipError_t launch_fused_fwd(int nkc, int waves, bool grad, int ns, const FusedFwdPtrs& a,
                            const Item* items, int n, const FusedQueue* q, hipStream_t st);
template <int PREC>
hipError_t launch_fused_bwd(int nkc, int waves, const FusedBwdPtrs& a, const Item* items, int n,
                            const FusedQueue* q, hipStream_t st);
hipError_t launch_fused_dz(const LayerDev* layers, const Item* items, int n, const float* z,
                           const float* s, const float* p, const float* ev, const double* dlogp,
                           float* dz, float* dsp, hipStream_t st);
hipError_t launch_fused_fwd_init(const ChainDev* chains, int n_chains, const LayerDev* layers,
                                 const float* u, double* alpha, double* wmax, int* heads,
                                 int n_heads, hipStream_t st);
hipError_t launch_fused_bwd_init(const ChainDev* chains, int n_chains, const LayerDev* layers,
                                 const double* alpha, const double* logp_ws, const double* dlogp,
                                 const float* rl, float* lam, float* p, float* du, float* dz,
                                 int* heads, int n_heads, hipStream_t st);

}  // namespace tmc

// Internal declarations shared by the host runtime and the kernels of libtmc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmc {

constexpr int kPlainMaxK = 4096;      // plain engine: one column vector must fit in LDS
constexpr int kPlainMaxD = 4096;
constexpr int kFusedMaxD = 256;       // fused engine: row operands held in registers
constexpr int kFusedMaxK = 1 << 16;

// Device flag bits (plan-owned word, read by tmc_plan_check).
constexpr int kFlagNonFinite = 1;

// Per latent layer of every chain, indexed by the global layer id of the problem.
// A non-top layer l is the row layer of pair (l, l+1); its fields *_up describe
// the layer above (the column layer of that pair).
struct LayerDev {
  int32_t K, D;          // samples and dimension of this layer
  int32_t Kc;            // samples of the layer above (0 for a top layer)
  int32_t chain;         // owning chain
  int32_t up;            // global id of the layer above, -1 for a top layer
  int32_t depth;         // index within the chain (0 = next to the data)
  // caller buffer offsets (elements)
  int64_t z_off, u_off, mu_off, s_off, f_off;
  int64_t u_up_off;      // u offset of the layer above
  // workspace offsets (elements of the region they index)
  int64_t alpha_off;     // double alpha[K]
  int64_t p_off;         // T p[K]            (marginal of this layer's samples)
  int64_t rl_off;        // T rowlse[K]       (row log-sum-exp of the pair's forward)
  int64_t alpha_up_off;  // alpha of the layer above
  int64_t p_up_off;      // p of the layer above
  int64_t wf_off;        // plain: T f/G[K][Kc]
  int64_t gtz_off;       // plain: T (G^T z)[Kc][D]
  int64_t dsp_off;       // T ds partial rows [dsp_parts][D] of this pair
  int64_t ev_off;        // fused: float softmax-weighted mean of mu per row [K][D]
  int64_t q_off;         // fused: double column norms q_j of this pair [Kc]
  int64_t wmax_off;      // fused: double maxima of alpha per 128 rows [ceil(K/128)]
  int32_t dsp_parts;     // partial rows of the log-std gradient of this pair
  int32_t up_top;        // 1 if the layer above is the top of its chain
  int64_t wmax_up_off;   // fused: wmax offset of the layer above
  int32_t nwmax_up;      // fused: number of wmax partials of the layer above
  int32_t dz_fused;      // fused: an 8-wave backward of this pair may write dz and the
                         // ds row part itself (aligned rows of z and e)
  double lnKc;           // ln K of the layer above
  double kappa;          // exponent of the weights (1: the estimator of eq. (is))
};

struct ChainDev {
  int32_t L;
  int32_t first;         // global id of layer 0
  int32_t top;           // global id of layer L-1
  int32_t pad;
};

// Byte offsets of the workspace regions.
struct WsLayout {
  size_t alpha, p, rl, pairM, logp, wmax;
  size_t wf, wg, gtz, dsp;          // plain engine (dsp shared)
  size_t anchor;                    // plain engine: FP64 row anchors of the stored factors
  size_t ev, lam, q, cnt;           // fused engine (cnt: int counters of persistent launches)
  size_t total;
};

// Work item of a level-synchronous launch: a layer (pair) and a block start.
struct Item {
  int32_t layer;
  int32_t start;
};

}  // namespace tmc

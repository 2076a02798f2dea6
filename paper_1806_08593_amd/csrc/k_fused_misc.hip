// Fused engine: column norms and the start of the backward pass.
#include <math.h>

#include "dev_util.h"
#include "fused.h"
#include "fused_kernels.h"

namespace tmc {

using fused::load_f4;

// q_j = -1/2 sum_d lam_d mu_jd^2 (FP64) for every column sample of every pair; read
// by both passes so their column terms agree bitwise.  8 threads per row.
__global__ __launch_bounds__(256) void k_fused_colnorm(const LayerDev* __restrict__ Ls,
                                                       const Item* __restrict__ items,
                                                       const float* __restrict__ mu,
                                                       const float* __restrict__ s,
                                                       double* __restrict__ qcol) {
  const Item it = items[blockIdx.x];
  const LayerDev& L = Ls[it.layer];
  const int t = threadIdx.x, sub = t & 7;
  const int j = it.start + (t >> 3);
  const bool valid = j < L.Kc;
  const bool vec = (L.D % 4 == 0) && (L.mu_off % 4 == 0);
  const float* rowp = mu + L.mu_off + (int64_t)(valid ? j : 0) * L.D;
  double q = 0.0;
  for (int d = 4 * sub; d < L.D; d += 32) {
    const float4 v = load_f4(rowp, d, L.D, valid, vec);
    const float x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (d + e < L.D) q += (double)expf(-2.0f * s[L.s_off + d + e]) * (double)x[e] * (double)x[e];
  }
  q += __shfl_xor(q, 1, kWave);
  q += __shfl_xor(q, 2, kWave);
  q += __shfl_xor(q, 4, kWave);
  if (sub == 0 && valid) qcol[L.q_off + j] = -0.5 * q;
}


// p_0[i] = exp(alpha_0[i] - ln K_0 - log P), du_0 = dlogp p_0,
// Lam_0[i] = ell_0[i] - log2 p_0[i] (the row shift the first backward step uses),
// and dz of the top layer = 0.  A chain with log P = -inf gets zero marginals.
__global__ __launch_bounds__(256) void k_fused_bwd_init(const ChainDev* __restrict__ chains,
                                                        const LayerDev* __restrict__ layers,
                                                        const double* __restrict__ alpha,
                                                        const double* __restrict__ logp_ws,
                                                        const double* __restrict__ dlogp,
                                                        const float* __restrict__ rl,
                                                        float* __restrict__ lam,
                                                        float* __restrict__ p,
                                                        float* __restrict__ du,
                                                        float* __restrict__ dz) {
  const int c = blockIdx.x;
  const ChainDev ch = chains[c];
  const LayerDev& l0 = layers[ch.first];
  const double lp = logp_ws[c];
  const double g = dlogp[c];
  const double lk = log((double)l0.K);
  const bool has_pair = l0.up >= 0;
  for (int k = threadIdx.x; k < l0.K; k += blockDim.x) {
    double v;
    if (isnan(lp)) v = lp;
    else if (lp == -INFINITY) v = 0.0;
    else v = exp(alpha[l0.alpha_off + k] - lk - lp);
    const float pv = (float)v;
    p[l0.p_off + k] = pv;
    if (du) du[l0.u_off + k] = (float)(g * v);
    if (has_pair) lam[l0.rl_off + k] = (pv == 0.0f) ? INFINITY : rl[l0.rl_off + k] - log2f(pv);
  }
  if (dz) {
    const LayerDev& t = layers[ch.top];
    const int64_t n = (int64_t)t.K * t.D;
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) dz[t.z_off + e] = 0.0f;
  }
}

hipError_t launch_fused_bwd_init(const ChainDev* chains, int n_chains, const LayerDev* layers,
                                 const double* alpha, const double* logp_ws, const double* dlogp,
                                 const float* rl, float* lam, float* p, float* du, float* dz,
                                 hipStream_t st) {
  if (n_chains <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fused_bwd_init, dim3(n_chains), dim3(256), 0, st, chains, layers, alpha,
                     logp_ws, dlogp, rl, lam, p, du, dz);
  return hipGetLastError();
}

hipError_t launch_fused_colnorm(const LayerDev* layers, const Item* items, int n, const float* mu,
                                const float* s, double* qcol, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fused_colnorm, dim3(n), dim3(256), 0, st, layers, items, mu, s, qcol);
  return hipGetLastError();
}

}  // namespace tmc

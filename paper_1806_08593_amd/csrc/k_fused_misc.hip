// Fused engine: start of the backward pass and the per-pair row epilogue.
#include <math.h>

#include "dev_util.h"
#include "fused.h"

namespace tmc {

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

// Per layer pair (rows = samples of layer l), with e_i the softmax-weighted mean of
// mu from the forward pass and p the marginals:
//   dz_i  = -dlogp * lam * p_i (z_i - e_i)
//   ds    =  dlogp * [lam * (sum_i p_i z_i^2 - 2 sum_i p_i z_i e_i + sum_j p'_j mu_j^2)
//                     - sum_i p_i]
// (sum_ij G_ij (lam (z_i - mu_j)^2 - 1) with G_ij = p_i softmax_ij expanded).
__global__ __launch_bounds__(256) void k_fused_rowep(const LayerDev* __restrict__ Ls,
                                                     const int* __restrict__ pair_ids,
                                                     const float* __restrict__ z,
                                                     const float* __restrict__ mu,
                                                     const float* __restrict__ s,
                                                     const float* __restrict__ p,
                                                     const float* __restrict__ ev,
                                                     const double* __restrict__ dlogp,
                                                     float* __restrict__ dz,
                                                     float* __restrict__ dsp) {
  __shared__ float red[3][4][64];
  __shared__ float redp[kMaxWaves];
  const LayerDev& L = Ls[pair_ids[blockIdx.x]];
  const int K = L.K, Kc = L.Kc, D = L.D;
  const int tid = threadIdx.x, dl = tid % 64, rg = tid / 64;
  const float* pr = p + L.p_off;
  const float* pc = p + L.p_up_off;
  const float g = (float)dlogp[L.chain];
  float P = 0.0f;
  for (int i = tid; i < K; i += blockDim.x) P += pr[i];
  P = block_sum(P, redp);
  for (int d0 = 0; d0 < D; d0 += 64) {
    const int d = d0 + dl;
    const bool act = d < D;
    const float lam = act ? expf(-2.0f * s[L.s_off + d]) : 0.0f;
    float A = 0.0f, X = 0.0f, C = 0.0f;
    if (act) {
      for (int i = rg; i < K; i += 4) {
        const int64_t o = (int64_t)i * D + d;
        const float zv = z[L.z_off + o], e = ev[L.ev_off + o], pi = pr[i];
        if (dz) dz[L.z_off + o] = -g * lam * pi * (zv - e);
        A += pi * zv * zv;
        X += pi * zv * e;
      }
      for (int j = rg; j < Kc; j += 4) {
        const float mv = mu[L.mu_off + (int64_t)j * D + d];
        C += pc[j] * mv * mv;
      }
    }
    __syncthreads();
    red[0][rg][dl] = A;
    red[1][rg][dl] = X;
    red[2][rg][dl] = C;
    __syncthreads();
    if (rg == 0 && act && dsp) {
      const float At = red[0][0][dl] + red[0][1][dl] + red[0][2][dl] + red[0][3][dl];
      const float Xt = red[1][0][dl] + red[1][1][dl] + red[1][2][dl] + red[1][3][dl];
      const float Ct = red[2][0][dl] + red[2][1][dl] + red[2][2][dl] + red[2][3][dl];
      dsp[L.dsp_off + d] = g * (lam * (At - 2.0f * Xt + Ct) - P);
    }
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

hipError_t launch_fused_rowep(const LayerDev* layers, const int* pair_ids, int n_pairs,
                              const float* z, const float* mu, const float* s, const float* p,
                              const float* ev, const double* dlogp, float* dz, float* dsp,
                              hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fused_rowep, dim3(n_pairs), dim3(256), 0, st, layers, pair_ids, z, mu, s, p,
                     ev, dlogp, dz, dsp);
  return hipGetLastError();
}

}  // namespace tmc

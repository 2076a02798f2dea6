// Fused engine: the start of the forward and of the backward pass.
#include <math.h>

#include "dev_util.h"
#include "fused.h"
#include "fused_kernels.h"
#include "tmc_kernels.h"

namespace tmc {

// Start of the fused forward, one workgroup per chain: alpha of the top layer = u,
// and the per-128-row maxima of u_top (the same layout the forward leaves for every
// other layer), one wave per 128-row part.  Workgroup 0 clears the queue heads of the
// persistent forward launches.
__global__ __launch_bounds__(256) void k_fused_fwd_init(const ChainDev* __restrict__ chains,
                                                        const LayerDev* __restrict__ layers,
                                                        const float* __restrict__ u,
                                                        double* __restrict__ alpha,
                                                        double* __restrict__ wmax,
                                                        int* __restrict__ heads, int n_heads) {
  const ChainDev ch = chains[blockIdx.x];
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < n_heads; k += blockDim.x) heads[k] = 0;
  const LayerDev& t = layers[ch.top];
  const int nparts = (t.K + 127) / 128;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int q = w; q < nparts; q += blockDim.x >> 6) {
    double m = -INFINITY;
    for (int k = q * 128 + lane; k < min(t.K, (q + 1) * 128); k += 64) {
      const double v = t.kappa * (double)u[t.u_off + k];
      alpha[t.alpha_off + k] = v;
      m = nan_max(m, v);
    }
    m = wave_max(m);
    if (lane == 0) wmax[t.wmax_off + q] = m;
  }
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
                                                        float* __restrict__ dz,
                                                        int* __restrict__ heads, int n_heads) {
  const int c = blockIdx.x;
  const ChainDev ch = chains[c];
  if (c == 0)
    for (int k = threadIdx.x; k < n_heads; k += blockDim.x) heads[k] = 0;
  const LayerDev& l0 = layers[ch.first];
  const double lp = logp_ws[c];
  const double g = dlogp[c] * l0.kappa;   // d/d(kappa u) -> d/du
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
    // dz of the top layer is 0: a scalar head up to 16-byte alignment, float4 stores,
    // a scalar tail
    const LayerDev& t = layers[ch.top];
    const int64_t n = (int64_t)t.K * t.D;
    float* o = dz + t.z_off;
    int64_t head = (4 - (int64_t)(((uintptr_t)o / sizeof(float)) % 4)) % 4;
    if (head > n) head = n;
    const int64_t n4 = (n - head) / 4;
    float4* o4 = reinterpret_cast<float4*>(o + head);
    for (int64_t e = threadIdx.x; e < head; e += blockDim.x) o[e] = 0.0f;
    for (int64_t e = threadIdx.x; e < n4; e += blockDim.x) o4[e] = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int64_t e = head + 4 * n4 + threadIdx.x; e < n; e += blockDim.x) o[e] = 0.0f;
  }
}

// Row part of the backward of one pair, 64 rows of layer l per workgroup, with e_i the
// softmax-weighted mean of mu left by the forward and p the marginals (cw lanes of 4
// columns per row, cw the smallest power of two from 4 to 32 with 4 cw >= D, so narrow
// layers keep every lane busy; 256 / cw rows at a time):
//   dz_i = -dlogp * lam * p_i (z_i - e_i)
//   ds row part = dlogp * (lam_d * sum_i p_i z_id^2 - sum_i p_i)
// (the partial row follows the pair's column parts; fixed summation order).
__global__ __launch_bounds__(256) void k_fused_dz(const LayerDev* __restrict__ Ls,
                                                  const Item* __restrict__ items,
                                                  const float* __restrict__ z,
                                                  const float* __restrict__ s,
                                                  const float* __restrict__ p,
                                                  const float* __restrict__ ev,
                                                  const double* __restrict__ dlogp,
                                                  float* __restrict__ dz, float* __restrict__ dsp) {
  __shared__ float lam[kFusedMaxD];
  __shared__ float4 red[256];
  __shared__ float redp[kMaxWaves];
  const Item it = items[blockIdx.x];
  const LayerDev& L = Ls[it.layer];
  const int D = L.D, K = L.K, r0 = it.start;
  int cw = 4;
  while (cw < 32 && 4 * cw < D) cw *= 2;
  const int tid = threadIdx.x, c4 = tid & (cw - 1), rg = tid / cw;
  const int nrg = 256 / cw, nrr = kFusedDzRows / nrg;
  for (int d = tid; d < D; d += blockDim.x) lam[d] = expf(-2.0f * s[L.s_off + d]);
  const float* pr = p + L.p_off;
  const float g = (float)(dlogp[L.chain] * L.kappa);
  float P = 0.0f;
  if (tid < 64 && r0 + tid < K) P = pr[r0 + tid];
  P = block_sum(P, redp);     // (contains a barrier: lam is visible after it)
  const bool vec = (D % 4 == 0) && (L.z_off % 4 == 0) && (L.ev_off % 4 == 0);
  const int ncol = (L.Kc + kFusedBwdCols - 1) / kFusedBwdCols;
  float* part = dsp ? dsp + L.dsp_off + (int64_t)(ncol + r0 / kFusedDzRows) * D : nullptr;
  for (int d0 = 0; d0 < D; d0 += 4 * cw) {
    const int d = d0 + 4 * c4;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (d < D) {
      for (int rr = 0; rr < nrr; ++rr) {
        const int i = r0 + rg + nrg * rr;
        if (i < K) {
          const float pi = pr[i];
          const int64_t o = (int64_t)i * D + d;
          float zv[4], ev4[4];
          if (vec && d + 3 < D) {
            const float4 a = *reinterpret_cast<const float4*>(z + L.z_off + o);
            const float4 b = *reinterpret_cast<const float4*>(ev + L.ev_off + o);
            zv[0] = a.x; zv[1] = a.y; zv[2] = a.z; zv[3] = a.w;
            ev4[0] = b.x; ev4[1] = b.y; ev4[2] = b.z; ev4[3] = b.w;
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              zv[e] = (d + e < D) ? z[L.z_off + o + e] : 0.0f;
              ev4[e] = (d + e < D) ? ev[L.ev_off + o + e] : 0.0f;
            }
          }
          float out[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float lm = (d + e < D) ? lam[d + e] : 0.0f;
            out[e] = -g * lm * pi * (zv[e] - ev4[e]);
          }
          acc.x += pi * zv[0] * zv[0];
          acc.y += pi * zv[1] * zv[1];
          acc.z += pi * zv[2] * zv[2];
          acc.w += pi * zv[3] * zv[3];
          if (dz) {
            if (vec && d + 3 < D) {
              *reinterpret_cast<float4*>(dz + L.z_off + o) = make_float4(out[0], out[1], out[2], out[3]);
            } else {
#pragma unroll
              for (int e = 0; e < 4; ++e)
                if (d + e < D) dz[L.z_off + o + e] = out[e];
            }
          }
        }
      }
    }
    red[rg * cw + c4] = acc;
    __syncthreads();
    if (rg == 0 && d < D && part) {
      float4 t = red[c4];
      for (int q = 1; q < nrg; ++q) {
        const float4 u = red[q * cw + c4];
        t.x += u.x; t.y += u.y; t.z += u.z; t.w += u.w;
      }
      const float tv[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (d + e < D) part[d + e] = g * (lam[d + e] * tv[e] - P);
    }
    __syncthreads();
  }
}

hipError_t launch_fused_dz(const LayerDev* layers, const Item* items, int n, const float* z,
                           const float* s, const float* p, const float* ev, const double* dlogp,
                           float* dz, float* dsp, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fused_dz, dim3(n), dim3(256), 0, st, layers, items, z, s, p, ev, dlogp, dz,
                     dsp);
  return hipGetLastError();
}

hipError_t launch_fused_bwd_init(const ChainDev* chains, int n_chains, const LayerDev* layers,
                                 const double* alpha, const double* logp_ws, const double* dlogp,
                                 const float* rl, float* lam, float* p, float* du, float* dz,
                                 int* heads, int n_heads, hipStream_t st) {
  if (n_chains <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fused_bwd_init, dim3(n_chains), dim3(256), 0, st, chains, layers, alpha,
                     logp_ws, dlogp, rl, lam, p, du, dz, heads, n_heads);
  return hipGetLastError();
}

hipError_t launch_fused_fwd_init(const ChainDev* chains, int n_chains, const LayerDev* layers,
                                 const float* u, double* alpha, double* wmax, int* heads,
                                 int n_heads, hipStream_t st) {
  if (n_chains <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fused_fwd_init, dim3(n_chains), dim3(256), 0, st, chains, layers, u,
                     alpha, wmax, heads, n_heads);
  return hipGetLastError();
}

}  // namespace tmc

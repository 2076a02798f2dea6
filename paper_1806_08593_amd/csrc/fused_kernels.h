// Fused engine kernels (device templates).  The pairwise log-factor
//   f_l[i,j] = log N(z_l^i; mu_l^j, diag exp(2 s_l))
//            = r_i + c + q_j + <lam * z_i, mu_j>,
//   r_i = -1/2 sum_d lam_d z_id^2,  q_j = -1/2 sum_d lam_d mu_jd^2,
//   c   = -sum_d s_d - D/2 ln 2 pi,  lam = exp(-2 s)
// (the diagonal-Gaussian conditional of Sec. "Computational costs for TMC and IWAE")
// is never stored: the inner product runs on MFMA tile by tile and feeds an online
// log-sum-exp (forward) or the pairwise marginals (backward).  The per-sample norms
// r_i, q_j are accumulated in FP64 (O(K D) work) so the large, cancelling terms of the
// expansion never pass through FP32; the per-entry arithmetic is FP32.
//
// MFMA layouts (v_mfma_f32_32x32x16_bf16 and v_mfma_f32_32x32x2_f32 on gfx950):
//   operand fragment: lane l holds vector (l % 32) and a k-slice selected by l / 32;
//   accumulator: lane l holds column n = l % 32, rows m = 8(v/4) + 4(l/32) + v%4.
// Operands are read from the caller's row-major FP32 z and mu and split in
// registers: BF16X3 keeps x = hi + lo (both bf16) and forms hi*hi + hi*lo + lo*hi;
// FP32 feeds the values directly.  A 16-wide d chunk gives each lane 8 consecutive d
// (d = 16 kc + 8 (l/32) + s); both operands use that same k order.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "../../include/tmc.h"
#include "dev_util.h"
#include "tmc_internal.h"

namespace tmc {
namespace fused {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr float kLog2e = 1.4426950408889634f;
constexpr double kLn2 = 0.69314718055994530942;
constexpr float kRescale = 8.0f;   // lazy online-max threshold (log2 units)

template <int PREC>
struct Frag;
template <>
struct Frag<TMC_FP32> {
  float x[8];
};
template <>
struct Frag<TMC_BF16X3> {
  bf16x8 hi, lo;
};

template <int PREC>
__device__ __forceinline__ void make_frag(const float (&x)[8], Frag<PREC>& f) {
  if constexpr (PREC == TMC_FP32) {
#pragma unroll
    for (int s = 0; s < 8; ++s) f.x[s] = x[s];
  } else {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const __bf16 h = (__bf16)x[s];
      f.hi[s] = h;
      f.lo[s] = (__bf16)(x[s] - (float)h);
    }
  }
}

// acc[m][n] += sum_k A[m][k] B[k][n] over one 16-wide k chunk
template <int PREC>
__device__ __forceinline__ void mma_chunk(f32x16& acc, const Frag<PREC>& a, const Frag<PREC>& b) {
  if constexpr (PREC == TMC_FP32) {
#pragma unroll
    for (int s = 0; s < 8; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x[s], b.x[s], acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.lo, b.hi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi, b.lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi, b.hi, acc, 0, 0, 0);
  }
}

// Eight consecutive values row[d0 .. d0+7] with zeros past D (vector loads when the
// row is 16-byte aligned and the chunk is whole).
__device__ __forceinline__ void load8(const float* __restrict__ row, int d0, int D, bool vec,
                                      float (&x)[8]) {
  if (vec && d0 + 8 <= D) {
    const float4 a = *reinterpret_cast<const float4*>(row + d0);
    const float4 b = *reinterpret_cast<const float4*>(row + d0 + 4);
    x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
    x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
  } else {
#pragma unroll
    for (int s = 0; s < 8; ++s) x[s] = (d0 + s < D) ? row[d0 + s] : 0.0f;
  }
}

__device__ __forceinline__ float lam_f(const float* __restrict__ s, int d, int D) {
  return d < D ? expf(-2.0f * s[d]) : 0.0f;
}

// Column constant pieces shared by forward and backward (must agree bitwise):
// maxa = max_j alpha_{l+1}[j];  cs = -sum_d s_d - D/2 ln 2 pi.
__device__ __forceinline__ void pair_constants(const LayerDev& L, const double* __restrict__ alpha,
                                               const float* __restrict__ s, double& maxa,
                                               double& cs) {
  const int lane = threadIdx.x;
  const double* aup = alpha + L.alpha_up_off;
  double m = -INFINITY;
  for (int j = lane; j < L.Kc; j += kWave) m = nan_max(m, aup[j]);
  m = wave_max(m);
  maxa = (m == -INFINITY) ? 0.0 : m;
  double ss = 0.0;
  for (int d = lane; d < L.D; d += kWave) ss += (double)s[L.s_off + d];
  ss = wave_sum(ss);
  cs = -ss - 0.5 * (double)L.D * log(2.0 * M_PI);
}

// Loads the mu fragments of the 32 columns j0..j0+31 (lane -> column j0 + l%32) and
// returns, for the lane's own column, gamma_j = log2e (q_j + alpha_{l+1}[j] - maxa)
// (-inf past Kc).  Identical in forward and backward.
template <int PREC, int NKC>
__device__ __forceinline__ float load_cols(const LayerDev& L, const float* __restrict__ mu,
                                           const float* __restrict__ lamv,
                                           const double* __restrict__ alpha, double maxa, int j0,
                                           Frag<PREC> (&B)[NKC]) {
  const int lane = threadIdx.x, jr = lane % 32, h = lane / 32;
  const int j = j0 + jr;
  const int D = L.D;
  const bool valid = j < L.Kc;
  const float* row = mu + L.mu_off + (int64_t)(valid ? j : 0) * D;
  const bool vec = (D % 4 == 0) && (L.mu_off % 4 == 0);
  double q = 0.0;
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc) {
    float x[8];
    const int d0 = kc * 16 + 8 * h;
    if (valid) load8(row, d0, D, vec, x);
    else
#pragma unroll
      for (int t = 0; t < 8; ++t) x[t] = 0.0f;
#pragma unroll
    for (int t = 0; t < 8; ++t) q += (double)lamv[kc * 8 + t] * (double)x[t] * (double)x[t];
    make_frag<PREC>(x, B[kc]);
  }
  q = q + __shfl_xor(q, 32, kWave);
  if (!valid) return -INFINITY;
  const double g = -0.5 * q + (alpha[L.alpha_up_off + j] - maxa);
  return (float)(g * (double)kLog2e);
}

// Row operand fragments a_i = log2e * lam * z_i for rows i0..i0+31 (lane -> row
// i0 + l%32); optionally r_i = -1/2 sum lam z^2 (FP64) for the lane's row.
template <int PREC, int NKC, bool WANT_R>
__device__ __forceinline__ double load_rows(const LayerDev& L, const float* __restrict__ z,
                                            const float* __restrict__ lamv, int i0,
                                            Frag<PREC> (&A)[NKC]) {
  const int lane = threadIdx.x, ir = lane % 32, h = lane / 32;
  const int i = i0 + ir;
  const int D = L.D;
  const bool valid = i < L.K;
  const float* row = z + L.z_off + (int64_t)(valid ? i : 0) * D;
  const bool vec = (D % 4 == 0) && (L.z_off % 4 == 0);
  double r = 0.0;
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc) {
    float x[8];
    const int d0 = kc * 16 + 8 * h;
    if (valid) load8(row, d0, D, vec, x);
    else
#pragma unroll
      for (int t = 0; t < 8; ++t) x[t] = 0.0f;
    if (WANT_R) {
#pragma unroll
      for (int t = 0; t < 8; ++t) r += (double)lamv[kc * 8 + t] * (double)x[t] * (double)x[t];
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) x[t] *= lamv[kc * 8 + t] * kLog2e;
    make_frag<PREC>(x, A[kc]);
  }
  if (WANT_R) r = r + __shfl_xor(r, 32, kWave);
  return -0.5 * r;
}

// lam_d for the lane's 8 d of every chunk
template <int NKC>
__device__ __forceinline__ void lane_lams(const LayerDev& L, const float* __restrict__ s,
                                          float (&lamv)[NKC * 8]) {
  const int h = threadIdx.x / 32;
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
    for (int t = 0; t < 8; ++t) lamv[kc * 8 + t] = lam_f(s + L.s_off, kc * 16 + 8 * h + t, L.D);
}

// Transposed operand for a 32x32 block of an [n][D] row-major matrix X whose rows
// are the k index: lane (d = d0 + l%32, h = l/32) gets, for k-step t (bf16) or step v
// (fp32), the values X[k0 + kidx][d] where kidx follows the accumulator row order
// 8(v/4) + 4h + v%4.  BF16X3: one fragment per t in {0,1}, slots s -> v = 8t + s.
template <int PREC>
struct TFrag;
template <>
struct TFrag<TMC_FP32> {
  float x[16];
};
template <>
struct TFrag<TMC_BF16X3> {
  Frag<TMC_BF16X3> f[2];
};

template <int PREC>
__device__ __forceinline__ void load_tfrag(const float* __restrict__ X, int64_t off, int nrows,
                                           int D, int k0, int d0, TFrag<PREC>& T) {
  const int lane = threadIdx.x, h = lane / 32;
  const int d = d0 + lane % 32;
  float x[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int k = k0 + 8 * (v / 4) + 4 * h + (v % 4);
    x[v] = (k < nrows && d < D) ? X[off + (int64_t)k * D + d] : 0.0f;
  }
  if constexpr (PREC == TMC_FP32) {
#pragma unroll
    for (int v = 0; v < 16; ++v) T.x[v] = x[v];
  } else {
    float a[8], b[8];
#pragma unroll
    for (int s2 = 0; s2 < 8; ++s2) {
      a[s2] = x[s2];
      b[s2] = x[8 + s2];
    }
    make_frag<TMC_BF16X3>(a, T.f[0]);
    make_frag<TMC_BF16X3>(b, T.f[1]);
  }
}

// acc[d][n] += sum_k T[d][k] P[k][n] where P is this lane's accumulator column
// (16 values in accumulator row order) used as the B operand.
template <int PREC>
__device__ __forceinline__ void mma_t(f32x16& acc, const TFrag<PREC>& T, const float (&p)[16]) {
  if constexpr (PREC == TMC_FP32) {
#pragma unroll
    for (int v = 0; v < 16; ++v) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(T.x[v], p[v], acc, 0, 0, 0);
  } else {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      float a[8];
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) a[s2] = p[8 * t + s2];
      Frag<TMC_BF16X3> pf;
      make_frag<TMC_BF16X3>(a, pf);
      mma_chunk<TMC_BF16X3>(acc, T.f[t], pf);
    }
  }
}

// ---------------------------------------------------------------------------
// forward: one wave owns 32 rows of one layer pair and sweeps every column tile.
//   ell_i   = log2 sum_j exp2(S_ij + gamma_j)            (S = log2e <lam z_i, mu_j>)
//   alpha_i = u_i + r_i + c + maxa + ln2 * ell_i - ln K_{l+1}
//   e_i     = sum_j softmax_j(S_ij + gamma_j) mu_j          (GRAD: used for dz)
// ---------------------------------------------------------------------------
template <int PREC, int NKC, bool GRAD>
__global__ __launch_bounds__(64) void k_fused_fwd(const LayerDev* __restrict__ Ls,
                                                  const Item* __restrict__ items,
                                                  const float* __restrict__ z,
                                                  const float* __restrict__ mu,
                                                  const float* __restrict__ s,
                                                  const float* __restrict__ u,
                                                  double* __restrict__ alpha,
                                                  float* __restrict__ rl,
                                                  float* __restrict__ ev) {
  constexpr int ND32 = (NKC + 1) / 2;
  __shared__ __align__(16) float gam[32];
  const Item it = items[blockIdx.x];
  const LayerDev L = Ls[it.layer];
  const int lane = threadIdx.x, h = lane / 32, ir = lane % 32;
  const int i0 = it.start;

  float lamv[NKC * 8];
  lane_lams<NKC>(L, s, lamv);
  double maxa, cs;
  pair_constants(L, alpha, s, maxa, cs);

  Frag<PREC> A[NKC];
  const double r_i = load_rows<PREC, NKC, true>(L, z, lamv, i0, A);

  float m = -INFINITY, ssum = 0.0f;
  f32x16 O[GRAD ? ND32 : 1];
  if (GRAD) {
#pragma unroll
    for (int q = 0; q < ND32; ++q)
#pragma unroll
      for (int v = 0; v < 16; ++v) O[q][v] = 0.0f;
  }

  for (int j0 = 0; j0 < L.Kc; j0 += 32) {
    Frag<PREC> Bf[NKC];
    const float gj = load_cols<PREC, NKC>(L, mu, lamv, alpha, maxa, j0, Bf);
    f32x16 S;
#pragma unroll
    for (int v = 0; v < 16; ++v) S[v] = 0.0f;
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) mma_chunk<PREC>(S, Bf[kc], A[kc]);   // S[j][i]
    __syncthreads();
    if (h == 0) gam[ir] = gj;
    __syncthreads();
    float x[16];
    float tmax = -INFINITY;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 g4 = *reinterpret_cast<const float4*>(&gam[8 * q + 4 * h]);
      x[4 * q + 0] = S[4 * q + 0] + g4.x;
      x[4 * q + 1] = S[4 * q + 1] + g4.y;
      x[4 * q + 2] = S[4 * q + 2] + g4.z;
      x[4 * q + 3] = S[4 * q + 3] + g4.w;
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) tmax = nan_max(tmax, x[v]);
    tmax = nan_max(tmax, __shfl_xor(tmax, 32, kWave));
    const bool need = tmax > m + kRescale;
    if (__any(need)) {
      const float mn = need ? tmax : m;
      const float f = need ? ((m == -INFINITY) ? 0.0f : __builtin_amdgcn_exp2f(m - mn)) : 1.0f;
      ssum *= f;
      if (GRAD) {
#pragma unroll
        for (int q = 0; q < ND32; ++q)
#pragma unroll
          for (int v = 0; v < 16; ++v) O[q][v] *= f;
      }
      m = mn;
    }
    const float msafe = (m == -INFINITY) ? 0.0f : m;
    float p[16];
    float ps = 0.0f;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      p[v] = __builtin_amdgcn_exp2f(x[v] - msafe);
      ps += p[v];
    }
    ssum += ps;
    if (GRAD) {
#pragma unroll
      for (int q = 0; q < ND32; ++q) {
        TFrag<PREC> T;
        load_tfrag<PREC>(mu, L.mu_off, L.Kc, L.D, j0, 32 * q, T);
        mma_t<PREC>(O[q], T, p);
      }
    }
  }
  const float stot = ssum + __shfl_xor(ssum, 32, kWave);
  float ell;
  if (m != m || stot != stot) ell = NAN;
  else if (m == -INFINITY || stot == 0.0f) ell = -INFINITY;
  else ell = m + log2f(stot);
  const int i = i0 + ir;
  if (h == 0 && i < L.K) {
    rl[L.rl_off + i] = ell;
    alpha[L.alpha_off + i] = (double)u[L.u_off + i] + r_i + cs + maxa + kLn2 * (double)ell -
                             log((double)L.Kc);
  }
  if (GRAD && i < L.K) {
    const float inv = (stot > 0.0f) ? 1.0f / stot : 0.0f;
#pragma unroll
    for (int q = 0; q < ND32; ++q)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int d = 32 * q + 8 * (v / 4) + 4 * h + (v % 4);
        if (d < L.D) ev[L.ev_off + (int64_t)i * L.D + d] = O[q][v] * inv;
      }
  }
}

// ---------------------------------------------------------------------------
// backward: one wave owns 32 columns (samples j of layer l+1) and sweeps every row
// tile of layer l:
//   G_ij   = exp2(S_ij + gamma_j - Lam_i),   Lam_i = ell_i - log2 p_l[i]
//   p_{l+1}[j] = sum_i G_ij,  (G^T z)_j = sum_i G_ij z_i
//   dmu_j  = dlogp * lam * ((G^T z)_j - p_{l+1}[j] mu_j)
// ---------------------------------------------------------------------------
template <int PREC, int NKC>
__global__ __launch_bounds__(64) void k_fused_bwd(const LayerDev* __restrict__ Ls,
                                                  const Item* __restrict__ items,
                                                  const float* __restrict__ z,
                                                  const float* __restrict__ mu,
                                                  const float* __restrict__ s,
                                                  const double* __restrict__ alpha,
                                                  const float* __restrict__ rl,
                                                  float* __restrict__ lam_ws,
                                                  const double* __restrict__ dlogp,
                                                  float* __restrict__ p,
                                                  float* __restrict__ dmu,
                                                  float* __restrict__ du) {
  constexpr int ND32 = (NKC + 1) / 2;
  const Item it = items[blockIdx.x];
  const LayerDev L = Ls[it.layer];
  const int lane = threadIdx.x, h = lane / 32, jr = lane % 32;
  const int j0 = it.start;

  float lamv[NKC * 8];
  lane_lams<NKC>(L, s, lamv);
  double maxa, cs;
  pair_constants(L, alpha, s, maxa, cs);
  Frag<PREC> Bf[NKC];
  const float gj = load_cols<PREC, NKC>(L, mu, lamv, alpha, maxa, j0, Bf);

  f32x16 GT[ND32];
#pragma unroll
  for (int q = 0; q < ND32; ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) GT[q][v] = 0.0f;
  float csum = 0.0f;
  const float* lamrow = lam_ws + L.rl_off;   // Lam shares the per-layer indexing of rl

  for (int i0 = 0; i0 < L.K; i0 += 32) {
    Frag<PREC> A[NKC];
    (void)load_rows<PREC, NKC, false>(L, z, lamv, i0, A);
    f32x16 S;
#pragma unroll
    for (int v = 0; v < 16; ++v) S[v] = 0.0f;
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc) mma_chunk<PREC>(S, A[kc], Bf[kc]);   // S[i][j]
    float g[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ib = i0 + 8 * q + 4 * h;
      float lm[4];
      if (ib + 3 < L.K && ((L.rl_off + ib) % 4 == 0)) {
        const float4 t = *reinterpret_cast<const float4*>(lamrow + ib);
        lm[0] = t.x; lm[1] = t.y; lm[2] = t.z; lm[3] = t.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) lm[e] = (ib + e < L.K) ? lamrow[ib + e] : INFINITY;
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        g[4 * q + e] = __builtin_amdgcn_exp2f(S[4 * q + e] + gj - lm[e]);
        csum += g[4 * q + e];
      }
    }
#pragma unroll
    for (int q = 0; q < ND32; ++q) {
      TFrag<PREC> T;
      load_tfrag<PREC>(z, L.z_off, L.K, L.D, i0, 32 * q, T);
      mma_t<PREC>(GT[q], T, g);
    }
  }
  const float ctot = csum + __shfl_xor(csum, 32, kWave);
  const int j = j0 + jr;
  const double gl = dlogp[L.chain];
  if (j < L.Kc) {
    if (h == 0) {
      p[L.p_up_off + j] = ctot;
      if (du) du[L.u_up_off + j] = (float)(gl * (double)ctot);
      const LayerDev& U = Ls[L.up];
      if (U.up >= 0) {
        const float ell = rl[U.rl_off + j];
        lam_ws[U.rl_off + j] = (ctot == 0.0f) ? INFINITY : ell - log2f(ctot);
      }
    }
    if (dmu) {
      const float g32 = (float)gl;
#pragma unroll
      for (int q = 0; q < ND32; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int d = 32 * q + 8 * (v / 4) + 4 * h + (v % 4);
          if (d < L.D) {
            const int64_t mi = L.mu_off + (int64_t)j * L.D + d;
            const float lam = expf(-2.0f * s[L.s_off + d]);
            dmu[mi] = g32 * lam * (GT[q][v] - ctot * mu[mi]);
          }
        }
    }
  }
}

}  // namespace fused
}  // namespace tmc

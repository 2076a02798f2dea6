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

#include <type_traits>

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
constexpr int kFusedRowsPerGroup = 128;   // forward rows per workgroup (4 waves x 32)

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

// Column constant pieces shared by forward and backward (identical in both):
// maxa = max_j alpha_{l+1}[j], reduced from the per-workgroup maxima the pass that
// wrote alpha_{l+1} left in wmax (fixed order); cs = -sum_d s_d - D/2 ln 2 pi (per
// pair, written at the start of the forward).
__device__ __forceinline__ void pair_constants(const LayerDev& L, const LayerDev& U,
                                               const double* __restrict__ wmax,
                                               const double* __restrict__ pair_c, double& maxa,
                                               double& cs) {
  const int n = (U.K + kFusedRowsPerGroup - 1) / kFusedRowsPerGroup;
  double m = -INFINITY;
  for (int k = 0; k < n; ++k) m = nan_max(m, wmax[U.wmax_off + k]);
  maxa = (m == -INFINITY) ? 0.0 : m;
  cs = pair_c[L.up - 1];
}

// Transposed operand of a 32-row tile X[k][d] (rows k are the contraction index):
// lane (d = 32q + l%32, h = l/32) holds, for step v (fp32) or k-step t with slots
// s -> v = 8t + s (bf16), the value X[8(v/4) + 4h + v%4][d] -- the same k order as
// the rows of an accumulator tile, so an accumulator column can be the other operand.
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
// LDS staging of NS operand tiles of 32 samples (rows of mu or of z), written once
// per workgroup and read by all four waves.  Per 32-row subtile:
//   row-major copy: fragments with the d chunk along k (factor GEMM);
//   d-major copy:   fragments with the tile rows along k (G^T z, softmax * mu),
//                   row r stored at column perm(r) (bits 2 and 3 of r swapped) so the
//                   8 rows a lane needs for one k-step are adjacent.
// Every fragment is one or two 128-bit LDS reads.  BF16X3 keeps two bf16 planes
// (hi, lo), FP32 one float plane.  NS independent subtiles give each wave NS
// independent MFMA chains per stage.
// ---------------------------------------------------------------------------
template <int PREC, int NKC, int NS_>
struct TileSmem {
  static constexpr int NS = NS_;
  static constexpr int DP = NKC * 16;               // padded width
  static constexpr int ND32 = (NKC + 1) / 2;        // 32-wide d blocks
  static constexpr int DT = ND32 * 32;              // rows of the d-major copy
  static constexpr bool BF = PREC == TMC_BF16X3;
  static constexpr int NPL = BF ? 2 : 1;
  static constexpr int RS = BF ? DP + 8 : DP + 4;   // row stride (elements)
  static constexpr int CS = BF ? 40 : 36;           // d-major stride (elements)
  static constexpr int ROWN = 32 * RS, COLN = DT * CS;
  typedef typename std::conditional<BF, __bf16, float>::type E;
  E row[NPL][NS * ROWN];
  E col[NPL][NS * COLN];
  float lamf[DP];        // lam_d = exp(-2 s_d)            (0 past D)
  float lam2[DP];        // log2(e) * lam_d
  float gam[NS * 32];    // column terms of the staged tiles
  float lamT[NS * 32];   // row shifts of the staged tiles (backward)
  double wm[4];          // per-wave maxima of alpha (forward)
};

__device__ __forceinline__ int tile_perm(int r) {
  return (r & 0x13) | ((r & 4) << 1) | ((r & 8) >> 1);
}

template <int PREC, int NKC, int NS>
__device__ __forceinline__ void tile_init(TileSmem<PREC, NKC, NS>& T, const LayerDev& L,
                                          const float* __restrict__ s) {
  using TS = TileSmem<PREC, NKC, NS>;
  for (int d = threadIdx.x; d < TS::DP; d += blockDim.x) {
    const float lf = lam_f(s + L.s_off, d, L.D);
    T.lamf[d] = lf;
    T.lam2[d] = lf * kLog2e;
  }
  for (int e = threadIdx.x; e < TS::NPL * TS::NS * TS::COLN; e += blockDim.x)
    (&T.col[0][0])[e] = (typename TS::E)0.0f;
}

// Register stage of NS tiles (blockDim 256): thread t serves row t / 8 of every
// subtile and float4 columns 4 (t % 8 + 8 m).  Rows >= nvalid and d >= D read as zero.
template <int NKC, int NS_>
struct TilePrefetch {
  static constexpr int NS = NS_;
  static constexpr int NF = (NKC + 1) / 2;
  float4 v[NS][NF];
  double a[NS], q[NS];   // column tiles: alpha_{l+1}[j] and stored q_j (thread t%8 == 0)
  float lam;         // backward: row shift of row t (t < 32 NS)
};

__device__ __forceinline__ float4 load_f4(const float* __restrict__ rowp, int d, int D, bool valid,
                                          bool vec) {
  if (valid && vec && d < D) return *reinterpret_cast<const float4*>(rowp + d);
  float4 r;
  r.x = (valid && d + 0 < D) ? rowp[d + 0] : 0.0f;
  r.y = (valid && d + 1 < D) ? rowp[d + 1] : 0.0f;
  r.z = (valid && d + 2 < D) ? rowp[d + 2] : 0.0f;
  r.w = (valid && d + 3 < D) ? rowp[d + 3] : 0.0f;
  return r;
}

// Column tiles of pair L: mu rows r0.. (samples of layer l+1), their alpha and
// (when qcol is given) the stored q.
template <int NKC, int NS>
__device__ __forceinline__ void fetch_cols(TilePrefetch<NKC, NS>& pf, const LayerDev& L,
                                           const float* __restrict__ mu,
                                           const double* __restrict__ alpha,
                                           const double* __restrict__ qcol, int r0) {
  const int t = threadIdx.x, sub = t & 7;
  const bool vec = (L.D % 4 == 0) && (L.mu_off % 4 == 0);
#pragma unroll
  for (int sb = 0; sb < NS; ++sb) {
    const int gr = r0 + 32 * sb + (t >> 3);
    const bool valid = gr < L.Kc;
    const float* rowp = mu + L.mu_off + (int64_t)(valid ? gr : 0) * L.D;
#pragma unroll
    for (int m = 0; m < TilePrefetch<NKC, NS>::NF; ++m)
      pf.v[sb][m] = load_f4(rowp, 4 * (sub + 8 * m), L.D, valid, vec);
    if (sub == 0 && valid) {
      pf.a[sb] = alpha[L.alpha_up_off + gr];
      if (qcol) pf.q[sb] = qcol[L.q_off + gr];
    }
  }
}

// Row tiles of pair L (samples of layer l): z rows r0.. and their shifts Lam.
template <int NKC, int NS>
__device__ __forceinline__ void fetch_rows(TilePrefetch<NKC, NS>& pf, const LayerDev& L,
                                           const float* __restrict__ z,
                                           const float* __restrict__ lamrow, int r0) {
  const int t = threadIdx.x, sub = t & 7;
  const bool vec = (L.D % 4 == 0) && (L.z_off % 4 == 0);
#pragma unroll
  for (int sb = 0; sb < NS; ++sb) {
    const int gr = r0 + 32 * sb + (t >> 3);
    const bool valid = gr < L.K;
    const float* rowp = z + L.z_off + (int64_t)(valid ? gr : 0) * L.D;
#pragma unroll
    for (int m = 0; m < TilePrefetch<NKC, NS>::NF; ++m)
      pf.v[sb][m] = load_f4(rowp, 4 * (sub + 8 * m), L.D, valid, vec);
  }
  if (t < 32 * NS) pf.lam = (r0 + t < L.K) ? lamrow[r0 + t] : INFINITY;
}

// Writes fetched tiles to LDS: row-major copy = x * lam2 when `scale`, else x;
// d-major copy (when `want_col`) = x.
template <int PREC, int NKC, int NS>
__device__ __forceinline__ void tile_store(TileSmem<PREC, NKC, NS>& T,
                                           const TilePrefetch<NKC, NS>& pf, bool scale,
                                           bool want_col) {
  using TS = TileSmem<PREC, NKC, NS>;
  const int t = threadIdx.x, r = t >> 3, sub = t & 7;
  const int pr = tile_perm(r);
#pragma unroll
  for (int sb = 0; sb < TS::NS; ++sb) {
#pragma unroll
    for (int m = 0; m < TilePrefetch<NKC, NS>::NF; ++m) {
      const int k = sub + 8 * m;
      if (k >= TS::DP / 4) break;
      const int d = 4 * k;
      const float x[4] = {pf.v[sb][m].x, pf.v[sb][m].y, pf.v[sb][m].z, pf.v[sb][m].w};
      const int ro = sb * TS::ROWN + r * TS::RS + d;
      const int co = sb * TS::COLN + d * TS::CS + pr;
      if constexpr (TS::BF) {
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        bf16x4 xh, xl;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const __bf16 hb = (__bf16)x[e];
          xh[e] = hb;
          xl[e] = (__bf16)(x[e] - (float)hb);
        }
        if (want_col) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            T.col[0][co + e * TS::CS] = xh[e];
            T.col[1][co + e * TS::CS] = xl[e];
          }
        }
        if (scale) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float y = x[e] * T.lam2[d + e];
            const __bf16 hb = (__bf16)y;
            xh[e] = hb;
            xl[e] = (__bf16)(y - (float)hb);
          }
        }
        *reinterpret_cast<bf16x4*>(&T.row[0][ro]) = xh;
        *reinterpret_cast<bf16x4*>(&T.row[1][ro]) = xl;
      } else {
        if (want_col) {
#pragma unroll
          for (int e = 0; e < 4; ++e) T.col[0][co + e * TS::CS] = x[e];
        }
        float y[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) y[e] = scale ? x[e] * T.lam2[d + e] : x[e];
        *reinterpret_cast<float4*>(&T.row[0][ro]) = make_float4(y[0], y[1], y[2], y[3]);
      }
    }
  }
}

// q_j = -1/2 sum_d lam_d mu_jd^2 (FP64) of the fetched column row of subtile sb,
// complete in all 8 threads serving the row (fixed reduction order).
template <int PREC, int NKC, int NS>
__device__ __forceinline__ double tile_colq(const TileSmem<PREC, NKC, NS>& T,
                                            const TilePrefetch<NKC, NS>& pf, int sb) {
  using TS = TileSmem<PREC, NKC, NS>;
  const int sub = threadIdx.x & 7;
  double q = 0.0;
#pragma unroll
  for (int m = 0; m < TilePrefetch<NKC, NS>::NF; ++m) {
    const int k = sub + 8 * m;
    if (k >= TS::DP / 4) break;
    const int d = 4 * k;
    const float x[4] = {pf.v[sb][m].x, pf.v[sb][m].y, pf.v[sb][m].z, pf.v[sb][m].w};
#pragma unroll
    for (int e = 0; e < 4; ++e) q += (double)T.lamf[d + e] * (double)x[e] * (double)x[e];
  }
  q += __shfl_xor(q, 1, kWave);
  q += __shfl_xor(q, 2, kWave);
  q += __shfl_xor(q, 4, kWave);
  return -0.5 * q;
}

// gamma_j = log2(e) (q_j + alpha_{l+1}[j] - maxa) of staged column j (-inf past Kc).
template <int PREC, int NKC, int NS>
__device__ __forceinline__ void tile_gamma(TileSmem<PREC, NKC, NS>& T, double a, double q,
                                           const LayerDev& L, int sb, int j, double maxa) {
  const int t = threadIdx.x, r = t >> 3;
  if ((t & 7) == 0)
    T.gam[32 * sb + r] = (j < L.Kc) ? (float)((q + (a - maxa)) * (double)kLog2e) : -INFINITY;
}

// Fragment of staged row (lane % 32) of subtile sb for d chunk kc (d = 16 kc + 8 h + s).
template <int PREC, int NKC, int NS>
__device__ __forceinline__ void tile_row_frag(const TileSmem<PREC, NKC, NS>& T, int sb, int kc,
                                              Frag<PREC>& f) {
  using TS = TileSmem<PREC, NKC, NS>;
  const int lane = threadIdx.x & 63, r = lane & 31, h = lane >> 5;
  const int o = sb * TS::ROWN + r * TS::RS + kc * 16 + 8 * h;
  if constexpr (TS::BF) {
    f.hi = *reinterpret_cast<const bf16x8*>(&T.row[0][o]);
    f.lo = *reinterpret_cast<const bf16x8*>(&T.row[1][o]);
  } else {
    const float4 a = *reinterpret_cast<const float4*>(&T.row[0][o]);
    const float4 b = *reinterpret_cast<const float4*>(&T.row[0][o + 4]);
    f.x[0] = a.x; f.x[1] = a.y; f.x[2] = a.z; f.x[3] = a.w;
    f.x[4] = b.x; f.x[5] = b.y; f.x[6] = b.z; f.x[7] = b.w;
  }
}

// Transposed fragment of subtile sb for d block q (lane -> d = 32 q + lane % 32).
template <int PREC, int NKC, int NS>
__device__ __forceinline__ void tile_col_frag(const TileSmem<PREC, NKC, NS>& T, int sb, int q,
                                              TFrag<PREC>& f) {
  using TS = TileSmem<PREC, NKC, NS>;
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const int o = sb * TS::COLN + (32 * q + (lane & 31)) * TS::CS + 8 * h;
  if constexpr (TS::BF) {
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
      f.f[tt].hi = *reinterpret_cast<const bf16x8*>(&T.col[0][o + 16 * tt]);
      f.f[tt].lo = *reinterpret_cast<const bf16x8*>(&T.col[1][o + 16 * tt]);
    }
  } else {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const float4 a = *reinterpret_cast<const float4*>(&T.col[0][o + 4 * (g & 1) + 16 * (g >> 1)]);
      f.x[4 * g + 0] = a.x; f.x[4 * g + 1] = a.y; f.x[4 * g + 2] = a.z; f.x[4 * g + 3] = a.w;
    }
  }
}

// Row operand of the wave's rows i0 .. i0+31 straight from global memory:
// a_i = log2(e) lam z_i as fragments, and r_i = -1/2 sum_d lam_d z_id^2 (FP64).
template <int PREC, int NKC, int NS>
__device__ __forceinline__ double wave_rows(const TileSmem<PREC, NKC, NS>& T, const LayerDev& L,
                                            const float* __restrict__ z, int i0,
                                            Frag<PREC> (&A)[NKC]) {
  const int lane = threadIdx.x & 63, ir = lane & 31, h = lane >> 5;
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
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      r += (double)T.lamf[d0 + t] * (double)x[t] * (double)x[t];
      x[t] *= T.lam2[d0 + t];
    }
    make_frag<PREC>(x, A[kc]);
  }
  r = r + __shfl_xor(r, 32, kWave);
  return -0.5 * r;
}

// ---------------------------------------------------------------------------
// forward: a workgroup of 4 waves owns 128 rows of one layer pair (wave w: rows
// start + 32 w ..); the samples of the layer above are staged NS x 32 at a time in
// LDS (prefetched into registers one stage ahead) and swept by all waves.
//   ell_i   = log2 sum_j exp2(S_ij + gamma_j)          (S = log2e <lam z_i, mu_j>)
//   alpha_i = u_i + r_i + c + maxa + ln2 * ell_i - ln K_{l+1}
//   e_i     = sum_j softmax_j(S_ij + gamma_j) mu_j        (GRAD: used for dz)
// ---------------------------------------------------------------------------
template <int PREC, int NKC, bool GRAD, int NS>
__global__ __launch_bounds__(256, (NKC <= 8 ? 2 : 1)) void k_fused_fwd(const LayerDev* __restrict__ Ls,
                                                   const Item* __restrict__ items,
                                                   const float* __restrict__ z,
                                                   const float* __restrict__ mu,
                                                   const float* __restrict__ s,
                                                   const float* __restrict__ u,
                                                   double* __restrict__ qcol,
                                                   double* __restrict__ alpha,
                                                   double* __restrict__ wmax,
                                                   const double* __restrict__ pair_c,
                                                   float* __restrict__ rl,
                                                   float* __restrict__ ev) {
  using TS = TileSmem<PREC, NKC, NS>;
  constexpr int ND32 = TS::ND32;
  __shared__ __align__(16) TS T;
  const Item it = items[blockIdx.x];
  const LayerDev L = Ls[it.layer];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, h = lane >> 5, ir = lane & 31;
  double maxa, cs;
  pair_constants(L, Ls[L.up], wmax, pair_c, maxa, cs);
  tile_init<PREC, NKC, NS>(T, L, s);
  __syncthreads();

  const int i0 = it.start + 32 * w;
  const bool active = i0 < L.K;
  Frag<PREC> A[NKC];
  double r_i = 0.0;
  if (active) r_i = wave_rows<PREC, NKC, NS>(T, L, z, i0, A);
  TilePrefetch<NKC, NS> pf;
  fetch_cols<NKC, NS>(pf, L, mu, alpha, nullptr, 0);

  float m = -INFINITY, ssum = 0.0f;
  f32x16 O[GRAD ? ND32 : 1];
#pragma unroll
  for (int q = 0; q < (GRAD ? ND32 : 1); ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) O[q][v] = 0.0f;

  // The forward computes the column norms q_j (FP64) of every column it stages; the
  // workgroup that starts at row 0 stores them for the backward.
  const bool qwriter = GRAD && it.start == 0;
  for (int j0 = 0; j0 < L.Kc; j0 += 32 * NS) {
    __syncthreads();                       // waits for the prefetch and for readers of T
    tile_store<PREC, NKC, NS>(T, pf, false, GRAD);
#pragma unroll
    for (int sb = 0; sb < NS; ++sb) {
      const int j = j0 + 32 * sb + (tid >> 3);
      const double qj = tile_colq<PREC, NKC, NS>(T, pf, sb);
      tile_gamma<PREC, NKC, NS>(T, pf.a[sb], qj, L, sb, j, maxa);
      if (qwriter && (tid & 7) == 0 && j < L.Kc) qcol[L.q_off + j] = qj;
    }
    __syncthreads();
    if (j0 + 32 * NS < L.Kc) fetch_cols<NKC, NS>(pf, L, mu, alpha, nullptr, j0 + 32 * NS);
    if (!active) continue;
    f32x16 S[NS];
#pragma unroll
    for (int sb = 0; sb < NS; ++sb)
#pragma unroll
      for (int v = 0; v < 16; ++v) S[sb][v] = 0.0f;
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
      for (int sb = 0; sb < NS; ++sb) {
        Frag<PREC> Bf;
        tile_row_frag<PREC, NKC, NS>(T, sb, kc, Bf);
        mma_chunk<PREC>(S[sb], Bf, A[kc]);     // S[j][i]
      }
    float x[NS][16];
    float tmax = -INFINITY;
#pragma unroll
    for (int sb = 0; sb < NS; ++sb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 g4 = *reinterpret_cast<const float4*>(&T.gam[32 * sb + 8 * q + 4 * h]);
        x[sb][4 * q + 0] = S[sb][4 * q + 0] + g4.x;
        x[sb][4 * q + 1] = S[sb][4 * q + 1] + g4.y;
        x[sb][4 * q + 2] = S[sb][4 * q + 2] + g4.z;
        x[sb][4 * q + 3] = S[sb][4 * q + 3] + g4.w;
      }
    // (a NaN entry is dropped by fmaxf here but reaches ssum through exp2 below)
#pragma unroll
    for (int sb = 0; sb < NS; ++sb)
#pragma unroll
      for (int v = 0; v < 16; ++v) tmax = fmaxf(tmax, x[sb][v]);
    tmax = fmaxf(tmax, __shfl_xor(tmax, 32, kWave));
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
    float p[NS][16];
    float ps = 0.0f;
#pragma unroll
    for (int sb = 0; sb < NS; ++sb)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        p[sb][v] = __builtin_amdgcn_exp2f(x[sb][v] - msafe);
        ps += p[sb][v];
      }
    ssum += ps;
    if (GRAD) {
#pragma unroll
      for (int q = 0; q < ND32; ++q)
#pragma unroll
        for (int sb = 0; sb < NS; ++sb) {
          TFrag<PREC> Tf;
          tile_col_frag<PREC, NKC, NS>(T, sb, q, Tf);
          mma_t<PREC>(O[q], Tf, p[sb]);
        }
    }
  }
  const float stot = ssum + __shfl_xor(ssum, 32, kWave);
  float ell;
  if (m != m || stot != stot) ell = NAN;
  else if (m == -INFINITY || stot == 0.0f) ell = -INFINITY;
  else ell = m + log2f(stot);
  const int i = active ? i0 + ir : L.K;
  const double a_i = (double)u[L.u_off + (i < L.K ? i : 0)] + r_i + cs + maxa +
                     kLn2 * (double)ell - log((double)L.Kc);
  if (h == 0 && i < L.K) {
    rl[L.rl_off + i] = ell;
    alpha[L.alpha_off + i] = a_i;
  }
  // this workgroup's max_i alpha_l[i], for the next step's column terms
  const double wm = wave_max(i < L.K ? a_i : -INFINITY);
  if (lane == 0) T.wm[w] = wm;
  __syncthreads();
  if (tid == 0)
    wmax[L.wmax_off + it.start / kFusedRowsPerGroup] =
        nan_max(nan_max(T.wm[0], T.wm[1]), nan_max(T.wm[2], T.wm[3]));
  if (GRAD && i < L.K) {
    const float inv = (stot > 0.0f) ? 1.0f / stot : 0.0f;
    float* erow = ev + L.ev_off + (int64_t)i * L.D;
    const bool vec = (L.D % 4 == 0) && (L.ev_off % 4 == 0);
#pragma unroll
    for (int q = 0; q < ND32; ++q)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int d = 32 * q + 8 * g + 4 * h;
        const float4 o4 = make_float4(O[q][4 * g] * inv, O[q][4 * g + 1] * inv,
                                      O[q][4 * g + 2] * inv, O[q][4 * g + 3] * inv);
        if (vec && d + 3 < L.D) {
          *reinterpret_cast<float4*>(erow + d) = o4;
        } else {
          if (d + 0 < L.D) erow[d + 0] = o4.x;
          if (d + 1 < L.D) erow[d + 1] = o4.y;
          if (d + 2 < L.D) erow[d + 2] = o4.z;
          if (d + 3 < L.D) erow[d + 3] = o4.w;
        }
      }
  }
}

// ---------------------------------------------------------------------------
// backward: a workgroup of 4 waves owns 128 columns (samples j of layer l+1; wave
// w: columns start + 32 w ..) and sweeps every row of layer l, NS x 32 rows per LDS
// stage (scaled row-major copy for the factor, raw d-major copy for G^T z):
//   G_ij   = exp2(S_ij + gamma_j - Lam_i),   Lam_i = ell_i - log2 p_l[i]
//   p_{l+1}[j] = sum_i G_ij,  (G^T z)_j = sum_i G_ij z_i
//   dmu_j  = dlogp * lam * ((G^T z)_j - p_{l+1}[j] mu_j)
// and writes the column part of the log-std gradient of its columns,
//   dlogp * lam * sum_j (p_{l+1}[j] mu_j^2 - 2 mu_j (G^T z)_j)
// (sum_ij G_ij (z_i - mu_j)^2 expanded; the row terms come from k_fused_dz).
// ---------------------------------------------------------------------------
template <int PREC, int NKC, int NS>
__global__ __launch_bounds__(256, (NKC <= 8 ? 2 : 1)) void k_fused_bwd(const LayerDev* __restrict__ Ls,
                                                   const Item* __restrict__ items,
                                                   const float* __restrict__ z,
                                                   const float* __restrict__ mu,
                                                   const float* __restrict__ s,
                                                   const double* __restrict__ alpha,
                                                   const double* __restrict__ wmax,
                                                   const double* __restrict__ pair_c,
                                                   const double* __restrict__ qcol,
                                                   const float* __restrict__ rl,
                                                   float* __restrict__ lam_ws,
                                                   const double* __restrict__ dlogp,
                                                   float* __restrict__ p,
                                                   float* __restrict__ dmu,
                                                   float* __restrict__ du,
                                                   float* __restrict__ dsp) {
  using TS = TileSmem<PREC, NKC, NS>;
  constexpr int ND32 = TS::ND32;
  __shared__ __align__(16) TS T;
  __shared__ float accD[TS::DT];
  const Item it = items[blockIdx.x];
  const LayerDev L = Ls[it.layer];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, h = lane >> 5, jr = lane & 31;
  tile_init<PREC, NKC, NS>(T, L, s);
  for (int d = tid; d < TS::DT; d += blockDim.x) accD[d] = 0.0f;
  double maxa, cs;
  pair_constants(L, Ls[L.up], wmax, pair_c, maxa, cs);
  const int jw = it.start + 32 * w;
  const bool active = jw < L.Kc;
  const float g32 = (float)dlogp[L.chain];

  // the waves' column operands and column terms, staged NS waves at a time
  Frag<PREC> Bf[NKC];
  float gj = -INFINITY;
  for (int w0 = 0; w0 < 4; w0 += NS) {
    const int jt = it.start + 32 * w0;
    if (jt >= L.Kc) break;
    TilePrefetch<NKC, NS> pm;
    fetch_cols<NKC, NS>(pm, L, mu, alpha, qcol, jt);
    __syncthreads();
    tile_store<PREC, NKC, NS>(T, pm, false, false);
#pragma unroll
    for (int sb = 0; sb < NS; ++sb)
      tile_gamma<PREC, NKC, NS>(T, pm.a[sb], pm.q[sb], L, sb, jt + 32 * sb + (tid >> 3), maxa);
    __syncthreads();
    if (w >= w0 && w < w0 + NS) {
#pragma unroll
      for (int kc = 0; kc < NKC; ++kc) tile_row_frag<PREC, NKC, NS>(T, w - w0, kc, Bf[kc]);
      gj = T.gam[32 * (w - w0) + jr];
    }
  }

  f32x16 GT[ND32];
#pragma unroll
  for (int q = 0; q < ND32; ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) GT[q][v] = 0.0f;
  float csum = 0.0f;
  const float* lamrow = lam_ws + L.rl_off;   // Lam shares the per-layer indexing of rl

  TilePrefetch<NKC, NS> pf;
  fetch_rows<NKC, NS>(pf, L, z, lamrow, 0);
  for (int i0 = 0; i0 < L.K; i0 += 32 * NS) {
    __syncthreads();                       // waits for the prefetch and for readers of T
    tile_store<PREC, NKC, NS>(T, pf, true, true);
    if (tid < 32 * NS) T.lamT[tid] = pf.lam;
    __syncthreads();
    if (i0 + 32 * NS < L.K) fetch_rows<NKC, NS>(pf, L, z, lamrow, i0 + 32 * NS);
    if (!active) continue;
    f32x16 S[NS];
#pragma unroll
    for (int sb = 0; sb < NS; ++sb)
#pragma unroll
      for (int v = 0; v < 16; ++v) S[sb][v] = 0.0f;
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
      for (int sb = 0; sb < NS; ++sb) {
        Frag<PREC> Af;
        tile_row_frag<PREC, NKC, NS>(T, sb, kc, Af);
        mma_chunk<PREC>(S[sb], Af, Bf[kc]);    // S[i][j]
      }
    float g[NS][16];
#pragma unroll
    for (int sb = 0; sb < NS; ++sb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 l4 = *reinterpret_cast<const float4*>(&T.lamT[32 * sb + 8 * q + 4 * h]);
        g[sb][4 * q + 0] = __builtin_amdgcn_exp2f(S[sb][4 * q + 0] + gj - l4.x);
        g[sb][4 * q + 1] = __builtin_amdgcn_exp2f(S[sb][4 * q + 1] + gj - l4.y);
        g[sb][4 * q + 2] = __builtin_amdgcn_exp2f(S[sb][4 * q + 2] + gj - l4.z);
        g[sb][4 * q + 3] = __builtin_amdgcn_exp2f(S[sb][4 * q + 3] + gj - l4.w);
      }
#pragma unroll
    for (int sb = 0; sb < NS; ++sb)
#pragma unroll
      for (int v = 0; v < 16; ++v) csum += g[sb][v];
#pragma unroll
    for (int q = 0; q < ND32; ++q)
#pragma unroll
      for (int sb = 0; sb < NS; ++sb) {
        TFrag<PREC> Tf;
        tile_col_frag<PREC, NKC, NS>(T, sb, q, Tf);
        mma_t<PREC>(GT[q], Tf, g[sb]);
      }
  }

  // ---- column epilogue: marginals of layer l+1, dmu, column part of ds ----
  const float ctot = csum + __shfl_xor(csum, 32, kWave);
  const int j = jw + jr;
  const bool jv = active && j < L.Kc;
  const double gl = dlogp[L.chain];
  if (jv && h == 0) {
    p[L.p_up_off + j] = ctot;
    if (du) du[L.u_up_off + j] = (float)(gl * (double)ctot);
    const LayerDev& U = Ls[L.up];
    if (U.up >= 0) {
      const float ell = rl[U.rl_off + j];
      lam_ws[U.rl_off + j] = (ctot == 0.0f) ? INFINITY : ell - log2f(ctot);
    }
  }
  // per-lane column terms p'_j mu_jd^2 - 2 mu_jd (G^T z)_jd, reduced over the wave's
  // 32 columns through LDS (wave by wave, fixed order)
  float colt[ND32][16];
  {
    const bool mvec = (L.D % 4 == 0) && (L.mu_off % 4 == 0);
    const float* murow = mu + L.mu_off + (int64_t)(jv ? j : 0) * L.D;
    float* dmurow = dmu ? dmu + L.mu_off + (int64_t)(jv ? j : 0) * L.D : nullptr;
#pragma unroll
    for (int q = 0; q < ND32; ++q)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int d = 32 * q + 8 * g + 4 * h;
        const float4 m4 = load_f4(murow, d, L.D, jv, mvec);
        const float mv[4] = {m4.x, m4.y, m4.z, m4.w};
        float o[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float gt = GT[q][4 * g + e];
          colt[q][4 * g + e] = jv ? (ctot * mv[e] - 2.0f * gt) * mv[e] : 0.0f;
          o[e] = (d + e < L.D) ? g32 * T.lamf[d + e] * (gt - ctot * mv[e]) : 0.0f;
        }
        if (jv && dmurow) {
          if (mvec && d + 3 < L.D) {
            *reinterpret_cast<float4*>(dmurow + d) = make_float4(o[0], o[1], o[2], o[3]);
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (d + e < L.D) dmurow[d + e] = o[e];
          }
        }
      }
  }
  if (!dsp) return;
  float* buf = reinterpret_cast<float*>(&T.col[0][0]);   // >= 32 x DT floats
  for (int w2 = 0; w2 < 4; ++w2) {
    __syncthreads();
    if (w == w2) {
#pragma unroll
      for (int q = 0; q < ND32; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) buf[jr * TS::DT + 32 * q + 8 * (v / 4) + 4 * h + (v % 4)] = colt[q][v];
    }
    __syncthreads();
    for (int d = tid; d < TS::DT; d += blockDim.x) {
      float acc = 0.0f;
      for (int c = 0; c < 32; ++c) acc += buf[c * TS::DT + d];
      accD[d] += acc;
    }
  }
  __syncthreads();
  const int part = it.start / 128;
  for (int d = tid; d < L.D; d += blockDim.x)
    dsp[L.dsp_off + (int64_t)part * L.D + d] = g32 * T.lamf[d] * accD[d];
}

}  // namespace fused
}  // namespace tmc

// Plain engine: the pairwise log-factors are materialised in device memory and the
// message pass streams them.  Used for FP64, as the FP32 comparator of the fused
// engine, and for chains whose log-factors the caller supplies.
//
//   forward  (Sec. "Efficient averaging", Appendix log-domain product):
//     alpha_l[i] = u_l[i] + logsumexp_j(f_l[i,j] + alpha_{l+1}[j]) - ln K_{l+1}
//   backward (derivative of the same log-sum-exp):
//     G_l[i,j]   = p_l[i] * exp(f_l[i,j] + alpha_{l+1}[j] - rowlse_l[i])
//     p_{l+1}[j] = sum_i G_l[i,j]
// The column vector alpha_{l+1} is shifted by its FP64 maximum M before it is cast
// to the element type, so the per-entry arithmetic sees O(|f|) magnitudes only.
#include <math.h>

#include "dev_util.h"
#include "tmc_kernels.h"

namespace tmc {

template <typename T>
struct Vec;
template <>
struct Vec<float> {
  typedef float4 t4;
};
template <>
struct Vec<double> {
  typedef double2 t2;
};

template <typename T, int V>
__device__ __forceinline__ void load_vec(const T* __restrict__ p, T (&x)[V]) {
  if constexpr (V == 1) {
    x[0] = p[0];
  } else if constexpr (sizeof(T) == 4 && V == 4) {
    const float4 q = *reinterpret_cast<const float4*>(p);
    x[0] = q.x; x[1] = q.y; x[2] = q.z; x[3] = q.w;
  } else if constexpr (sizeof(T) == 8 && V == 2) {
    const double2 q = *reinterpret_cast<const double2*>(p);
    x[0] = q.x; x[1] = q.y;
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) x[v] = p[v];
  }
}

template <typename T, int V>
__device__ __forceinline__ void store_vec(T* __restrict__ p, const T (&x)[V]) {
  if constexpr (sizeof(T) == 4 && V == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(x[0], x[1], x[2], x[3]);
  } else if constexpr (sizeof(T) == 8 && V == 2) {
    *reinterpret_cast<double2*>(p) = make_double2(x[0], x[1]);
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) p[v] = x[v];
  }
}

// ---------------------------------------------------------------------------
// f_l[i,j] = sum_d -1/2 exp(-2 s_d) (z_id - mu_jd)^2 - sum_d s_d - D/2 ln 2 pi
// (direct difference; tile of 32 rows x 64 columns per workgroup).  Each term is
// formed in the element type and summed in FP64, so the sum over d (hundreds at
// D = 100) carries no FP32 accumulation error.  For the message pass (anchor != 0) row
// i is stored relative to its own FP64 value at column 0,
//   f~[i,j] = f[i,j] - a_i,   a_i = f[i,0]   (a_i written to anchor[] by the
// workgroups of column tile 0),
// so the element type holds differences of O(the spread of a row) instead of values
// of O(|f|): an FP32 row near -480 keeps ~1e-6 absolute precision instead of ~3e-5.
// With anchor == 0 (tmc_gauss_factors) f itself is written.
// PP (parent-dependent scale): s is [Kc][D], row j the log standard deviation produced
// from parent sample j, so lam and the constant are per column:
//   f_l[i,j] = sum_d -1/2 exp(-2 s_jd) (z_id - mu_jd)^2 - sum_d s_jd - D/2 ln 2 pi.
// ---------------------------------------------------------------------------
template <typename T, bool PP>
__global__ __launch_bounds__(256) void k_plain_factor(const LayerDev* __restrict__ Ls,
                                                      const Item* __restrict__ items,
                                                      const T* __restrict__ z,
                                                      const T* __restrict__ mu,
                                                      const T* __restrict__ s,
                                                      T* __restrict__ f, int caller_off,
                                                      double* __restrict__ anchor) {
  constexpr int TR = kPlainFactorRows, TC = kPlainFactorCols, DC = 32;
  __shared__ T zt[TR][DC + 1];
  __shared__ T mt[TC][DC + 1];
  __shared__ T m0[DC];
  __shared__ T lam[DC];                       // lam of the layer (PP: of column 0)
  __shared__ T lamt[PP ? TC : 1][DC + 1];       // PP: lam of the tile's columns
  __shared__ double cj[PP ? TC : 1];            // PP: constant of each column minus c0
  __shared__ double red[kMaxWaves];
  __shared__ double arow[TR];
  const Item it = items[blockIdx.x];
  const LayerDev& L = Ls[it.layer];
  const int K = L.K, Kc = L.Kc, D = L.D;
  const int64_t zo = L.z_off, mo = L.mu_off, so = L.s_off;
  const int tiles_c = (Kc + TC - 1) / TC;
  const int i0 = (it.start / tiles_c) * TR, j0 = (it.start % tiles_c) * TC;
  const int tid = threadIdx.x;
  const bool anchored = anchor != nullptr;

  // (PP: s[so + d] is row 0 of the block, so c0 is column 0's constant)
  double ssum = 0.0;
  for (int d = tid; d < D; d += blockDim.x) ssum += (double)s[so + d];
  ssum = block_sum(ssum, red);
  const double c0 = -ssum - 0.5 * (double)D * log(2.0 * M_PI);
  if constexpr (PP) {
    // column constants relative to c0, each an FP64 sum over d in increasing d
    if (tid < TC) {
      double sj = 0.0;
      if (j0 + tid < Kc)
        for (int d = 0; d < D; ++d) sj += (double)s[so + (int64_t)(j0 + tid) * D + d];
      cj[tid] = -sj - 0.5 * (double)D * log(2.0 * M_PI) - c0;
    }
  }

  const int col = tid % TC, rsub = tid / TC;
  double acc[TR / 4];
#pragma unroll
  for (int q = 0; q < TR / 4; ++q) acc[q] = 0.0;
  double aacc = 0.0;   // threads tid < TR: FP64 sum of row tid against column 0

  for (int d0 = 0; d0 < D; d0 += DC) {
    __syncthreads();
    for (int e = tid; e < TR * DC; e += 256) {
      const int r = e / DC, dd = e % DC;
      zt[r][dd] = (i0 + r < K && d0 + dd < D) ? z[zo + (int64_t)(i0 + r) * D + d0 + dd] : (T)0;
    }
    for (int e = tid; e < TC * DC; e += 256) {
      const int c = e / DC, dd = e % DC;
      mt[c][dd] = (j0 + c < Kc && d0 + dd < D) ? mu[mo + (int64_t)(j0 + c) * D + d0 + dd] : (T)0;
    }
    if (tid < DC) {
      lam[tid] = (d0 + tid < D) ? (T)exp(-2.0 * (double)s[so + d0 + tid]) : (T)0;
      m0[tid] = (d0 + tid < D) ? mu[mo + d0 + tid] : (T)0;
    }
    if constexpr (PP) {
      for (int e = tid; e < TC * DC; e += 256) {
        const int c = e / DC, dd = e % DC;
        lamt[c][dd] = (j0 + c < Kc && d0 + dd < D)
                          ? (T)exp(-2.0 * (double)s[so + (int64_t)(j0 + c) * D + d0 + dd])
                          : (T)0;
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int dd = 0; dd < DC; ++dd) {
      const T m = mt[col][dd], l = PP ? lamt[col][dd] : lam[dd];
#pragma unroll
      for (int q = 0; q < TR / 4; ++q) {
        const T t = zt[rsub + 4 * q][dd] - m;
        acc[q] += (double)(l * t * t);
      }
    }
    if (anchored && tid < TR) {
      // the same terms, in the same order, as the column-0 entry of row tid
      for (int dd = 0; dd < DC; ++dd) {
        const T t = zt[tid][dd] - m0[dd];
        aacc += (double)(lam[dd] * t * t);
      }
    }
  }
  if (anchored) {
    if (tid < TR) arow[tid] = aacc;
    __syncthreads();
    if (j0 == 0 && tid < TR && i0 + tid < K) anchor[L.rl_off + i0 + tid] = -0.5 * aacc + c0;
  }
  T* fb = f + (caller_off ? L.f_off : L.wf_off);
  const int j = j0 + col;
  if (j < Kc) {
    const double cc = PP ? cj[col] : 0.0;   // this column's constant minus c0
#pragma unroll
    for (int q = 0; q < TR / 4; ++q) {
      const int i = i0 + rsub + 4 * q;
      if (i < K)
        fb[(int64_t)i * Kc + j] = anchored ? (T)(-0.5 * (acc[q] - arow[rsub + 4 * q]) + cc)
                                           : (T)(-0.5 * acc[q] + c0 + cc);
    }
  }
}

// ---------------------------------------------------------------------------
// forward message: a wave owns kPlainFwdRowsPerWave rows and streams them together,
// one vector of V elements per lane and row per step, so that every lane has that many
// loads in flight; each lane keeps an online (max, sum) per row over the columns it
// reads (no cross-lane work inside the loop), merged across the wave at the end.  Few
// rows per wave keep the register count low, so many waves stay resident per CU and
// they, not deep per-wave buffers, hold the bytes in flight; the kPlainFwdWaves waves
// of a workgroup share one copy of the column shifts, formed once in its prologue.
// ---------------------------------------------------------------------------
template <typename T, int V, int R>
__device__ __forceinline__ void rows_lse(const T* __restrict__ fb, int64_t row0, int nrow,
                                         const T* __restrict__ gam, int Kc, int lane, T kap,
                                         T (&lse)[R]) {
  const T NEG = (T)(-INFINITY);
  T m[R], sm[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    m[r] = NEG;
    sm[r] = (T)0;
  }
  for (int base = 0; base < Kc; base += kWave * V) {
    const int j = base + lane * V;
    const bool ok = j < Kc;   // Kc % V == 0 when V > 1, so a vector is whole or absent
    T x[R][V];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int rr = min(r, nrow - 1);   // rows past the block repeat its last row
      if (ok) load_vec<T, V>(fb + (row0 + rr) * (int64_t)Kc + j, x[r]);
    }
    T g[V];
    if (ok) load_vec<T, V>(gam + j, g);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      T cm = NEG;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        x[r][v] = ok ? kap * x[r][v] + g[v] : NEG;
        cm = nan_max(cm, x[r][v]);
      }
      const T nm = nan_max(m[r], cm);
      const T sh = (nm == NEG) ? (T)0 : nm;
      T acc = (T)0;
#pragma unroll
      for (int v = 0; v < V; ++v) acc += fast_exp(x[r][v] - sh);
      sm[r] = sm[r] * fast_exp(m[r] - sh) + acc;
      m[r] = nm;
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const T M = wave_max(m[r]);
    const T sh = (M == NEG || M != M) ? (T)0 : M;
    const T S = wave_sum(sm[r] * fast_exp(m[r] - sh));
    lse[r] = (M != M) ? M : (M == NEG ? NEG : M + fast_log(S));
  }
}

template <typename T, int V>
__global__ __launch_bounds__(64 * kPlainFwdWaves) void k_plain_lse_fwd(const LayerDev* __restrict__ Ls,
                                                       const Item* __restrict__ items,
                                                       const T* __restrict__ f, int caller_off,
                                                       const T* __restrict__ u,
                                                       double* __restrict__ alpha,
                                                       T* __restrict__ rl,
                                                       double* __restrict__ pairM,
                                                       const double* __restrict__ anchor) {
  constexpr int R = kPlainFwdRowsPerWave;
  extern __shared__ unsigned char smem_raw[];
  T* gam = reinterpret_cast<T*>(smem_raw);
  __shared__ double red[kMaxWaves];
  const Item it = items[blockIdx.x];
  const LayerDev& L = Ls[it.layer];
  const int Kc = L.Kc, K = L.K;
  const double* aup = alpha + L.alpha_up_off;
  const int tid = threadIdx.x;

  double m = -INFINITY;
  for (int j = tid; j < Kc; j += blockDim.x) m = nan_max(m, aup[j]);
  m = block_max(m, red);
  const double M = (m == -INFINITY) ? 0.0 : m;
  for (int j = tid; j < Kc; j += blockDim.x) gam[j] = (T)(aup[j] - M);
  if (it.start == 0 && tid == 0) pairM[it.layer] = M;
  __syncthreads();

  const int w = tid / kWave, lane = tid % kWave;
  const int i0 = it.start + w * R;
  if (i0 >= K) return;
  const int nrow = min(R, K - i0);
  const T* fb = f + (caller_off ? L.f_off : L.wf_off);
  T lse[R];
  rows_lse<T, V, R>(fb, i0, nrow, gam, Kc, lane, (T)L.kappa, lse);
  const double lkc = log((double)Kc);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = i0 + r;
    if (lane == r && r < nrow) {
      rl[L.rl_off + i] = lse[r];
      const double a = anchor ? anchor[L.rl_off + i] : 0.0;
      alpha[L.alpha_off + i] = L.kappa * ((double)u[L.u_off + i] + a) + M + (double)lse[r] - lkc;
    }
  }
}

// ---------------------------------------------------------------------------
// backward message: a workgroup of kPlainBwdWaves waves owns a strip of 64 V columns
// and walks every row (wave w: rows w, w + kPlainBwdWaves, ..., kPlainBwdRowsPerStep of
// them per step with all their loads issued first), so the column sums p_{l+1}[j] are
// complete inside it: per-wave partial sums, then a fixed-order sum over the waves (no
// atomics).  Reads f and writes G once per entry.
// ---------------------------------------------------------------------------
template <typename T, int V>
__global__ __launch_bounds__(64 * kPlainBwdWaves) void k_plain_lse_bwd(
    const LayerDev* __restrict__ Ls, const Item* __restrict__ items, const T* __restrict__ f,
    int caller_off, const double* __restrict__ alpha, const T* __restrict__ rl,
    const double* __restrict__ pairM, const double* __restrict__ dlogp, T* __restrict__ p,
    T* __restrict__ gout, int g_caller_off, int scale, T* __restrict__ du) {
  constexpr int NW = kPlainBwdWaves, RS = kPlainBwdRowsPerStep;
  __shared__ T red[NW][kWave * V];
  const Item it = items[blockIdx.x];
  const LayerDev& L = Ls[it.layer];
  const int Kc = L.Kc, K = L.K;
  const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
  const int j = it.start + lane * V;
  const bool active = j < Kc;
  const double M = pairM[it.layer];
  const double* aup = alpha + L.alpha_up_off;
  const double g = dlogp[L.chain] * L.kappa;   // d/d(kappa f) -> d/df
  const T gs = scale ? (T)g : (T)1;
  const T kap = (T)L.kappa;
  T gam[V], cs[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    gam[v] = active ? (T)(aup[j + v] - M) : (T)0;
    cs[v] = (T)0;
  }
  const T* fb = f + (caller_off ? L.f_off : L.wf_off);
  T* gb = gout + (g_caller_off ? L.f_off : L.wf_off);
  const T* pr = p + L.p_off;
  const T* rr = rl + L.rl_off;
  const int jc = active ? j : 0;   // inactive lanes read column 0 of a valid row
  for (int i0 = w; i0 < K; i0 += NW * RS) {
    T x[RS][V], pi[RS], li[RS];
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int i = min(i0 + NW * r, K - 1);   // rows past K repeat row K-1 (not stored)
      pi[r] = pr[i];
      li[r] = rr[i];
      load_vec<T, V>(fb + (int64_t)i * Kc + jc, x[r]);
    }
#pragma unroll
    for (int r = 0; r < RS; ++r) {
      const int i = i0 + NW * r;
      const bool live = i < K && active;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        // p_i == 0 (a row outside the support) gives G = 0 even where exp overflows
        const T gv = (pi[r] == (T)0) ? (T)0 : pi[r] * fast_exp(kap * x[r][v] + gam[v] - li[r]);
        cs[v] += live ? gv : (T)0;
        x[r][v] = gv * gs;
      }
      if (gout && live) store_vec<T, V>(gb + (int64_t)i * Kc + j, x[r]);
    }
  }
#pragma unroll
  for (int v = 0; v < V; ++v) red[w][lane * V + v] = cs[v];
  __syncthreads();
  if (w == 0 && active) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      T t = red[0][lane * V + v];
#pragma unroll
      for (int q = 1; q < NW; ++q) t += red[q][lane * V + v];
      p[L.p_up_off + j + v] = t;
      if (du) du[L.u_up_off + j + v] = (T)(g * (double)t);
    }
  }
}

// ---------------------------------------------------------------------------
// Gaussian gradients from the materialised marginals G (plain engine)
//   dz_l[i]  = -dlogp * lam * (p_l[i] z_l[i] - (G mu)_i)
//   dmu_l[j] =  dlogp * lam * ((G^T z)_j - p_{l+1}[j] mu_j)
// PP (lam_j per parent sample): the same sums with lam inside, by direct difference,
//   dz_l[i]  = -dlogp * sum_j G_ij lam_j (z_i - mu_j)
//   dmu_l[j] =  dlogp * lam_j sum_i G_ij (z_i - mu_j)
//   ds_l[j]  =  dlogp * (lam_j sum_i G_ij (z_i - mu_j)^2 - p_{l+1}[j])
// ---------------------------------------------------------------------------
template <typename T, bool PP>
__global__ __launch_bounds__(256) void k_plain_gmu(const LayerDev* __restrict__ Ls,
                                                   const Item* __restrict__ items,
                                                   const T* __restrict__ G,
                                                   const T* __restrict__ z,
                                                   const T* __restrict__ mu,
                                                   const T* __restrict__ s,
                                                   const T* __restrict__ p,
                                                   const double* __restrict__ dlogp,
                                                   T* __restrict__ dz) {
  constexpr int TR = kPlainGemmRows, TD = kPlainGemmD, TJ = 32;
  __shared__ T gt[TR][TJ + 1];
  __shared__ T mt[TJ][TD + 1];
  __shared__ T lt[PP ? TJ : 1][TD + 1];
  const Item it = items[blockIdx.x];
  const LayerDev& L = Ls[it.layer];
  const int K = L.K, Kc = L.Kc, D = L.D;
  const int nd = (D + TD - 1) / TD;
  const int i0 = (it.start / nd) * TR, d0 = (it.start % nd) * TD;
  const int tid = threadIdx.x, dl = tid % TD, rs = tid / TD;
  const T* Gb = G + L.wf_off;
  const int64_t mo = L.mu_off;
  T acc[TR / 4], zr[PP ? TR / 4 : 1];
#pragma unroll
  for (int q = 0; q < TR / 4; ++q) acc[q] = (T)0;
  if constexpr (PP) {
#pragma unroll
    for (int q = 0; q < TR / 4; ++q) {
      const int i = i0 + rs + 4 * q;
      zr[q] = (i < K && d0 + dl < D) ? z[L.z_off + (int64_t)i * D + d0 + dl] : (T)0;
    }
  }
  for (int j0 = 0; j0 < Kc; j0 += TJ) {
    __syncthreads();
    for (int e = tid; e < TR * TJ; e += 256) {
      const int r = e / TJ, jj = e % TJ;
      gt[r][jj] = (i0 + r < K && j0 + jj < Kc) ? Gb[(int64_t)(i0 + r) * Kc + j0 + jj] : (T)0;
    }
    for (int e = tid; e < TJ * TD; e += 256) {
      const int jj = e / TD, dd = e % TD;
      mt[jj][dd] = (j0 + jj < Kc && d0 + dd < D) ? mu[mo + (int64_t)(j0 + jj) * D + d0 + dd] : (T)0;
      if constexpr (PP)
        lt[jj][dd] = (j0 + jj < Kc && d0 + dd < D)
                         ? (T)exp(-2.0 * (double)s[L.s_off + (int64_t)(j0 + jj) * D + d0 + dd])
                         : (T)0;
    }
    __syncthreads();
#pragma unroll 8
    for (int jj = 0; jj < TJ; ++jj) {
      const T m = mt[jj][dl];
      if constexpr (PP) {
        const T lm = lt[jj][dl];
#pragma unroll
        for (int q = 0; q < TR / 4; ++q) acc[q] += gt[rs + 4 * q][jj] * (lm * (zr[q] - m));
      } else {
#pragma unroll
        for (int q = 0; q < TR / 4; ++q) acc[q] += gt[rs + 4 * q][jj] * m;
      }
    }
  }
  const int d = d0 + dl;
  if (d >= D) return;
  const T g = (T)(dlogp[L.chain] * L.kappa);
  if constexpr (PP) {
#pragma unroll
    for (int q = 0; q < TR / 4; ++q) {
      const int i = i0 + rs + 4 * q;
      if (i < K) dz[L.z_off + (int64_t)i * D + d] = -g * acc[q];
    }
    return;
  }
  const T lam = (T)exp(-2.0 * (double)s[L.s_off + d]);
#pragma unroll
  for (int q = 0; q < TR / 4; ++q) {
    const int i = i0 + rs + 4 * q;
    if (i < K) {
      const int64_t zi = L.z_off + (int64_t)i * D + d;
      dz[zi] = -g * lam * (p[L.p_off + i] * z[zi] - acc[q]);
    }
  }
}

template <typename T, bool PP>
__global__ __launch_bounds__(256) void k_plain_gtz(const LayerDev* __restrict__ Ls,
                                                   const Item* __restrict__ items,
                                                   const T* __restrict__ G,
                                                   const T* __restrict__ z,
                                                   const T* __restrict__ mu,
                                                   const T* __restrict__ s,
                                                   const T* __restrict__ p,
                                                   const double* __restrict__ dlogp,
                                                   T* __restrict__ gtz, T* __restrict__ dmu,
                                                   T* __restrict__ ds_pp) {
  constexpr int TC = kPlainGemmRows, TD = kPlainGemmD, TI = 32;
  __shared__ T gt[TI][TC + 1];
  __shared__ T zt[TI][TD + 1];
  const Item it = items[blockIdx.x];
  const LayerDev& L = Ls[it.layer];
  const int K = L.K, Kc = L.Kc, D = L.D;
  const int nd = (D + TD - 1) / TD;
  const int j0 = (it.start / nd) * TC, d0 = (it.start % nd) * TD;
  const int tid = threadIdx.x, dl = tid % TD, cs = tid / TD;
  const T* Gb = G + L.wf_off;
  const int64_t zo = L.z_off;
  T acc[TC / 4], acc2[PP ? TC / 4 : 1], mr[PP ? TC / 4 : 1];
#pragma unroll
  for (int q = 0; q < TC / 4; ++q) acc[q] = (T)0;
  if constexpr (PP) {
#pragma unroll
    for (int q = 0; q < TC / 4; ++q) {
      const int j = j0 + cs + 4 * q;
      acc2[q] = (T)0;
      mr[q] = (j < Kc && d0 + dl < D) ? mu[L.mu_off + (int64_t)j * D + d0 + dl] : (T)0;
    }
  }
  for (int i0 = 0; i0 < K; i0 += TI) {
    __syncthreads();
    for (int e = tid; e < TI * TC; e += 256) {
      const int ii = e / TC, jj = e % TC;
      gt[ii][jj] = (i0 + ii < K && j0 + jj < Kc) ? Gb[(int64_t)(i0 + ii) * Kc + j0 + jj] : (T)0;
    }
    for (int e = tid; e < TI * TD; e += 256) {
      const int ii = e / TD, dd = e % TD;
      zt[ii][dd] = (i0 + ii < K && d0 + dd < D) ? z[zo + (int64_t)(i0 + ii) * D + d0 + dd] : (T)0;
    }
    __syncthreads();
#pragma unroll 8
    for (int ii = 0; ii < TI; ++ii) {
      const T zv = zt[ii][dl];
      if constexpr (PP) {
#pragma unroll
        for (int q = 0; q < TC / 4; ++q) {
          const T gv = gt[ii][cs + 4 * q], df = zv - mr[q];
          acc[q] += gv * df;
          acc2[q] += gv * df * df;
        }
      } else {
#pragma unroll
        for (int q = 0; q < TC / 4; ++q) acc[q] += gt[ii][cs + 4 * q] * zv;
      }
    }
  }
  const int d = d0 + dl;
  if (d >= D) return;
  const T g = (T)(dlogp[L.chain] * L.kappa);
  if constexpr (PP) {
#pragma unroll
    for (int q = 0; q < TC / 4; ++q) {
      const int j = j0 + cs + 4 * q;
      if (j < Kc) {
        const int64_t e = (int64_t)j * D + d;
        const T lam = (T)exp(-2.0 * (double)s[L.s_off + e]);
        if (dmu) dmu[L.mu_off + e] = g * lam * acc[q];
        if (ds_pp) ds_pp[L.s_off + e] = g * (lam * acc2[q] - p[L.p_up_off + j]);
      }
    }
    return;
  }
  const T lam = (T)exp(-2.0 * (double)s[L.s_off + d]);
#pragma unroll
  for (int q = 0; q < TC / 4; ++q) {
    const int j = j0 + cs + 4 * q;
    if (j < Kc) {
      gtz[L.gtz_off + (int64_t)j * D + d] = acc[q];
      if (dmu) {
        const int64_t mi = L.mu_off + (int64_t)j * D + d;
        dmu[mi] = g * lam * (acc[q] - p[L.p_up_off + j] * mu[mi]);
      }
    }
  }
}

// ds partial of one pair:
//   dlogp * [ lam_d * (sum_i p_i z_id^2 - 2 sum_j mu_jd (G^T z)_jd + sum_j p'_j mu_jd^2)
//             - sum_i p_i ]
// which is sum_ij G_ij (lam (z_i - mu_j)^2 - 1) with the double sum expanded.
template <typename T>
__global__ __launch_bounds__(256) void k_pair_dsp(const LayerDev* __restrict__ Ls,
                                                  const int* __restrict__ pair_ids,
                                                  const T* __restrict__ z,
                                                  const T* __restrict__ mu,
                                                  const T* __restrict__ s,
                                                  const T* __restrict__ p,
                                                  const T* __restrict__ gtz,
                                                  const double* __restrict__ dlogp,
                                                  T* __restrict__ dsp) {
  const int l = pair_ids[blockIdx.x];
  const LayerDev& L = Ls[l];
  const int K = L.K, Kc = L.Kc, D = L.D;
  const T* pr = p + L.p_off;
  const T* pc = p + L.p_up_off;
  const T g = (T)(dlogp[L.chain] * L.kappa);
  T P = (T)0;
  for (int i = 0; i < K; ++i) P += pr[i];
  for (int d = threadIdx.x; d < D; d += blockDim.x) {
    T A = 0, B = 0, C = 0;
    for (int i = 0; i < K; ++i) {
      const T zv = z[L.z_off + (int64_t)i * D + d];
      A += pr[i] * zv * zv;
    }
    for (int j = 0; j < Kc; ++j) {
      const T mv = mu[L.mu_off + (int64_t)j * D + d];
      B += mv * gtz[L.gtz_off + (int64_t)j * D + d];
      C += pc[j] * mv * mv;
    }
    const T lam = (T)exp(-2.0 * (double)s[L.s_off + d]);
    dsp[L.dsp_off + d] = g * (lam * (A - (T)2 * B + C) - P);
  }
}

// ---- launchers ----
template <typename T>
hipError_t launch_plain_factor(const LayerDev* layers, const Item* items, int n_items,
                               const T* z, const T* mu, const T* s, T* f, bool caller_off,
                               double* anchor, bool parent_scale, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  if (parent_scale)
    hipLaunchKernelGGL((k_plain_factor<T, true>), dim3(n_items), dim3(256), 0, st, layers, items, z,
                       mu, s, f, (int)caller_off, anchor);
  else
    hipLaunchKernelGGL((k_plain_factor<T, false>), dim3(n_items), dim3(256), 0, st, layers, items, z,
                       mu, s, f, (int)caller_off, anchor);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_plain_lse_fwd(const LayerDev* layers, const Item* items, int n_items, int max_kc,
                                int vec, const T* f, bool caller_off, const T* u, double* alpha,
                                T* rl, double* pairM, const double* anchor, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  constexpr int VV = sizeof(T) == 4 ? 4 : 2;
  const size_t smem = (size_t)max_kc * sizeof(T);
  if (vec)
    hipLaunchKernelGGL((k_plain_lse_fwd<T, VV>), dim3(n_items), dim3(64 * kPlainFwdWaves), smem, st, layers, items,
                       f, (int)caller_off, u, alpha, rl, pairM, anchor);
  else
    hipLaunchKernelGGL((k_plain_lse_fwd<T, 1>), dim3(n_items), dim3(64 * kPlainFwdWaves), smem, st, layers, items,
                       f, (int)caller_off, u, alpha, rl, pairM, anchor);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_plain_lse_bwd(const LayerDev* layers, const Item* items, int n_items, int vec,
                                const T* f, bool caller_off, const double* alpha, const T* rl,
                                const double* pairM, const double* dlogp, T* p, T* g_out,
                                bool g_caller_off, bool scale_by_dlogp, T* du, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  constexpr int VV = sizeof(T) == 4 ? 4 : 2;
  if (vec)
    hipLaunchKernelGGL((k_plain_lse_bwd<T, VV>), dim3(n_items), dim3(64 * kPlainBwdWaves), 0, st, layers, items, f,
                       (int)caller_off, alpha, rl, pairM, dlogp, p, g_out, (int)g_caller_off,
                       (int)scale_by_dlogp, du);
  else
    hipLaunchKernelGGL((k_plain_lse_bwd<T, 1>), dim3(n_items), dim3(64 * kPlainBwdWaves), 0, st, layers, items, f,
                       (int)caller_off, alpha, rl, pairM, dlogp, p, g_out, (int)g_caller_off,
                       (int)scale_by_dlogp, du);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_plain_gmu(const LayerDev* layers, const Item* items, int n_items, const T* g,
                            const T* z, const T* mu, const T* s, const T* p, const double* dlogp,
                            T* dz, bool parent_scale, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  if (parent_scale)
    hipLaunchKernelGGL((k_plain_gmu<T, true>), dim3(n_items), dim3(256), 0, st, layers, items, g, z,
                       mu, s, p, dlogp, dz);
  else
    hipLaunchKernelGGL((k_plain_gmu<T, false>), dim3(n_items), dim3(256), 0, st, layers, items, g, z,
                       mu, s, p, dlogp, dz);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_plain_gtz(const LayerDev* layers, const Item* items, int n_items, const T* g,
                            const T* z, const T* mu, const T* s, const T* p, const double* dlogp,
                            T* gtz, T* dmu, T* ds_pp, bool parent_scale, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  if (parent_scale)
    hipLaunchKernelGGL((k_plain_gtz<T, true>), dim3(n_items), dim3(256), 0, st, layers, items, g, z,
                       mu, s, p, dlogp, gtz, dmu, ds_pp);
  else
    hipLaunchKernelGGL((k_plain_gtz<T, false>), dim3(n_items), dim3(256), 0, st, layers, items, g, z,
                       mu, s, p, dlogp, gtz, dmu, ds_pp);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_pair_dsp(const LayerDev* layers, const int* pair_ids, int n_pairs, const T* z,
                           const T* mu, const T* s, const T* p, const T* gtz, const double* dlogp,
                           T* dsp, hipStream_t st) {
  if (n_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pair_dsp<T>, dim3(n_pairs), dim3(256), 0, st, layers, pair_ids, z, mu, s,
                     p, gtz, dlogp, dsp);
  return hipGetLastError();
}

#define TMC_INST(T)                                                                              \
  template hipError_t launch_plain_factor<T>(const LayerDev*, const Item*, int, const T*,        \
                                             const T*, const T*, T*, bool, double*, bool,        \
                                             hipStream_t);                                       \
  template hipError_t launch_plain_lse_fwd<T>(const LayerDev*, const Item*, int, int, int,       \
                                              const T*, bool, const T*, double*, T*, double*,    \
                                              const double*, hipStream_t);                       \
  template hipError_t launch_plain_lse_bwd<T>(const LayerDev*, const Item*, int, int, const T*,  \
                                              bool, const double*, const T*, const double*,      \
                                              const double*, T*, T*, bool, bool, T*,             \
                                              hipStream_t);                                      \
  template hipError_t launch_plain_gmu<T>(const LayerDev*, const Item*, int, const T*,           \
                                          const T*, const T*, const T*, const T*,                \
                                          const double*, T*, bool, hipStream_t);                 \
  template hipError_t launch_plain_gtz<T>(const LayerDev*, const Item*, int, const T*,           \
                                          const T*, const T*, const T*, const T*,                \
                                          const double*, T*, T*, T*, bool, hipStream_t);         \
  template hipError_t launch_pair_dsp<T>(const LayerDev*, const int*, int, const T*, const T*,   \
                                         const T*, const T*, const T*, const double*, T*,        \
                                         hipStream_t);
TMC_INST(float)
TMC_INST(double)
#undef TMC_INST

}  // namespace tmc

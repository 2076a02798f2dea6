// Star-shaped model (Sec. "Efficient averaging", the latent-variable example: one global
// latent theta with K_t samples shared by N data points, each with its own local latent
// of K samples).  The local indices are summed out first, then theta:
//   m_i[kt] = logsumexp_k(u_i[k] + f_i[kt, k]) - ln K
//   log P   = logsumexp_kt(uth[kt] + sum_i m_i[kt]) - ln K_t
// with the Gaussian factor f_i[kt, k] = log N(z_i^k; mth^kt, diag exp(2 s)), mth^kt the
// mean of the local latents given global sample kt.  The local latents of such models
// are low-dimensional (the paper's workload has D = 1), so each factor is formed by
// direct difference on the vector ALU; with D this small there is no contraction to put
// on MFMA, and the cost is the exponential of every entry.  Backward, with
//   w[kt]      = exp(uth[kt] + sum_i m_i[kt] - ln K_t - log P)        (d log P / d uth)
//   G_i[kt, k] = w[kt] exp(u_i[k] + f_i[kt, k] - m_i[kt] - ln K)      (d log P / d f_i):
//   d u_i[k] = sum_kt G,  d z_ik = -lam sum_kt G (z_ik - mth[kt]),
//   d mth[kt] = lam sum_i sum_k G (z_ik - mth[kt]),
//   d s = sum_i sum_{kt,k} G (lam (z_ik - mth[kt])^2 - 1),  lam = exp(-2 s).
// Workgroups are 8 waves: the 64 lanes of a wave take 64 samples of one index, the waves
// split the other; every sum across lanes, waves, points or workgroups runs in a fixed
// order, so results are deterministic.  Per-entry arithmetic is in T (the plan's
// precision); per-row results and sums over rows are double.
#include <math.h>

#include "dev_util.h"
#include "tmc_internal.h"
#include "tmc_star.h"

namespace tmc {

namespace {

constexpr int kStarThreads = kStarWaves * kWave;
constexpr int kRowsPerWave = kStarChunk / kStarWaves;
constexpr double kLn2Pi = 1.8378770664093454836;

// lam_d = exp(-2 s_d) (0 past D); returns c = -sum_d s_d - D/2 ln(2 pi).
template <typename T, int DB>
__device__ __forceinline__ T star_consts(const T* __restrict__ s, int D, T (&lam)[DB]) {
  double ssum = 0.0;
#pragma unroll
  for (int d = 0; d < DB; ++d) {
    const double sd = d < D ? (double)s[d] : 0.0;
    lam[d] = d < D ? (T)exp(-2.0 * sd) : (T)0;
    ssum += sd;
  }
  return (T)(-ssum - 0.5 * (double)D * kLn2Pi);
}

// -1/2 sum_d lam_d (x_d - y_d)^2; entries past D are 0 on both sides and lam is 0 there.
template <typename T, int DB, class X, class Y>
__device__ __forceinline__ T star_quad(const X& x, const Y& y, const T (&lam)[DB]) {
  T acc = (T)0;
#pragma unroll
  for (int d = 0; d < DB; ++d) {
    const T t = x[d] - y[d];
    acc += lam[d] * t * t;
  }
  return (T)(-0.5) * acc;
}

// Rows [r0, r0 + n) of a row-major [*][D] array into LDS rows of stride DB (the padding
// columns d >= D keep the zeros written at kernel start).
template <typename T, int DB>
__device__ __forceinline__ void star_stage(T* dst, const T* __restrict__ src, int r0, int n, int D) {
  for (int e = threadIdx.x; e < n * D; e += blockDim.x) {
    const int r = e / D;
    dst[r * DB + (e - r * D)] = src[(int64_t)r0 * D + e];
  }
}

template <typename T, int N>
__device__ __forceinline__ void lds_zero(T* dst) {
  for (int e = threadIdx.x; e < N; e += blockDim.x) dst[e] = (T)0;
}

// Sum over the waves, in wave order, of each lane's v; the result is valid in wave 0.
// Every thread of the workgroup must call it.
template <typename T>
__device__ __forceinline__ double waves_sum(T v, T (*cb)[kStarLanes], int wv, int lane) {
  __syncthreads();
  cb[wv][lane] = v;
  __syncthreads();
  double r = 0.0;
  if (wv == 0) {
#pragma unroll
    for (int w = 0; w < kStarWaves; ++w) r += (double)cb[w][lane];
  }
  return r;
}

}  // namespace

// Messages: a workgroup per (instance, group of P points, 64 global samples).  Lane ->
// global sample kt; wave wv takes local rows wv, wv + 8, .. of each staged chunk of 64,
// keeping a running (max, sum) per lane; the waves' pairs are merged in wave order.
template <typename T, int DB>
__global__ __launch_bounds__(kStarThreads) void k_star_msg(StarArgs<T> a) {
  __shared__ T zs[kStarChunk * DB];
  __shared__ T us[kStarChunk];
  __shared__ T cm[kStarWaves][kStarLanes];
  __shared__ T cs[kStarWaves][kStarLanes];
  const int inst = blockIdx.x / a.ngrp, grp = blockIdx.x - inst * a.ngrp;
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int D = a.D, K = a.K, Kt = a.Kt;
  const int kt = blockIdx.y * kStarLanes + lane;
  const bool ktv = kt < Kt;
  T lam[DB], mt[DB];
  const T c0 = star_consts<T, DB>(a.s + (int64_t)inst * D, D, lam);
#pragma unroll
  for (int d = 0; d < DB; ++d) mt[d] = (ktv && d < D) ? a.mth[((int64_t)inst * Kt + kt) * D + d] : (T)0;
  lds_zero<T, kStarChunk * DB>(zs);
  const T ninf = (T)(-INFINITY);
  const double lnK = log((double)K);
  double gacc = 0.0;
  const int p0 = grp * a.P, p1 = min(a.N, p0 + a.P);
  for (int pt = p0; pt < p1; ++pt) {
    const int64_t pi = (int64_t)inst * a.N + pt;
    const T* z = a.z + pi * K * D;
    const T* u = a.u + pi * K;
    T mx = ninf, sm = (T)0;
    for (int k0 = 0; k0 < K; k0 += kStarChunk) {
      const int nk = min(kStarChunk, K - k0);
      __syncthreads();   // (also orders the previous point's reads of cm, cs)
      star_stage<T, DB>(zs, z, k0, nk, D);
      for (int e = threadIdx.x; e < nk; e += blockDim.x) us[e] = u[k0 + e];
      __syncthreads();
      T x[kRowsPerWave];
      T m = ninf;
#pragma unroll
      for (int r = 0; r < kRowsPerWave; ++r) {
        const int k = wv + kStarWaves * r;
        x[r] = k < nk ? us[k] + c0 + star_quad<T, DB>(&zs[k * DB], mt, lam) : ninf;
        m = nan_max(m, x[r]);
      }
      if (m != m) {
        mx = m;
        sm = m;
      } else if (m != ninf && mx == mx) {
        if (m > mx) {
          sm *= fast_exp(mx - m);
          mx = m;
        }
#pragma unroll
        for (int r = 0; r < kRowsPerWave; ++r) sm += fast_exp(x[r] - mx);
      }
    }
    cm[wv][lane] = mx;
    cs[wv][lane] = sm;
    __syncthreads();
    if (wv == 0) {
      T M = cm[0][lane];
#pragma unroll
      for (int w = 1; w < kStarWaves; ++w) M = nan_max(M, cm[w][lane]);
      double mi;
      if (M != M) {
        mi = (double)M;
      } else if (M == ninf) {
        mi = -INFINITY;
      } else {
        T S = (T)0;
#pragma unroll
        for (int w = 0; w < kStarWaves; ++w) S += cs[w][lane] * fast_exp(cm[w][lane] - M);
        mi = (double)M + log((double)S) - lnK;
      }
      if (ktv) a.msg[pi * Kt + kt] = mi;
      gacc += mi;
    }
  }
  if (wv == 0 && ktv) a.gsum[((int64_t)inst * a.ngrp + grp) * Kt + kt] = gacc;
}

// Logits of the global samples: w[kt] = uth[kt] + sum over groups of gsum (wave wv sums
// groups wv, wv + 8, ..; then the waves in order).  A workgroup per (instance, 64 kt).
template <typename T>
__global__ __launch_bounds__(kStarThreads) void k_star_colsum(StarArgs<T> a) {
  __shared__ double part[kStarWaves][kStarLanes];
  const int inst = blockIdx.x;
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int kt = blockIdx.y * kStarLanes + lane;
  const bool ktv = kt < a.Kt;
  double acc = 0.0;
  if (ktv)
    for (int g = wv; g < a.ngrp; g += kStarWaves) acc += a.gsum[((int64_t)inst * a.ngrp + g) * a.Kt + kt];
  part[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && ktv) {
    double v = (double)a.uth[(int64_t)inst * a.Kt + kt];
#pragma unroll
    for (int w = 0; w < kStarWaves; ++w) v += part[w][lane];
    a.w[(int64_t)inst * a.Kt + kt] = v;
  }
}

// log P of an instance from its logits, then the logits replaced by the weights w[kt].
template <typename T>
__global__ __launch_bounds__(256) void k_star_logp(StarArgs<T> a) {
  __shared__ double red[kMaxWaves];
  const int inst = blockIdx.x, Kt = a.Kt;
  double* w = a.w + (int64_t)inst * Kt;
  double mx = -INFINITY;
  for (int kt = threadIdx.x; kt < Kt; kt += blockDim.x) mx = nan_max(mx, w[kt]);
  mx = block_max(mx, red);
  const double lnKt = log((double)Kt);
  double lp;
  if (mx != mx || mx == -INFINITY || mx == INFINITY) {   // (uniform)
    lp = mx;
  } else {
    double sm = 0.0;
    for (int kt = threadIdx.x; kt < Kt; kt += blockDim.x) sm += exp(w[kt] - mx);
    sm = block_sum(sm, red);
    lp = mx + log(sm) - lnKt;
  }
  if (threadIdx.x == 0) {
    a.lp[inst] = lp;
    if (a.logp) a.logp[inst] = lp;
    if (lp != lp || lp == INFINITY) atomicOr(a.flag, kFlagNonFinite);
  }
  const bool fin = lp == lp && lp != INFINITY && lp != -INFINITY;
  for (int kt = threadIdx.x; kt < Kt; kt += blockDim.x)
    w[kt] = fin ? exp(w[kt] - lnKt - lp) : (lp == -INFINITY ? 0.0 : (double)NAN);
}

// Local gradients: a workgroup per (instance and point, 64 local samples).  Lane ->
// local sample k; wave wv takes global rows wv, wv + 8, .. of each staged chunk.
// Writes du, dz, and this block's part of ds: sum_{kt,k} G (lam diff^2 - 1).
template <typename T, int DB>
__global__ __launch_bounds__(kStarThreads) void k_star_bwd_local(StarArgs<T> a) {
  __shared__ T ms[kStarChunk * DB];
  __shared__ T wt[kStarChunk];
  __shared__ T mg[kStarChunk];
  __shared__ T cb[kStarWaves][kStarLanes];
  const int64_t pi = blockIdx.x;
  const int inst = (int)(pi / a.N);
  const int kb = blockIdx.y;
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int D = a.D, K = a.K, Kt = a.Kt;
  const int k = kb * kStarLanes + lane;
  const bool kv = k < K;
  T lam[DB], zk[DB];
  const T c0 = star_consts<T, DB>(a.s + (int64_t)inst * D, D, lam);
#pragma unroll
  for (int d = 0; d < DB; ++d) zk[d] = (kv && d < D) ? a.z[(pi * K + k) * D + d] : (T)0;
  const T uk = kv ? a.u[pi * K + k] : (T)0;
  lds_zero<T, kStarChunk * DB>(ms);
  const double lnK = log((double)K);
  const T* mth = a.mth + (int64_t)inst * Kt * D;
  T gs = (T)0, gz[DB], gq[DB];
#pragma unroll
  for (int d = 0; d < DB; ++d) gz[d] = gq[d] = (T)0;
  for (int t0 = 0; t0 < Kt; t0 += kStarChunk) {
    const int nt = min(kStarChunk, Kt - t0);
    __syncthreads();
    star_stage<T, DB>(ms, mth, t0, nt, D);
    for (int e = threadIdx.x; e < nt; e += blockDim.x) {
      wt[e] = (T)a.w[(int64_t)inst * Kt + t0 + e];
      mg[e] = (T)(a.msg[pi * Kt + t0 + e] + lnK);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRowsPerWave; ++r) {
      const int t = wv + kStarWaves * r;
      if (t < nt) {
        const T* mrow = &ms[t * DB];
        const T x = uk + c0 + star_quad<T, DB>(zk, mrow, lam);
        const T wtt = wt[t];
        const T G = (kv && wtt != (T)0) ? wtt * fast_exp(x - mg[t]) : (T)0;
        gs += G;
#pragma unroll
        for (int d = 0; d < DB; ++d) {
          const T df = zk[d] - mrow[d];
          gz[d] += G * df;
          gq[d] += G * df * df;
        }
      }
    }
  }
  const double g = a.dlogp[inst];
  const double Gs = waves_sum<T>(gs, cb, wv, lane);
  if (wv == 0 && kv && a.du) a.du[pi * K + k] = (T)(g * Gs);
  if (a.dz) {
#pragma unroll
    for (int d = 0; d < DB; ++d) {
      if (d < D) {   // (uniform)
        const double v = waves_sum<T>(gz[d], cb, wv, lane);
        if (wv == 0 && kv) a.dz[(pi * K + k) * D + d] = (T)(-g * (double)lam[d] * v);
      }
    }
  }
  if (a.ds) {
#pragma unroll
    for (int d = 0; d < DB; ++d) {
      if (d < D) {   // (uniform)
        const double v = waves_sum<T>(gq[d], cb, wv, lane);
        // sum_{kt} G (lam diff^2 - 1) of this lane's sample, then over the lanes
        const double lv = wave_sum(kv ? (double)lam[d] * v - Gs : 0.0);
        if (wv == 0 && lane == 0) a.dsp[(pi * a.nkb + kb) * D + d] = lv;
      }
    }
  }
}

// d mth parts: a workgroup per (instance, group of P points, 64 global samples), the
// loop structure of k_star_msg; per lane sum_i sum_k G (z_ik - mth[kt]) over the group.
template <typename T, int DB>
__global__ __launch_bounds__(kStarThreads) void k_star_bwd_global(StarArgs<T> a) {
  __shared__ T zs[kStarChunk * DB];
  __shared__ T us[kStarChunk];
  __shared__ T cb[kStarWaves][kStarLanes];
  const int inst = blockIdx.x / a.ngrp, grp = blockIdx.x - inst * a.ngrp;
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int D = a.D, K = a.K, Kt = a.Kt;
  const int kt = blockIdx.y * kStarLanes + lane;
  const bool ktv = kt < Kt;
  T lam[DB], mt[DB], gm[DB];
  const T c0 = star_consts<T, DB>(a.s + (int64_t)inst * D, D, lam);
#pragma unroll
  for (int d = 0; d < DB; ++d) {
    mt[d] = (ktv && d < D) ? a.mth[((int64_t)inst * Kt + kt) * D + d] : (T)0;
    gm[d] = (T)0;
  }
  lds_zero<T, kStarChunk * DB>(zs);
  const T wk = ktv ? (T)a.w[(int64_t)inst * Kt + kt] : (T)0;
  const double lnK = log((double)K);
  const int p0 = grp * a.P, p1 = min(a.N, p0 + a.P);
  for (int pt = p0; pt < p1; ++pt) {
    const int64_t pi = (int64_t)inst * a.N + pt;
    const T* z = a.z + pi * K * D;
    const T* u = a.u + pi * K;
    const T mgt = ktv ? (T)(a.msg[pi * Kt + kt] + lnK) : (T)0;
    for (int k0 = 0; k0 < K; k0 += kStarChunk) {
      const int nk = min(kStarChunk, K - k0);
      __syncthreads();
      star_stage<T, DB>(zs, z, k0, nk, D);
      for (int e = threadIdx.x; e < nk; e += blockDim.x) us[e] = u[k0 + e];
      __syncthreads();
      if (wk != (T)0) {
#pragma unroll
        for (int r = 0; r < kRowsPerWave; ++r) {
          const int k = wv + kStarWaves * r;
          if (k < nk) {
            const T* zrow = &zs[k * DB];
            const T G = wk * fast_exp(us[k] + c0 + star_quad<T, DB>(zrow, mt, lam) - mgt);
#pragma unroll
            for (int d = 0; d < DB; ++d) gm[d] += G * (zrow[d] - mt[d]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int d = 0; d < DB; ++d) {
    if (d < D) {   // (uniform)
      const double v = waves_sum<T>(gm[d], cb, wv, lane);
      if (wv == 0 && ktv) a.dm[(((int64_t)inst * a.ngrp + grp) * Kt + kt) * D + d] = v;
    }
  }
}

// Final sums.  Blocks y < ceil(Kt D / 64): d mth of 64 entries (wave wv sums groups
// wv, wv + 8, ..; then the waves in order), scaled by dlogp lam.  Block y = last: ds
// (the workgroup strides over the N * nkb parts, then a fixed-order tree) and
// d uth = dlogp w.
template <typename T>
__global__ __launch_bounds__(kStarThreads) void k_star_reduce(StarArgs<T> a) {
  __shared__ double part[kStarWaves][kStarLanes];
  __shared__ double red[kMaxWaves];
  const int inst = blockIdx.x;
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const int D = a.D, Kt = a.Kt;
  const int64_t KD = (int64_t)Kt * D;
  const double g = a.dlogp[inst];
  if (blockIdx.y + 1 < gridDim.y) {
    if (!a.dmth) return;   // (uniform)
    const int64_t e = (int64_t)blockIdx.y * kStarLanes + lane;
    const bool ev = e < KD;
    double acc = 0.0;
    if (ev)
      for (int gi = wv; gi < a.ngrp; gi += kStarWaves) acc += a.dm[((int64_t)inst * a.ngrp + gi) * KD + e];
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && ev) {
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < kStarWaves; ++w) v += part[w][lane];
      const int d = (int)(e % D);
      const double lam = exp(-2.0 * (double)a.s[(int64_t)inst * D + d]);
      a.dmth[(int64_t)inst * KD + e] = (T)(g * lam * v);
    }
    return;
  }
  if (a.ds) {
    const int64_t nparts = (int64_t)a.N * a.nkb;
    const double* dsp = a.dsp + (int64_t)inst * nparts * D;
    for (int d = 0; d < D; ++d) {
      double acc = 0.0;
      for (int64_t j = threadIdx.x; j < nparts; j += blockDim.x) acc += dsp[j * D + d];
      acc = block_sum(acc, red);
      if (threadIdx.x == 0) a.ds[(int64_t)inst * D + d] = (T)(g * acc);
    }
  }
  if (a.duth)
    for (int kt = threadIdx.x; kt < Kt; kt += blockDim.x)
      a.duth[(int64_t)inst * Kt + kt] = (T)(g * a.w[(int64_t)inst * Kt + kt]);
}

// ---- launchers ----
#define TMC_STAR_BY_WIDTH(KERNEL, grid)                                                      \
  do {                                                                                       \
    if (a.D <= 1) hipLaunchKernelGGL((KERNEL<T, 1>), grid, dim3(kStarThreads), 0, st, a);    \
    else if (a.D <= 4) hipLaunchKernelGGL((KERNEL<T, 4>), grid, dim3(kStarThreads), 0, st, a); \
    else if (a.D <= 16) hipLaunchKernelGGL((KERNEL<T, 16>), grid, dim3(kStarThreads), 0, st, a); \
    else hipLaunchKernelGGL((KERNEL<T, 32>), grid, dim3(kStarThreads), 0, st, a);            \
  } while (0)

template <typename T>
hipError_t launch_star_msg(const StarArgs<T>& a, hipStream_t st) {
  const dim3 grid(a.S * a.ngrp, (a.Kt + kStarLanes - 1) / kStarLanes);
  TMC_STAR_BY_WIDTH(k_star_msg, grid);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_star_colsum(const StarArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL((k_star_colsum<T>), dim3(a.S, (a.Kt + kStarLanes - 1) / kStarLanes),
                     dim3(kStarThreads), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_star_logp(const StarArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL((k_star_logp<T>), dim3(a.S), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_star_bwd_local(const StarArgs<T>& a, hipStream_t st) {
  const dim3 grid(a.S * a.N, a.nkb);
  TMC_STAR_BY_WIDTH(k_star_bwd_local, grid);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_star_bwd_global(const StarArgs<T>& a, hipStream_t st) {
  const dim3 grid(a.S * a.ngrp, (a.Kt + kStarLanes - 1) / kStarLanes);
  TMC_STAR_BY_WIDTH(k_star_bwd_global, grid);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_star_reduce(const StarArgs<T>& a, hipStream_t st) {
  const int64_t KD = (int64_t)a.Kt * a.D;
  const int ny = (int)((KD + kStarLanes - 1) / kStarLanes) + 1;
  hipLaunchKernelGGL((k_star_reduce<T>), dim3(a.S, ny), dim3(kStarThreads), 0, st, a);
  return hipGetLastError();
}
#undef TMC_STAR_BY_WIDTH

#define TMC_STAR_INST(T)                                                       \
  template hipError_t launch_star_msg<T>(const StarArgs<T>&, hipStream_t);     \
  template hipError_t launch_star_colsum<T>(const StarArgs<T>&, hipStream_t);  \
  template hipError_t launch_star_logp<T>(const StarArgs<T>&, hipStream_t);    \
  template hipError_t launch_star_bwd_local<T>(const StarArgs<T>&, hipStream_t); \
  template hipError_t launch_star_bwd_global<T>(const StarArgs<T>&, hipStream_t); \
  template hipError_t launch_star_reduce<T>(const StarArgs<T>&, hipStream_t);
TMC_STAR_INST(float)
TMC_STAR_INST(double)
#undef TMC_STAR_INST

}  // namespace tmc

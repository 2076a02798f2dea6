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
// The 64 lanes of a wave take 64 samples of one index and the wave walks the other,
// reading those rows (shared by all its lanes) with scalar loads: no LDS staging and no
// barrier in the loops.  Every sum across lanes, waves, points or workgroups runs in a
// fixed order, so results are deterministic.  Per-entry arithmetic is in T (the plan's
// precision); per-row results and sums over rows are double.
#include <math.h>

#include <limits>

#include "dev_util.h"
#include "tmc_internal.h"
#include "tmc_star.h"

namespace tmc {

namespace {

constexpr int kStarThreads = kStarWaves * kWave;
constexpr double kLn2Pi = 1.8378770664093454836;
constexpr double kLog2eD = 1.4426950408889634074;

// The wave's index as a wave-uniform value: addresses built from it stay in scalar
// registers, so rows that every lane of a wave reads (a point's local samples, a global
// sample's mean) are fetched once per wave by scalar loads and used as scalar operands.
__device__ __forceinline__ int wave_index() { return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave); }

__device__ __forceinline__ float exp2_t(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double exp2_t(double x) { return exp2(x); }

// Per-instance constants: nlam_d = -1/2 exp(-2 s_d) (0 past D); returns
// c = -sum_d s_d - D/2 ln(2 pi) (FP64).
template <typename T, int DB>
__device__ __forceinline__ double star_consts(const T* __restrict__ s, int D, T (&nlam)[DB]) {
  double ssum = 0.0;
#pragma unroll
  for (int d = 0; d < DB; ++d) {
    const double sd = d < D ? (double)s[d] : 0.0;
    nlam[d] = d < D ? (T)(-0.5 * exp(-2.0 * sd)) : (T)0;
    ssum += sd;
  }
  return -ssum - 0.5 * (double)D * kLn2Pi;
}

// u + f - c for one (local row zr, global mean mt): u + sum_d nlam_d (zr_d - mt_d)^2.
// For DB = 1 the width is 1 (rows are consecutive values).
template <typename T, int DB>
__device__ __forceinline__ T star_x(const T* __restrict__ zr, const T (&mt)[DB], const T (&nlam)[DB],
                                    int D, T u) {
  T x = u;
#pragma unroll
  for (int d = 0; d < DB; ++d) {
    if (DB == 1 || d < D) {   // (uniform)
      const T t = zr[d] - mt[d];
      x = fma(nlam[d] * t, t, x);
    }
  }
  return x;
}

// Adds rows [k0, k0 + NR) of one point to a lane's running log-sum-exp (mx, sm), sm in
// units of exp(mx): the rows' maximum first, one rescale, then the exponentials, each
// exp(x - mx) as exp2 of one fused multiply-add.  Branch-free: the maximum ignores NaN
// (fmax) while a NaN row still makes the sum NaN; an all -inf prefix keeps (mx, sm) =
// (-inf, 0).
// Rows a step batches (loads first): kStarRows for narrow latents, fewer for wide ones
// (a row's working set is DB values per lane; batching 8 of them at d = 32 exceeds the
// register file).  The rows are still taken in order, so the sums do not change.
template <typename T, int DB>
constexpr int kRowsFor = (DB * (int)sizeof(T) <= 16)    ? kStarRows
                         : (DB * (int)sizeof(T) <= 64)  ? kStarRows / 2
                         : (DB * (int)sizeof(T) <= 128) ? kStarRows / 4
                                                        : 1;

template <typename T, int DB, int NR>
__device__ __forceinline__ void star_rows(const T* __restrict__ z, const T* __restrict__ u, int k0,
                                          int D, const T (&mt)[DB], const T (&nlam)[DB], T& mx, T& sm) {
  const T l2e = (T)kLog2eD;
  const int stride = DB == 1 ? 1 : D;
  T ur[NR], x[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) ur[r] = u[k0 + r];   // (all loads of the step first)
#pragma unroll
  for (int r = 0; r < NR; ++r) x[r] = star_x<T, DB>(z + (int64_t)(k0 + r) * stride, mt, nlam, D, ur[r]);
  T m = mx;
#pragma unroll
  for (int r = 0; r < NR; ++r) m = fmax(m, x[r]);
  const T nsh = m == (T)(-INFINITY) ? (T)0 : -m * l2e;
  T acc = sm * exp2_t(fma(mx, l2e, nsh));
#pragma unroll
  for (int r = 0; r < NR; ++r) acc += exp2_t(fma(x[r], l2e, nsh));
  sm = acc;
  mx = m;
}

}  // namespace

// Messages.  A workgroup per (instance, group of P points, 64 global samples); lane ->
// global sample kt, and the waves take the group's points in turn (wave wv: points
// wv, wv + 4, ..).  A wave walks all K local samples of its point, kRowsFor at a time,
// reading them with scalar loads, and keeps a running (max, sum) per lane; no LDS and no
// barrier until the group's sums of m_i are combined in wave order.
template <typename T, int DB>
__global__ __launch_bounds__(kStarThreads) void k_star_msg(StarArgs<T> a) {
  __shared__ double part[kStarWaves][kStarLanes];
  const int inst = blockIdx.x / a.ngrp, grp = blockIdx.x - inst * a.ngrp;
  const int lane = threadIdx.x % kWave, wv = wave_index();
  const int D = a.D, K = a.K, Kt = a.Kt;
  const int kt = blockIdx.y * kStarLanes + lane;
  const bool ktv = kt < Kt;
  T nlam[DB], mt[DB];
  const double c0 = star_consts<T, DB>(a.s + (int64_t)inst * D, D, nlam);
#pragma unroll
  for (int d = 0; d < DB; ++d) mt[d] = (ktv && d < D) ? a.mth[((int64_t)inst * Kt + kt) * D + d] : (T)0;
  const double cK = c0 - log((double)K);
  double gacc = 0.0;
  const int p1 = min(a.N, (grp + 1) * a.P);
  for (int pt = grp * a.P + wv; pt < p1; pt += kStarWaves) {
    const int64_t pi = (int64_t)inst * a.N + pt;
    const T* z = a.z + pi * K * D;
    const T* u = a.u + pi * K;
    T mx = (T)(-INFINITY), sm = (T)0;
    int k = 0;
    constexpr int NRB = kRowsFor<T, DB>;
    for (; k + NRB <= K; k += NRB) star_rows<T, DB, NRB>(z, u, k, D, mt, nlam, mx, sm);
    for (; k < K; ++k) star_rows<T, DB, 1>(z, u, k, D, mt, nlam, mx, sm);
    // (all -inf: -inf + log 0 = -inf; a NaN row: log NaN = NaN)
    const double lse = (double)mx + log((double)sm);   // m_i + ln K - c
    const double mi = lse + cK;
    if (ktv) {
      a.msg[pi * Kt + kt] = mi;
      // clamped: an all -inf point meets only -inf exponents there (never inf - inf)
      a.nsh[pi * Kt + kt] = (T)fmin(-lse * kLog2eD, (double)std::numeric_limits<T>::max());
    }
    gacc += mi;
  }
  part[wv][lane] = gacc;
  __syncthreads();
  if (wv == 0 && ktv) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kStarWaves; ++w) v += part[w][lane];
    a.gsum[((int64_t)inst * a.ngrp + grp) * Kt + kt] = v;
  }
}

// The sums over point groups (logits of the global samples, the d mth parts) are few
// but long: a workgroup of kRedWaves waves per 64 sums, each wave a strided share of the
// groups with kRedUnroll loads in flight, so that the latency of the loads is spread
// over many waves.
constexpr int kRedWaves = 16;
constexpr int kRedUnroll = 16;

// Logits of the global samples: w[kt] = uth[kt] + sum over groups of gsum.  A workgroup
// per (instance, 64 kt); wave wv sums groups wv, wv + kRedWaves, .. (added in group
// order), then the waves in order.
template <typename T>
__global__ __launch_bounds__(kRedWaves * kWave) void k_star_colsum(StarArgs<T> a) {
  __shared__ double part[kRedWaves][kStarLanes];
  const int inst = blockIdx.x;
  const int lane = threadIdx.x % kWave, wv = wave_index();
  const int kt = blockIdx.y * kStarLanes + lane;
  const bool ktv = kt < a.Kt;
  const double* gs = a.gsum + (int64_t)inst * a.ngrp * a.Kt + (ktv ? kt : 0);
  double acc = 0.0;
  constexpr int U = kRedUnroll;
  for (int g0 = wv; g0 < a.ngrp; g0 += kRedWaves * U) {
    double v[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int g = g0 + kRedWaves * q;
      v[q] = g < a.ngrp ? gs[(int64_t)g * a.Kt] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < U; ++q) acc += v[q];
  }
  part[wv][lane] = acc;
  __syncthreads();
  if (wv == 0 && ktv) {
    double v = (double)a.uth[(int64_t)inst * a.Kt + kt];
#pragma unroll
    for (int w = 0; w < kRedWaves; ++w) v += part[w][lane];
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
  for (int kt = threadIdx.x; kt < Kt; kt += blockDim.x) {
    const double v = fin ? exp(w[kt] - lnKt - lp) : (lp == -INFINITY ? 0.0 : (double)NAN);
    w[kt] = v;
    a.wT[(int64_t)inst * Kt + kt] = (T)v;
  }
}

// Local gradients.  A wave per (instance and point, 64 local samples): lane -> local
// sample k; the wave walks every global sample t, kRowsFor at a time (mean, weight and
// this point's message by scalar loads; samples of weight 0 add 0) and accumulates
//   gs = sum_t G,  gz_d = sum_t G (z_kd - mth_td),  gq_d = sum_t G (z_kd - mth_td)^2
// with G = w_t exp(u_k + f[t, k] - m_i[t] - ln K).  Writes du, dz and this block's part of
// ds: sum_k (lam_d gq_d - gs) over its lanes.
template <typename T, int DB>
__global__ __launch_bounds__(kStarThreads) void k_star_bwd_local(StarArgs<T> a) {
  const int lane = threadIdx.x % kWave, wv = wave_index();
  const int64_t task = (int64_t)blockIdx.x * kStarWaves + wv;
  if (task >= (int64_t)a.S * a.N * a.nkb) return;   // (uniform per wave; no barrier below)
  const int64_t pi = task / a.nkb;
  const int kb = (int)(task - pi * a.nkb);
  const int inst = (int)(pi / a.N);
  const int D = a.D, K = a.K, Kt = a.Kt;
  const int k = kb * kStarLanes + lane;
  const bool kv = k < K;
  T nlam[DB], zk[DB];
  (void)star_consts<T, DB>(a.s + (int64_t)inst * D, D, nlam);
#pragma unroll
  for (int d = 0; d < DB; ++d) zk[d] = (kv && d < D) ? a.z[(pi * K + k) * D + d] : (T)0;
  const T uk = kv ? a.u[pi * K + k] : (T)(-INFINITY);
  const T* mth = a.mth + (int64_t)inst * Kt * D;
  const T* w = a.wT + (int64_t)inst * Kt;
  const T* nshp = a.nsh + pi * Kt;
  const T l2e = (T)kLog2eD;
  T gs = (T)0, gz[DB], gq[DB];
#pragma unroll
  for (int d = 0; d < DB; ++d) gz[d] = gq[d] = (T)0;
  // one global sample (weight wt, exponent offset nt) into the lane's sums; a sample of
  // weight 0 adds 0 (its offset is finite, or the lane's exponent is -inf)
  auto row = [&](const T* mr, T wt, T nt) {
    T x = uk, df[DB];
#pragma unroll
    for (int d = 0; d < DB; ++d) {
      df[d] = (DB == 1 || d < D) ? zk[d] - mr[d] : (T)0;
      x = fma(nlam[d] * df[d], df[d], x);
    }
    const T G = wt * exp2_t(fma(x, l2e, nt));
    gs += G;
#pragma unroll
    for (int d = 0; d < DB; ++d) {
      gz[d] = fma(G, df[d], gz[d]);
      gq[d] = fma(G * df[d], df[d], gq[d]);
    }
  };
  const int stride = DB == 1 ? 1 : D;
  int t = 0;
  constexpr int NRB = kRowsFor<T, DB>;
  for (; t + NRB <= Kt; t += NRB) {
    T wr[NRB], nr[NRB];
#pragma unroll
    for (int r = 0; r < NRB; ++r) {   // (all loads of the step first)
      wr[r] = w[t + r];
      nr[r] = nshp[t + r];
    }
#pragma unroll
    for (int r = 0; r < NRB; ++r) row(mth + (int64_t)(t + r) * stride, wr[r], nr[r]);
  }
  for (; t < Kt; ++t) row(mth + (int64_t)t * stride, w[t], nshp[t]);
  const double g = a.dlogp[inst];
  if (kv && a.du) a.du[pi * K + k] = (T)(g * (double)gs);
  if (a.dz && kv) {
    // dz = -dlogp lam sum_t G (z - mth_t),  -lam = 2 nlam
#pragma unroll
    for (int d = 0; d < DB; ++d)
      if (d < D) a.dz[(pi * K + k) * D + d] = (T)(g * 2.0 * (double)nlam[d] * (double)gz[d]);
  }
  if (a.ds) {
#pragma unroll
    for (int d = 0; d < DB; ++d) {
      if (d < D) {   // (uniform)
        const double lam = -2.0 * (double)nlam[d];
        const double lv = wave_sum(kv ? lam * (double)gq[d] - (double)gs : 0.0);
        if (lane == 0) a.dsp[(pi * a.nkb + kb) * D + d] = g * lv;
      }
    }
  }
}

// d mth parts: a workgroup per (instance, group of P points, 64 global samples) as in
// k_star_msg; per lane, gm_d = sum over the wave's points and their local samples of
// G (z_kd - mth_d), with G = w exp(u_k + f - m_i - ln K) (lanes of weight 0: G = 0); the
// waves' sums combined in wave order.
template <typename T, int DB>
__global__ __launch_bounds__(kStarThreads) void k_star_bwd_global(StarArgs<T> a) {
  __shared__ double part[kStarWaves][kStarLanes];
  const int inst = blockIdx.x / a.ngrp, grp = blockIdx.x - inst * a.ngrp;
  const int lane = threadIdx.x % kWave, wv = wave_index();
  const int D = a.D, K = a.K, Kt = a.Kt;
  const int kt = blockIdx.y * kStarLanes + lane;
  const bool ktv = kt < Kt;
  T nlam[DB], mt[DB], gm[DB];
  (void)star_consts<T, DB>(a.s + (int64_t)inst * D, D, nlam);
#pragma unroll
  for (int d = 0; d < DB; ++d) {
    mt[d] = (ktv && d < D) ? a.mth[((int64_t)inst * Kt + kt) * D + d] : (T)0;
    gm[d] = (T)0;
  }
  const T wk = ktv ? a.wT[(int64_t)inst * Kt + kt] : (T)0;
  const T l2e = (T)kLog2eD;
  const int stride = DB == 1 ? 1 : D;
  const int p1 = min(a.N, (grp + 1) * a.P);
  for (int pt = grp * a.P + wv; pt < p1; pt += kStarWaves) {
    const int64_t pi = (int64_t)inst * a.N + pt;
    const T* z = a.z + pi * K * D;
    const T* u = a.u + pi * K;
    // (a lane of weight 0 has a finite offset or only -inf exponents: its G are 0)
    const T nsh = ktv ? a.nsh[pi * Kt + kt] : (T)0;
    int k = 0;
    constexpr int NRB = kRowsFor<T, DB>;
    for (; k + NRB <= K; k += NRB) {
      T ur[NRB];
#pragma unroll
      for (int r = 0; r < NRB; ++r) ur[r] = u[k + r];
#pragma unroll
      for (int r = 0; r < NRB; ++r) {
        const T* zr = z + (int64_t)(k + r) * stride;
        T x = ur[r], df[DB];
#pragma unroll
        for (int d = 0; d < DB; ++d) {
          df[d] = (DB == 1 || d < D) ? zr[d] - mt[d] : (T)0;
          x = fma(nlam[d] * df[d], df[d], x);
        }
        const T G = (T)wk * exp2_t(fma(x, l2e, nsh));
#pragma unroll
        for (int d = 0; d < DB; ++d) gm[d] = fma(G, df[d], gm[d]);
      }
    }
    for (; k < K; ++k) {
      const T* zr = z + (int64_t)k * stride;
      T x = u[k], df[DB];
#pragma unroll
      for (int d = 0; d < DB; ++d) {
        df[d] = (DB == 1 || d < D) ? zr[d] - mt[d] : (T)0;
        x = fma(nlam[d] * df[d], df[d], x);
      }
      const T G = (T)wk * exp2_t(fma(x, l2e, nsh));
#pragma unroll
      for (int d = 0; d < DB; ++d) gm[d] = fma(G, df[d], gm[d]);
    }
  }
#pragma unroll
  for (int d = 0; d < DB; ++d) {
    if (d < D) {   // (uniform)
      __syncthreads();
      part[wv][lane] = (double)gm[d];
      __syncthreads();
      if (wv == 0 && ktv) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < kStarWaves; ++w) v += part[w][lane];
        a.dm[(((int64_t)inst * a.ngrp + grp) * Kt + kt) * D + d] = v;
      }
    }
  }
}

// Final sums.  Blocks y < ceil(Kt D / 64): d mth of 64 entries (wave wv sums groups
// wv, wv + kRedWaves, ..; then the waves in order), scaled by dlogp lam.  Block y = last:
// ds (the workgroup strides over the N nkb parts, then a fixed-order tree) and
// d uth = dlogp w.
template <typename T>
__global__ __launch_bounds__(kRedWaves * kWave) void k_star_reduce(StarArgs<T> a) {
  __shared__ double part[kRedWaves][kStarLanes];
  __shared__ double red[kMaxWaves];
  const int inst = blockIdx.x;
  const int lane = threadIdx.x % kWave, wv = wave_index();
  const int D = a.D, Kt = a.Kt;
  const int64_t KD = (int64_t)Kt * D;
  const double g = a.dlogp[inst];
  constexpr int U = kRedUnroll;
  if (blockIdx.y + 1 < gridDim.y) {
    if (!a.dmth) return;   // (uniform)
    const int64_t e = (int64_t)blockIdx.y * kStarLanes + lane;
    const bool ev = e < KD;
    const double* dm = a.dm + (int64_t)inst * a.ngrp * KD + (ev ? e : 0);
    double acc = 0.0;
    for (int g0 = wv; g0 < a.ngrp; g0 += kRedWaves * U) {
      double v[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int gi = g0 + kRedWaves * q;
        v[q] = gi < a.ngrp ? dm[(int64_t)gi * KD] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < U; ++q) acc += v[q];
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && ev) {
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < kRedWaves; ++w) v += part[w][lane];
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
      for (int64_t j0 = threadIdx.x; j0 < nparts; j0 += (int64_t)blockDim.x * U) {
        double v[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
          const int64_t j = j0 + (int64_t)blockDim.x * q;
          v[q] = j < nparts ? dsp[j * D + d] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < U; ++q) acc += v[q];
      }
      acc = block_sum(acc, red);
      if (threadIdx.x == 0) a.ds[(int64_t)inst * D + d] = (T)acc;
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
                     dim3(kRedWaves * kWave), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_star_logp(const StarArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL((k_star_logp<T>), dim3(a.S), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_star_bwd_local(const StarArgs<T>& a, hipStream_t st) {
  const int64_t tasks = (int64_t)a.S * a.N * a.nkb;
  const dim3 grid((unsigned)((tasks + kStarWaves - 1) / kStarWaves));
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
  hipLaunchKernelGGL((k_star_reduce<T>), dim3(a.S, ny), dim3(kRedWaves * kWave), 0, st, a);
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

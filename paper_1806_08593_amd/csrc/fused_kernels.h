// Fused engine kernels (device templates).  The pairwise log-factor
//   f_l[i,j] = log N(z_l^i; mu_l^j, diag exp(2 s_l))
//            = r_i + c + q_j + <lam * z_i, mu_j>,
//   r_i = -1/2 sum_d lam_d z_id^2,  q_j = -1/2 sum_d lam_d mu_jd^2,
//   c   = -sum_d s_d - D/2 ln 2 pi,  lam = exp(-2 s)
// (the diagonal-Gaussian conditional of Sec. "Computational costs for TMC and IWAE")
// is never stored: the inner product runs on MFMA tile by tile and feeds an online
// log-sum-exp (forward) or the pairwise marginals (backward).  The per-sample norms
// r_i, q_j and the constant c are accumulated in FP64 (O(K D) work) so the large,
// cancelling terms of the expansion never pass through FP32; the per-entry arithmetic
// is FP32.
//
// MFMA layouts (v_mfma_f32_32x32x16_bf16 and v_mfma_f32_32x32x2_f32 on gfx950):
//   operand fragment: lane l holds vector (l % 32) and a k-slice selected by l / 32;
//   accumulator: lane l holds column n = l % 32, rows m = 8(v/4) + 4(l/32) + v%4.
// Operands are read from the caller's row-major FP32 z and mu and split in
// registers: BF16X3 keeps x = hi + lo (both bf16) and forms hi*hi + hi*lo + lo*hi;
// FP32 feeds the values directly.  A 16-wide d chunk gives each lane 8 consecutive d
// (d = 16 kc + 8 (l/32) + s); both operands use that same k order.
//
// Pipelining.  Global loads are issued branch-free (clamped addresses, zeros
// selected afterwards) so that a wave's loads are all in flight together, and the
// workgroup barriers wait for LDS traffic only (lds_barrier), never for global loads
// in flight.  Staged operand tiles are double-buffered in LDS when two buffers fit
// beside a second workgroup (d <= 128): tile t+1 is written and tile t+2 fetched while
// tile t is consumed, one barrier per tile.
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
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr float kLog2e = 1.4426950408889634f;
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kHalfLn2Pi = 0.91893853320467274178;
constexpr float kRescale = 8.0f;   // lazy online-max threshold (log2 units)
constexpr int kFusedRowsPerGroup = 128;   // rows per alpha-max partial / ds column part;
                                          // also the rows (columns) of a 4-wave workgroup
constexpr int kFusedBwdColsDev = 128;     // backward columns of a 4-wave workgroup
constexpr int kFusedDzRowsDev = 64;       // rows per row-term item (one ds row partial)

// Kernel arguments (device pointers; see the launchers for their regions).
struct FwdArgs {
  const LayerDev* Ls;
  const Item* items;
  const float *z, *mu, *s, *u;
  double *qcol, *alpha, *wmax;
  float *rl, *ev;
};
struct BwdArgs {
  const LayerDev* Ls;
  const Item* items;
  const float *z, *mu, *s;
  const double *alpha, *wmax, *qcol;
  const float* rl;
  float* lam;
  const double* dlogp;
  float *p, *dmu, *du, *dsp;
  const float* ev;   // softmax-weighted means left by the forward (dz of the row layer)
  float* dz;
  int rows;          // 1: 8-wave items of dz_fused pairs at column 0 write the row terms
};
// Chain queue of a persistent launch: chains[0 .. n) (most expensive first); a
// workgroup takes the next chain from the head counter and runs all of its layer
// pairs itself, so no workgroup ever waits for another.
struct ChainQueue {
  const int* chains;
  int n;
  int* head;
  const ChainDev* cd;
};

// Workgroup barrier that orders LDS traffic only: outstanding global loads stay in
// flight across it (a fence-based __syncthreads would wait for them).
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Two values split at once: x = hi + lo with hi = bf16(x) (nearest even) and
// lo = bf16(x - hi); each plane packs the pair (first value in the low half), so one
// conversion instruction serves two values and hi is widened back by bit operations.
__device__ __forceinline__ void split2(float a, float b, uint32_t& hi, uint32_t& lo) {
  const uint32_t hu = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
  const float ha = __uint_as_float(hu << 16), hb = __uint_as_float(hu & 0xffff0000u);
  hi = hu;
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a - ha, b - hb}, bf16x2));
}

// v combined with the value of lane (l xor 32): the permlane swap hands every lane
// the pair {x[l % 32], x[l % 32 + 32]}; sum and max are symmetric in the pair, so
// both halves of the wave get the identical result.
__device__ __forceinline__ float xor32_sum(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float xor32_max(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
}

// v + (the value of lane l xor m) for m = 1, 2 (quad permutes), 4 (swizzle) and 8 (row
// rotation), FP64: a butterfly built from these leaves the same sum in all its lanes.
template <int M>
__device__ __forceinline__ double xor_add_f64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
  int lo2, hi2;
  if constexpr (M == 1) {
    lo2 = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    hi2 = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
  } else if constexpr (M == 2) {
    lo2 = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    hi2 = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
  } else if constexpr (M == 4) {
    lo2 = __builtin_amdgcn_ds_swizzle(lo, 0x1F | (4 << 10));      // bitmask mode, xor 4
    hi2 = __builtin_amdgcn_ds_swizzle(hi, 0x1F | (4 << 10));
  } else {
    static_assert(M == 8, "xor 1, 2, 4 or 8");
    lo2 = __builtin_amdgcn_mov_dpp(lo, 0x128, 0xF, 0xF, false);  // row_ror:8 = xor 8 in 16 lanes
    hi2 = __builtin_amdgcn_mov_dpp(hi, 0x128, 0xF, 0xF, false);
  }
  return v + __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi2 << 32) | (uint32_t)lo2);
}

// Scheduling hint for a block that holds a chain of N dependent MFMAs and independent
// staging work: one MFMA, then an LDS read, a few VALU instructions and LDS writes, N
// times, so that the staging issues while the matrix core works through the chain.
template <int N>
__device__ __forceinline__ void interleave_mfma() {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
    __builtin_amdgcn_sched_group_barrier(0x002, 5, 0);   // VALU
    __builtin_amdgcn_sched_group_barrier(0x200, 2, 0);   // LDS write
  }
}

// Scheduling hints of the pipelined sweep.  Phase A: the factor-GEMM MFMAs of the next
// tile (two LDS fragment reads ahead of every three MFMAs) with the exponentials and
// operand splits of the current tile between them.  Phase B: the second-GEMM MFMAs
// with the staging of a later tile (VALU and LDS writes) between them.
template <int NMFMA, int NVALU>
__device__ __forceinline__ void interleave_phase_a() {
#pragma unroll
  for (int i = 0; i < NMFMA; ++i) {
    if (i % 3 == 0) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);   // LDS read
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                   // MFMA
    __builtin_amdgcn_sched_group_barrier(0x002, NVALU, 0);               // VALU
  }
}
template <int NMFMA>
__device__ __forceinline__ void interleave_phase_b() {
#pragma unroll
  for (int i = 0; i < NMFMA; ++i) {
    if (i % 6 == 0) __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);   // LDS read
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                   // MFMA
    __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);                   // VALU
    __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);                   // LDS write
  }
}

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
    uint32_t h[4], l[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) split2(x[2 * p], x[2 * p + 1], h[p], l[p]);
    f.hi = __builtin_bit_cast(bf16x8, (u32x4){h[0], h[1], h[2], h[3]});
    f.lo = __builtin_bit_cast(bf16x8, (u32x4){l[0], l[1], l[2], l[3]});
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

// Eight consecutive values row[d0 .. d0+7], zeros past D, without branches: the
// addresses are clamped into the row (which must be a valid row of D >= 1 values).
// `vec`: D % 4 == 0 and the row is 16-byte aligned.
__device__ __forceinline__ void load8(const float* __restrict__ row, int d0, int D, bool vec,
                                      float (&x)[8]) {
  if (vec) {
    const float4 a = *reinterpret_cast<const float4*>(row + min(d0, D - 4));
    const float4 b = *reinterpret_cast<const float4*>(row + min(d0 + 4, D - 4));
    const bool va = d0 < D, vb = d0 + 4 < D;
    x[0] = va ? a.x : 0.0f; x[1] = va ? a.y : 0.0f; x[2] = va ? a.z : 0.0f; x[3] = va ? a.w : 0.0f;
    x[4] = vb ? b.x : 0.0f; x[5] = vb ? b.y : 0.0f; x[6] = vb ? b.z : 0.0f; x[7] = vb ? b.w : 0.0f;
  } else {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const float v = row[min(d0 + s, D - 1)];
      x[s] = (d0 + s < D) ? v : 0.0f;
    }
  }
}

// Four values row[d .. d+3] (zeros past D, or everywhere when !valid), branch-free.
__device__ __forceinline__ float4 load_f4(const float* __restrict__ row, int d, int D, bool valid,
                                          bool vec) {
  float4 r;
  if (vec) {
    r = *reinterpret_cast<const float4*>(row + min(d, D - 4));
    const bool v = valid && d < D;
    r.x = v ? r.x : 0.0f; r.y = v ? r.y : 0.0f; r.z = v ? r.z : 0.0f; r.w = v ? r.w : 0.0f;
  } else {
    const float a = row[min(d + 0, D - 1)], b = row[min(d + 1, D - 1)];
    const float c = row[min(d + 2, D - 1)], e = row[min(d + 3, D - 1)];
    r.x = (valid && d + 0 < D) ? a : 0.0f;
    r.y = (valid && d + 1 < D) ? b : 0.0f;
    r.z = (valid && d + 2 < D) ? c : 0.0f;
    r.w = (valid && d + 3 < D) ? e : 0.0f;
  }
  return r;
}

// The small per-pair inputs of a workgroup's prologue, loaded from clamped addresses
// before the bulk operand loads so that consuming them waits for them alone: this
// lane's partial max of alpha_{l+1} (see pair_maxa), this lane's s values for the
// constant c (d = lane + 64 k, D <= 256), and s_d for d = tix (lam into LDS).
struct PairPre {
  double wm;
  float sv[4];
  float slam;
};

__device__ __forceinline__ void pair_preload(int tix, const LayerDev& L, const double* __restrict__ wmax,
                                             const float* __restrict__ s, PairPre& P) {
  const int lane = tix & 63;
  P.wm = wmax[L.wmax_up_off + min(lane, L.nwmax_up - 1)];
#pragma unroll
  for (int k = 0; k < 4; ++k) P.sv[k] = s[L.s_off + min(lane + 64 * k, L.D - 1)];
  P.slam = s[L.s_off + min(tix, L.D - 1)];
}

// Column shift of pair L: maxa = max_j alpha_{l+1}[j], reduced over the
// per-workgroup maxima the pass that wrote alpha_{l+1} left in wmax (one lane per
// partial, then a wave reduction; exact, so the order does not matter).
__device__ __forceinline__ double pair_maxa(int tix, const LayerDev& L, const double* __restrict__ wmax,
                                            const PairPre& P) {
  const int lane = tix & 63;
  double m = (lane < L.nwmax_up) ? P.wm : -INFINITY;
  for (int k = lane + 64; k < L.nwmax_up; k += 64) m = nan_max(m, wmax[L.wmax_up_off + k]);
  m = wave_max(m);
  return (m == -INFINITY) ? 0.0 : m;
}

// c = -sum_d s_d - D/2 ln 2 pi of pair L in FP64 (fixed order: lane-strided partial
// sums, then a butterfly over the wave), complete in every lane of the calling wave.
__device__ __forceinline__ double pair_const(int tix, const LayerDev& L, const PairPre& P) {
  const int lane = tix & 63;
  double a = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) a += (lane + 64 * k < L.D) ? (double)P.sv[k] : 0.0;
  a = wave_sum(a);
  return -a - (double)L.D * kHalfLn2Pi;
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

// An accumulator column (16 values in accumulator row order) prepared as the B operand
// of mma_t: FP32 keeps the values, BF16X3 splits them once into hi/lo fragments.
template <int PREC>
struct PFrag;
template <>
struct PFrag<TMC_FP32> {
  float x[16];
};
template <>
struct PFrag<TMC_BF16X3> {
  Frag<TMC_BF16X3> f[2];
};

template <int PREC>
__device__ __forceinline__ void make_pfrag(const float (&p)[16], PFrag<PREC>& o) {
  if constexpr (PREC == TMC_FP32) {
#pragma unroll
    for (int v = 0; v < 16; ++v) o.x[v] = p[v];
  } else {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      float a[8];
#pragma unroll
      for (int s2 = 0; s2 < 8; ++s2) a[s2] = p[8 * t + s2];
      make_frag<TMC_BF16X3>(a, o.f[t]);
    }
  }
}

// acc[d][n] += sum_k T[d][k] P[k][n] where P is this lane's accumulator column.
template <int PREC>
__device__ __forceinline__ void mma_t(f32x16& acc, const TFrag<PREC>& T, const PFrag<PREC>& P) {
  if constexpr (PREC == TMC_FP32) {
#pragma unroll
    for (int v = 0; v < 16; ++v) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(T.x[v], P.x[v], acc, 0, 0, 0);
  } else {
#pragma unroll
    for (int t = 0; t < 2; ++t) mma_chunk<TMC_BF16X3>(acc, T.f[t], P.f[t]);
  }
}

// ---------------------------------------------------------------------------
// LDS staging of NS operand tiles of 32 samples (rows of mu or of z), written once
// per workgroup and read by all four waves, in NB buffers.  Per 32-row subtile:
//   row-major copy: fragments with the d chunk along k (factor GEMM);
//   d-major copy:   fragments with the tile rows along k (G^T z, softmax * mu),
//                   row r stored at column perm(r) (bits 2 and 3 of r swapped) so the
//                   8 rows a lane needs for one k-step are adjacent (only when COL).
// Every fragment is one or two 128-bit LDS reads.  BF16X3 keeps two bf16 planes
// (hi, lo), FP32 one float plane.  BF16X3 has no d-major copies: the second GEMM reads
// the row-major copy through LDS transpose reads (tile_rowT_frag).
// ---------------------------------------------------------------------------
// Row stride (elements) of the BF16 row-major copy.  The LDS has 64 banks of 4 bytes
// and serves 16 lanes of a 64- or 128-bit access per pass.  With a stride of sigma
// dwords, sigma = 4 s (mod 64), the 16 rows of one pass of a fragment read (16 bytes
// each, same columns) sit at 16-byte slots s r (mod 16): distinct for odd s.  The four
// rows of one pass of a transpose read (32 bytes each) sit at slots 0, s, 2 s, 3 s, which
// must stay two slots apart: s in {3, 7, 9, 13}.  One-subtile layouts (the ones read
// through transpose reads) take the smallest such stride from DT + 8; two-subtile
// layouts (no transpose reads) keep DT + 8, which leaves room for two workgroups per CU.
constexpr int bf_row_stride(int DT, int NS) {
  if (NS != 1) return DT + 8;
  int rs = DT + 8;
  for (;; rs += 8) {
    const int sl = ((rs / 2) % 64) / 4;
    if (sl == 3 || sl == 7 || sl == 9 || sl == 13) break;
  }
  return rs;
}

template <int PREC, int NKC, int NS_, int NB_, bool COL_, bool RAW_ = false>
struct TileSmem {
  static constexpr int NS = NS_, NB = NB_;
  static constexpr bool COL = COL_;   // d-major copy of the raw values
  static constexpr bool RAW = RAW_;   // second row-major copy holding the raw values (the
                                      // first one scaled), read through transpose reads
  static constexpr int DP = NKC * 16;               // padded width
  static constexpr int ND32 = (NKC + 1) / 2;        // 32-wide d blocks
  static constexpr int DT = ND32 * 32;              // rows of the d-major copy; also the
                                                    // d span the staging threads cover
  static constexpr bool BF = PREC == TMC_BF16X3;
  static constexpr int NPL = BF ? 2 : 1;
  static constexpr int RS = BF ? bf_row_stride(DT, NS) : DT + 4;   // row stride (elements)
  static constexpr int CS = BF ? 40 : 36;           // d-major stride (elements)
  static constexpr int ROWN = 32 * RS, COLN = DT * CS;
  static constexpr int COLSZ = COL ? NS * COLN : 2;
  typedef typename std::conditional<BF, __bf16, float>::type E;
  E row[NB][NPL][NS * ROWN];
  E col[NB][NPL][COLSZ];
  E raw[NB][NPL][RAW ? NS * ROWN : 2];
  // lam_d in FP64 (column norms), split so that the staging threads' reads of 4
  // consecutive d (two 16-byte reads each) are contiguous across threads:
  // lamdA[f] = (lam_4f, lam_4f+1), lamdB[f] = (lam_4f+2, lam_4f+3)
  double2 lamdA[DT / 4];
  double2 lamdB[DT / 4];
  float lamf[DT];        // lam_d = exp(-2 s_d)            (0 past D)
  float lam2[DT];        // log2(e) * lam_d
  float rlam2[DT];       // 1 / (log2(e) lam_d)             (0 past D)
  float gam[NB][NS * 32];   // column terms of the staged tiles (forward)
  float lamT[NB][NS * 32];  // row shifts of the staged tiles (backward)
  double wm[8];          // per-wave maxima of alpha (forward)
};

__device__ __forceinline__ int tile_perm(int r) {
  return (r & 0x13) | ((r & 4) << 1) | ((r & 8) >> 1);
}

// lam into LDS (thread d holds s_d, DT <= blockDim; zeros past D).
template <class TS>
__device__ __forceinline__ void tile_init(int tix, TS& T, const LayerDev& L, const PairPre& P) {
  const int d = tix;
  if (d < TS::DT) {
    const float lf = d < L.D ? expf(-2.0f * P.slam) : 0.0f;
    T.lamf[d] = lf;
    const float k2 = (float)L.kappa * kLog2e;   // weights raised to the power kappa
    T.lam2[d] = lf * k2;
    T.rlam2[d] = lf > 0.0f ? 1.0f / (lf * k2) : 0.0f;
    reinterpret_cast<double*>((d & 2) ? &T.lamdB[d >> 2] : &T.lamdA[d >> 2])[d & 1] = (double)lf;
  }
}

// Register stage of NS tiles (blockDim 64 WV): thread t serves row t / TPR of every
// subtile and float4 columns 4 (t % TPR + TPR m), d < DT, with TPR = 2 WV threads per
// row.  Slots past the data -- rows
// past the block's end, d >= D -- hold zeros (unaligned path) or copies of real values
// of the block (aligned path: clamped addresses).  Either is harmless: such d meet an
// exact zero (lam_d = 0, zero padding of the register operand) or land in outputs that
// are discarded, and such rows get a -inf shift (gamma_j, or Lam_i = +inf).
template <int NKC, int NS_, int WV = 4>
struct TilePrefetch {
  static constexpr int NS = NS_;
  static constexpr int NF = (NKC + 1) / 2;       // float4 columns of a row (4 NF = DT)
  static constexpr int TPR = 2 * WV;             // threads per row
  static constexpr int NFT = NF * 8 / TPR;       // float4 columns per thread
  static_assert(WV == 4 || WV == 8, "4 or 8 waves");
  static_assert(NKC <= 8 || WV == 4, "8-wave workgroups for d <= 128 only");
  static_assert(NFT * TPR == NF * 8, "8-wave staging needs an even float4 count");
  float4 v[NS][NFT];
  double a[NS];      // column tiles: alpha_{l+1}[j]
  float lam;         // row tiles: row shift of row t % (32 NS) (+inf applied at the store)
  int rem;           // rows of the stage that exist, counted from its first row
  int r0;            // row tiles: first row of the stage
  float4 e[NS][NFT]; // row tiles with dz: e of the thread's row (same columns as v)
  float prow[NS];    // row tiles with dz: marginal p of the thread's row (0 past K)
};

// Column tiles of pair L: mu rows r0.. (samples of layer l+1) and their alpha.
template <int NKC, int NS, int WV>
__device__ __forceinline__ void fetch_cols(int tix, TilePrefetch<NKC, NS, WV>& pf, const LayerDev& L,
                                           const float* __restrict__ mu,
                                           const double* __restrict__ alpha, int r0) {
  constexpr int TPR = TilePrefetch<NKC, NS, WV>::TPR, NFT = TilePrefetch<NKC, NS, WV>::NFT;
  const int t = tix, sub = t % TPR;
  const bool vec = (L.D % 4 == 0) && (L.mu_off % 4 == 0);
  pf.rem = L.Kc - r0;
  if (vec) {
    // loads only (clamped into the block): the values are not used until the stage is
    // written to LDS, so the loads stay in flight across the compute of the current tile
#pragma unroll
    for (int sb = 0; sb < NS; ++sb) {
      const int gc = min(r0 + 32 * sb + (t / TPR), L.Kc - 1);
      const float* rowp = mu + L.mu_off + (int64_t)gc * L.D;
#pragma unroll
      for (int m = 0; m < NFT; ++m)
        pf.v[sb][m] = *reinterpret_cast<const float4*>(rowp + min(opaque(4 * (sub + TPR * m)), L.D - 4));
      pf.a[sb] = alpha[L.alpha_up_off + gc];
    }
    return;
  }
#pragma unroll
  for (int sb = 0; sb < NS; ++sb) {
    const int gr = r0 + 32 * sb + (t / TPR);
    const bool valid = gr < L.Kc;
    const int gc = valid ? gr : L.Kc - 1;
    const float* rowp = mu + L.mu_off + (int64_t)gc * L.D;
#pragma unroll
    for (int m = 0; m < NFT; ++m)
      pf.v[sb][m] = load_f4(rowp, opaque(4 * (sub + TPR * m)), L.D, valid, false);
    pf.a[sb] = alpha[L.alpha_up_off + gc];
  }
}

// Row tiles of pair L (samples of layer l): z rows r0.. and their shifts Lam.
template <int NKC, int NS, int WV>
__device__ __forceinline__ void fetch_rows(int tix, TilePrefetch<NKC, NS, WV>& pf, const LayerDev& L,
                                           const float* __restrict__ z,
                                           const float* __restrict__ lamrow, int r0,
                                           const float* __restrict__ ev = nullptr,
                                           const float* __restrict__ pl = nullptr,
                                           bool dzw = false) {
  constexpr int TPR = TilePrefetch<NKC, NS, WV>::TPR, NFT = TilePrefetch<NKC, NS, WV>::NFT;
  const int t = tix, sub = t % TPR;
  const bool vec = (L.D % 4 == 0) && (L.z_off % 4 == 0);
  const int rr = r0 + (t & (32 * NS - 1));
  pf.rem = L.K - r0;
  pf.r0 = r0;
  if (vec) {
    // loads only (see fetch_cols)
#pragma unroll
    for (int sb = 0; sb < NS; ++sb) {
      const int gr = min(r0 + 32 * sb + (t / TPR), L.K - 1);
      const float* rowp = z + L.z_off + (int64_t)gr * L.D;
#pragma unroll
      for (int m = 0; m < NFT; ++m)
        pf.v[sb][m] = *reinterpret_cast<const float4*>(rowp + min(opaque(4 * (sub + TPR * m)), L.D - 4));
      if (dzw) {   // (uniform)
        const float* erow = ev + L.ev_off + (int64_t)gr * L.D;
#pragma unroll
        for (int m = 0; m < NFT; ++m)
          pf.e[sb][m] = *reinterpret_cast<const float4*>(erow + min(opaque(4 * (sub + TPR * m)), L.D - 4));
        const float pv = pl[L.p_off + gr];
        pf.prow[sb] = (r0 + 32 * sb + (t / TPR) < L.K) ? pv : 0.0f;
      }
    }
    pf.lam = lamrow[min(rr, L.K - 1)];
    return;
  }
#pragma unroll
  for (int sb = 0; sb < NS; ++sb) {
    const int gr = r0 + 32 * sb + (t / TPR);
    const bool valid = gr < L.K;
    const float* rowp = z + L.z_off + (int64_t)(valid ? gr : L.K - 1) * L.D;
#pragma unroll
    for (int m = 0; m < NFT; ++m)
      pf.v[sb][m] = load_f4(rowp, opaque(4 * (sub + TPR * m)), L.D, valid, false);
  }
  const float lv = lamrow[min(rr, L.K - 1)];
  pf.lam = (rr < L.K) ? lv : INFINITY;
}

// Writes fetched tiles to LDS buffer b: row-major copy = x * lam2 when `scale`, else
// x; d-major copy and second row-major copy (when the layout has them) = x.  With Q,
// also the column norms of the
// staged rows, q[sb] = -1/2 sum_d lam_d x_d^2 in FP64, in one fixed order for 4 and 8
// waves: float4 column f of the row goes to partial A if f mod 16 < 8, else to B, each
// partial summed in increasing f; then A + B, then a butterfly over f mod 8 (so both
// workgroup sizes give identical norms, complete in every thread of the row).
// tile_store_part writes float4 column m of subtile sb and adds its terms to the
// partials qa; tile_store_norm completes a subtile's norm; tile_store does it all.
template <class TS, int NKC, bool Q, int WV>
__device__ __forceinline__ void tile_store_part(int tix, TS& T, int b, const TilePrefetch<NKC, TS::NS, WV>& pf,
                                                bool scale, int sb, int m, double (&qa)[2]) {
  constexpr int TPR = TilePrefetch<NKC, TS::NS, WV>::TPR;
  const int t = tix, r = t / TPR, sub = t % TPR;
  const int pr = tile_perm(r);
  // d < DT always (the row stride and the lam tables cover DT, so no thread
  // branches here); slots past the data are harmless (see TilePrefetch)
  const int d = 4 * (sub + TPR * m);
  double& qp = qa[WV == 4 ? (m & 1) : 0];
  const float x[4] = {pf.v[sb][m].x, pf.v[sb][m].y, pf.v[sb][m].z, pf.v[sb][m].w};
  if constexpr (Q) {
    const double2 la = T.lamdA[d >> 2];
    const double2 lb = T.lamdB[d >> 2];
    qp += la.x * (double)x[0] * (double)x[0];
    qp += la.y * (double)x[1] * (double)x[1];
    qp += lb.x * (double)x[2] * (double)x[2];
    qp += lb.y * (double)x[3] * (double)x[3];
  }
  const int ro = sb * TS::ROWN + r * TS::RS + d;
  const int co = sb * TS::COLN + d * TS::CS + pr;
  if constexpr (TS::BF) {
    uint32_t xh[2], xl[2];
    split2(x[0], x[1], xh[0], xl[0]);
    split2(x[2], x[3], xh[1], xl[1]);
    if constexpr (TS::RAW) {
      *reinterpret_cast<bf16x4*>(&T.raw[b][0][ro]) = __builtin_bit_cast(bf16x4, (u32x2){xh[0], xh[1]});
      *reinterpret_cast<bf16x4*>(&T.raw[b][1][ro]) = __builtin_bit_cast(bf16x4, (u32x2){xl[0], xl[1]});
    }
    if constexpr (TS::COL) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        T.col[b][0][co + e * TS::CS] =
            __builtin_bit_cast(__bf16, (uint16_t)(xh[e >> 1] >> (16 * (e & 1))));
        T.col[b][1][co + e * TS::CS] =
            __builtin_bit_cast(__bf16, (uint16_t)(xl[e >> 1] >> (16 * (e & 1))));
      }
    }
    if (scale) {
      const float4 l2 = *reinterpret_cast<const float4*>(&T.lam2[d]);
      split2(x[0] * l2.x, x[1] * l2.y, xh[0], xl[0]);
      split2(x[2] * l2.z, x[3] * l2.w, xh[1], xl[1]);
    }
    *reinterpret_cast<bf16x4*>(&T.row[b][0][ro]) = __builtin_bit_cast(bf16x4, (u32x2){xh[0], xh[1]});
    *reinterpret_cast<bf16x4*>(&T.row[b][1][ro]) = __builtin_bit_cast(bf16x4, (u32x2){xl[0], xl[1]});
  } else {
    if constexpr (TS::COL) {
#pragma unroll
      for (int e = 0; e < 4; ++e) T.col[b][0][co + e * TS::CS] = x[e];
    }
    float y[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) y[e] = scale ? x[e] * T.lam2[d + e] : x[e];
    *reinterpret_cast<float4*>(&T.row[b][0][ro]) = make_float4(y[0], y[1], y[2], y[3]);
  }
}

// The norm of one subtile from its two partials (see tile_store).
template <int WV>
__device__ __forceinline__ double tile_store_norm(const double (&qa)[2]) {
  // 4 waves: this thread holds A (even m) and B (odd m); 8 waves: threads with
  // sub < 8 hold A, their xor-8 partners B
  double qs = (WV == 4) ? qa[0] + qa[1] : xor_add_f64<8>(qa[0]);
  qs = xor_add_f64<1>(qs);
  qs = xor_add_f64<2>(qs);
  qs = xor_add_f64<4>(qs);
  return -0.5 * qs;
}

template <class TS, int NKC, bool Q, int WV>
__device__ __forceinline__ void tile_store(int tix, TS& T, int b, const TilePrefetch<NKC, TS::NS, WV>& pf,
                                           bool scale, double (&q)[TS::NS]) {
  constexpr int NFT = TilePrefetch<NKC, TS::NS, WV>::NFT;
#pragma unroll
  for (int sb = 0; sb < TS::NS; ++sb) {
    double qa[2] = {0.0, 0.0};
#pragma unroll
    for (int m = 0; m < NFT; ++m) tile_store_part<TS, NKC, Q, WV>(tix, T, b, pf, scale, sb, m, qa);
    if constexpr (Q) q[sb] = tile_store_norm<WV>(qa);
  }
}

// gamma_j = log2(e) (kappa q_j + alpha_{l+1}[j] - maxa), -inf past Kc.
__device__ __forceinline__ float col_gamma(double q, double a, int j, int Kc, double maxa,
                                           double kappa) {
  return (j < Kc) ? (float)((kappa * q + (a - maxa)) * (double)kLog2e) : -INFINITY;
}

// Fragment of staged row (lane % 32) of subtile sb for d chunk kc (d = 16 kc + 8 h + s).
template <class TS, int PREC>
__device__ __forceinline__ void tile_row_frag(int tix, const TS& T, int b, int sb, int kc, Frag<PREC>& f) {
  const int lane = tix & 63, r = lane & 31, h = lane >> 5;
  const int o = sb * TS::ROWN + r * TS::RS + kc * 16 + 8 * h;
  if constexpr (TS::BF) {
    f.hi = *reinterpret_cast<const bf16x8*>(&T.row[b][0][o]);
    f.lo = *reinterpret_cast<const bf16x8*>(&T.row[b][1][o]);
  } else {
    const float4 a = *reinterpret_cast<const float4*>(&T.row[b][0][o]);
    const float4 c = *reinterpret_cast<const float4*>(&T.row[b][0][o + 4]);
    f.x[0] = a.x; f.x[1] = a.y; f.x[2] = a.z; f.x[3] = a.w;
    f.x[4] = c.x; f.x[5] = c.y; f.x[6] = c.z; f.x[7] = c.w;
  }
}

// Transposed fragment of subtile sb for d block q (lane -> d = 32 q + lane % 32).
template <class TS, int PREC>
__device__ __forceinline__ void tile_col_frag(int tix, const TS& T, int b, int sb, int q, TFrag<PREC>& f) {
  const int lane = tix & 63, h = lane >> 5;
  const int o = sb * TS::COLN + (32 * q + (lane & 31)) * TS::CS + 8 * h;
  if constexpr (TS::BF) {
#pragma unroll
    for (int tt = 0; tt < 2; ++tt) {
      f.f[tt].hi = *reinterpret_cast<const bf16x8*>(&T.col[b][0][o + 16 * tt]);
      f.f[tt].lo = *reinterpret_cast<const bf16x8*>(&T.col[b][1][o + 16 * tt]);
    }
  } else {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const float4 a = *reinterpret_cast<const float4*>(&T.col[b][0][o + 4 * (g & 1) + 16 * (g >> 1)]);
      f.x[4 * g + 0] = a.x; f.x[4 * g + 1] = a.y; f.x[4 * g + 2] = a.z; f.x[4 * g + 3] = a.w;
    }
  }
}

// LDS transpose read (ds_read_b64_tr_b16): in each group of 16 lanes, output lane i
// receives element i % 4 of the 4-element (64-bit) chunks addressed by lanes i / 4 + 4 e
// of its group, e = 0..3 (one column gathered from four rows).
__device__ __forceinline__ bf16x4 lds_read_tr16(const __bf16* p) {
  typedef __attribute__((address_space(3))) bf16x4 lds_bf16x4;
  return __builtin_amdgcn_ds_read_tr16_b64_v4bf16((lds_bf16x4*)(p));
}

// Transposed BF16 fragment of subtile sb for d block q read from the row-major copy
// (no d-major copy needed).  Lane l addresses row 16 t + 8 half + 4 (l / 32) + (l % 16) / 4
// at column 32 q + 16 ((l / 16) % 2) + 4 (l % 4), so that it receives rows
// 16 t + 8 half + 4 (l / 32) + e, e = 0..3, of column d = 32 q + l % 32: for k-step t,
// slots 4 half + e, the k order of an accumulator column (see TFrag).
template <class TS, bool FROM_RAW = false>
__device__ __forceinline__ void tile_rowT_frag(int tix, const TS& T, int b, int sb, int q,
                                               TFrag<TMC_BF16X3>& f) {
  const __bf16* hi = FROM_RAW ? &T.raw[b][0][0] : &T.row[b][0][0];
  const __bf16* lo = FROM_RAW ? &T.raw[b][1][0] : &T.row[b][1][0];
  const int lane = tix & 63;
  const int rb = 4 * (lane >> 5) + ((lane & 15) >> 2);
  const int cb = 32 * q + 16 * ((lane >> 4) & 1) + 4 * (lane & 3);
#pragma unroll
  for (int tt = 0; tt < 2; ++tt) {
    const int o0 = sb * TS::ROWN + (16 * tt + rb) * TS::RS + cb;
    const int o1 = o0 + 8 * TS::RS;
    const bf16x4 h0 = lds_read_tr16(hi + o0), h1 = lds_read_tr16(hi + o1);
    const bf16x4 l0 = lds_read_tr16(lo + o0), l1 = lds_read_tr16(lo + o1);
    f.f[tt].hi = __builtin_shufflevector(h0, h1, 0, 1, 2, 3, 4, 5, 6, 7);
    f.f[tt].lo = __builtin_shufflevector(l0, l1, 0, 1, 2, 3, 4, 5, 6, 7);
  }
}

// The wave's own 32 rows of a row-major [n][D] block as raw values: x[kc] holds
// row (lane % 32), d = 16 kc + 8 (lane / 32) + s.  Rows past n read the last row.
template <int NKC>
__device__ __forceinline__ void wave_load(int tix, const float* __restrict__ base, int64_t off, int n, int D,
                                          int r0, float (&x)[NKC][8]) {
  const int lane = tix & 63, h = lane >> 5;
  const int r = min(r0 + (lane & 31), n - 1);
  const float* row = base + off + (int64_t)r * D;
  if ((D % 4 == 0) && (off % 4 == 0)) {
    // all loads first (one round trip), then the padding zeros
    float4 a[NKC][2];
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
      for (int e = 0; e < 2; ++e)
        a[kc][e] = *reinterpret_cast<const float4*>(row + min(kc * 16 + 8 * h + 4 * e, D - 4));
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const bool v = kc * 16 + 8 * h + 4 * e < D;
        x[kc][4 * e + 0] = v ? a[kc][e].x : 0.0f;
        x[kc][4 * e + 1] = v ? a[kc][e].y : 0.0f;
        x[kc][4 * e + 2] = v ? a[kc][e].z : 0.0f;
        x[kc][4 * e + 3] = v ? a[kc][e].w : 0.0f;
      }
    return;
  }
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc) load8(row, kc * 16 + 8 * h, D, false, x[kc]);
}

// ---------------------------------------------------------------------------
// forward: a workgroup of 4 waves owns 128 rows of one layer pair (wave w: rows
// start + 32 w ..); the samples of the layer above are staged NS x 32 at a time in
// LDS and swept by all waves.
//   ell_i   = log2 sum_j exp2(S_ij + gamma_j)          (S = kappa log2e <lam z_i, mu_j>)
//   alpha_i = kappa (u_i + r_i + c) + maxa + ln2 * ell_i - ln K_{l+1}
// (kappa: the weight exponent of the plan, 1 for the estimator itself)
//   e_i     = sum_j softmax_j(S_ij + gamma_j) mu_j        (GRAD: used for dz)
// ---------------------------------------------------------------------------
// MFMAs of one 32-column (32-row) tile's factor GEMM per subtile
template <int PREC, int NKC>
constexpr int kGemmMfma = NKC * (PREC == TMC_BF16X3 ? 3 : 8);

// LDS stages of a sweep: three for BF16X3 at d <= 128 with one subtile per stage (the
// pipelined sweep, below), two otherwise at d <= 128, one for wider layers.
template <int PREC, int NKC, int NS>
constexpr int kStages = NKC <= 8 ? ((PREC == TMC_BF16X3 && NS == 1) ? 3 : 2) : 1;

template <int PREC, int NKC, bool GRAD, int NS>
using FwdSmem = TileSmem<PREC, NKC, NS, kStages<PREC, NKC, NS>, GRAD && PREC != TMC_BF16X3>;

template <int PREC, int NKC, bool GRAD, int NS, int WV>
__device__ __forceinline__ void fwd_item(int tix, FwdSmem<PREC, NKC, GRAD, NS>& T, const Item it,
                                         const LayerDev& L, const FwdArgs& args) {
  using TS = FwdSmem<PREC, NKC, GRAD, NS>;
  constexpr int NB = TS::NB;
  constexpr int ND32 = TS::ND32;
  const float* __restrict__ z = args.z;
  const float* __restrict__ mu = args.mu;
  const float* __restrict__ s = args.s;
  const float* __restrict__ u = args.u;
  double* __restrict__ qcol = args.qcol;
  double* __restrict__ alpha = args.alpha;
  double* __restrict__ wmax = args.wmax;
  float* __restrict__ rl = args.rl;
  float* __restrict__ ev = args.ev;
  const int tid = tix, w = tid >> 6, lane = tid & 63, h = lane >> 5, ir = lane & 31;
  const int i0 = it.start + 32 * w;
  const bool active = i0 < L.K;
  const int i = i0 + ir;
  const int nt = (L.Kc + 32 * NS - 1) / (32 * NS);

  // small inputs first, then the bulk operand loads; consuming the small ones waits
  // for them alone
  PairPre pre;
  pair_preload(tix, L, wmax, s, pre);
  const float u_i = u[L.u_off + min(i, L.K - 1)];
  float xz[NKC][8];
  wave_load<NKC>(tix, z, L.z_off, L.K, L.D, i0, xz);
  TilePrefetch<NKC, NS, WV> pf;
  fetch_cols(tix, pf, L, mu, alpha, 0);
  const double maxa = pair_maxa(tix, L, wmax, pre);
  const double cs = pair_const(tix, L, pre);
  tile_init(tix, T, L, pre);
  lds_barrier();

  // row operand a_i = log2(e) lam z_i as fragments, r_i = -1/2 sum_d lam_d z_id^2 (FP64)
  Frag<PREC> A[NKC];
  double r_i = 0.0;
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc) {
    const int d0 = kc * 16 + 8 * h;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      r_i += (double)T.lamf[d0 + t] * (double)xz[kc][t] * (double)xz[kc][t];
      xz[kc][t] *= T.lam2[d0 + t];
    }
    make_frag<PREC>(xz[kc], A[kc]);
  }
  r_i = -0.5 * (r_i + __shfl_xor(r_i, 32, kWave));

  // The forward computes the column norms q_j (FP64) of every column it stages; the
  // workgroup that starts at row 0 stores them for the backward.
  const bool qwriter = GRAD && it.start == 0;
  constexpr int TPR = TilePrefetch<NKC, NS, WV>::TPR;
  const int srow = tid / TPR;   // staged row of this thread
  // Stages the fetched columns j0.. into buffer b; the TPR threads of a row hold the
  // same norm and write the same gamma.  The norms are returned for the q store, which is
  // kept apart (a divergent store would split the block the stage is scheduled in).
  auto stage = [&](int b, int j0, double (&qs)[NS]) {
    tile_store<TS, NKC, true, WV>(tix, T, b, pf, false, qs);
#pragma unroll
    for (int sb = 0; sb < NS; ++sb)
      T.gam[b][32 * sb + srow] = col_gamma(qs[sb], pf.a[sb], j0 + 32 * sb + srow, L.Kc, maxa, L.kappa);
  };
  auto store_q = [&](int j0, const double (&qs)[NS]) {
#pragma unroll
    for (int sb = 0; sb < NS; ++sb) {
      const int j = j0 + 32 * sb + srow;
      if (qwriter && tid % TPR == 0 && j < L.Kc) qcol[L.q_off + j] = qs[sb];
    }
  };
  float m = -INFINITY, ssum = 0.0f;
  f32x16 O[GRAD ? ND32 : 1];
#pragma unroll
  for (int q = 0; q < (GRAD ? ND32 : 1); ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) O[q][v] = 0.0f;

  // S[j][i] over the staged tile in buffer cur
  auto s_gemm = [&](int cur, f32x16 (&S)[NS]) {
#pragma unroll
    for (int sb = 0; sb < NS; ++sb)
#pragma unroll
      for (int v = 0; v < 16; ++v) S[sb][v] = 0.0f;
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
      for (int sb = 0; sb < NS; ++sb) {
        Frag<PREC> Bf;
        tile_row_frag<TS, PREC>(tix, T, cur, sb, kc, Bf);
        mma_chunk<PREC>(S[sb], Bf, A[kc]);     // S[j][i]
      }
  };
  // online log-sum-exp, first half: x = S + gamma and the running max of the tile (a
  // rescale of the running sums when it grows by more than kRescale, rare)
  auto soft_max = [&](int cur, const f32x16 (&S)[NS], float (&x)[NS][16]) {
    float tmax = -INFINITY;
#pragma unroll
    for (int sb = 0; sb < NS; ++sb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 g4 = *reinterpret_cast<const float4*>(&T.gam[cur][32 * sb + 8 * q + 4 * h]);
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
    tmax = xor32_max(tmax);
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
  };
  // second half: the exponentials, their sum and (GRAD) the split operand of the
  // softmax-weighted sum of mu
  auto soft_exp = [&](float (&x)[NS][16], PFrag<PREC> (&P)[NS]) {
    const float msafe = (m == -INFINITY) ? 0.0f : m;
    float ps = 0.0f;
#pragma unroll
    for (int sb = 0; sb < NS; ++sb)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        x[sb][v] = __builtin_amdgcn_exp2f(x[sb][v] - msafe);
        ps += x[sb][v];
      }
    ssum += ps;
    if (GRAD) {
#pragma unroll
      for (int sb = 0; sb < NS; ++sb) make_pfrag<PREC>(x[sb], P[sb]);
    }
  };
  // O[d][i] += sum_j mu_j[d] P[j][i] over the staged tile in buffer cur
  auto o_gemm = [&](int cur, const PFrag<PREC> (&P)[NS]) {
#pragma unroll
    for (int q = 0; q < ND32; ++q)
#pragma unroll
      for (int sb = 0; sb < NS; ++sb) {
        TFrag<PREC> Tf;
        if constexpr (PREC == TMC_BF16X3)
          tile_rowT_frag<TS>(tix, T, cur, sb, q, Tf);   // transpose reads of the row copy
        else
          tile_col_frag<TS, PREC>(tix, T, cur, sb, q, Tf);
        mma_t<PREC>(O[q], Tf, P[sb]);
      }
  };
  auto softmax_e = [&](int cur, const f32x16 (&S)[NS]) {
    float x[NS][16];
    PFrag<PREC> P[NS];
    soft_max(cur, S, x);
    soft_exp(x, P);
    if (GRAD) o_gemm(cur, P);
  };

  // BF16X3, one subtile, 8 waves, gradient forward: the two phases of the pipelined sweep in
  // issue order with their LDS fragments read ahead.  Phase A: d chunk kc of the next
  // tile's factor GEMM (three MFMAs; its fragment read two chunks earlier), then the
  // exponentials of two entries of the current tile and their hi/lo split.  Phase B: d
  // block q of the current tile's second GEMM (six MFMAs; fragments read one block
  // earlier), then a share of the staging of tile t+2 (its float4 columns, then the
  // norm and the column term) and finally the fetch of tile t+3.  Every sum keeps the
  // order of s_gemm, soft_exp and o_gemm.
  constexpr bool kAhead = PREC == TMC_BF16X3 && GRAD && NS == 1 && NKC == 8 && WV == 8;
  auto phase_a = [&](int nb, float (&x)[NS][16], f32x16 (&Sn)[NS], PFrag<PREC> (&P)[NS]) {
    if constexpr (kAhead) {
      const float msafe = (m == -INFINITY) ? 0.0f : m;
      float ps = 0.0f;
#pragma unroll
      for (int v = 0; v < 16; ++v) Sn[0][v] = 0.0f;
      Frag<PREC> B3[3];
      tile_row_frag<TS, PREC>(tix, T, nb, 0, 0, B3[0]);
      tile_row_frag<TS, PREC>(tix, T, nb, 0, 1, B3[1]);
#pragma unroll
      for (int kc = 0; kc < NKC; ++kc) {
        if (kc + 2 < NKC) tile_row_frag<TS, PREC>(tix, T, nb, 0, kc + 2, B3[(kc + 2) % 3]);
        mma_chunk<PREC>(Sn[0], B3[kc % 3], A[kc]);
#pragma unroll
        for (int e = 2 * kc; e < 2 * kc + 2; ++e) {
          x[0][e] = __builtin_amdgcn_exp2f(x[0][e] - msafe);
          ps += x[0][e];
        }
        uint32_t hu, lu;
        split2(x[0][2 * kc], x[0][2 * kc + 1], hu, lu);
        Frag<TMC_BF16X3>& f = P[0].f[kc / 4];
        u32x4 hv = __builtin_bit_cast(u32x4, f.hi), lv = __builtin_bit_cast(u32x4, f.lo);
        hv[kc % 4] = hu;
        lv[kc % 4] = lu;
        f.hi = __builtin_bit_cast(bf16x8, hv);
        f.lo = __builtin_bit_cast(bf16x8, lv);
      }
      ssum += ps;
    }
  };
  auto phase_b = [&](int cb, int b, int t, const PFrag<PREC> (&P)[NS], double (&qs)[NS]) {
    if constexpr (kAhead) {
      constexpr int NFT = TilePrefetch<NKC, NS, WV>::NFT;
      constexpr int NA = NFT + 2;   // staging parts: NFT columns, norm + gamma, fetch
      const int j0 = 32 * (t + 2);
      double qa[2] = {0.0, 0.0};
      TFrag<PREC> T2[2];
      tile_rowT_frag<TS>(tix, T, cb, 0, 0, T2[0]);
#pragma unroll
      for (int q = 0; q < ND32; ++q) {
        if (q + 1 < ND32) tile_rowT_frag<TS>(tix, T, cb, 0, q + 1, T2[(q + 1) & 1]);
        mma_t<PREC>(O[q], T2[q & 1], P[0]);
#pragma unroll
        for (int k = 0; k < NA; ++k) {
          if (k * ND32 / NA != q) continue;
          if (k < NFT) {
            tile_store_part<TS, NKC, true, WV>(tix, T, b, pf, false, 0, k, qa);
          } else if (k == NFT) {
            qs[0] = tile_store_norm<WV>(qa);
            T.gam[b][srow] = col_gamma(qs[0], pf.a[0], j0 + srow, L.Kc, maxa, L.kappa);
          } else {
            fetch_cols(tix, pf, L, mu, alpha, 32 * (t + 3));
          }
        }
      }
    }
  };

  if constexpr (NB == 3) {
    // Pipelined sweep over three LDS stages.  While the wave works on tile t, tile t+1
    // is already staged and tile t+2 is being staged: phase A issues the factor-GEMM
    // MFMAs of tile t+1 and, between them, the exponentials of tile t; phase B issues
    // the second-GEMM MFMAs of tile t and, between them, the staging of tile t+2 (and
    // the fetch of tile t+3).  So the matrix cores and the vector ALU of a wave work
    // at the same time instead of in turns.  Stage b of tile t is t mod 3; every
    // access past the last tile is in bounds (clamped fetches) and its results are
    // never read.  Rows past K compute on clamped rows and are discarded at the end.
    {
      double qs[NS];
      stage(0, 0, qs);
      store_q(0, qs);
    }
    fetch_cols(tix, pf, L, mu, alpha, 32 * NS);
    lds_barrier();                                   // tile 0 visible
    {
      double qs[NS];
      stage(1, 32 * NS, qs);
      store_q(32 * NS, qs);
    }
    fetch_cols(tix, pf, L, mu, alpha, 64 * NS);
    f32x16 S[NS];
    s_gemm(0, S);
    lds_barrier();                                   // tile 1 visible
    int cur = 0;
    for (int t = 0; t + 1 < nt; ++t) {
      const int nxt = cur == 2 ? 0 : cur + 1;
      const int stg = nxt == 2 ? 0 : nxt + 1;
      float x[NS][16];
      soft_max(cur, S, x);
      f32x16 Sn[NS];
      PFrag<PREC> P[NS];
      double qs[NS];
      if constexpr (kAhead) {
        phase_a(nxt, x, Sn, P);
        phase_b(cur, stg, t, P, qs);
      } else {
        // phase A
        s_gemm(nxt, Sn);
        soft_exp(x, P);
        interleave_phase_a<kGemmMfma<PREC, NKC> * NS, 8>();
        // phase B
        if (GRAD) o_gemm(cur, P);
        stage(stg, 32 * NS * (t + 2), qs);
        fetch_cols(tix, pf, L, mu, alpha, 32 * NS * (t + 3));
        if (GRAD) interleave_phase_b<ND32 * NS * 2 * (PREC == TMC_BF16X3 ? 3 : 8)>();
      }
      store_q(32 * NS * (t + 2), qs);
      lds_barrier();
#pragma unroll
      for (int sb = 0; sb < NS; ++sb) S[sb] = Sn[sb];
      cur = nxt;
    }
    // the last tile: no next tile to multiply, stage or fetch
    softmax_e(cur, S);
  } else {
    {
      double qs[NS];
      stage(0, 0, qs);
      store_q(0, qs);
    }
    if (nt > 1) fetch_cols(tix, pf, L, mu, alpha, 32 * NS);
    lds_barrier();
    // One tile.  Double-buffered: the S MFMAs are issued first, and the next stage is
    // written to the idle buffer behind them (straight-line code, so the scheduler can
    // interleave the staging with the MFMAs); past the last tile that stage repeats
    // data into a buffer that is never read again.
    auto tile = [&](auto bc, int t) {
      constexpr int cur = decltype(bc)::value;
      if constexpr (NB == 2) {
        double qs[NS];
        if (active) {
          f32x16 S[NS];
          s_gemm(cur, S);
          stage(cur ^ 1, 32 * NS * (t + 1), qs);
          interleave_mfma<kGemmMfma<PREC, NKC> * NS>();
          if (t + 2 < nt) fetch_cols(tix, pf, L, mu, alpha, 32 * NS * (t + 2));
          softmax_e(cur, S);
        } else {
          stage(cur ^ 1, 32 * NS * (t + 1), qs);
          if (t + 2 < nt) fetch_cols(tix, pf, L, mu, alpha, 32 * NS * (t + 2));
        }
        store_q(32 * NS * (t + 1), qs);
        lds_barrier();
      } else {
        if (active) {
          f32x16 S[NS];
          s_gemm(cur, S);
          softmax_e(cur, S);
        }
        lds_barrier();
        if (t + 1 < nt) {
          double qs[NS];
          stage(0, 32 * NS * (t + 1), qs);
          store_q(32 * NS * (t + 1), qs);
          if (t + 2 < nt) fetch_cols(tix, pf, L, mu, alpha, 32 * NS * (t + 2));
          lds_barrier();
        }
      }
    };
    if constexpr (NB == 2) {
      int t = 0;
      for (; t + 1 < nt; t += 2) {
        tile(std::integral_constant<int, 0>{}, t);
        tile(std::integral_constant<int, 1>{}, t + 1);
      }
      if (t < nt) tile(std::integral_constant<int, 0>{}, t);
    } else {
      for (int t = 0; t < nt; ++t) tile(std::integral_constant<int, 0>{}, t);
    }
  }
  const float stot = xor32_sum(ssum);
  float ell;
  if (m != m || stot != stot) ell = NAN;
  else if (m == -INFINITY || stot == 0.0f) ell = -INFINITY;
  else ell = m + log2f(stot);
  const bool iv = active && i < L.K;
  const double a_i = L.kappa * ((double)u_i + r_i + cs) + maxa + kLn2 * (double)ell - L.lnKc;
  if (h == 0 && iv) {
    rl[L.rl_off + i] = ell;
    alpha[L.alpha_off + i] = a_i;
  }
  // this workgroup's max_i alpha_l[i], for the next step's column shift
  const double wm = wave_max(iv ? a_i : -INFINITY);
  if (lane == 0) T.wm[w] = wm;
  lds_barrier();
  // one partial per 128 rows (waves 4 h .. 4 h + 3), whatever the workgroup size
  if (tid < WV / 4 && it.start + kFusedRowsPerGroup * tid < L.K) {
    const double* pw = &T.wm[4 * tid];
    wmax[L.wmax_off + it.start / kFusedRowsPerGroup + tid] =
        nan_max(nan_max(pw[0], pw[1]), nan_max(pw[2], pw[3]));
  }
  if (GRAD && iv) {
    const float inv = (stot > 0.0f) ? 1.0f / stot : 0.0f;
    float* erow = ev + L.ev_off + (int64_t)i * L.D;
    const bool vec = (L.D % 4 == 0) && (L.ev_off % 4 == 0);
    if (vec) {
      // D % 4 == 0: a float4 at d < D is whole
#pragma unroll
      for (int q = 0; q < ND32; ++q)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int d = 32 * q + 8 * g + 4 * h;
          if (d < L.D)
            *reinterpret_cast<float4*>(erow + d) =
                make_float4(O[q][4 * g] * inv, O[q][4 * g + 1] * inv, O[q][4 * g + 2] * inv,
                            O[q][4 * g + 3] * inv);
        }
    } else {
#pragma unroll
    for (int q = 0; q < ND32; ++q)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int d = 32 * q + 8 * g + 4 * h;
        const float4 o4 = make_float4(O[q][4 * g] * inv, O[q][4 * g + 1] * inv,
                                      O[q][4 * g + 2] * inv, O[q][4 * g + 3] * inv);
        {
          if (d + 0 < L.D) erow[d + 0] = o4.x;
          if (d + 1 < L.D) erow[d + 1] = o4.y;
          if (d + 2 < L.D) erow[d + 2] = o4.z;
          if (d + 3 < L.D) erow[d + 3] = o4.w;
        }
      }
    }
  }
}

// Work item of workgroup b of n: the hardware hands workgroup b to XCD b mod 8, and
// consecutive items (the row or column blocks of one layer pair, which sweep the same
// operand) go to workgroups of one XCD, so that they share its L2.  A tail of n mod 8
// workgroups keeps its own index (a bijection on [0, n)).
__device__ __forceinline__ int xcd_item(int b, int n) {
  constexpr int X = 8;
  const int per = n / X;
  return b < per * X ? (b % X) * per + b / X : b;
}

// One workgroup of WV waves (32 WV rows) per work item (level-synchronous launch):
// 4 waves, two workgroups per compute unit, or 8 waves, one per compute unit.
template <int PREC, int NKC, bool GRAD, int NS, int WV>
__global__ __launch_bounds__(64 * WV, (WV == 8 ? 1 : (NKC <= 8 ? 2 : 1))) void k_fused_fwd(FwdArgs args) {
  __shared__ __align__(16) FwdSmem<PREC, NKC, GRAD, NS> T;
  const Item it = args.items[xcd_item(blockIdx.x, gridDim.x)];
  const LayerDev L = args.Ls[it.layer];
  fwd_item<PREC, NKC, GRAD, NS, WV>((int)threadIdx.x, T, it, L, args);
}

// The thread index of a 256-thread workgroup as a value the compiler cannot treat as
// invariant: the persistent kernels take it afresh for every item, so the addressing the
// sweep derives from it stays inside the item.  (With threadIdx.x itself it was hoisted out
// of the chain and pair loops, held across the whole loop nest and spilled: hundreds of
// VGPRs.)  The helpers of the sweep take the thread index as an argument for this reason.
__device__ __forceinline__ int item_tid() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  __builtin_assume(t >= 0 && t < 256);
  return t;
}

// Persistent launch: each workgroup takes whole chains from the queue and runs their
// pairs top-down (pair l reads the alpha_{l+1} and maxima its own earlier pair wrote;
// the workgroup barrier between pairs orders those global writes and reads).
template <int PREC, int NKC, bool GRAD, int NS>
__global__ __launch_bounds__(256, (NKC <= 8 ? 2 : 1)) void k_fused_fwd_persist(FwdArgs args,
                                                                               ChainQueue q) {
  __shared__ __align__(16) FwdSmem<PREC, NKC, GRAD, NS> T;
  __shared__ int s_k;
  for (;;) {
    if (threadIdx.x == 0) s_k = atomicAdd(q.head, 1);
    __syncthreads();
    // uniform across the workgroup: keep it (and all that derives from it) scalar
    const int k = __builtin_amdgcn_readfirstlane(s_k);
    __syncthreads();
    if (k >= q.n) return;
    const ChainDev ch = q.cd[q.chains[k]];
    for (int l = ch.top - 1; l >= ch.first; --l) {
      const LayerDev L = args.Ls[l];
      for (int x = 0; x < L.K; x += kFusedRowsPerGroup) {
        fwd_item<PREC, NKC, GRAD, NS, 4>(item_tid(), T, Item{l, x}, L, args);
        __syncthreads();
      }
    }
  }
}

// ---------------------------------------------------------------------------
// backward: a workgroup of 4 waves owns 128 columns (samples j of layer l+1; wave
// w: columns start + 32 w ..) and sweeps every row of layer l, NS x 32 rows per LDS
// stage (a log2(e) lam-scaled row-major copy for the factor; for G^T z, BF16X3 reads
// the same copy through transpose reads and divides the sums by log2(e) lam_d, FP32
// keeps a raw d-major copy):
//   G_ij   = exp2(S_ij + gamma_j - Lam_i),   Lam_i = ell_i - log2 p_l[i]
//   p_{l+1}[j] = sum_i G_ij,  (G^T z)_j = sum_i G_ij z_i
//   dmu_j  = dlogp * lam * ((G^T z)_j - p_{l+1}[j] mu_j)
// and writes the column part of the log-std gradient of its columns,
//   dlogp * lam * sum_j (p_{l+1}[j] mu_j^2 - 2 mu_j (G^T z)_j)
// (sum_ij G_ij (z_i - mu_j)^2 expanded).  The row terms, dz and the ds row part, come
// from k_fused_dz, or for aligned pairs from the 8-wave workgroups themselves (below).
// With 8 waves a workgroup owns 256 columns.
// The constant c cancels between the forward's ell_i and G, so it is not needed here.
// ---------------------------------------------------------------------------
template <int PREC, int NKC, int NS>
using BwdSmem = TileSmem<PREC, NKC, NS, kStages<PREC, NKC, NS>, PREC != TMC_BF16X3>;

template <int PREC, int NKC, int NS, int WV>
__device__ __forceinline__ void bwd_item(int tix, BwdSmem<PREC, NKC, NS>& T, float* accD, const Item it,
                                         const LayerDev& L, const BwdArgs& args) {
  using TS = BwdSmem<PREC, NKC, NS>;
  constexpr int NB = TS::NB;
  constexpr int ND32 = TS::ND32;
  const float* __restrict__ z = args.z;
  const float* __restrict__ mu = args.mu;
  const float* __restrict__ s = args.s;
  const double* __restrict__ alpha = args.alpha;
  const double* __restrict__ wmax = args.wmax;
  const double* __restrict__ qcol = args.qcol;
  const float* __restrict__ rl = args.rl;
  float* __restrict__ lam_ws = args.lam;
  const double* __restrict__ dlogp = args.dlogp;
  float* __restrict__ p = args.p;
  float* __restrict__ dmu = args.dmu;
  float* __restrict__ du = args.du;
  float* __restrict__ dsp = args.dsp;
  const int tid = tix, w = tid >> 6, lane = tid & 63, h = lane >> 5, jr = lane & 31;
  const int jw = it.start + 32 * w;
  const bool active = jw < L.Kc;
  const int j = jw + jr;
  const int jc = min(j, L.Kc - 1);
  const int nt = (L.K + 32 * NS - 1) / (32 * NS);
  const float* lamrow = lam_ws + L.rl_off;   // Lam shares the per-layer indexing of rl
  // Every workgroup of a pair sweeps all rows of layer l, so the 8-wave workgroups of a
  // flagged pair also write the row terms (dz and the ds row part) from the rows they
  // stage: workgroup c of nwg takes the row tiles t with t % nwg == c and writes the
  // pair's row partial c (uniform; the host leaves those pairs out of the row-term
  // launch and flags them only when nwg <= ceil(K / 64)).
  const bool dzw = WV == 8 && args.rows && L.dz_fused;
  const int wg_c = it.start / (32 * WV), nwg = (L.Kc + 32 * WV - 1) / (32 * WV);
  auto own = [&](int tt) { return dzw && (tt % nwg) == wg_c; };
  const float* __restrict__ evp = args.ev;
  float* __restrict__ dzp = args.dz;
  constexpr int NFT = TilePrefetch<NKC, NS, WV>::NFT, TPR = TilePrefetch<NKC, NS, WV>::TPR;
  float rsum[NFT][4];   // sum over the thread's rows of p_i z_id^2, its column slots
#pragma unroll
  for (int m = 0; m < NFT; ++m)
#pragma unroll
    for (int e = 0; e < 4; ++e) rsum[m][e] = 0.0f;
  float psum = 0.0f;    // sum of p_i over the thread's rows

  // prologue loads: the wave's own column operands (mu rows), their column terms and
  // the first row tile
  PairPre pre;
  pair_preload(tix, L, wmax, s, pre);
  const double qj = qcol[L.q_off + jc];
  const double aj = alpha[L.alpha_up_off + jc];
  const double gl = dlogp[L.chain] * L.kappa;   // d/d(kappa log w) -> d/d(log w)
  float xm[NKC][8];
  wave_load<NKC>(tix, mu, L.mu_off, L.Kc, L.D, jw, xm);
  TilePrefetch<NKC, NS, WV> pf;
  fetch_rows(tix, pf, L, z, lamrow, 0, evp, p, own(0));
  const double maxa = pair_maxa(tix, L, wmax, pre);
  tile_init(tix, T, L, pre);
  for (int d = tid; d < (WV / 4) * TS::DT; d += blockDim.x) accD[d] = 0.0f;
  lds_barrier();

  Frag<PREC> Bf[NKC];
#pragma unroll
  for (int kc = 0; kc < NKC; ++kc) make_frag<PREC>(xm[kc], Bf[kc]);
  const float gj = col_gamma(qj, aj, j, L.Kc, maxa, L.kappa);
  const float g32 = (float)gl;

  // Stages the fetched rows into buffer b.  Threads t and t + 32 NS hold the shift of
  // the same row, so every thread writes (equal values to equal slots, no branch).
  // Row terms of the staged rows when the workgroup owns them (fresh; a 2-buffer sweep
  // also re-stages its last tile, which is never fresh),
  //   dz_i = -dlogp lam p_i (z_i - e_i),  sums of p_i z_id^2 and of p_i;
  // thread t serves the rows and column slots it staged.
  auto row_terms = [&](bool fresh) {
    if (fresh) {
      const int sub = tid % TPR;
#pragma unroll
      for (int sb = 0; sb < NS; ++sb) {
        const int row = pf.r0 + 32 * sb + tid / TPR;
        const float pr = pf.prow[sb];   // 0 past K
        psum += pr;
        float* drow = dzp ? dzp + L.z_off + (int64_t)row * L.D : nullptr;
#pragma unroll
        for (int m = 0; m < NFT; ++m) {
          const int c = 4 * (sub + TPR * m);   // < DT; lamf is 0 past D
          const float4 l4 = *reinterpret_cast<const float4*>(&T.lamf[c]);
          const float zv[4] = {pf.v[sb][m].x, pf.v[sb][m].y, pf.v[sb][m].z, pf.v[sb][m].w};
          const float ev[4] = {pf.e[sb][m].x, pf.e[sb][m].y, pf.e[sb][m].z, pf.e[sb][m].w};
          const float lv[4] = {l4.x, l4.y, l4.z, l4.w};
          float o[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            o[e] = -g32 * lv[e] * pr * (zv[e] - ev[e]);
            rsum[m][e] += pr * zv[e] * zv[e];
          }
          // D % 4 == 0: a float4 at c < D is whole
          if (drow && row < L.K && c < L.D)
            *reinterpret_cast<float4*>(drow + c) = make_float4(o[0], o[1], o[2], o[3]);
        }
      }
    }
  };
  auto stage = [&](int b, bool fresh) {
    double qs[NS];
    tile_store<TS, NKC, false, WV>(tix, T, b, pf, true, qs);
    const int rr = tid & (32 * NS - 1);
    T.lamT[b][rr] = (rr < pf.rem) ? pf.lam : INFINITY;
    row_terms(fresh);
  };
  f32x16 GT[ND32];
#pragma unroll
  for (int q = 0; q < ND32; ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) GT[q][v] = 0.0f;
  float csum = 0.0f;

  // S[i][j] over the staged row tile in buffer cur
  auto s_gemm = [&](int cur, f32x16 (&S)[NS]) {
#pragma unroll
    for (int sb = 0; sb < NS; ++sb)
#pragma unroll
      for (int v = 0; v < 16; ++v) S[sb][v] = 0.0f;
#pragma unroll
    for (int kc = 0; kc < NKC; ++kc)
#pragma unroll
      for (int sb = 0; sb < NS; ++sb) {
        Frag<PREC> Af;
        tile_row_frag<TS, PREC>(tix, T, cur, sb, kc, Af);
        mma_chunk<PREC>(S[sb], Af, Bf[kc]);    // S[i][j]
      }
  };
  // pairwise marginals of the tile, their column sums, and the split G operand
  auto marg_exp = [&](int cur, const f32x16 (&S)[NS], PFrag<PREC> (&P)[NS]) {
    float g[NS][16];
#pragma unroll
    for (int sb = 0; sb < NS; ++sb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float4 l4 = *reinterpret_cast<const float4*>(&T.lamT[cur][32 * sb + 8 * q + 4 * h]);
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
    for (int sb = 0; sb < NS; ++sb) make_pfrag<PREC>(g[sb], P[sb]);
  };
  // G^T z over the staged row tile in buffer cur
  auto gt_gemm = [&](int cur, const PFrag<PREC> (&P)[NS]) {
#pragma unroll
    for (int q = 0; q < ND32; ++q)
#pragma unroll
      for (int sb = 0; sb < NS; ++sb) {
        TFrag<PREC> Tf;
        if constexpr (PREC == TMC_BF16X3)
          tile_rowT_frag<TS>(tix, T, cur, sb, q, Tf);   // (log2e lam z)^T: transpose reads
        else
          tile_col_frag<TS, PREC>(tix, T, cur, sb, q, Tf);
        mma_t<PREC>(GT[q], Tf, P[sb]);
      }
  };
  auto marg = [&](int cur, const f32x16 (&S)[NS]) {
    PFrag<PREC> P[NS];
    marg_exp(cur, S, P);
    gt_gemm(cur, P);
  };

  // BF16X3, one subtile, 8 waves: the two phases in issue order with their LDS fragments
  // read ahead, as in the forward.  Phase A: d chunk kc of the next tile's factor GEMM
  // (fragment read two chunks earlier), then the marginals of two entries of the current
  // tile and their hi/lo split.  Phase B: d block q of G^T z (fragments read one block
  // earlier), then a share of the staging of tile t+2 (its float4 columns, then the row
  // shifts and row terms) and finally the fetch of tile t+3.  Every sum keeps the order
  // of s_gemm, marg_exp and gt_gemm.
  constexpr bool kAhead = PREC == TMC_BF16X3 && NS == 1 && NKC == 8 && WV == 8;
  auto phase_a = [&](int nb, int cb, const f32x16 (&S)[NS], f32x16 (&Sn)[NS], PFrag<PREC> (&P)[NS]) {
    if constexpr (kAhead) {
#pragma unroll
      for (int v = 0; v < 16; ++v) Sn[0][v] = 0.0f;
      Frag<PREC> B3[3];
      tile_row_frag<TS, PREC>(tix, T, nb, 0, 0, B3[0]);
      tile_row_frag<TS, PREC>(tix, T, nb, 0, 1, B3[1]);
      float2 l2[2];
      l2[0] = *reinterpret_cast<const float2*>(&T.lamT[cb][4 * h]);
#pragma unroll
      for (int kc = 0; kc < NKC; ++kc) {
        if (kc + 2 < NKC) tile_row_frag<TS, PREC>(tix, T, nb, 0, kc + 2, B3[(kc + 2) % 3]);
        if (kc + 1 < NKC)   // row shifts of entries 2 kc + 2, 2 kc + 3
          l2[(kc + 1) & 1] = *reinterpret_cast<const float2*>(
              &T.lamT[cb][8 * ((kc + 1) / 2) + 4 * h + 2 * ((kc + 1) % 2)]);
        mma_chunk<PREC>(Sn[0], B3[kc % 3], Bf[kc]);
        const float2 lv = l2[kc & 1];
        const float g0 = __builtin_amdgcn_exp2f(S[0][2 * kc] + gj - lv.x);
        const float g1 = __builtin_amdgcn_exp2f(S[0][2 * kc + 1] + gj - lv.y);
        csum += g0;
        csum += g1;
        uint32_t hu, lu;
        split2(g0, g1, hu, lu);
        Frag<TMC_BF16X3>& f = P[0].f[kc / 4];
        u32x4 hv = __builtin_bit_cast(u32x4, f.hi), lv4 = __builtin_bit_cast(u32x4, f.lo);
        hv[kc % 4] = hu;
        lv4[kc % 4] = lu;
        f.hi = __builtin_bit_cast(bf16x8, hv);
        f.lo = __builtin_bit_cast(bf16x8, lv4);
      }
    }
  };
  auto phase_b = [&](int cb, int b, bool fresh, int r3, bool fresh3, const PFrag<PREC> (&P)[NS]) {
    if constexpr (kAhead) {
      constexpr int NFT = TilePrefetch<NKC, NS, WV>::NFT;
      constexpr int NA = NFT + 2;   // staging parts: NFT columns, row shifts + row terms, fetch
      double qa[2] = {0.0, 0.0};
      TFrag<PREC> T2[2];
      tile_rowT_frag<TS>(tix, T, cb, 0, 0, T2[0]);
#pragma unroll
      for (int q = 0; q < ND32; ++q) {
        if (q + 1 < ND32) tile_rowT_frag<TS>(tix, T, cb, 0, q + 1, T2[(q + 1) & 1]);
        mma_t<PREC>(GT[q], T2[q & 1], P[0]);
#pragma unroll
        for (int k = 0; k < NA; ++k) {
          if (k * ND32 / NA != q) continue;
          if (k < NFT) {
            tile_store_part<TS, NKC, false, WV>(tix, T, b, pf, true, 0, k, qa);
          } else if (k == NFT) {
            const int rr = tid & 31;
            T.lamT[b][rr] = (rr < pf.rem) ? pf.lam : INFINITY;
            row_terms(fresh);
          } else {
            fetch_rows(tix, pf, L, z, lamrow, r3, evp, p, fresh3);
          }
        }
      }
    }
  };

  if constexpr (NB == 3) {
    // Pipelined sweep over three LDS stages (see the forward): phase A issues the
    // factor-GEMM MFMAs of tile t+1 with the marginals of tile t between them, phase B
    // the G^T z MFMAs of tile t with the staging of tile t+2 (row terms included) and
    // the fetch of tile t+3 between them.  Columns past Kc compute on clamped columns
    // with gamma = -inf (zero marginals) and are discarded in the epilogue.
    stage(0, own(0));
    fetch_rows(tix, pf, L, z, lamrow, 32 * NS, evp, p, nt > 1 && own(1));
    lds_barrier();                                   // tile 0 visible
    stage(1, nt > 1 && own(1));
    fetch_rows(tix, pf, L, z, lamrow, 64 * NS, evp, p, nt > 2 && own(2));
    f32x16 S[NS];
    s_gemm(0, S);
    lds_barrier();                                   // tile 1 visible
    int cur = 0;
    for (int t = 0; t + 1 < nt; ++t) {
      const int nxt = cur == 2 ? 0 : cur + 1;
      const int stg = nxt == 2 ? 0 : nxt + 1;
      f32x16 Sn[NS];
      PFrag<PREC> P[NS];
      if constexpr (kAhead) {
        phase_a(nxt, cur, S, Sn, P);
        phase_b(cur, stg, t + 2 < nt && own(t + 2), 32 * (t + 3), t + 3 < nt && own(t + 3), P);
      } else {
        // phase A
        s_gemm(nxt, Sn);
        marg_exp(cur, S, P);
        interleave_phase_a<kGemmMfma<PREC, NKC> * NS, 8>();
        // phase B
        gt_gemm(cur, P);
        stage(stg, t + 2 < nt && own(t + 2));
        fetch_rows(tix, pf, L, z, lamrow, 32 * NS * (t + 3), evp, p, t + 3 < nt && own(t + 3));
        interleave_phase_b<ND32 * NS * 2 * (PREC == TMC_BF16X3 ? 3 : 8)>();
      }
      lds_barrier();
#pragma unroll
      for (int sb = 0; sb < NS; ++sb) S[sb] = Sn[sb];
      cur = nxt;
    }
    // the last tile: no next tile to multiply, stage or fetch
    marg(cur, S);
  } else {
    stage(0, own(0));
    if (nt > 1) fetch_rows(tix, pf, L, z, lamrow, 32 * NS, evp, p, own(1));
    lds_barrier();
    // One tile (see the forward: S MFMAs first, the next stage behind them).
    auto tile = [&](auto bc, int t) {
      constexpr int cur = decltype(bc)::value;
      if constexpr (NB == 2) {
        if (active) {
          f32x16 S[NS];
          s_gemm(cur, S);
          stage(cur ^ 1, t + 1 < nt && own(t + 1));
          interleave_mfma<kGemmMfma<PREC, NKC> * NS>();
          if (t + 2 < nt) fetch_rows(tix, pf, L, z, lamrow, 32 * NS * (t + 2), evp, p, own(t + 2));
          marg(cur, S);
        } else {
          stage(cur ^ 1, t + 1 < nt && own(t + 1));
          if (t + 2 < nt) fetch_rows(tix, pf, L, z, lamrow, 32 * NS * (t + 2), evp, p, own(t + 2));
        }
        lds_barrier();
      } else {
        if (active) {
          f32x16 S[NS];
          s_gemm(cur, S);
          marg(cur, S);
        }
        lds_barrier();
        if (t + 1 < nt) {
          stage(0, own(t + 1));
          if (t + 2 < nt) fetch_rows(tix, pf, L, z, lamrow, 32 * NS * (t + 2), evp, p, own(t + 2));
          lds_barrier();
        }
      }
    };
    if constexpr (NB == 2) {
      int t = 0;
      for (; t + 1 < nt; t += 2) {
        tile(std::integral_constant<int, 0>{}, t);
        tile(std::integral_constant<int, 1>{}, t + 1);
      }
      if (t < nt) tile(std::integral_constant<int, 0>{}, t);
    } else {
      for (int t = 0; t < nt; ++t) tile(std::integral_constant<int, 0>{}, t);
    }
  }

  // ---- column epilogue: marginals of layer l+1, dmu, column part of ds ----
  if constexpr (PREC == TMC_BF16X3) {
    // the BF16X3 sweep formed sum_i G_ij log2(e) lam_d z_id from the scaled row copy
#pragma unroll
    for (int q = 0; q < ND32; ++q)
#pragma unroll
      for (int v = 0; v < 16; ++v) GT[q][v] *= T.rlam2[32 * q + 8 * (v / 4) + 4 * h + (v % 4)];
  }
  const float ctot = xor32_sum(csum);
  const bool jv = active && j < L.Kc;
  if (jv && h == 0) {
    p[L.p_up_off + j] = ctot;
    if (du) du[L.u_up_off + j] = (float)(gl * (double)ctot);
    if (!L.up_top) {
      // row shift of layer l+1 for the next backward step (rl and Lam share indexing)
      const float ell = rl[L.alpha_up_off + j];
      lam_ws[L.alpha_up_off + j] = (ctot == 0.0f) ? INFINITY : ell - log2f(ctot);
    }
  }
  // per-lane column terms p'_j mu_jd^2 - 2 mu_jd (G^T z)_jd, reduced over the wave's
  // 32 columns through LDS (wave by wave, fixed order)
  float colt[ND32][16];
  if ((L.D % 4 == 0) && (L.mu_off % 4 == 0)) {
    // all loads of mu_j first (one round trip), then the column terms and dmu
    const float* murow = mu + L.mu_off + (int64_t)jc * L.D;
    float4 mr[ND32][4];
#pragma unroll
    for (int q = 0; q < ND32; ++q)
#pragma unroll
      for (int g = 0; g < 4; ++g)
        mr[q][g] = *reinterpret_cast<const float4*>(murow + min(32 * q + 8 * g + 4 * h, L.D - 4));
    float* dmurow = dmu ? dmu + L.mu_off + (int64_t)jc * L.D : nullptr;
#pragma unroll
    for (int q = 0; q < ND32; ++q)
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int d = 32 * q + 8 * g + 4 * h;
        const bool v = jv && d < L.D;
        const float mv[4] = {v ? mr[q][g].x : 0.0f, v ? mr[q][g].y : 0.0f, v ? mr[q][g].z : 0.0f,
                             v ? mr[q][g].w : 0.0f};
        float o[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float gt = GT[q][4 * g + e];
          colt[q][4 * g + e] = jv ? (ctot * mv[e] - 2.0f * gt) * mv[e] : 0.0f;
          o[e] = (d < L.D) ? g32 * T.lamf[d + e] * (gt - ctot * mv[e]) : 0.0f;
        }
        // D % 4 == 0: a float4 at d < D is whole
        if (v && dmurow)
          *reinterpret_cast<float4*>(dmurow + d) = make_float4(o[0], o[1], o[2], o[3]);
      }
  } else {
    const bool mvec = false;
    const float* murow = mu + L.mu_off + (int64_t)jc * L.D;
    float* dmurow = dmu ? dmu + L.mu_off + (int64_t)jc * L.D : nullptr;
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
  if (!dsp) return;   // (uniform: ends this item)
  // one column part per 128 columns (waves 4 h .. 4 h + 3), whatever the workgroup size;
  // the two halves of an 8-wave workgroup are reduced side by side in their own buffers
  // (the tile copies are free once the sweep is done)
  // (rows of the reduction buffer are DT + 1 floats apart: the 32 lanes of a wave that
  // write one slot of 32 different rows then hit distinct banks, not one or a few)
  constexpr int RB = TS::DT + 1;
  float* buf = reinterpret_cast<float*>(TS::COL ? (void*)&T.col[0][0][0] : (void*)&T.row[0][0][0]);
  static_assert((TS::COL ? sizeof(T.col) : sizeof(T.row)) >= (WV / 4) * 32 * RB * sizeof(float),
                "reduction buffer");
  if constexpr (WV == 8) {
    if (dzw) {
      // row part of ds over the workgroup's rows: the 32 row slots' sums, reduced in a
      // fixed order, into row partial wg_c (workgroup 0 zeroes partials nwg .. nrow - 1)
      static_assert((WV / 4) * 32 * RB >= 32 * RB + 32, "row reduction buffer");
      lds_barrier();
      const int r = tid / TPR, sub = tid % TPR;
#pragma unroll
      for (int m = 0; m < NFT; ++m)
#pragma unroll
        for (int e = 0; e < 4; ++e) buf[r * RB + 4 * (sub + TPR * m) + e] = rsum[m][e];
      if (sub == 0) buf[32 * RB + r] = psum;
      lds_barrier();
      float P = 0.0f;
      for (int c = 0; c < 32; ++c) P += buf[32 * RB + c];
      const int ncol = (L.Kc + kFusedBwdColsDev - 1) / kFusedBwdColsDev;
      const int nrow = (L.K + kFusedDzRowsDev - 1) / kFusedDzRowsDev;
      float* part = dsp + L.dsp_off + (int64_t)(ncol + wg_c) * L.D;
      for (int d = tid; d < L.D; d += blockDim.x) {
        float acc = 0.0f;
        for (int c = 0; c < 32; ++c) acc += buf[c * RB + d];
        part[d] = g32 * (T.lamf[d] * acc - P);
      }
      if (wg_c == 0)
        for (int e = tid; e < (nrow - nwg) * L.D; e += blockDim.x) part[(int64_t)nwg * L.D + e] = 0.0f;
    }
  }
  for (int w2 = 0; w2 < 4; ++w2) {
    lds_barrier();
    if ((w & 3) == w2) {
      float* bw = buf + (w >> 2) * 32 * RB;
#pragma unroll
      for (int q = 0; q < ND32; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) bw[jr * RB + 32 * q + 8 * (v / 4) + 4 * h + (v % 4)] = colt[q][v];
    }
    lds_barrier();
    for (int e = tid; e < (WV / 4) * TS::DT; e += blockDim.x) {
      const float* bh = buf + (e / TS::DT) * 32 * RB;
      const int d = e % TS::DT;
      float acc = 0.0f;
      for (int c = 0; c < 32; ++c) acc += bh[c * RB + d];
      accD[e] += acc;
    }
  }
  lds_barrier();
#pragma unroll
  for (int hh = 0; hh < WV / 4; ++hh) {
    if (it.start + kFusedBwdColsDev * hh >= L.Kc) break;   // (uniform)
    const int part = it.start / kFusedBwdColsDev + hh;
    for (int d = tid; d < L.D; d += blockDim.x)
      dsp[L.dsp_off + (int64_t)part * L.D + d] = g32 * T.lamf[d] * accD[hh * TS::DT + d];
  }
}

template <int PREC, int NKC, int NS, int WV>
__global__ __launch_bounds__(64 * WV, (WV == 8 ? 1 : (NKC <= 8 ? 2 : 1))) void k_fused_bwd(BwdArgs args) {
  __shared__ __align__(16) BwdSmem<PREC, NKC, NS> T;
  __shared__ float accD[(WV / 4) * BwdSmem<PREC, NKC, NS>::DT];
  const Item it = args.items[xcd_item(blockIdx.x, gridDim.x)];
  const LayerDev L = args.Ls[it.layer];
  bwd_item<PREC, NKC, NS, WV>((int)threadIdx.x, T, accD, it, L, args);
}

// Persistent backward: each workgroup takes whole chains and runs their pairs
// bottom-up (pair l reads the row shifts Lam_l its own pair l-1 wrote).
template <int PREC, int NKC, int NS>
__global__ __launch_bounds__(256, (NKC <= 8 ? 2 : 1)) void k_fused_bwd_persist(BwdArgs args,
                                                                               ChainQueue q) {
  __shared__ __align__(16) BwdSmem<PREC, NKC, NS> T;
  __shared__ float accD[BwdSmem<PREC, NKC, NS>::DT];
  __shared__ int s_k;
  for (;;) {
    if (threadIdx.x == 0) s_k = atomicAdd(q.head, 1);
    __syncthreads();
    // uniform across the workgroup: keep it (and all that derives from it) scalar
    const int k = __builtin_amdgcn_readfirstlane(s_k);
    __syncthreads();
    if (k >= q.n) return;
    const ChainDev ch = q.cd[q.chains[k]];
    for (int l = ch.first; l < ch.top; ++l) {
      const LayerDev L = args.Ls[l];
      for (int x = 0; x < L.Kc; x += kFusedBwdColsDev) {
        bwd_item<PREC, NKC, NS, 4>(item_tid(), T, accD, Item{l, x}, L, args);
        __syncthreads();
      }
    }
  }
}

}  // namespace fused
}  // namespace tmc

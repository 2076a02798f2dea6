// Log-domain matrix product (Appendix "Numerically stable matrix (tensor) products in the
// log-domain"), batched:
//   Z_b[i,k] = log sum_j exp(X_b[i,j] + Y_b[j,k]),  X_b [M][K], Y_b [K][N], Z_b [M][N].
// The Appendix's shift, x_i = max_j X_ij and y_k = max_j Y_jk, makes every exponential
// at most 1, so the sum is an ordinary matrix product C = exp(X - x) exp(Y - y) on the
// matrix cores; the shifted exponentials are formed once, in the operand layout of the
// product (BF16 hi/lo planes, FP32 or FP64, Y's transposed, the reduction index padded
// with zeros to a multiple of 32), and Z = log C + x + y.  Where that shift underflows
// (log C below the floor, -60 in FP32 / BF16X3 and -600 in FP64: the maxima of X's row
// and Y's column sit at indices j far apart), the epilogue recomputes the entry exactly,
// with its own maximum over j, on the vector ALU.
#include <math.h>

#include "../../include/tmc.h"
#include "dev_util.h"
#include "tmc_logmm.h"

namespace tmc {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
// (register arrays of the operand staging use native vector types: arrays of HIP's
// float4 / double2 structs are not promoted to registers here)
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

constexpr int kTile = kLogmmTile;   // output rows and columns of a workgroup
constexpr int kKC = 32;             // reduction indices staged per step
constexpr int kColmaxCW = 32;       // columns of a column-maximum workgroup
constexpr int kPadB = 8;            // bf16 row padding of the LDS tiles (16 B)
constexpr int kPadF = 4;            // float row padding
constexpr float kLogmmFloor = -60.0f;
constexpr double kLogmmFloorD = -600.0;   // FP64: far above the underflow of a product
                                          // of two exponentials (e^-745) summed K times

// x = hi + lo for two values at once (hi = bf16(x), lo = bf16(x - hi), round to nearest).
__device__ __forceinline__ void split_pair(float a, float b, uint32_t& hi, uint32_t& lo) {
  const uint32_t hu = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a, b}, bf16x2));
  const float ha = __uint_as_float(hu << 16), hb = __uint_as_float(hu & 0xffff0000u);
  hi = hu;
  lo = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){a - ha, b - hb}, bf16x2));
}

template <int PREC>
struct LogmmSmem;
template <>
struct LogmmSmem<TMC_BF16X3> {
  __bf16 a[2][kTile][kKC + kPadB];   // [hi/lo][row i][j]
  __bf16 b[2][kTile][kKC + kPadB];   // [hi/lo][column k][j]
};
template <>
struct LogmmSmem<TMC_FP32> {
  float a[kTile][kKC + kPadF];
  float b[kTile][kKC + kPadF];
};

// Prepared operand element e (one row of 8 consecutive j): BF16X3 writes its hi part at
// e in the first plane and its lo part at e in the second (plane stride ps); FP32 the values.
template <int PREC, typename T>
__device__ __forceinline__ void store_operand(void* base, int64_t ps, int64_t e, const T (&v)[8]) {
  if constexpr (PREC == TMC_FP64) {
    double* dp = static_cast<double*>(base);
#pragma unroll
    for (int q = 0; q < 4; ++q) *reinterpret_cast<double2*>(dp + e + 2 * q) = make_double2(v[2 * q], v[2 * q + 1]);
  } else if constexpr (PREC == TMC_BF16X3) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) split_pair(v[2 * p], v[2 * p + 1], h[p], l[p]);
    __bf16* bp = static_cast<__bf16*>(base);
    *reinterpret_cast<u32x4*>(bp + e) = (u32x4){h[0], h[1], h[2], h[3]};
    *reinterpret_cast<u32x4*>(bp + ps + e) = (u32x4){l[0], l[1], l[2], l[3]};
  } else {
    float* fp = static_cast<float*>(base);
    *reinterpret_cast<float4*>(fp + e) = make_float4(v[0], v[1], v[2], v[3]);
    *reinterpret_cast<float4*>(fp + e + 4) = make_float4(v[4], v[5], v[6], v[7]);
  }
}

// 16 consecutive j of one operand row, as loaded (BF16X3: hi and lo, 32 B each; FP32: 64 B).
template <int PREC>
struct OperandRegs;
template <>
struct OperandRegs<TMC_BF16X3> {
  u32x4 h[2], l[2];
};
template <>
struct OperandRegs<TMC_FP32> {
  f32x4 v[4];
};

template <int PREC>
__device__ __forceinline__ void load_operand(const void* base, int64_t ps, int64_t e, OperandRegs<PREC>& r) {
  if constexpr (PREC == TMC_BF16X3) {
    const __bf16* bp = static_cast<const __bf16*>(base);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      r.h[q] = *reinterpret_cast<const u32x4*>(bp + e + 8 * q);
      r.l[q] = *reinterpret_cast<const u32x4*>(bp + ps + e + 8 * q);
    }
  } else {
    const float* fp = static_cast<const float*>(base);
#pragma unroll
    for (int q = 0; q < 4; ++q) r.v[q] = *reinterpret_cast<const f32x4*>(fp + e + 4 * q);
  }
}

template <int PREC>
__device__ __forceinline__ void stage_operand(LogmmSmem<PREC>& S, bool is_a, int row, int j,
                                              const OperandRegs<PREC>& r) {
  if constexpr (PREC == TMC_BF16X3) {
    __bf16* hp = is_a ? &S.a[0][row][j] : &S.b[0][row][j];
    __bf16* lp = is_a ? &S.a[1][row][j] : &S.b[1][row][j];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      *reinterpret_cast<u32x4*>(hp + 8 * q) = r.h[q];
      *reinterpret_cast<u32x4*>(lp + 8 * q) = r.l[q];
    }
  } else {
    float* p = is_a ? &S.a[row][j] : &S.b[row][j];
#pragma unroll
    for (int q = 0; q < 4; ++q) *reinterpret_cast<f32x4*>(p + 4 * q) = r.v[q];
  }
}

// log sum_j exp(x[j] + y[j N]) by its own maximum over j (two passes); -inf when every
// term is -inf, NaN when one is NaN.
template <typename T>
__device__ T exact_entry(const T* __restrict__ x, const T* __restrict__ y, int K, int N) {
  T m = (T)(-INFINITY);
  for (int j = 0; j < K; ++j) m = nan_max(m, x[j] + y[(int64_t)j * N]);
  if (m == (T)(-INFINITY) || m != m) return m;
  T s = (T)0;
  for (int j = 0; j < K; ++j) s += exp(x[j] + y[(int64_t)j * N] - m);
  return m + log(s);
}

}  // namespace

// Shifts: xs[b][i] = max_j X_b[i,j] (in k_logmm_prep_x) and ys[b][k] = max_j Y_b[j,k]
// (below); an all -inf row or column gets 0 (its exponentials are then 0, never NaN).
// Column maxima: a workgroup of 16 waves per CW columns; lane l of wave w takes column
// l % CW and rows (64 / CW) w + l / CW + 1024 / CW * q (loads issued 8 at a time), so a
// wave reads 64 / CW rows of CW consecutive columns per load and the grid has 64 / CW
// times as many workgroups as with one column per lane (at 8 x 1024 x 1024 and CW = 64
// only 128 workgroups for 256 CUs); the partial maxima are merged in LDS.  CW = 32
// (128-byte row pieces in FP32) measured best: 10.2 us at 8 x 1024 x 1024 FP32, against
// 11.5 at CW = 64 and 17.5 at CW = 16 (64-byte pieces).
template <typename T, int CW>
__global__ __launch_bounds__(1024) void k_logmm_colmax(LogmmArgs a, const T* __restrict__ Y,
                                                       T* __restrict__ ys) {
  constexpr int RG = kWave / CW;    // row groups of a wave
  constexpr int RS = 16 * RG;       // rows of one load step of the workgroup
  __shared__ T part[16 * RG][CW];
  const int b = blockIdx.z;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int c = lane % CW, g = RG * w + lane / CW;   // column in the block, row group
  const int64_t col = (int64_t)blockIdx.x * CW + c;
  const bool cv = col < a.N;
  const T* y = Y + (int64_t)b * a.K * a.N + (cv ? col : 0);
  T m = (T)(-INFINITY);
  constexpr int U = 8;
  for (int j0 = g; j0 < a.K; j0 += RS * U) {
    T v[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int j = j0 + RS * q;
      v[q] = j < a.K ? y[(int64_t)j * a.N] : (T)(-INFINITY);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) m = nan_max(m, v[q]);
  }
  part[g][c] = m;
  __syncthreads();
  if (threadIdx.x < CW) {
    const int cc = threadIdx.x;
    const int64_t colc = (int64_t)blockIdx.x * CW + cc;
    T mm = part[0][cc];
#pragma unroll 4
    for (int q = 1; q < 16 * RG; ++q) mm = nan_max(mm, part[q][cc]);
    if (colc < a.N) ys[(int64_t)b * a.N + colc] = (mm == (T)(-INFINITY)) ? (T)0 : mm;
  }
}

// exp in the operand's precision (FP64: the libm exp; otherwise the fast FP32 one)
__device__ __forceinline__ float op_exp(float v) { return __expf(v); }
__device__ __forceinline__ double op_exp(double v) { return exp(v); }

// Operands of the product: A[b][i][j] = exp(X_b[i,j] - x_i) and Bt[b][k][j] =
// exp(Y_b[j,k] - y_k) (Y transposed), j padded with zeros to Kp; BF16X3 stores hi and lo
// planes (one after the other, each [B][rows][Kp]), FP32 the values.  Rows of X: a wave per
// row finds the row maximum x_i (written to xs; an all -inf row gets 0), then writes the
// row, 8 consecutive j per lane and step.
template <int PREC>
__global__ __launch_bounds__(256) void k_logmm_prep_x(LogmmArgs a) {
  typedef typename std::conditional<PREC == TMC_FP64, double, float>::type T;
  const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;   // b M + i
  if (row >= (int64_t)a.B * a.M) return;   // (uniform per wave)
  const int lane = threadIdx.x % kWave;
  const T* x = (PREC == TMC_FP64 ? (const T*)a.Xd : (const T*)a.X) + row * a.K;
  if constexpr (PREC != TMC_FP64) {
    // Rows of at most 1024 floats, 16-byte aligned: one read into registers (lane: 4
    // consecutive j of each 256-wide chunk), the maximum, then the exponentials from the
    // registers -- X is read once instead of twice (FP64 below: 2 j of 8 chunks).
    if (a.Kp <= 1024 && (a.K % 4) == 0 && (reinterpret_cast<uintptr_t>(a.X) % 16) == 0) {
      f32x4 v[4];
      float m = -INFINITY;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int e = 4 * (lane + kWave * c);
        v[c] = e < a.K ? *reinterpret_cast<const f32x4*>(x + e)
                       : (f32x4){-INFINITY, -INFINITY, -INFINITY, -INFINITY};
#pragma unroll
        for (int i = 0; i < 4; ++i) m = nan_max(m, v[c][i]);
      }
      m = wave_max(m);
      const float sh = (m == -INFINITY) ? 0.0f : m;
      if (lane == 0) a.xs[row] = sh;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int e = 4 * (lane + kWave * c);
        if (e >= a.Kp) continue;
        float o[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) o[i] = e + i < a.K ? __expf(v[c][i] - sh) : 0.0f;
        const int64_t eo = row * a.Kp + e;
        if constexpr (PREC == TMC_BF16X3) {
          uint32_t h[2], l[2];
          split_pair(o[0], o[1], h[0], l[0]);
          split_pair(o[2], o[3], h[1], l[1]);
          __bf16* bp = static_cast<__bf16*>(a.opa);
          const int64_t ps = (int64_t)a.B * a.M * a.Kp;
          *reinterpret_cast<u32x2*>(bp + eo) = (u32x2){h[0], h[1]};
          *reinterpret_cast<u32x2*>(bp + ps + eo) = (u32x2){l[0], l[1]};
        } else {
          *reinterpret_cast<f32x4*>(static_cast<float*>(a.opa) + eo) = (f32x4){o[0], o[1], o[2], o[3]};
        }
      }
      return;
    }
  } else {
    // FP64 rows of at most 1024 doubles: lane j pairs 2 (lane + 64 c), c < 8
    if (a.Kp <= 1024 && (a.K % 2) == 0 && (reinterpret_cast<uintptr_t>(a.Xd) % 16) == 0) {
      f64x2 v[8];
      double m = -INFINITY;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int e = 2 * (lane + kWave * c);
        v[c] = e < a.K ? *reinterpret_cast<const f64x2*>(x + e) : (f64x2){-INFINITY, -INFINITY};
        m = nan_max(m, nan_max(v[c][0], v[c][1]));
      }
      m = wave_max(m);
      const double sh = (m == -INFINITY) ? 0.0 : m;
      if (lane == 0) a.xsd[row] = sh;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int e = 2 * (lane + kWave * c);
        if (e >= a.Kp) continue;
        const f64x2 o = {e < a.K ? exp(v[c][0] - sh) : 0.0, e + 1 < a.K ? exp(v[c][1] - sh) : 0.0};
        *reinterpret_cast<f64x2*>(static_cast<double*>(a.opa) + row * a.Kp + e) = o;
      }
      return;
    }
  }
  T m = (T)(-INFINITY);
  for (int j = lane; j < a.K; j += kWave) m = nan_max(m, x[j]);
  m = wave_max(m);
  const T sh = (m == (T)(-INFINITY)) ? (T)0 : m;
  if (lane == 0) (PREC == TMC_FP64 ? (T*)a.xsd : (T*)a.xs)[row] = sh;
  for (int j0 = 8 * lane; j0 < a.Kp; j0 += 8 * kWave) {
    T v[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = j0 + s < a.K ? op_exp(x[j0 + s] - sh) : (T)0;
    store_operand<PREC>(a.opa, (int64_t)a.B * a.M * a.Kp, row * a.Kp + j0, v);
  }
}

// Columns of Y into rows of Bt: a workgroup per 64 j x 64 k tile, read along k (coalesced),
// transposed through LDS, written along j.
template <int PREC>
__global__ __launch_bounds__(256) void k_logmm_prep_y(LogmmArgs a) {
  typedef typename std::conditional<PREC == TMC_FP64, double, float>::type T;
  __shared__ T tile[64][64 + 1];
  const int b = blockIdx.z, j0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
  const int t = threadIdx.x;
  {
    const int kl = t % 64, k = k0 + kl;
    const T* ysp = PREC == TMC_FP64 ? (const T*)a.ysd : (const T*)a.ys;
    const T ysh = k < a.N ? ysp[(int64_t)b * a.N + k] : (T)0;
    const T* y = (PREC == TMC_FP64 ? (const T*)a.Yd : (const T*)a.Y) + (int64_t)b * a.K * a.N;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int jl = 16 * (t / 64) + r, j = j0 + jl;
      tile[kl][jl] = (j < a.K && k < a.N) ? op_exp(y[(int64_t)j * a.N + k] - ysh) : (T)0;
    }
  }
  __syncthreads();
  const int kl = t / 4, k = k0 + kl, jc = (t % 4) * 16;
  if (k >= a.N) return;
  const int64_t rowo = ((int64_t)b * a.N + k) * a.Kp + j0 + jc;
  T v[8];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int s = 0; s < 8; ++s) v[s] = tile[kl][jc + 8 * h + s];
    if (j0 + jc + 8 * h < a.Kp) store_operand<PREC>(a.opb, (int64_t)a.B * a.N * a.Kp, rowo + 8 * h, v);
  }
}

// Output tile of this workgroup, XCD-aware: workgroups are handed to the 8 XCDs in turn
// by flattened index, so workgroup w runs on XCD w mod 8.  The first 8 floor(n / 8) tiles
// (x fastest, then y, then the batch) are dealt out in 8 contiguous ranges, range c to the
// workgroups of XCD c, so the tiles one XCD runs share their row and column panels in its
// L2 (at 8 x 1024^3 an XCD runs one product of the batch); the rest keep their own index.
__device__ __forceinline__ void logmm_tile(int& bx, int& by, int& bz) {
  const int nx = gridDim.x, ny = gridDim.y;
  const int n = nx * ny * gridDim.z;
  int w = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
  const int full = n & ~7;
  if (w < full) w = (w & 7) * (full >> 3) + (w >> 3);
  bx = w % nx;
  by = (w / nx) % ny;
  bz = w / (nx * ny);
}

// The shifted product on MFMA: a workgroup of 4 waves per 128 x 128 output tile (wave w:
// rows 64 (w / 2), columns 64 (w % 2), as 2 x 2 accumulators of 32 x 32), the reduction
// index staged 32 at a time from the prepared operands (thread t: row t / 2 of each
// operand tile, 16 consecutive j; rows past the matrix edge read the last row and their
// results are discarded); the global loads of the next slice are in flight during the
// current slice's MFMAs.  Operand fragments: lane l holds row (column) l % 32 of its block
// and j = 16 s + 8 (l / 32) .. + 7 of step s (both operands in that order); accumulator
// value v of lane l is row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32.
template <int PREC>
__global__ __launch_bounds__(256) void k_logmm_mfma(LogmmArgs a) {
  __shared__ LogmmSmem<PREC> SB[2];   // slice s is read from SB[s % 2]
  int bx, by, b;
  logmm_tile(bx, by, b);
  const int i0 = by * kTile, k0 = bx * kTile;
  const int M = a.M, N = a.N, Kp = a.Kp;
  const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
  const int r = t / 2, jg = (t % 2) * 16;
  const int64_t ra = ((int64_t)b * M + min(i0 + r, M - 1)) * Kp + jg;
  const int64_t rb = ((int64_t)b * N + min(k0 + r, N - 1)) * Kp + jg;
  const int64_t pa = (int64_t)a.B * M * Kp, pb = (int64_t)a.B * N * Kp;   // plane sizes
  OperandRegs<PREC> xa, xb;
  f32x16 acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = (f32x16){};
  const int wr = 64 * (w / 2), wc = 64 * (w % 2);
  const int ns = Kp / kKC;
  load_operand<PREC>(a.opa, pa, ra, xa);
  load_operand<PREC>(a.opb, pb, rb, xb);
  stage_operand<PREC>(SB[0], true, r, jg, xa);
  stage_operand<PREC>(SB[0], false, r, jg, xb);
  {
    const int jn = min(kKC, Kp - kKC);
    load_operand<PREC>(a.opa, pa, ra + jn, xa);
    load_operand<PREC>(a.opb, pb, rb + jn, xb);
  }
  __syncthreads();
  for (int sl = 0; sl < ns; ++sl) {
    const LogmmSmem<PREC>& S = SB[sl & 1];
#pragma unroll
    for (int st = 0; st < kKC / 16; ++st) {
      const int jj = 16 * st + 8 * (lane / 32);
      if constexpr (PREC == TMC_BF16X3) {
        bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          ah[p] = *reinterpret_cast<const bf16x8*>(&S.a[0][wr + 32 * p + lane % 32][jj]);
          al[p] = *reinterpret_cast<const bf16x8*>(&S.a[1][wr + 32 * p + lane % 32][jj]);
          bh[p] = *reinterpret_cast<const bf16x8*>(&S.b[0][wc + 32 * p + lane % 32][jj]);
          bl[p] = *reinterpret_cast<const bf16x8*>(&S.b[1][wc + 32 * p + lane % 32][jj]);
        }
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[p], bh[q], acc[p][q], 0, 0, 0);
            acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[p], bl[q], acc[p][q], 0, 0, 0);
            acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[p], bh[q], acc[p][q], 0, 0, 0);
          }
      } else {
        float af[2][8], bfv[2][8];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          const float4 a0 = *reinterpret_cast<const float4*>(&S.a[wr + 32 * p + lane % 32][jj]);
          const float4 a1 = *reinterpret_cast<const float4*>(&S.a[wr + 32 * p + lane % 32][jj + 4]);
          const float4 b0 = *reinterpret_cast<const float4*>(&S.b[wc + 32 * p + lane % 32][jj]);
          const float4 b1 = *reinterpret_cast<const float4*>(&S.b[wc + 32 * p + lane % 32][jj + 4]);
          af[p][0] = a0.x; af[p][1] = a0.y; af[p][2] = a0.z; af[p][3] = a0.w;
          af[p][4] = a1.x; af[p][5] = a1.y; af[p][6] = a1.z; af[p][7] = a1.w;
          bfv[p][0] = b0.x; bfv[p][1] = b0.y; bfv[p][2] = b0.z; bfv[p][3] = b0.w;
          bfv[p][4] = b1.x; bfv[p][5] = b1.y; bfv[p][6] = b1.z; bfv[p][7] = b1.w;
        }
#pragma unroll
        for (int s2 = 0; s2 < 8; ++s2)
#pragma unroll
          for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q)
              acc[p][q] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[p][s2], bfv[q][s2], acc[p][q], 0, 0, 0);
      }
    }
    // Slice sl + 1 into the other buffer (its last reads, slice sl - 1, ended before the
    // barrier that closed the previous step), then slice sl + 2 in flight.  Both are
    // unconditional -- past the end they repeat the last slice into a buffer no one reads
    // again -- so the operands stay in registers.
    stage_operand<PREC>(SB[(sl + 1) & 1], true, r, jg, xa);
    stage_operand<PREC>(SB[(sl + 1) & 1], false, r, jg, xb);
    const int jn = min((sl + 2) * kKC, Kp - kKC);
    load_operand<PREC>(a.opa, pa, ra + jn, xa);
    load_operand<PREC>(a.opb, pb, rb + jn, xb);
    __syncthreads();
  }
  // Z = log C + x + y; the entries whose shifted product fell below the floor (or is
  // not a number) are marked and recomputed exactly afterwards (rare: the lane loops
  // over j on its own)
  const float floor_c = __expf(kLogmmFloor);
  uint64_t redo = 0;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int k = k0 + wc + 32 * q + lane % 32;
    const float ys = k < N ? a.ys[(int64_t)b * N + k] : 0.0f;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int i = i0 + wr + 32 * p + 8 * (v / 4) + 4 * (lane / 32) + v % 4;
        const float c = acc[p][q][v];
        if (k < N && i < M) {
          if (c >= floor_c)
            a.Z[((int64_t)b * M + i) * N + k] = __logf(c) + a.xs[(int64_t)b * M + i] + ys;
          else
            redo |= 1ull << (32 * q + 16 * p + v);
        }
      }
  }
  while (redo) {
    const int e = __builtin_ctzll(redo);
    redo &= redo - 1;
    const int q = e / 32, p = (e / 16) % 2, v = e % 16;
    const int k = k0 + wc + 32 * q + lane % 32;
    const int i = i0 + wr + 32 * p + 8 * (v / 4) + 4 * (lane / 32) + v % 4;
    a.Z[((int64_t)b * M + i) * N + k] =
        exact_entry<float>(a.X + ((int64_t)b * M + i) * a.K, a.Y + (int64_t)b * a.K * N + k, a.K, N);
  }
}

// The shifted product in FP64 (v_mfma_f64_16x16x4_f64): a workgroup of 8 waves per
// 128 x 128 output tile (wave w: rows 64 (w / 4), columns 32 (w % 4), as 4 x 2
// accumulators of 16 x 16), the reduction index staged 16 at a time (thread t: row t / 4
// of each operand tile, 4 consecutive j; rows past the matrix edge read the last row and
// their results are discarded), the next slice's global loads in flight during the
// current slice's MFMAs.  Operand fragments of k-step s: lane l holds row (column)
// l % 16 of its block at j = 4 s + l / 16; accumulator value v of lane l is row
// l / 16 + 4 v, column l % 16.
constexpr int kKCd = 16;   // reduction indices per FP64 slice
constexpr int kPadD = 2;   // row padding of the FP64 LDS tiles (keeps 16-byte rows aligned)
typedef double f64x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(512) void k_logmm_mfma_f64(LogmmArgs a) {
  __shared__ __attribute__((aligned(16))) double SA[kTile][kKCd + kPadD];
  __shared__ __attribute__((aligned(16))) double SB[kTile][kKCd + kPadD];
  int bx, by, b;
  logmm_tile(bx, by, b);
  const int i0 = by * kTile, k0 = bx * kTile;
  const int M = a.M, N = a.N, Kp = a.Kp;
  const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
  const int r = t / 4, jg = (t % 4) * 4;
  const double* opa = static_cast<const double*>(a.opa);
  const double* opb = static_cast<const double*>(a.opb);
  const double* pa = opa + ((int64_t)b * M + min(i0 + r, M - 1)) * Kp + jg;
  const double* pb = opb + ((int64_t)b * N + min(k0 + r, N - 1)) * Kp + jg;
  f64x2 xa[2], xb[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    xa[q] = *reinterpret_cast<const f64x2*>(pa + 2 * q);
    xb[q] = *reinterpret_cast<const f64x2*>(pb + 2 * q);
  }
  f64x4 acc[4][2];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = (f64x4){0.0, 0.0, 0.0, 0.0};
  const int wr = 64 * (w / 4), wc = 32 * (w % 4);
  const int fr = lane % 16, fj = lane / 16;
  for (int j0 = 0; j0 < Kp; j0 += kKCd) {
    __syncthreads();   // (the previous slice's fragment reads are done)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      *reinterpret_cast<f64x2*>(&SA[r][jg + 2 * q]) = xa[q];
      *reinterpret_cast<f64x2*>(&SB[r][jg + 2 * q]) = xb[q];
    }
    __syncthreads();
    {
      // the next slice, in flight during the MFMAs below (after the last slice, the last
      // slice again: unconditional, so the operands stay in registers)
      const int jn = min(j0 + kKCd, Kp - kKCd);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        xa[q] = *reinterpret_cast<const f64x2*>(pa + jn + 2 * q);
        xb[q] = *reinterpret_cast<const f64x2*>(pb + jn + 2 * q);
      }
    }
#pragma unroll
    for (int st = 0; st < kKCd / 4; ++st) {
      double fa[4], fb[2];
#pragma unroll
      for (int p = 0; p < 4; ++p) fa[p] = SA[wr + 16 * p + fr][4 * st + fj];
#pragma unroll
      for (int q = 0; q < 2; ++q) fb[q] = SB[wc + 16 * q + fr][4 * st + fj];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          acc[p][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[p], fb[q], acc[p][q], 0, 0, 0);
    }
  }
  // Z = log C + x + y; the entries whose shifted product fell below the floor (or is
  // not a number) are marked and recomputed exactly afterwards (rare)
  const double floor_c = exp(kLogmmFloorD);
  uint32_t redo = 0;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int k = k0 + wc + 16 * q + fr;
    const double ys = k < N ? a.ysd[(int64_t)b * N + k] : 0.0;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wr + 16 * p + fj + 4 * v;
        const double c = acc[p][q][v];
        if (k < N && i < M) {
          if (c >= floor_c)
            a.Zd[((int64_t)b * M + i) * N + k] = log(c) + a.xsd[(int64_t)b * M + i] + ys;
          else
            redo |= 1u << (16 * q + 4 * p + v);
        }
      }
  }
  while (redo) {
    const int e = __builtin_ctz(redo);
    redo &= redo - 1;
    const int q = e / 16, p = (e / 4) % 4, v = e % 4;
    const int k = k0 + wc + 16 * q + fr, i = i0 + wr + 16 * p + fj + 4 * v;
    a.Zd[((int64_t)b * M + i) * N + k] =
        exact_entry<double>(a.Xd + ((int64_t)b * M + i) * a.K, a.Yd + (int64_t)b * a.K * N + k, a.K, N);
  }
}

hipError_t launch_logmm(const LogmmArgs& a, int precision, hipStream_t st) {
  const dim3 gc((a.N + kColmaxCW - 1) / kColmaxCW, 1, a.B);
  const dim3 grid((a.N + kTile - 1) / kTile, (a.M + kTile - 1) / kTile, a.B);
  const dim3 gx((unsigned)(((int64_t)a.B * a.M + 3) / 4));
  const dim3 gy((a.Kp + 63) / 64, (a.N + 63) / 64, a.B);
  if (precision == TMC_FP64) {
    hipLaunchKernelGGL((k_logmm_colmax<double, kColmaxCW>), gc, dim3(1024), 0, st, a, a.Yd, a.ysd);
    hipLaunchKernelGGL((k_logmm_prep_x<TMC_FP64>), gx, dim3(256), 0, st, a);
    hipLaunchKernelGGL((k_logmm_prep_y<TMC_FP64>), gy, dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_logmm_mfma_f64, grid, dim3(512), 0, st, a);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_logmm_colmax<float, kColmaxCW>), gc, dim3(1024), 0, st, a, a.Y, a.ys);
  if (precision == TMC_BF16X3) {
    hipLaunchKernelGGL((k_logmm_prep_x<TMC_BF16X3>), gx, dim3(256), 0, st, a);
    hipLaunchKernelGGL((k_logmm_prep_y<TMC_BF16X3>), gy, dim3(256), 0, st, a);
    hipLaunchKernelGGL((k_logmm_mfma<TMC_BF16X3>), grid, dim3(256), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_logmm_prep_x<TMC_FP32>), gx, dim3(256), 0, st, a);
    hipLaunchKernelGGL((k_logmm_prep_y<TMC_FP32>), gy, dim3(256), 0, st, a);
    hipLaunchKernelGGL((k_logmm_mfma<TMC_FP32>), grid, dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace tmc

// Log-domain matrix product (Appendix "Numerically stable matrix (tensor) products in the
// log-domain"), batched:
//   Z_b[i,k] = log sum_j exp(X_b[i,j] + Y_b[j,k]),  X_b [M][K], Y_b [K][N], Z_b [M][N].
// Matrix-core path (FP32, BF16X3): the Appendix's shift, x_i = max_j X_ij and
// y_k = max_j Y_jk, makes every exponential at most 1, so the sum is an ordinary matrix
// product C = exp(X - x) exp(Y - y) on MFMA, with the exponentials formed while the
// operand tiles are staged in LDS; Z = log C + x + y.  Where that shift underflows (log C
// below kLogmmFloor: the maxima of X's row and Y's column sit at indices j far apart), a
// fix-up pass recomputes the entry exactly, with its own maximum over j, on the vector
// ALU.  FP64: every entry exactly on the vector ALU.
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

constexpr int kTile = kLogmmTile;   // output rows and columns of a workgroup
constexpr int kKC = 32;             // reduction indices staged per step
constexpr int kPadB = 8;            // bf16 row padding of the LDS tiles (16 B)
constexpr int kPadF = 4;            // float row padding
constexpr float kLogmmFloor = -60.0f;

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

// Stores 16 consecutive reduction-index values of one row (column) of a staged tile.
template <int PREC>
__device__ __forceinline__ void stage16(LogmmSmem<PREC>& S, bool is_a, int row, int j, const float (&v)[16]) {
  if constexpr (PREC == TMC_BF16X3) {
    uint32_t h[8], l[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) split_pair(v[2 * p], v[2 * p + 1], h[p], l[p]);
    __bf16* hp = is_a ? &S.a[0][row][j] : &S.b[0][row][j];
    __bf16* lp = is_a ? &S.a[1][row][j] : &S.b[1][row][j];
    *reinterpret_cast<u32x4*>(hp) = (u32x4){h[0], h[1], h[2], h[3]};
    *reinterpret_cast<u32x4*>(hp + 8) = (u32x4){h[4], h[5], h[6], h[7]};
    *reinterpret_cast<u32x4*>(lp) = (u32x4){l[0], l[1], l[2], l[3]};
    *reinterpret_cast<u32x4*>(lp + 8) = (u32x4){l[4], l[5], l[6], l[7]};
  } else {
    float* p = is_a ? &S.a[row][j] : &S.b[row][j];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      *reinterpret_cast<float4*>(p + 4 * q) = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
  }
}

}  // namespace

// Shifts: xs[b][i] = max_j X_b[i,j] (a wave per row, lanes over j) and ys[b][k] =
// max_j Y_b[j,k] (below); an all -inf row or column gets 0 (its exponentials are then 0,
// never NaN).
__global__ __launch_bounds__(256) void k_logmm_rowmax(LogmmArgs a) {
  const int b = blockIdx.z;
  const int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
  if (row >= a.M) return;   // (uniform per wave)
  const float* x = a.X + ((int64_t)b * a.M + row) * a.K;
  float m = -INFINITY;
  for (int j = threadIdx.x % kWave; j < a.K; j += kWave) m = nan_max(m, x[j]);
  m = wave_max(m);
  if (threadIdx.x % kWave == 0) a.xs[(int64_t)b * a.M + row] = (m == -INFINITY) ? 0.0f : m;
}

// Column maxima: a workgroup of 16 waves per 64 columns (lane -> column), wave w takes
// rows w, w + 16, .. (loads issued 8 at a time); the waves' maxima are merged in LDS.
__global__ __launch_bounds__(1024) void k_logmm_colmax(LogmmArgs a) {
  __shared__ float part[16][kWave];
  const int b = blockIdx.z;
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int64_t col = (int64_t)blockIdx.x * kWave + lane;
  const bool cv = col < a.N;
  const float* y = a.Y + (int64_t)b * a.K * a.N + (cv ? col : 0);
  float m = -INFINITY;
  constexpr int U = 8;
  for (int j0 = w; j0 < a.K; j0 += 16 * U) {
    float v[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int j = j0 + 16 * q;
      v[q] = j < a.K ? y[(int64_t)j * a.N] : -INFINITY;
    }
#pragma unroll
    for (int q = 0; q < U; ++q) m = nan_max(m, v[q]);
  }
  part[w][lane] = m;
  __syncthreads();
  if (w == 0 && cv) {
#pragma unroll
    for (int q = 1; q < 16; ++q) m = nan_max(m, part[q][lane]);
    a.ys[(int64_t)b * a.N + col] = (m == -INFINITY) ? 0.0f : m;
  }
}

// The shifted product on MFMA: a workgroup of 4 waves per 128 x 128 output tile (wave w:
// rows 64 (w / 2), columns 64 (w % 2), as 2 x 2 accumulators of 32 x 32), the reduction
// index staged 32 at a time.  Thread t stages row t / 2 of the X tile and column t % 128
// of the Y tile, 16 consecutive j each, as exponentials of the shifted values (0 past the
// matrix edges); the global loads of the next slice are issued before the current
// slice's MFMAs.  Operand fragments: lane l holds row (column) l % 32 of its block and
// j = 16 s + 8 (l / 32) .. + 7 of step s (both operands in that order); accumulator
// value v of lane l is row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32.
template <int PREC>
__global__ __launch_bounds__(256) void k_logmm_mfma(LogmmArgs a) {
  __shared__ LogmmSmem<PREC> S;
  const int b = blockIdx.z;
  const int i0 = blockIdx.y * kTile, k0 = blockIdx.x * kTile;
  const int M = a.M, K = a.K, N = a.N;
  const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
  const float* X = a.X + (int64_t)b * M * K;
  const float* Y = a.Y + (int64_t)b * K * N;
  // staging roles
  const int ar = t / 2, ajg = (t % 2) * 16;          // X tile row, first j
  const int bc = t % kTile, bjg = (t / kTile) * 16;  // Y tile column, first j
  const int ai = i0 + ar, bk = k0 + bc;
  const bool av = ai < M, bv = bk < N;
  const float xsh = av ? a.xs[(int64_t)b * M + ai] : 0.0f;
  const float ysh = bv ? a.ys[(int64_t)b * N + bk] : 0.0f;
  const float* xrow = X + (int64_t)(av ? ai : 0) * K;
  const float* ycol = Y + (bv ? bk : 0);
  float ra[16], rb[16];   // raw values of the next slice (clamped addresses, masked below)
  auto fetch = [&](int j0) {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int ja = min(j0 + ajg + s, K - 1), jb = min(j0 + bjg + s, K - 1);
      ra[s] = xrow[ja];
      rb[s] = ycol[(int64_t)jb * N];
    }
  };
  f32x16 acc[2][2];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[p][q] = (f32x16){};
  const int wr = 64 * (w / 2), wc = 64 * (w % 2);
  fetch(0);
  for (int j0 = 0; j0 < K; j0 += kKC) {
    float va[16], vb[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      va[s] = (av && j0 + ajg + s < K) ? __expf(ra[s] - xsh) : 0.0f;
      vb[s] = (bv && j0 + bjg + s < K) ? __expf(rb[s] - ysh) : 0.0f;
    }
    __syncthreads();   // (the previous slice's fragment reads are done)
    stage16<PREC>(S, true, ar, ajg, va);
    stage16<PREC>(S, false, bc, bjg, vb);
    __syncthreads();
    if (j0 + kKC < K) fetch(j0 + kKC);   // in flight during the MFMAs below
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
  }
  // Z = log C + x + y
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int k = k0 + wc + 32 * q + lane % 32;
    if (k >= N) continue;
    const float ys = a.ys[(int64_t)b * N + k];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int i = i0 + wr + 32 * p + 8 * (v / 4) + 4 * (lane / 32) + v % 4;
        if (i < M) a.Z[((int64_t)b * M + i) * N + k] = __logf(acc[p][q][v]) + a.xs[(int64_t)b * M + i] + ys;
      }
    }
  }
}

// Exact entries: a thread per column k of one output row (the row of X read by scalar
// loads, Y's row j coalesced across the threads): m = max_j (X_ij + Y_jk), then
// m + log sum_j exp(X_ij + Y_jk - m).  With fix_only, only entries whose shifted product
// fell below kLogmmFloor (log C = Z - x_i - y_k) are recomputed.
template <typename T>
__global__ __launch_bounds__(256) void k_logmm_exact(LogmmArgs a, const T* __restrict__ X,
                                                     const T* __restrict__ Y, T* __restrict__ Z,
                                                     int fix_only) {
  const int b = blockIdx.z, i = blockIdx.y;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= a.N) return;
  const int K = a.K;
  T* zp = Z + ((int64_t)b * a.M + i) * a.N + k;
  if (fix_only) {
    const float r = (float)*zp - a.xs[(int64_t)b * a.M + i] - a.ys[(int64_t)b * a.N + k];
    if (r >= kLogmmFloor) return;
  }
  const T* x = X + ((int64_t)b * a.M + i) * K;
  const T* y = Y + (int64_t)b * K * a.N + k;
  T m = (T)(-INFINITY);
  for (int j = 0; j < K; ++j) m = nan_max(m, x[j] + y[(int64_t)j * a.N]);
  if (m == (T)(-INFINITY) || m != m) {
    *zp = m;
    return;
  }
  T s = (T)0;
  for (int j = 0; j < K; ++j) s += exp(x[j] + y[(int64_t)j * a.N] - m);
  *zp = m + log(s);
}

hipError_t launch_logmm(const LogmmArgs& a, int precision, hipStream_t st) {
  if (precision == TMC_FP64) {
    hipLaunchKernelGGL((k_logmm_exact<double>), dim3((a.N + 255) / 256, a.M, a.B), dim3(256), 0, st, a,
                       a.Xd, a.Yd, a.Zd, 0);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_logmm_rowmax, dim3((a.M + 3) / 4, 1, a.B), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_logmm_colmax, dim3((a.N + kWave - 1) / kWave, 1, a.B), dim3(1024), 0, st, a);
  const dim3 grid((a.N + kTile - 1) / kTile, (a.M + kTile - 1) / kTile, a.B);
  if (precision == TMC_BF16X3)
    hipLaunchKernelGGL((k_logmm_mfma<TMC_BF16X3>), grid, dim3(256), 0, st, a);
  else
    hipLaunchKernelGGL((k_logmm_mfma<TMC_FP32>), grid, dim3(256), 0, st, a);
  hipLaunchKernelGGL((k_logmm_exact<float>), dim3((a.N + 255) / 256, a.M, a.B), dim3(256), 0, st, a,
                     a.X, a.Y, a.Z, 1);
  return hipGetLastError();
}

}  // namespace tmc

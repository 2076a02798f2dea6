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
constexpr int kPadB = 8;            // bf16 row padding of the LDS tiles
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

// Stores 8 consecutive reduction-index values of one row of a tile.
template <int PREC>
__device__ __forceinline__ void stage8(LogmmSmem<PREC>& S, bool is_a, int row, int j, const float (&v)[8]) {
  if constexpr (PREC == TMC_BF16X3) {
    uint32_t h[4], l[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) split_pair(v[2 * p], v[2 * p + 1], h[p], l[p]);
    __bf16* hp = is_a ? &S.a[0][row][j] : &S.b[0][row][j];
    __bf16* lp = is_a ? &S.a[1][row][j] : &S.b[1][row][j];
    *reinterpret_cast<u32x4*>(hp) = (u32x4){h[0], h[1], h[2], h[3]};
    *reinterpret_cast<u32x4*>(lp) = (u32x4){l[0], l[1], l[2], l[3]};
  } else {
    float* p = is_a ? &S.a[row][j] : &S.b[row][j];
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
    *reinterpret_cast<float4*>(p + 4) = make_float4(v[4], v[5], v[6], v[7]);
  }
}

}  // namespace

// Shifts: xs[b][i] = max_j X_b[i,j] (a wave per row, lanes over j) and ys[b][k] =
// max_j Y_b[j,k] (a thread per column); an all -inf row or column gets 0 (its
// exponentials are then 0, never NaN).
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

__global__ __launch_bounds__(256) void k_logmm_colmax(LogmmArgs a) {
  const int b = blockIdx.z;
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col >= a.N) return;
  const float* y = a.Y + (int64_t)b * a.K * a.N + col;
  float m = -INFINITY;
  for (int j = 0; j < a.K; ++j) m = nan_max(m, y[(int64_t)j * a.N]);
  a.ys[(int64_t)b * a.N + col] = (m == -INFINITY) ? 0.0f : m;
}

// The shifted product on MFMA: a workgroup of 4 waves per 64 x 64 output tile (wave w:
// rows 32 (w / 2), columns 32 (w % 2)), the reduction index staged 32 at a time.  Thread
// t stages row t / 4 of the X tile and column t % 64 of the Y tile, 8 consecutive j each,
// as exponentials of the shifted values (0 past the matrix edges).  Operand fragments:
// lane l holds row (column) l % 32 and j = 16 s + 8 (l / 32) .. + 7 of step s (both
// operands in that order); accumulator value v of lane l is row 8 (v / 4) + 4 (l / 32)
// + v % 4, column l % 32.
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
  const int ar = t / 4, ajg = (t % 4) * 8;          // X tile row, first j
  const int bc = t % kTile, bjg = (t / kTile) * 8;  // Y tile column, first j
  const int ai = i0 + ar, bk = k0 + bc;
  const float xsh = ai < M ? a.xs[(int64_t)b * M + ai] : 0.0f;
  const float ysh = bk < N ? a.ys[(int64_t)b * N + bk] : 0.0f;
  const float* xrow = X + (int64_t)(ai < M ? ai : 0) * K;
  const float* ycol = Y + (bk < N ? bk : 0);
  f32x16 acc = {};
  const int wr = 32 * (w / 2), wc = 32 * (w % 2);
  for (int j0 = 0; j0 < K; j0 += kKC) {
    float va[8], vb[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const int ja = j0 + ajg + s, jb = j0 + bjg + s;
      va[s] = (ai < M && ja < K) ? __expf(xrow[ja] - xsh) : 0.0f;
      vb[s] = (bk < N && jb < K) ? __expf(ycol[(int64_t)jb * N] - ysh) : 0.0f;
    }
    __syncthreads();   // (the previous step's fragment reads are done)
    stage8<PREC>(S, true, ar, ajg, va);
    stage8<PREC>(S, false, bc, bjg, vb);
    __syncthreads();
#pragma unroll
    for (int st = 0; st < kKC / 16; ++st) {
      const int jj = 16 * st + 8 * (lane / 32);
      if constexpr (PREC == TMC_BF16X3) {
        const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&S.a[0][wr + lane % 32][jj]);
        const bf16x8 al = *reinterpret_cast<const bf16x8*>(&S.a[1][wr + lane % 32][jj]);
        const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&S.b[0][wc + lane % 32][jj]);
        const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&S.b[1][wc + lane % 32][jj]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
      } else {
        const float4 a0 = *reinterpret_cast<const float4*>(&S.a[wr + lane % 32][jj]);
        const float4 a1 = *reinterpret_cast<const float4*>(&S.a[wr + lane % 32][jj + 4]);
        const float4 b0 = *reinterpret_cast<const float4*>(&S.b[wc + lane % 32][jj]);
        const float4 b1 = *reinterpret_cast<const float4*>(&S.b[wc + lane % 32][jj + 4]);
        const float av[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
        const float bv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
#pragma unroll
        for (int s = 0; s < 8; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s], bv[s], acc, 0, 0, 0);
      }
    }
  }
  // Z = log C + x + y
  const int k = k0 + wc + lane % 32;
  if (k >= N) return;
  const float ys = a.ys[(int64_t)b * N + k];
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int i = i0 + wr + 8 * (v / 4) + 4 * (lane / 32) + v % 4;
    if (i < M) a.Z[((int64_t)b * M + i) * N + k] = __logf(acc[v]) + a.xs[(int64_t)b * M + i] + ys;
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
  hipLaunchKernelGGL(k_logmm_colmax, dim3((a.N + 255) / 256, 1, a.B), dim3(256), 0, st, a);
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

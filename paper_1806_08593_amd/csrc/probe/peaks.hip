// Measured machine peaks of the GPU the library runs on: the rates the rooflines are
// judged against, re-measured instead of taken from the datasheet.  Built as its own
// library (libtmc_peaks.so), not part of the estimator's C ABI.
//
//   tmc_peaks_run(kind, &value) runs one probe on the current device and returns
//   its rate; kinds:
//     0  HBM copy: bytes read + written per second (1 GiB -> 1 GiB, float4 loads/stores)
//     1  HBM read: bytes read per second (1 GiB, float4 loads, one sum per thread)
//     2  MFMA BF16: flop/s of v_mfma_f32_32x32x16_bf16 (4 independent chains per wave)
//     3  MFMA FP32: flop/s of v_mfma_f32_32x32x2f32
//     4  VALU FP32 FMA: flop/s (2 per lane FMA; no packed instructions)
//     5  VALU exp2: lane results per second of v_exp_f32
//     6  VALU FP64 FMA: flop/s
//     7  LDS: bytes per second of ds_read_b128 summed over the CUs
//     8  MFMA FP64: flop/s of v_mfma_f64_16x16x4_f64
// Every probe launches 4 x (number of CUs) workgroups of 512 threads and times 5
// launches after one warm-up with HIP events; the matrix-core probes also run with one
// workgroup per CU (2 waves per SIMD, the occupancy of the fused kernels) and report the
// faster of the two (the clock under matrix-core load depends on the occupancy).
// Returns 0, or a HIP error code.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(512) void k_copy(const float4* __restrict__ a, float4* __restrict__ b,
                                              int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}

__global__ __launch_bounds__(512) void k_read(const float4* __restrict__ a, float* __restrict__ out,
                                              int64_t n) {
  float s = 0.0f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float4 v = a[i];
    s += v.x + v.y + v.z + v.w;
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// 4 chains x 16 MFMAs per iteration
__global__ __launch_bounds__(512) void k_mfma_bf16(float* out, int iters) {
  const int l = threadIdx.x & 63;
  bf16x8 a, b;
  for (int i = 0; i < 8; ++i) {
    a[i] = (__bf16)(1e-3f * (float)(l + i));
    b[i] = (__bf16)(1e-3f * (float)(l - i));
  }
  f32x16 c[4];
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < 16; ++i) c[k][i] = 0.0f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int k = 0; k < 4; ++k) c[k] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c[k], 0, 0, 0);
  }
  float s = 0.0f;
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < 16; ++i) s += c[k][i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(512) void k_mfma_f32(float* out, int iters) {
  const int l = threadIdx.x & 63;
  const float a = 1e-3f * (float)l, b = 2e-3f * (float)l;
  f32x16 c[4];
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < 16; ++i) c[k][i] = 0.0f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int k = 0; k < 4; ++k) c[k] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c[k], 0, 0, 0);
  }
  float s = 0.0f;
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < 16; ++i) s += c[k][i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(512) void k_mfma_f64(float* out, int iters) {
  const int l = threadIdx.x & 63;
  const double a = 1e-3 * (double)l, b = 2e-3 * (double)l;
  f64x4 c[4];
  for (int k = 0; k < 4; ++k) c[k] = (f64x4){0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int k = 0; k < 4; ++k) c[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[k], 0, 0, 0);
  }
  double s = 0.0;
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < 4; ++i) s += c[k][i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

// 8 independent chains x 8 steps per iteration
__global__ __launch_bounds__(512) void k_fma_f32(float* out, int iters, float m) {
  float v[8];
  for (int j = 0; j < 8; ++j) v[j] = 1e-3f * (float)(threadIdx.x + j);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = __builtin_fmaf(v[j], m, 0.25f);
  }
  float s = 0.0f;
  for (int j = 0; j < 8; ++j) s += v[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// y <- 2^(-y) stays in [0.5, 1]; the negation is a source modifier of the exponential
__global__ __launch_bounds__(512) void k_exp2(float* out, int iters) {
  float v[8];
  for (int j = 0; j < 8; ++j) v[j] = 1e-3f * (float)(threadIdx.x + j);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = __builtin_amdgcn_exp2f(-v[j]);
  }
  float s = 0.0f;
  for (int j = 0; j < 8; ++j) s += v[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(512) void k_fma_f64(float* out, int iters, double m) {
  double v[8];
  for (int j = 0; j < 8; ++j) v[j] = 1e-3 * (double)(threadIdx.x + j);
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = __builtin_fma(v[j], m, 0.25);
  }
  double s = 0.0;
  for (int j = 0; j < 8; ++j) s += v[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = (float)s;
}

// every lane reads 16 contiguous bytes, lanes contiguous (no bank conflicts); the
// compiler barrier keeps the reads inside the loop
__global__ __launch_bounds__(512) void k_lds(float* out, int iters) {
  __shared__ __attribute__((aligned(16))) float buf[8192];   // 32 KB
  for (int i = threadIdx.x; i < 8192; i += blockDim.x) buf[i] = (float)i;
  __syncthreads();
  const int base = (threadIdx.x & 63) * 4;   // floats; a wave covers 1 KB
  float s = 0.0f;
  for (int it = 0; it < iters; ++it) {
    asm volatile("" ::: "memory");
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const f32x4v v = *reinterpret_cast<const f32x4v*>(&buf[base + 1024 * k]);   // < 32 KB
      s += v[0] + v[1] + v[2] + v[3];
    }
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

struct Timer {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t init() {
    hipError_t e = hipEventCreate(&e0);
    return e != hipSuccess ? e : hipEventCreate(&e1);
  }
  ~Timer() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

}  // namespace

namespace {

int run_one(int kind, int per_cu, double* value) {
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return (int)e;
  const int grid = per_cu * cus, block = 512, reps = 5;
  Timer tm;
  if ((e = tm.init()) != hipSuccess) return (int)e;
  float* out = nullptr;
  if ((e = hipMalloc(&out, (size_t)grid * block * sizeof(float))) != hipSuccess) return (int)e;
  const int64_t n4 = (int64_t)1 << 26;   // float4 elements: 1 GiB
  float4 *a = nullptr, *b = nullptr;
  double work = 0.0;   // per launch
  auto launch = [&]() {
    switch (kind) {
      case 0: hipLaunchKernelGGL(k_copy, dim3(grid), dim3(block), 0, 0, a, b, n4); break;
      case 1: hipLaunchKernelGGL(k_read, dim3(grid), dim3(block), 0, 0, a, out, n4); break;
      case 2: hipLaunchKernelGGL(k_mfma_bf16, dim3(grid), dim3(block), 0, 0, out, 1024); break;
      case 3: hipLaunchKernelGGL(k_mfma_f32, dim3(grid), dim3(block), 0, 0, out, 1024); break;
      case 4: hipLaunchKernelGGL(k_fma_f32, dim3(grid), dim3(block), 0, 0, out, 2048, 0.999f); break;
      case 5: hipLaunchKernelGGL(k_exp2, dim3(grid), dim3(block), 0, 0, out, 1024); break;
      case 6: hipLaunchKernelGGL(k_fma_f64, dim3(grid), dim3(block), 0, 0, out, 1024, 0.999); break;
      case 7: hipLaunchKernelGGL(k_lds, dim3(grid), dim3(block), 0, 0, out, 4096); break;
      case 8: hipLaunchKernelGGL(k_mfma_f64, dim3(grid), dim3(block), 0, 0, out, 256); break;
    }
  };
  const double waves = (double)grid * block / 64;
  switch (kind) {
    case 0: work = 2.0 * 16.0 * (double)n4; break;
    case 1: work = 16.0 * (double)n4; break;
    case 2: work = waves * 1024 * 16 * 32768.0; break;
    case 3: work = waves * 1024 * 16 * 4096.0; break;
    case 4: work = (double)grid * block * 2048 * 64 * 2.0; break;
    case 5: work = (double)grid * block * 1024 * 64; break;
    case 6: work = (double)grid * block * 1024 * 64 * 2.0; break;
    case 7: work = (double)grid * block * 4096 * 8 * 16.0; break;
    case 8: work = waves * 256 * 16 * 2048.0; break;
    default: (void)hipFree(out); return (int)hipErrorInvalidValue;
  }
  if (kind <= 1) {
    e = hipMalloc(&a, (size_t)n4 * sizeof(float4));
    if (e == hipSuccess && kind == 0) e = hipMalloc(&b, (size_t)n4 * sizeof(float4));
    if (e == hipSuccess) e = hipMemset(a, 0, (size_t)n4 * sizeof(float4));
  }
  float ms = 0.0f;
  if (e == hipSuccess) {
    launch();
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(tm.e0, 0);
  for (int r = 0; r < reps && e == hipSuccess; ++r) {
    launch();
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(tm.e1, 0);
  if (e == hipSuccess) e = hipEventSynchronize(tm.e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, tm.e0, tm.e1);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  (void)hipFree(out);
  if (e != hipSuccess) return (int)e;
  *value = work * reps / (ms * 1e-3);
  return 0;
}

}  // namespace

extern "C" int tmc_peaks_run(int kind, double* value) {
  if (!value || kind < 0 || kind > 8) return (int)hipErrorInvalidValue;
  int rc = run_one(kind, 4, value);
  if (rc == 0 && (kind == 2 || kind == 3 || kind == 8)) {
    double v1 = 0.0;
    rc = run_one(kind, 1, &v1);
    if (rc == 0 && v1 > *value) *value = v1;
  }
  return rc;
}

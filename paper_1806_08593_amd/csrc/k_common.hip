// Kernels shared by both engines: top-of-chain initialisation, the per-chain FP64
// log-normaliser, the start of the backward pass and the deterministic reduction of
// log-std gradients over layers that share one s block.
#include <math.h>

#include "dev_util.h"
#include "tmc_kernels.h"

namespace tmc {

// alpha of the top layer is its unary term (nothing left to sum above it), times the
// exponent of the weights.
template <typename T>
__global__ __launch_bounds__(256) void k_init_top(const ChainDev* __restrict__ chains,
                                                  const LayerDev* __restrict__ layers,
                                                  const T* __restrict__ u,
                                                  double* __restrict__ alpha) {
  const ChainDev c = chains[blockIdx.x];
  const LayerDev& t = layers[c.top];
  const int K = t.K;
  const int64_t uo = t.u_off, ao = t.alpha_off;
  for (int k = threadIdx.x; k < K; k += blockDim.x) alpha[ao + k] = t.kappa * (double)u[uo + k];
}

// log P_TMC = logsumexp_i alpha_0[i] - ln K_0 (eq. (is)), in double.
__global__ __launch_bounds__(256) void k_finalize(const ChainDev* __restrict__ chains,
                                                  const LayerDev* __restrict__ layers,
                                                  const double* __restrict__ alpha,
                                                  double* __restrict__ logp,
                                                  double* __restrict__ logp_ws,
                                                  int* __restrict__ flag) {
  __shared__ double red[kMaxWaves];
  const ChainDev c = chains[blockIdx.x];
  const LayerDev& l0 = layers[c.first];
  const int K = l0.K;
  const double* a = alpha + l0.alpha_off;
  double m = -INFINITY;
  for (int k = threadIdx.x; k < K; k += blockDim.x) m = nan_max(m, a[k]);
  m = block_max(m, red);
  const double sh = isfinite(m) ? m : 0.0;
  double s = 0.0;
  for (int k = threadIdx.x; k < K; k += blockDim.x) s += exp(a[k] - sh);
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    double r;
    if (isnan(m)) r = m;
    else if (m == INFINITY) r = INFINITY;
    else r = sh + log(s) - log((double)K);
    logp[blockIdx.x] = r;
    logp_ws[blockIdx.x] = r;
    if (isnan(r) || r == INFINITY) atomicOr(flag, kFlagNonFinite);
  }
}

// Marginal of layer 0 samples: p_0[i] = exp(alpha_0[i] - ln K_0 - log P); du_0 = dlogp p_0.
// A chain with log P = -inf has no gradient: its marginals are set to 0.
// Also clears dz of the top layer (the top samples enter only through mu and u).
template <typename T>
__global__ __launch_bounds__(256) void k_bwd_init(const ChainDev* __restrict__ chains,
                                                  const LayerDev* __restrict__ layers,
                                                  const double* __restrict__ alpha,
                                                  const double* __restrict__ logp_ws,
                                                  const double* __restrict__ dlogp,
                                                  T* __restrict__ p, T* __restrict__ du,
                                                  T* __restrict__ dz) {
  const int c = blockIdx.x;
  const ChainDev ch = chains[c];
  const LayerDev& l0 = layers[ch.first];
  const double lp = logp_ws[c];
  const double g = dlogp[c] * l0.kappa;   // d/d(kappa u) -> d/du
  const double lk = log((double)l0.K);
  for (int k = threadIdx.x; k < l0.K; k += blockDim.x) {
    double v;
    if (isnan(lp)) v = lp;
    else if (lp == -INFINITY) v = 0.0;
    else v = exp(alpha[l0.alpha_off + k] - lk - lp);
    p[l0.p_off + k] = (T)v;
    if (du) du[l0.u_off + k] = (T)(g * v);
  }
  if (dz) {
    const LayerDev& t = layers[ch.top];
    const int64_t n = (int64_t)t.K * t.D;
    for (int64_t e = threadIdx.x; e < n; e += blockDim.x) dz[t.z_off + e] = (T)0;
  }
}

// ds[s block] = sum of the partial rows that belong to the block, in a fixed order:
// part_off[slot_start[sl] .. slot_start[sl+1]) are element offsets of [D] partial
// rows in dsp.  Workgroup = (slot, 16 d), 256 threads: 16 groups of 16 threads split the
// parts (group g takes parts g, g + 16, ..), then the 16 group sums are combined in LDS
// in two fixed-order steps (4 x 4).  Most slots of a ragged batch hold a few parts, so
// the workgroup is small (many resident at once) and one whose 16 d lie past the slot's
// width ends at once.
template <typename T>
__global__ __launch_bounds__(256) void k_ds_reduce(const int64_t* __restrict__ part_off,
                                                  const int* __restrict__ slot_start,
                                                  const int64_t* __restrict__ slot_soff,
                                                  const int* __restrict__ slot_D,
                                                  const T* __restrict__ dsp, T* __restrict__ ds) {
  __shared__ double red[16][16];
  __shared__ double red2[4][16];
  const int sl = blockIdx.x;
  const int D = slot_D[sl];
  if (blockIdx.y * 16 >= D) return;   // (uniform)
  const int b = slot_start[sl], e = slot_start[sl + 1];
  const int dl = threadIdx.x & 15, g = threadIdx.x >> 4;
  const int d = blockIdx.y * 16 + dl;
  double acc = 0.0;
  if (d < D) {
#pragma unroll 4
    for (int q = b + g; q < e; q += 16) acc += (double)dsp[part_off[q] + d];
  }
  red[g][dl] = acc;
  __syncthreads();
  if (g < 4) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) t += red[4 * g + k][dl];
    red2[g][dl] = t;
  }
  __syncthreads();
  if (g == 0 && d < D) {
    double t = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) t += red2[k][dl];
    ds[slot_soff[sl] + d] = (T)t;
  }
}

// ---- launchers ----
template <typename T>
hipError_t launch_init_top(const ChainDev* chains, int n_chains, const LayerDev* layers,
                           const T* u, double* alpha, hipStream_t st) {
  if (n_chains <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_top<T>, dim3(n_chains), dim3(256), 0, st, chains, layers, u, alpha);
  return hipGetLastError();
}

hipError_t launch_finalize(const ChainDev* chains, int n_chains, const LayerDev* layers,
                           const double* alpha, double* logp, double* logp_ws, int* flag,
                           hipStream_t st) {
  if (n_chains <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3(n_chains), dim3(256), 0, st, chains, layers, alpha, logp,
                     logp_ws, flag);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_bwd_init(const ChainDev* chains, int n_chains, const LayerDev* layers,
                           const double* alpha, const double* logp_ws, const double* dlogp,
                           T* p, T* du, T* dz, hipStream_t st) {
  if (n_chains <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bwd_init<T>, dim3(n_chains), dim3(256), 0, st, chains, layers, alpha,
                     logp_ws, dlogp, p, du, dz);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ds_reduce(const int64_t* part_off, const int* slot_start, const int64_t* slot_soff,
                            const int* slot_D, int n_slots, int max_D, const T* dsp, T* ds,
                            hipStream_t st) {
  if (n_slots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ds_reduce<T>, dim3(n_slots, (max_D + 15) / 16), dim3(256), 0, st, part_off,
                     slot_start, slot_soff, slot_D, dsp, ds);
  return hipGetLastError();
}

#define TMC_INST(T)                                                                            \
  template hipError_t launch_init_top<T>(const ChainDev*, int, const LayerDev*, const T*,      \
                                         double*, hipStream_t);                                \
  template hipError_t launch_bwd_init<T>(const ChainDev*, int, const LayerDev*, const double*, \
                                         const double*, const double*, T*, T*, T*,             \
                                         hipStream_t);                                         \
  template hipError_t launch_ds_reduce<T>(const int64_t*, const int*, const int64_t*,         \
                                          const int*, int, int, const T*, T*, hipStream_t);
TMC_INST(float)
TMC_INST(double)
#undef TMC_INST

}  // namespace tmc

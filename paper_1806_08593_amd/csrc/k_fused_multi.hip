// Fused engine, gradient forward and backward launches that mix the chunk buckets 1..4
// (d <= 64) of one depth step: each workgroup takes the sweep of its own item's bucket.
// A ragged batch (many widths at every depth) then runs one 4-wave launch per step and
// direction instead of one per bucket: the buckets' workgroups share the GPU instead of
// running one launch after another, and the step pays one launch's fixed cost.  Every
// item runs the same sweep as in its bucket's own kernel, so the results are identical.
#include "fused.h"
#include "fused_kernels.h"

namespace tmc {
namespace fused {

template <class A, class B>
constexpr size_t cmax(A a, B b) { return a > b ? (size_t)a : (size_t)b; }

template <int PREC>
constexpr size_t fwd_multi_smem() {
  return cmax(cmax(sizeof(FwdSmem<PREC, 1, true, 1>), sizeof(FwdSmem<PREC, 2, true, 1>)),
              cmax(sizeof(FwdSmem<PREC, 3, true, 1>), sizeof(FwdSmem<PREC, 4, true, 1>)));
}
template <int PREC>
constexpr size_t bwd_multi_smem() {
  return cmax(cmax(sizeof(BwdSmem<PREC, 1, 1>), sizeof(BwdSmem<PREC, 2, 1>)),
              cmax(sizeof(BwdSmem<PREC, 3, 1>), sizeof(BwdSmem<PREC, 4, 1>)));
}

template <int PREC>
__global__ __launch_bounds__(256, 2) void k_fused_fwd_multi(FwdArgs args) {
  __shared__ __align__(16) unsigned char raw[fwd_multi_smem<PREC>()];
  const Item it = args.items[xcd_item(blockIdx.x, gridDim.x)];
  const LayerDev L = args.Ls[it.layer];
  const int tix = (int)threadIdx.x;
  switch ((L.D + 15) / 16) {   // uniform: the item's chunk bucket
    case 1: fwd_item<PREC, 1, true, 1, 4>(tix, *reinterpret_cast<FwdSmem<PREC, 1, true, 1>*>(raw), it, L, args); break;
    case 2: fwd_item<PREC, 2, true, 1, 4>(tix, *reinterpret_cast<FwdSmem<PREC, 2, true, 1>*>(raw), it, L, args); break;
    case 3: fwd_item<PREC, 3, true, 1, 4>(tix, *reinterpret_cast<FwdSmem<PREC, 3, true, 1>*>(raw), it, L, args); break;
    default: fwd_item<PREC, 4, true, 1, 4>(tix, *reinterpret_cast<FwdSmem<PREC, 4, true, 1>*>(raw), it, L, args); break;
  }
}

template <int PREC>
__global__ __launch_bounds__(256, 2) void k_fused_bwd_multi(BwdArgs args) {
  __shared__ __align__(16) unsigned char raw[bwd_multi_smem<PREC>()];
  __shared__ float accD[BwdSmem<PREC, 4, 1>::DT];
  const Item it = args.items[xcd_item(blockIdx.x, gridDim.x)];
  const LayerDev L = args.Ls[it.layer];
  const int tix = (int)threadIdx.x;
  switch ((L.D + 15) / 16) {
    case 1: bwd_item<PREC, 1, 1, 4>(tix, *reinterpret_cast<BwdSmem<PREC, 1, 1>*>(raw), accD, it, L, args); break;
    case 2: bwd_item<PREC, 2, 1, 4>(tix, *reinterpret_cast<BwdSmem<PREC, 2, 1>*>(raw), accD, it, L, args); break;
    case 3: bwd_item<PREC, 3, 1, 4>(tix, *reinterpret_cast<BwdSmem<PREC, 3, 1>*>(raw), accD, it, L, args); break;
    default: bwd_item<PREC, 4, 1, 4>(tix, *reinterpret_cast<BwdSmem<PREC, 4, 1>*>(raw), accD, it, L, args); break;
  }
}

}  // namespace fused

template <int PREC>
hipError_t launch_fused_fwd_multi(const FusedFwdPtrs& a, const Item* items, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  fused::FwdArgs A{a.layers, items, a.z, a.mu, a.s, a.u, a.qcol, a.alpha, a.wmax, a.rl, a.ev};
  hipLaunchKernelGGL((fused::k_fused_fwd_multi<PREC>), dim3(n), dim3(256), 0, st, A);
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_fused_bwd_multi(const FusedBwdPtrs& a, const Item* items, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  fused::BwdArgs A{a.layers, items, a.z,     a.mu, a.s,   a.alpha, a.wmax, a.qcol,
                   a.rl,     a.lam, a.dlogp, a.p,  a.dmu, a.du,    a.dsp, a.ev, a.dz, a.rows};
  hipLaunchKernelGGL((fused::k_fused_bwd_multi<PREC>), dim3(n), dim3(256), 0, st, A);
  return hipGetLastError();
}

template hipError_t launch_fused_fwd_multi<TMC_FP32>(const FusedFwdPtrs&, const Item*, int, hipStream_t);
template hipError_t launch_fused_fwd_multi<TMC_BF16X3>(const FusedFwdPtrs&, const Item*, int, hipStream_t);
template hipError_t launch_fused_bwd_multi<TMC_FP32>(const FusedBwdPtrs&, const Item*, int, hipStream_t);
template hipError_t launch_fused_bwd_multi<TMC_BF16X3>(const FusedBwdPtrs&, const Item*, int, hipStream_t);

}  // namespace tmc

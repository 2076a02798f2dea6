// Fused engine interface: factors recomputed on MFMA inside the message kernels.
#pragma once

#include <vector>

#include "../../include/tmc.h"
#include "tmc_internal.h"

namespace tmc {

constexpr bool kFusedAvailable = false;

struct FusedPlan {
  int prec = 0, flags = 0;
};

struct FusedArgs {
  const void *z, *mu, *s, *u;
  double* logp;
  const double* dlogp;
  void *dz, *dmu, *ds, *du;
  void* ws;
  hipStream_t stream;
  const ChainDev* chains_d;
  const LayerDev* layers_d;
  int n_chains;
  int* flag_d;
  const WsLayout* ws_layout;
  const int* ints_d;
  const int64_t* slot_soff_d;
  int n_slots, slot_layers_off, slot_start_off, slot_D_off;
};

inline tmc_status fused_build(FusedPlan&, int, int, std::vector<LayerDev>&, const std::vector<ChainDev>&,
                              const std::vector<int>&, WsLayout&, std::vector<Item>&) {
  return TMC_ERR_UNSUPPORTED;
}
inline tmc_status fused_upload(FusedPlan&) { return TMC_ERR_UNSUPPORTED; }
inline tmc_status fused_fwd(FusedPlan&, const FusedArgs&) { return TMC_ERR_UNSUPPORTED; }
inline tmc_status fused_bwd(FusedPlan&, const FusedArgs&) { return TMC_ERR_UNSUPPORTED; }
inline void fused_release(FusedPlan&) {}
inline void fused_info(const FusedPlan&, tmc_plan_info*) {}

}  // namespace tmc

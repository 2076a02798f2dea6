// Launchers of the libtmc kernels (host-callable, defined next to their kernels).
#pragma once

#include "tmc_internal.h"

namespace tmc {

// ---- common (k_common.hip) ----
template <typename T>
hipError_t launch_init_top(const ChainDev* chains, int n_chains, const LayerDev* layers,
                           const T* u, double* alpha, hipStream_t st);
hipError_t launch_finalize(const ChainDev* chains, int n_chains, const LayerDev* layers,
                           const double* alpha, double* logp, double* logp_ws, int* flag,
                           hipStream_t st);
template <typename T>
hipError_t launch_bwd_init(const ChainDev* chains, int n_chains, const LayerDev* layers,
                           const double* alpha, const double* logp_ws, const double* dlogp,
                           T* p, T* du, T* dz, hipStream_t st);
template <typename T>
hipError_t launch_ds_reduce(const int64_t* part_off, const int* slot_start, const int64_t* slot_soff,
                            const int* slot_D, int n_slots, int max_D, const T* dsp, T* ds,
                            hipStream_t st);

// ---- plain engine (k_plain.hip) ----
template <typename T>
hipError_t launch_plain_factor(const LayerDev* layers, const Item* items, int n_items,
                               const T* z, const T* mu, const T* s, T* f, bool caller_off,
                               double* anchor, bool parent_scale, hipStream_t st);
template <typename T>
hipError_t launch_plain_lse_fwd(const LayerDev* layers, const Item* items, int n_items,
                                int max_kc, int vec, const T* f, bool caller_off, const T* u,
                                double* alpha, T* rl, double* pairM, const double* anchor,
                                hipStream_t st);
template <typename T>
hipError_t launch_plain_lse_bwd(const LayerDev* layers, const Item* items, int n_items, int vec,
                                const T* f, bool caller_off, const double* alpha,
                                const T* rl, const double* pairM, const double* dlogp, T* p,
                                T* g_out, bool g_caller_off, bool scale_by_dlogp, T* du,
                                hipStream_t st);
template <typename T>
hipError_t launch_plain_gmu(const LayerDev* layers, const Item* items, int n_items,
                            const T* g, const T* z, const T* mu, const T* s, const T* p,
                            const double* dlogp, T* dz, bool parent_scale, hipStream_t st);
template <typename T>
hipError_t launch_plain_gtz(const LayerDev* layers, const Item* items, int n_items,
                            const T* g, const T* z, const T* mu, const T* s, const T* p,
                            const double* dlogp, T* gtz, T* dmu, T* ds_pp, bool parent_scale,
                            hipStream_t st);
template <typename T>
hipError_t launch_pair_dsp(const LayerDev* layers, const int* pair_ids, int n_pairs,
                           const T* z, const T* mu, const T* s, const T* p, const T* gtz,
                           const double* dlogp, T* dsp, hipStream_t st);

// plain tiling constants (host and device agree)
constexpr int kPlainFactorRows = 32, kPlainFactorCols = 64;
constexpr int kPlainFwdRowsPerWave = 4;        // rows a forward wave streams together
constexpr int kPlainFwdWaves = 16;             // waves of a forward workgroup
constexpr int kPlainFwdRowsPerBlock = kPlainFwdWaves * kPlainFwdRowsPerWave;
constexpr int kPlainBwdWaves = 16;             // waves of a backward workgroup (one column strip)
constexpr int kPlainBwdRowsPerStep = 4;        // rows a backward wave loads before using them
constexpr int kPlainBwdColsScalar = 64;        // one column per lane
constexpr int kPlainBwdColsVec = 256;          // four columns per lane (float4 / 2x double2)
constexpr int kPlainGemmRows = 32, kPlainGemmD = 64;

}  // namespace tmc

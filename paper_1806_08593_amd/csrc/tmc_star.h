// Star-model kernels (one global latent shared by N local latents): argument block,
// launch constants and launchers.  Host runtime and k_star.hip share this header.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmc {

constexpr int kStarLanes = 64;     // samples of the lane index per wave
constexpr int kStarWaves = 4;      // waves per workgroup
constexpr int kStarRows = 8;       // rows of the other index a wave evaluates per step
constexpr int kStarMaxD = 32;      // widest local latent
constexpr int kStarTargetGroups = 2048;   // workgroups the forward grid aims for

// Workspace of one plan; every array is indexed by instance first.
//   msg   double [S][N][Kt]        m_i[kt] = logsumexp_k(u_i[k] + f_i[kt, k]) - ln K
//   gsum  double [S][ngrp][Kt]     sum of m_i[kt] over the points of each point group
//   w     double [S][Kt]           uth[kt] + sum_i m_i[kt], then the normalised weight
//   nsh   T      [S][N][Kt]        -(m_i[kt] + ln K - c) log2 e, at most the largest finite
//                                  T (the exponent offset of the gradient passes)
//   wT    T      [S][Kt]           the weights in T
//   lp    double [S]               log P
//   dm    double [S][ngrp][Kt][D]  per group: sum_i sum_k G_i[kt, k] (z_ik - mth[kt])
//   dsp   double [S][N][nkb][D]    per (point, block of 64 local samples):
//                                  sum_{kt, k} G (lam (z - mth)^2 - 1)
// Point groups: P = max(min(N, kStarWaves), min(N, S N ceil(Kt/64) / kStarTargetGroups))
// consecutive points; the waves of a group's workgroup take its points in turn.
template <typename T>
struct StarArgs {
  int S, N, Kt, K, D;
  int P;       // points per group (forward and d mth passes)
  int ngrp;    // ceil(N / P)
  int nkb;     // ceil(K / kStarLanes)
  const T* mth;    // [S][Kt][D]
  const T* s;      // [S][D]
  const T* z;      // [S][N][K][D]
  const T* u;      // [S][N][K]
  const T* uth;    // [S][Kt]
  double* msg;
  double* gsum;
  double* w;
  T* nsh;
  T* wT;
  double* lp;
  double* dm;
  double* dsp;
  int* flag;
  double* logp;          // caller's output (forward)
  const double* dlogp;   // caller's upstream gradient (backward)
  T* dmth;               // caller's gradients (backward; each may be null)
  T* ds;
  T* dz;
  T* du;
  T* duth;
};

// forward: messages and group sums, then the weights' logits, then log P and the weights
template <typename T>
hipError_t launch_star_msg(const StarArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_star_colsum(const StarArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_star_logp(const StarArgs<T>& a, hipStream_t st);
// backward: local gradients (du, dz, ds parts), global parts (d mth), final sums
template <typename T>
hipError_t launch_star_bwd_local(const StarArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_star_bwd_global(const StarArgs<T>& a, hipStream_t st);
template <typename T>
hipError_t launch_star_reduce(const StarArgs<T>& a, hipStream_t st);

}  // namespace tmc

// Log-domain matrix product: argument block and launcher (host runtime and k_logmm.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tmc {

constexpr int kLogmmTile = 128;  // output rows and columns per workgroup of the MFMA pass

struct LogmmArgs {
  int B, M, K, N;
  int Kp;            // K rounded up to a multiple of 32 (the prepared operands' row length)
  const float* X;    // [B][M][K]  (FP32 and BF16X3)
  const float* Y;    // [B][K][N]
  float* Z;          // [B][M][N]
  float* xs;         // workspace [B][M]: row maxima of X
  float* ys;         // workspace [B][N]: column maxima of Y
  void* opa;         // workspace: exp(X - x) as the product's operand, [B][M][Kp] per plane
  void* opb;         // workspace: exp(Y - y) transposed, [B][N][Kp] per plane
  const double* Xd;  // FP64: inputs, output and the shifts (operands in opa, opb)
  const double* Yd;
  double* Zd;
  double* xsd;
  double* ysd;
};

// Enqueues the whole product on st: the shifts, the shifted product on MFMA (FP64,
// FP32 or BF16X3 hi/lo products) and the exact fix-up of underflowed entries.
hipError_t launch_logmm(const LogmmArgs& a, int precision, hipStream_t st);

}  // namespace tmc

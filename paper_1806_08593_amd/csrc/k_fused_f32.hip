// Fused engine kernels, FP32 MFMA instantiation.
#define TMC_FUSED_PREC TMC_FP32
// Built once per d-chunk bucket of fused.h (kNkcBuckets): -DTMC_FUSED_NKC=<bucket>.
#include "k_fused_inst.inc"

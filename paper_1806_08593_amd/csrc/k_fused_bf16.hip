// Fused engine kernels, BF16X3 (split bf16 on MFMA) instantiation.
#define TMC_FUSED_PREC TMC_BF16X3
// Built once per d-chunk bucket of fused.h (kNkcBuckets): -DTMC_FUSED_NKC=<bucket>.
#include "k_fused_inst.inc"

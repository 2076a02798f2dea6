// Fused engine kernels, BF16X3 (split bf16 on MFMA) instantiation.
#define TMC_FUSED_PREC TMC_BF16X3
#include "k_fused_inst.inc"

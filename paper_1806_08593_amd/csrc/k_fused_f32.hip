// Fused engine kernels, FP32 MFMA instantiation.
#define TMC_FUSED_PREC TMC_FP32
#include "k_fused_inst.inc"

// Batched ensemble kernels of stencil d3q27.
#define LBM_TU_STENCIL 2
#include "lbm_batch_instantiate.inc"

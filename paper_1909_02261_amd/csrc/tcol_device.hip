// The device code of libtcol as one translation unit: the separate kernels of the step, the
// MFMA contraction, and the persistent batch launch, which runs the other kernels' block
// bodies inline.
#include "tcol_kernels.hip"
#include "tcol_gemm.hip"
#include "tcol_batch.hip"

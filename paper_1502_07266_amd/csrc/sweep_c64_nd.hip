// Instantiations of the sweep kernel whose line solves use nested dissection: complex64
// sweeps, forward (M^{-1}), writing complex128 (z64) or complex64 output.
#include "sweep_kernel.h"
#include "sweep_variants.h"

const void* sweep_kernel_c64_nd(bool z64) {
  return z64 ? (const void*)sweepk::k_sweep_nd<double2, double2> : (const void*)sweepk::k_sweep_nd<double2, float2>;
}

// Instantiations of the sweep kernel: complex64 sweeps, forward (M^{-1}), writing complex128 output.
#include "sweep_kernel.h"
#include "sweep_variants.h"

const void* sweep_kernel_c64_fwd(bool z64, int k) {
  if (!z64) return sweep_kernel_c64_fwd_z32(k);
  int idx = 0;
#define X(NCA, CWA, DA, NCB, CWB, DB) \
  if (idx++ == k) return (const void*)sweepk::k_sweep<float, double2, double2, NCA, CWA, DA, NCB, CWB, DB, false>;
  HELM_SWEEP_VARIANTS_C64(X)
#undef X
  return nullptr;
}

// Instantiations of the sweep kernel: complex64 sweeps, adjoint (M^{-H}), writing complex64 output (the
// preconditioned directions of the mixed-precision FGMRES).
#include "sweep_kernel.h"
#include "sweep_variants.h"

const void* sweep_kernel_c64_adj_z32(int k) {
  int idx = 0;
#define X(NCA, CWA, DA, NCB, CWB, DB) \
  if (idx++ == k) return (const void*)sweepk::k_sweep<float, double2, float2, NCA, CWA, DA, NCB, CWB, DB, true>;
  HELM_SWEEP_VARIANTS_C64(X)
#undef X
  return nullptr;
}

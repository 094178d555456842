// Instantiations of the sweep kernel: complex128 sweeps, forward (M^{-1}) and adjoint (M^{-H}).
#include "sweep_kernel.h"
#include "sweep_variants.h"

const void* sweep_kernel_c128(bool adj, int k) {
  int idx = 0;
#define X(NCA, CWA, DA, NCB, CWB, DB)                                                             \
  if (idx++ == k)                                                                                \
    return adj ? (const void*)sweepk::k_sweep<double, double2, double2, NCA, CWA, DA, NCB, CWB, DB, true> \
               : (const void*)sweepk::k_sweep<double, double2, double2, NCA, CWA, DA, NCB, CWB, DB, false>;
  HELM_SWEEP_VARIANTS_C128(X)
#undef X
  return nullptr;
}

// The instantiated launch shapes of the sweep kernel (sweep_kernel.h): each variant is
// (NCA, CWA, DA, NCB, CWB, DB): lines with B <= NCA * CWA take shape A (NCA lanes per block
// row, CWA columns per lane, a ring of DA factor blocks), larger ones shape B.  The ring
// depths are sized so that the ring fits the register budget of the variant's widest shape
// (its thread count fixes the waves per SIMD).  Listed in order of preference: the host takes
// the first variant whose shapes cover the blocks, unless the autotuner chose another.
#pragma once

#include "common.h"

#define HELM_SWEEP_VARIANTS_C64(X)                                                          \
  X(8, 3, 16, 8, 3, 16) X(8, 4, 16, 8, 4, 16) X(8, 5, 8, 8, 5, 8) X(8, 7, 4, 8, 7, 4)        \
  X(8, 8, 4, 8, 8, 4) X(8, 11, 4, 8, 11, 4) X(8, 16, 2, 8, 16, 2)                            \
  X(8, 3, 16, 8, 5, 8) X(8, 4, 8, 8, 6, 8) X(8, 4, 8, 8, 11, 4) X(8, 7, 4, 8, 11, 4)         \
  X(8, 7, 2, 8, 11, 2) X(8, 7, 8, 8, 11, 2) X(8, 8, 4, 8, 11, 4) X(8, 7, 4, 8, 12, 4)        \
  X(8, 7, 4, 8, 16, 2) X(8, 11, 4, 8, 16, 2)

#define HELM_SWEEP_VARIANTS_C128(X)                                                         \
  X(8, 3, 12, 8, 3, 12) X(8, 4, 10, 8, 4, 10) X(8, 5, 4, 8, 5, 4) X(8, 7, 4, 8, 7, 4)        \
  X(8, 8, 2, 8, 8, 2) X(8, 11, 2, 8, 11, 2) X(8, 3, 12, 8, 5, 4) X(8, 4, 4, 8, 6, 4)         \
  X(8, 4, 4, 8, 11, 2) X(8, 7, 2, 8, 11, 2) X(8, 7, 2, 8, 12, 2)

struct SweepVariant {
  int nca, cwa, da, ncb, cwb, db;
  int capA() const { return nca * cwa; }
  int capB() const { return ncb * cwb; }
};

// the variants of one precision, in preference order
const std::vector<SweepVariant>& sweep_variants(bool c64);
// the kernel of variant k (sweep_c64_{fwd,adj}{,_z32}.hip, sweep_c128.hip): complex64
// sweeps writing complex128 (z64) or complex64 output, or complex128 sweeps; forward or adjoint
const void* sweep_kernel(bool c64, bool z64, bool adj, int k);
// the nested-dissection sweep kernel (complex64 forward sweeps; sweep_c64_nd.hip)
const void* sweep_kernel_c64_nd(bool z64);
const void* sweep_kernel_c64_fwd(bool z64, int k);
const void* sweep_kernel_c64_adj(bool z64, int k);
const void* sweep_kernel_c64_fwd_z32(int k);
const void* sweep_kernel_c64_adj_z32(int k);
const void* sweep_kernel_c128(bool adj, int k);

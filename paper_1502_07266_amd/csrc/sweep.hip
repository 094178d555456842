// Application of the recursive sweeping preconditioner, z = M^{-1} r (Algorithm 6 with
// Algorithm 4 inside, each line block solved exactly by its block LDU), and its adjoint.
//
// One workgroup runs the whole sweep for one right-hand side; a launch covers a batch of
// right-hand sides ("persistent": the workgroup loops over every slab and line itself, so the
// sweep's long chain of dependent block steps never returns to the host).  Workgroups of
// different right-hand sides are independent and read the same factor stream.
//
// Data flow for one right-hand side:
//   outer forward  g = 0..G-1 : slab input  f on the group's layers, minus A[k0,k0-1] u[k0-1]
//   outer backward g = G-2..0 : slab input  A[k1,k1+1] u[k1+1] on the group's last layer
//     inner forward  l = 0..G-1 : line input  slab input on the group's rows, minus
//                                              Ht[j0,j0-1] v[j0-1]   (all window layers)
//     inner backward l = G-2..0 : line input  Ht[j1,j1+1] v[j1+1]
//       line solve: y_i = T_i (q_i - l_i y_{i-1}),  x_i = y_i - u_i T_i x_{i+1}
// where v is the slab iterate (n x n x window layers, in global scratch), the line vector
// (n blocks of B = Wy*Wz) lives in LDS, and the T_i stream from HBM.  The adjoint uses the
// couplings of A^H and T_i^H (see the oracle's derivation: the same pass order).
//
// Block step mapping: thread t owns output row t / NC of the B x B block and a chunk of
// ceil(B/NC) columns; the NC partial sums of a row sit in adjacent lanes of one wavefront
// and are combined with cross-lane exchanges.  One barrier per block step.
#include "common.h"

namespace {

constexpr int kBMax = 64;

struct SweepArgs {
  int n, G, maxW, maxB;
  long long N, in_stride, out_stride;
  const GroupInfo* groups;
  const long long* line_off;
  const double2* coef;   // [4][n+2]
  const void* factors;
  const void* in;
  void* out;
  const int* rhs_idx;
  void* scratch;
};

template <int NC, typename C> __device__ inline C reduce_lanes(C a) {
#pragma unroll
  for (int off = NC / 2; off > 0; off >>= 1) {
    a.x += __shfl_xor(a.x, off);
    a.y += __shfl_xor(a.y, off);
  }
  return a;
}

// Exact solve of one line problem through its block LDU factors.  On entry ybuf[i*B + q]
// holds the right-hand side block i; on exit it holds the solution.  `emit(i, q, x)` is
// called once per solution entry (by the thread owning row q) as soon as x is final.
// cf[m], cb[m] are the x1 couplings of row m (m = i+1) towards m-1 and m+1.
template <typename R, int NC, bool ADJ, typename Emit>
__device__ inline void line_solve(const typename cx<R>::type* __restrict__ T, const int B,
                                  const int n, typename cx<R>::type* ybuf,
                                  const typename cx<R>::type* cf, const typename cx<R>::type* cb,
                                  Emit emit) {
  using C = typename cx<R>::type;
  constexpr int CWMAX = kBMax / NC;
  const int tid = threadIdx.x;
  const int row = tid / NC, lc = tid - row * NC;
  const int CW = (B + NC - 1) / NC;
  const int c0 = lc * CW;
  const bool act = row < B;
  const long long BB = (long long)B * B;
  C tcur[CWMAX], tnxt[CWMAX], qcur[CWMAX], qnxt[CWMAX];
  const C zero = mk((R)0, (R)0);

  // ---- forward: y_i = T_i (q_i - cf_i y_{i-1}) ----
#define HELM_LOAD_T(blk, dst)                                                        \
  _Pragma("unroll") for (int cc = 0; cc < CWMAX; ++cc) {                             \
    const int col = c0 + cc;                                                         \
    dst[cc] = (act && cc < CW && col < B) ? (ADJ ? (blk)[col * B + row] : (blk)[row * B + col]) \
                                          : zero;                                    \
  }
#define HELM_LOAD_Q(i, dst)                                                          \
  _Pragma("unroll") for (int cc = 0; cc < CWMAX; ++cc) {                             \
    const int col = c0 + cc;                                                         \
    dst[cc] = (cc < CW && col < B) ? ybuf[(i) * B + col] : zero;                     \
  }
  HELM_LOAD_T(T, tcur);
  HELM_LOAD_Q(0, qcur);
  for (int i = 0; i < n; ++i) {
    if (i + 1 < n) {
      HELM_LOAD_T(T + (i + 1) * BB, tnxt);
      HELM_LOAD_Q(i + 1, qnxt);
    }
    const C cfi = cf[i + 1];
    C acc = zero;
#pragma unroll
    for (int cc = 0; cc < CWMAX; ++cc) {
      const int col = c0 + cc;
      if (cc < CW && col < B) {
        C z = qcur[cc];
        if (i > 0) z = csub(z, cmul(cfi, ybuf[(i - 1) * B + col]));
        acc = ADJ ? cfma_conj(acc, tcur[cc], z) : cfma(acc, tcur[cc], z);
      }
    }
    acc = reduce_lanes<NC>(acc);
    if (lc == 0 && act) ybuf[i * B + row] = acc;
    __syncthreads();
#pragma unroll
    for (int cc = 0; cc < CWMAX; ++cc) {
      tcur[cc] = tnxt[cc];
      qcur[cc] = qnxt[cc];
    }
  }
  // ---- backward: x_{n-1} = y_{n-1};  x_i = y_i - cb_i T_i x_{i+1} ----
  if (lc == 0 && act) emit(n - 1, row, ybuf[(n - 1) * B + row]);
  if (n >= 2) { HELM_LOAD_T(T + (n - 2) * BB, tcur); }
  for (int i = n - 2; i >= 0; --i) {
    if (i > 0) { HELM_LOAD_T(T + (i - 1) * BB, tnxt); }
    const C cbi = cb[i + 1];
    C acc = zero;
#pragma unroll
    for (int cc = 0; cc < CWMAX; ++cc) {
      const int col = c0 + cc;
      if (cc < CW && col < B) {
        const C xv = ybuf[(i + 1) * B + col];
        acc = ADJ ? cfma_conj(acc, tcur[cc], xv) : cfma(acc, tcur[cc], xv);
      }
    }
    acc = reduce_lanes<NC>(acc);
    if (lc == 0 && act) {
      const C x = csub(ybuf[i * B + row], cmul(cbi, acc));
      ybuf[i * B + row] = x;
      emit(i, row, x);
    }
    __syncthreads();
#pragma unroll
    for (int cc = 0; cc < CWMAX; ++cc) tcur[cc] = tnxt[cc];
  }
#undef HELM_LOAD_T
#undef HELM_LOAD_Q
}

template <typename R, typename TI, typename TO, int NC, bool ADJ>
__global__ void __launch_bounds__(kBMax * NC) k_sweep(SweepArgs a) {
  using C = typename cx<R>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = a.n, G = a.G;
  C* ybuf = reinterpret_cast<C*>(smem_raw);
  C* cf = ybuf + (size_t)n * a.maxB;  // A'[m, m-1], m = 0..n+1
  C* cb = cf + (n + 2);               // A'[m, m+1]
  const int tid = threadIdx.x, NT = blockDim.x;
  const int q = a.rhs_idx ? a.rhs_idx[blockIdx.x] : (int)blockIdx.x;
  const TI* __restrict__ f = reinterpret_cast<const TI*>(a.in) + (long long)q * a.in_stride;
  TO* u = reinterpret_cast<TO*>(a.out) + (long long)q * a.out_stride;
  C* v = reinterpret_cast<C*>(a.scratch) + (long long)blockIdx.x * n * n * a.maxW;
  const C zero = mk((R)0, (R)0);
  for (int m = tid; m < n + 2; m += NT) {
    cf[m] = cvt<C>(a.coef[(ADJ ? 2 : 0) * (n + 2) + m]);
    cb[m] = cvt<C>(a.coef[(ADJ ? 3 : 1) * (n + 2) + m]);
  }
  __syncthreads();
  auto gidx = [&](int i, int j, int k) -> long long {  // i 0-based, j, k 1-based
    return ((long long)(k - 1) * n + (j - 1)) * n + i;
  };

  for (int pass = 0; pass < 2; ++pass) {
    const bool ofwd = pass == 0;
    for (int gi = 0; gi < (ofwd ? G : G - 1); ++gi) {
      const int g = ofwd ? gi : G - 2 - gi;
      const GroupInfo gz = a.groups[g];
      const int Wz = gz.W, k0 = gz.first, k1 = gz.last, zw0 = gz.w0;
      for (int lp = 0; lp < 2 * G - 1; ++lp) {
        const bool ifwd = lp < G;
        const int l = ifwd ? lp : 2 * G - 2 - lp;
        const GroupInfo gy = a.groups[l];
        const int Wy = gy.W, B = Wy * Wz, j0 = gy.first, j1 = gy.last, yw0 = gy.w0;
        // ---- line input ----
        for (int e = tid; e < n * B; e += NT) {
          const int qq = e / n, i = e - qq * n;
          const int jj = qq / Wz, kk = qq - jj * Wz;
          const int j = yw0 + jj, k = zw0 + kk;
          C val = zero;
          if (ifwd) {
            if (j >= j0) {
              if (ofwd) {
                if (k >= k0) {
                  val = cvt<C>(f[gidx(i, j, k)]);
                  if (g > 0 && k == k0) val = csub(val, cmul(cf[k0], cvt<C>(u[gidx(i, j, k0 - 1)])));
                }
              } else if (k == k1) {
                val = cmul(cb[k1], cvt<C>(u[gidx(i, j, k1 + 1)]));
              }
              if (l > 0 && j == j0) val = csub(val, cmul(cf[j0], v[((long long)kk * n + (j0 - 2)) * n + i]));
            }
          } else if (j == j1) {
            val = cmul(cb[j1], v[((long long)kk * n + j1) * n + i]);
          }
          ybuf[i * B + qq] = val;
        }
        __syncthreads();
        const C* T = reinterpret_cast<const C*>(a.factors) + a.line_off[(size_t)g * G + l];
        line_solve<R, NC, ADJ>(T, B, n, ybuf, cf, cb, [&](int i, int qq, C x) {
          const int jj = qq / Wz, kk = qq - jj * Wz;
          const int j = yw0 + jj;
          if (j >= j0) {
            C* p = v + ((long long)kk * n + (j - 1)) * n + i;
            *p = ifwd ? x : csub(*p, x);
          }
        });
      }
      // ---- slab output on the group's layers ----
      const int nph = k1 - k0 + 1;
      for (int e = tid; e < n * n * nph; e += NT) {
        const int i = e % n, jm = (e / n) % n, kp = e / (n * n);
        const int kk = Wz - nph + kp;
        const C val = v[((long long)kk * n + jm) * n + i];
        const long long id = gidx(i, jm + 1, k0 + kp);
        u[id] = ofwd ? cvt<TO>(val) : cvt<TO>(csub(cvt<C>(u[id]), val));
      }
      __syncthreads();
    }
  }
}

// Exact solve of a single line problem on its own grid (for testing the building block).
template <typename R, int NC, bool ADJ>
__global__ void __launch_bounds__(kBMax * NC) k_line_solve(SweepArgs a, int g, int l) {
  using C = typename cx<R>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = a.n, G = a.G;
  C* ybuf = reinterpret_cast<C*>(smem_raw);
  C* cf = ybuf + (size_t)n * a.maxB;
  C* cb = cf + (n + 2);
  const int tid = threadIdx.x, NT = blockDim.x;
  for (int m = tid; m < n + 2; m += NT) {
    cf[m] = cvt<C>(a.coef[(ADJ ? 2 : 0) * (n + 2) + m]);
    cb[m] = cvt<C>(a.coef[(ADJ ? 3 : 1) * (n + 2) + m]);
  }
  const int Wz = a.groups[g].W, Wy = a.groups[l].W, B = Wy * Wz;
  const double2* r = reinterpret_cast<const double2*>(a.in) + (long long)blockIdx.x * n * B;
  double2* x = reinterpret_cast<double2*>(a.out) + (long long)blockIdx.x * n * B;
  for (int e = tid; e < n * B; e += NT) {   // line grid: x1 fastest, then window row, then layer
    const int i = e % n, jj = (e / n) % Wy, kk = e / (n * Wy);
    ybuf[i * B + jj * Wz + kk] = cvt<C>(r[e]);
  }
  __syncthreads();
  const C* T = reinterpret_cast<const C*>(a.factors) + a.line_off[(size_t)g * G + l];
  line_solve<R, NC, ADJ>(T, B, n, ybuf, cf, cb, [&](int i, int qq, C val) {
    const int jj = qq / Wz, kk = qq - jj * Wz;
    x[i + (long long)n * (jj + (long long)Wy * kk)] = cvt<double2>(val);
  });
}

// threads per workgroup: NC lanes for each of the maxB block rows, whole wavefronts
inline int block_threads(int maxB, int nc) { return ((maxB * nc + 63) / 64) * 64; }

template <typename K>
hipError_t launch_k(K kern, int grid, int threads, size_t sm, hipStream_t s, SweepArgs a) {
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)sm);
  if (e != hipSuccess) return e;
  kern<<<grid, threads, sm, s>>>(a);
  return hipGetLastError();
}

template <typename R, typename TI, typename TO, bool ADJ>
hipError_t dispatch_nc(int nc, int maxB, int grid, size_t sm, hipStream_t s, SweepArgs a) {
  const int t = block_threads(maxB, nc);
  switch (nc) {
    case 4: return launch_k(k_sweep<R, TI, TO, 4, ADJ>, grid, t, sm, s, a);
    case 16: return launch_k(k_sweep<R, TI, TO, 16, ADJ>, grid, t, sm, s, a);
    default: return launch_k(k_sweep<R, TI, TO, 8, ADJ>, grid, t, sm, s, a);
  }
}

int auto_lanes(const helm_handle* h) {
  if (h->lanes_override) return h->lanes_override;
  return h->prec == HELM_C64 ? 8 : 8;
}

SweepArgs base_args(helm_handle* h) {
  SweepArgs a;
  a.n = h->n;
  a.G = h->plan.G;
  a.maxW = h->plan.maxW;
  a.maxB = h->plan.maxB;
  a.N = (long long)h->n * h->n * h->n;
  a.in_stride = a.out_stride = a.N;
  a.groups = h->d_groups;
  a.line_off = h->d_line_off;
  a.coef = h->coef;
  a.factors = h->factors;
  a.in = nullptr;
  a.out = nullptr;
  a.rhs_idx = nullptr;
  a.scratch = nullptr;
  return a;
}

}  // namespace

hipError_t launch_apply(helm_handle* h, const void* r, bool r64, long long r_stride, void* z,
                        bool z64, long long z_stride, int R, const int* rhs_idx, bool adjoint,
                        hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const int n = h->n;
  const bool c64 = h->prec == HELM_C64;
  const size_t csz = c64 ? sizeof(float2) : sizeof(double2);
  const size_t need = (size_t)R * n * n * h->plan.maxW * csz;
  if (need > h->slab_scratch_bytes) {
    if (h->slab_scratch) {
      hipError_t e = hipFree(h->slab_scratch);
      if (e != hipSuccess) return e;
      h->slab_scratch = nullptr;
      h->slab_scratch_bytes = 0;
    }
    hipError_t e = hipMalloc(&h->slab_scratch, need);
    if (e != hipSuccess) return e;
    h->slab_scratch_bytes = need;
  }
  SweepArgs a = base_args(h);
  a.in = r;
  a.out = z;
  a.in_stride = r_stride;
  a.out_stride = z_stride;
  a.rhs_idx = rhs_idx;
  a.scratch = h->slab_scratch;
  const size_t sm = ((size_t)n * h->plan.maxB + 2 * (n + 2)) * csz;
  const int nc = auto_lanes(h);
  const int mb = h->plan.maxB;
  if (!r64) return hipErrorInvalidValue;  // inputs are always complex128
  if (!c64) {
    if (!z64) return hipErrorInvalidValue;
    return adjoint ? dispatch_nc<double, double2, double2, true>(nc, mb, R, sm, s, a)
                   : dispatch_nc<double, double2, double2, false>(nc, mb, R, sm, s, a);
  }
  if (z64)
    return adjoint ? dispatch_nc<float, double2, double2, true>(nc, mb, R, sm, s, a)
                   : dispatch_nc<float, double2, double2, false>(nc, mb, R, sm, s, a);
  return adjoint ? dispatch_nc<float, double2, float2, true>(nc, mb, R, sm, s, a)
                 : dispatch_nc<float, double2, float2, false>(nc, mb, R, sm, s, a);
}

hipError_t launch_line_solve(helm_handle* h, int zg, int yg, const double2* r, double2* x, int R,
                             bool adjoint, hipStream_t s) {
  const int n = h->n;
  const bool c64 = h->prec == HELM_C64;
  const size_t csz = c64 ? sizeof(float2) : sizeof(double2);
  SweepArgs a = base_args(h);
  a.in = r;
  a.out = x;
  const size_t sm = ((size_t)n * h->plan.maxB + 2 * (n + 2)) * csz;
  const int nc = auto_lanes(h);
  auto go = [&](auto kern) -> hipError_t {
    hipError_t e = hipFuncSetAttribute((const void*)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    kern<<<R, block_threads(h->plan.maxB, nc), sm, s>>>(a, zg, yg);
    return hipGetLastError();
  };
  if (c64) {
    if (nc == 4) return adjoint ? go(k_line_solve<float, 4, true>) : go(k_line_solve<float, 4, false>);
    if (nc == 16) return adjoint ? go(k_line_solve<float, 16, true>) : go(k_line_solve<float, 16, false>);
    return adjoint ? go(k_line_solve<float, 8, true>) : go(k_line_solve<float, 8, false>);
  }
  if (nc == 4) return adjoint ? go(k_line_solve<double, 4, true>) : go(k_line_solve<double, 4, false>);
  if (nc == 16) return adjoint ? go(k_line_solve<double, 16, true>) : go(k_line_solve<double, 16, false>);
  return adjoint ? go(k_line_solve<double, 8, true>) : go(k_line_solve<double, 8, false>);
}

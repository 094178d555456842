// The 7-point PML operator of eq. (3), y = A u or y = A^H u, in FP64, batched over
// right-hand sides, and the adjoint-state velocity gradient.
//
// Row of node p: sum_d [ A[m,m-1] u_{p-e_d} + A[m,m+1] u_{p+e_d} ] + (kappa_p + sum_d diag_d) u_p
// with A[m,m-1] = s_m s_{m-1/2}/h^2, A[m,m+1] = s_m s_{m+1/2}/h^2, diag_d = -s_m (s_{m+1/2} +
// s_{m-1/2})/h^2 and m the node's index along axis d; neighbours outside the grid are zero.
// The adjoint row uses A^H[m, m-+1] = conj(A[m-+1, m]) and the conjugated diagonal.
// Each thread produces one output value: 40 bytes of algorithmic traffic per point
// (u 16 B, kappa 8 B, y 16 B); the neighbour reloads hit the caches.
#include "common.h"

namespace {

template <typename TU, bool ADJ>
__global__ void __launch_bounds__(256) k_matvec(const TU* __restrict__ u, long long us,
                                                const double2* __restrict__ f,
                                                double2* __restrict__ y, long long ys,
                                                const double* __restrict__ kappa,
                                                const double2* __restrict__ coef,
                                                const double2* __restrict__ diag, int n,
                                                const int* __restrict__ idx, int mode) {
  const long long N = (long long)n * n * n;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  const int q = idx ? idx[blockIdx.y] : (int)blockIdx.y;
  const TU* uq = u + (long long)q * us;
  const int i = (int)(e % n), j = (int)((e / n) % n), k = (int)(e / ((long long)n * n));
  const int L = n + 2;
  const double2* cf = coef + (ADJ ? 2 : 0) * L;
  const double2* cb = coef + (ADJ ? 3 : 1) * L;
  double2 d = cadd(cadd(diag[i + 1], diag[j + 1]), diag[k + 1]);
  d.x += kappa[e];
  if (ADJ) d = cconj(d);
  double2 acc = cmul(d, cvt<double2>(uq[e]));
  const long long sj = n, sk = (long long)n * n;
  if (i > 0) acc = cfma(acc, cf[i + 1], cvt<double2>(uq[e - 1]));
  if (i < n - 1) acc = cfma(acc, cb[i + 1], cvt<double2>(uq[e + 1]));
  if (j > 0) acc = cfma(acc, cf[j + 1], cvt<double2>(uq[e - sj]));
  if (j < n - 1) acc = cfma(acc, cb[j + 1], cvt<double2>(uq[e + sj]));
  if (k > 0) acc = cfma(acc, cf[k + 1], cvt<double2>(uq[e - sk]));
  if (k < n - 1) acc = cfma(acc, cb[k + 1], cvt<double2>(uq[e + sk]));
  double2* yq = y + (long long)q * ys;
  if (mode == 1) acc = csub(f[(long long)q * ys + e], acc);
  yq[e] = acc;
}

// grad_p = (2 omega^2 / c_p^3) Re sum_s conj(lam_s,p) u_s,p, with 2 omega^2/c^3 = 2 kappa^{3/2}/omega
__global__ void __launch_bounds__(256) k_grad(const double2* __restrict__ u,
                                              const double2* __restrict__ lam,
                                              const double* __restrict__ kappa, int R,
                                              long long N, double omega, double* __restrict__ g) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double s = 0.0;
  for (int r = 0; r < R; ++r) {
    const double2 a = lam[(long long)r * N + e], b = u[(long long)r * N + e];
    s += a.x * b.x + a.y * b.y;
  }
  const double kap = kappa[e];
  g[e] = 2.0 * kap * sqrt(kap) / omega * s;
}

// per-block partial sums of |P u - d|^2 and the adjoint source g = P^T (P u - d)
__global__ void __launch_bounds__(256) k_misfit(const double2* __restrict__ u,
                                                const double2* __restrict__ d, int n, int plane_k,
                                                double2* __restrict__ g, double* __restrict__ part) {
  __shared__ double red[4];
  const long long N = (long long)n * n * n;
  const int s = blockIdx.y;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long p0 = (long long)(plane_k - 1) * n * n;
  double acc = 0.0;
  if (e < N) {
    double2 r = make_double2(0.0, 0.0);
    if (e >= p0 && e < p0 + (long long)n * n) {
      r = csub(u[(long long)s * N + e], d[(long long)s * n * n + (e - p0)]);
      acc = cabs2(r);
    }
    if (g) g[(long long)s * N + e] = r;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    part[(long long)s * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_sum(const double* __restrict__ part, long long count, double scale,
                      double* __restrict__ out) {
  __shared__ double red[4];
  double acc = 0.0;
  for (long long i = threadIdx.x; i < count; i += blockDim.x) acc += part[i];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *out = scale * (red[0] + red[1] + red[2] + red[3]);
}

}  // namespace

hipError_t launch_misfit(helm_handle* h, const double2* u, const double2* d, int R, int plane_k,
                         double* J_dev, double2* g, hipStream_t s) {
  const int n = h->n;
  const long long N = (long long)n * n * n;
  const unsigned nb = (unsigned)((N + 255) / 256);
  double* part = nullptr;
  hipError_t e = pool_alloc((void**)&part, (size_t)nb * R * sizeof(double), s);
  if (e != hipSuccess) return e;
  k_misfit<<<dim3(nb, (unsigned)R), 256, 0, s>>>(u, d, n, plane_k, g, part);
  k_sum<<<1, 256, 0, s>>>(part, (long long)nb * R, 0.5, J_dev);
  e = hipGetLastError();
  pool_free(part, s);
  return e;
}

hipError_t launch_matvec(helm_handle* h, const void* u, bool u64, const double2* f, double2* y,
                         int R, const int* rhs_idx, long long u_stride, long long y_stride,
                         bool adjoint, int mode, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const int n = h->n;
  const long long N = (long long)n * n * n;
  dim3 grid((unsigned)((N + 255) / 256), (unsigned)R);
  hipEvent_t ev = h->t_matvec.begin(s);
  if (u64) {
    if (adjoint)
      k_matvec<double2, true><<<grid, 256, 0, s>>>((const double2*)u, u_stride, f, y, y_stride,
                                                   h->kappa, h->coef, h->diag, n, rhs_idx, mode);
    else
      k_matvec<double2, false><<<grid, 256, 0, s>>>((const double2*)u, u_stride, f, y, y_stride,
                                                    h->kappa, h->coef, h->diag, n, rhs_idx, mode);
  } else {
    if (adjoint)
      k_matvec<float2, true><<<grid, 256, 0, s>>>((const float2*)u, u_stride, f, y, y_stride,
                                                  h->kappa, h->coef, h->diag, n, rhs_idx, mode);
    else
      k_matvec<float2, false><<<grid, 256, 0, s>>>((const float2*)u, u_stride, f, y, y_stride,
                                                   h->kappa, h->coef, h->diag, n, rhs_idx, mode);
  }
  hipError_t e = hipGetLastError();
  h->t_matvec.end(ev, s, R);
  return e;
}

hipError_t launch_grad(helm_handle* h, const double2* u, const double2* lam, int R, double* grad,
                       hipStream_t s) {
  const long long N = (long long)h->n * h->n * h->n;
  k_grad<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(u, lam, h->kappa, R, N, h->omega, grad);
  return hipGetLastError();
}

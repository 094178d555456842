// Coefficients of eq. (3): kappa = omega^2/c^2 at the nodes and the O(n) stretching tables.
//
// Positions along an axis are integer half-steps t (position t h / 2): node m is t = 2m and
// half-node m - 1/2 is t = 2m - 1.  The cube, its PMLs and the sweep partitions are the same
// on all three axes, so one table serves x1, x2 and x3.
#include "common.h"

namespace {

// sigma of Sec. 2: (C/eta) ((xi - eta)/eta)^2 on [0, eta], zero beyond
__device__ inline double sigma(double xi, double eta, double C) {
  if (xi < 0.0 || xi > eta) return 0.0;
  double q = (xi - eta) / eta;
  return (C / eta) * q * q;
}

// s = 1 / (1 + i sigma / omega)
__device__ inline double2 stretch(double sig, double omega) {
  double a = sig / omega;
  double den = 1.0 + a * a;
  return make_double2(1.0 / den, -a / den);
}

__global__ void k_kappa(const double* __restrict__ c, double* __restrict__ kappa, long long N,
                        double omega2, int* __restrict__ bad) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double v = c[e];
  if (!(v > 0.0) || !isfinite(v)) atomicOr(bad, 1);
  kappa[e] = omega2 / (v * v);
}

__global__ void k_tables(int n, int b, int p, double C, double C_mv, double omega, double2* __restrict__ sbd,
                         double2* __restrict__ smv, double2* __restrict__ coef,
                         double2* __restrict__ diag) {
  const double h = 1.0 / (n + 1);
  const double eta = b * h, eta_mv = (p + 1) * h;
  const int T = 2 * (n + 1) + 1;
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < T) {  // boundary profile, mirrored on both faces (PML on all six faces)
    double x_lo = 0.5 * e * h, x_hi = 0.5 * (2 * (n + 1) - e) * h;
    sbd[e] = stretch(sigma(x_lo, eta, C) + sigma(x_hi, eta, C), omega);
  }
  if (e < 2 * p + 2) {  // moving profile, measured from its own Dirichlet plane
    smv[e] = stretch(sigma(0.5 * e * h, eta_mv, C_mv), omega);
  }
}

__global__ void k_coupling(int n, const double2* __restrict__ sbd, double2* __restrict__ coef,
                           double2* __restrict__ diag) {
  const double h = 1.0 / (n + 1);
  const double ih2 = 1.0 / (h * h);
  const int T = 2 * (n + 1);  // last valid half-step index
  int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m > n + 1) return;
  auto S = [&](int t) { return (t < 0 || t > T) ? make_double2(0.0, 0.0) : sbd[t]; };
  const int L = n + 2;
  // A[m, m-1] and A[m, m+1] (row m: s_m s_{m -+ 1/2} / h^2)
  coef[0 * L + m] = cscale(cmul(S(2 * m), S(2 * m - 1)), ih2);
  coef[1 * L + m] = cscale(cmul(S(2 * m), S(2 * m + 1)), ih2);
  // A^H[m, m-1] = conj(A[m-1, m]) and A^H[m, m+1] = conj(A[m+1, m])
  coef[2 * L + m] = cconj(cscale(cmul(S(2 * m - 2), S(2 * m - 1)), ih2));
  coef[3 * L + m] = cconj(cscale(cmul(S(2 * m + 2), S(2 * m + 1)), ih2));
  diag[m] = cscale(cmul(S(2 * m), cadd(S(2 * m + 1), S(2 * m - 1))), -ih2);
}

}  // namespace

hipError_t launch_coefficients(helm_handle* h, const double* c_dev, bool tables, hipStream_t s) {
  const int n = h->n;
  const long long N = (long long)n * n * n;
  hipError_t e = hipMemsetAsync(h->d_err, 0, 2 * sizeof(int), s);
  if (e != hipSuccess) return e;
  k_kappa<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(c_dev, h->kappa, N, h->omega * h->omega,
                                                      h->d_err);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (tables) {
    const int T = 2 * (n + 1) + 1;
    k_tables<<<(T + 255) / 256, 256, 0, s>>>(n, h->plan.b, h->plan.p, h->C, h->C_mv, h->omega, h->sbd,
                                             h->smv, h->coef, h->diag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_coupling<<<(n + 2 + 255) / 256, 256, 0, s>>>(n, h->sbd, h->coef, h->diag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

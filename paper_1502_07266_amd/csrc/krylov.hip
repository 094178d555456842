// Flexible GMRES(m) on the GPU, FP64, batched over right-hand sides: the outer Krylov solver
// of Sec. 5 (GMRES around the whole 3D system, preconditioned by the recursive sweep).
//
// Right preconditioning with stored directions z_j = M^{-1} v_j (Saad's flexible variant), so
// the complex64 sweep of the mixed-precision mode enters only through z_j, which is exact in
// complex64 storage; the basis V, the Hessenberg matrix, the Givens rotations, the residual
// and the update x += Z y are FP64.  Orthogonalisation is classical Gram-Schmidt applied twice
// (two batched reductions per step instead of j+1 dependent ones).  x0 is the caller's u.
// After each cycle (or when a right-hand side's residual estimate reaches tol) the true
// residual ||f - A x|| decides convergence.
//
// All right-hand sides of a call advance in lockstep through one launch per kernel; a
// right-hand side that converges leaves the active index list.  The host reads R residual
// estimates per iteration to decide.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "common.h"

namespace {

constexpr int kDotThreads = 256;
constexpr int kDotPerThread = 8;
constexpr int kDotChunk = kDotThreads * kDotPerThread;
constexpr int kMaxRestart = 200;
constexpr int kFuse = 8;   // k_update_dots keeps up to this many basis values per element in registers

__device__ inline double2 block_sum(double2 v, double2* red) {
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_xor(v.x, off);
    v.y += __shfl_xor(v.y, off);
  }
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double2 s = make_double2(0.0, 0.0);
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s = cadd(s, red[i]);
  return s;
}

// Krylov bases are allocated kChunk vectors at a time as the iterations need them (a solve
// that converges in 7 iterations never holds the restart length's worth of vectors); within a
// chunk the vectors of all R right-hand sides are stored k-major: vector k of right-hand side
// q starts at c[k / kChunk] + ((k % kChunk) R + q) N.
constexpr int kChunk = 4;
constexpr int kMaxChunks = (kMaxRestart + 1 + kChunk - 1) / kChunk;

template <typename T> struct Basis {
  T* c[kMaxChunks];
  long long N;
  int R;
  __host__ __device__ __forceinline__ T* at(int k, int q) const {
    return c[k / kChunk] + ((long long)(k % kChunk) * R + q) * N;
  }
};

// a basis holding one vector per right-hand side, R vectors of N values at v
template <typename T> Basis<T> single(T* v, int R, long long N) {
  Basis<T> b{};
  b.c[0] = v;
  b.N = N;
  b.R = R;
  return b;
}

// partial[(a*K + k)*nchunk + chunk] = sum over the chunk of conj(X_k) w, for the active vector a
template <typename TX>
__global__ void __launch_bounds__(kDotThreads) k_dots(Basis<TX> X, int K,
                                                      const double2* __restrict__ w, long long wr,
                                                      const int* __restrict__ idx,
                                                      double2* __restrict__ partial, int nchunk,
                                                      long long N) {
  __shared__ double2 red[kDotThreads / 64];
  const int a = blockIdx.y, q = idx[a], chunk = blockIdx.x;
  const long long base = (long long)chunk * kDotChunk + threadIdx.x;
  double2 wv[kDotPerThread];
#pragma unroll
  for (int t = 0; t < kDotPerThread; ++t) {
    const long long e = base + (long long)t * kDotThreads;
    wv[t] = e < N ? w[(long long)q * wr + e] : make_double2(0.0, 0.0);
  }
  for (int k = 0; k < K; ++k) {
    const TX* xp = X.at(k, q);
    double2 s = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < kDotPerThread; ++t) {
      const long long e = base + (long long)t * kDotThreads;
      if (e < N) s = cfma_conj(s, cvt<double2>(xp[e]), wv[t]);
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) partial[((long long)a * K + k) * nchunk + chunk] = s;
  }
}

// One Gram-Schmidt update followed by the next reduction over the updated vector, in one pass
// over w: w_q -= sum_{k < K} coef[q][k] X_{q,k}, then (NORM false) the chunk's partial sums of
// conj(X_k) w for every k, as k_dots writes them (the basis chunk just read comes back from
// L2), or (NORM true) the partial sum of |w|^2, as k_dots of w with itself.  The arithmetic
// of each element is that of k_axpy_multi followed by k_dots.
template <typename TX, bool NORM>
__global__ void __launch_bounds__(kDotThreads) k_update_dots(double2* __restrict__ w, long long wr,
                                                             Basis<TX> X, const double2* __restrict__ coef,
                                                             int cstride, int K, const int* __restrict__ idx,
                                                             double2* __restrict__ partial, int nchunk,
                                                             long long N) {
  __shared__ double2 red[kDotThreads / 64];
  __shared__ double2 c[kMaxRestart + 1];
  const int a = blockIdx.y, q = idx[a], chunk = blockIdx.x;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double2 v = coef[(long long)q * cstride + k];
    c[k] = make_double2(-v.x, -v.y);
  }
  __syncthreads();
  const long long base = (long long)chunk * kDotChunk + threadIdx.x;
  if (!NORM && K <= kFuse) {
    // element by element: its K basis values loaded once, the update, then its terms of the
    // K dot products (the same operations, in the same order, as the general path below) and
    // of |w|^2 after the update, written as a (K + 1)-th dot product
    const int KS = K + 1;
    const TX* xp[kFuse];
#pragma unroll
    for (int k = 0; k < kFuse; ++k) xp[k] = k < K ? X.at(k, q) : nullptr;
    double2 acc[kFuse];
#pragma unroll
    for (int k = 0; k < kFuse; ++k) acc[k] = make_double2(0.0, 0.0);
    double2 ww = make_double2(0.0, 0.0);
    for (int t = 0; t < kDotPerThread; ++t) {
      const long long e = base + (long long)t * kDotThreads;
      if (e >= N) break;
      double2 xv[kFuse];
#pragma unroll
      for (int k = 0; k < kFuse; ++k)
        if (k < K) xv[k] = cvt<double2>(xp[k][e]);
      double2 wv = w[(long long)q * wr + e];
#pragma unroll
      for (int k = 0; k < kFuse; ++k)
        if (k < K) wv = cfma(wv, c[k], xv[k]);
      w[(long long)q * wr + e] = wv;
#pragma unroll
      for (int k = 0; k < kFuse; ++k)
        if (k < K) acc[k] = cfma_conj(acc[k], xv[k], wv);
      ww = cfma_conj(ww, wv, wv);
    }
#pragma unroll
    for (int k = 0; k < kFuse; ++k) {
      if (k >= K) break;
      const double2 sum = block_sum(acc[k], red);
      if (threadIdx.x == 0) partial[((long long)a * KS + k) * nchunk + chunk] = sum;
    }
    const double2 sum = block_sum(ww, red);
    if (threadIdx.x == 0) partial[((long long)a * KS + K) * nchunk + chunk] = sum;
    return;
  }
  double2 wv[kDotPerThread];
#pragma unroll
  for (int t = 0; t < kDotPerThread; ++t) {
    const long long e = base + (long long)t * kDotThreads;
    wv[t] = e < N ? w[(long long)q * wr + e] : make_double2(0.0, 0.0);
  }
  for (int k = 0; k < K; ++k) {
    const TX* xp = X.at(k, q);
#pragma unroll
    for (int t = 0; t < kDotPerThread; ++t) {
      const long long e = base + (long long)t * kDotThreads;
      if (e < N) wv[t] = cfma(wv[t], c[k], cvt<double2>(xp[e]));
    }
  }
#pragma unroll
  for (int t = 0; t < kDotPerThread; ++t) {
    const long long e = base + (long long)t * kDotThreads;
    if (e < N) w[(long long)q * wr + e] = wv[t];
  }
  if constexpr (NORM) {
    double2 sum = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < kDotPerThread; ++t) {
      const long long e = base + (long long)t * kDotThreads;
      if (e < N) sum = cfma_conj(sum, wv[t], wv[t]);
    }
    sum = block_sum(sum, red);
    if (threadIdx.x == 0) partial[(long long)a * nchunk + chunk] = sum;
  } else {
    for (int k = 0; k < K; ++k) {
      const TX* xp = X.at(k, q);
      double2 sum = make_double2(0.0, 0.0);
#pragma unroll
      for (int t = 0; t < kDotPerThread; ++t) {
        const long long e = base + (long long)t * kDotThreads;
        if (e < N) sum = cfma_conj(sum, cvt<double2>(xp[e]), wv[t]);
      }
      sum = block_sum(sum, red);
      if (threadIdx.x == 0) partial[((long long)a * K + k) * nchunk + chunk] = sum;
    }
  }
}

// out[q*ostride + k] = sum_chunks partial (mode 0), or sqrt(Re sum) (mode 1, norms): one
// workgroup per (k, active vector), the chunks' partial sums reduced across its threads
__global__ void __launch_bounds__(kDotThreads) k_dots_final(const double2* __restrict__ partial, int K,
                                                            int nchunk, const int* __restrict__ idx,
                                                            double2* __restrict__ out, int ostride,
                                                            int mode) {
  __shared__ double2 red[kDotThreads / 64];
  const int k = blockIdx.x, a = blockIdx.y, q = idx[a];
  const double2* p = partial + ((long long)a * K + k) * nchunk;
  double2 s = make_double2(0.0, 0.0);
  for (int c = threadIdx.x; c < nchunk; c += blockDim.x) s = cadd(s, p[c]);
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    // a norm keeps NaN (fmax would turn it into 0 and a broken vector would look converged)
    if (mode == 1) s = make_double2(s.x > 0.0 ? sqrt(s.x) : (s.x == s.x ? 0.0 : s.x), 0.0);
    out[(long long)q * ostride + k] = s;
  }
}

// y_q += sign * sum_{k < K_q} coef[q][k] X_{q,k}
template <typename TX>
__global__ void __launch_bounds__(256) k_axpy_multi(double2* __restrict__ y, long long yr,
                                                    Basis<TX> X, const double2* __restrict__ coef,
                                                    int cstride, int K, const int* __restrict__ kq,
                                                    double sign, const int* __restrict__ idx,
                                                    long long N) {
  __shared__ double2 c[kMaxRestart + 1];
  const int a = blockIdx.y, q = idx[a];
  const int Kq = kq ? kq[q] : K;
  for (int k = threadIdx.x; k < Kq; k += blockDim.x) {
    double2 v = coef[(long long)q * cstride + k];
    c[k] = make_double2(sign * v.x, sign * v.y);
  }
  __syncthreads();
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double2 acc = y[(long long)q * yr + e];
  for (int k = 0; k < Kq; ++k) acc = cfma(acc, c[k], cvt<double2>(X.at(k, q)[e]));
  y[(long long)q * yr + e] = acc;
}

// V_q = W_q / nrm_q (0 if the norm vanished: breakdown, the residual is then exactly zero)
__global__ void __launch_bounds__(256) k_scale(double2* __restrict__ V, long long vr,
                                               const double2* __restrict__ W, long long wr,
                                               const double2* __restrict__ nrm,
                                               const int* __restrict__ idx, long long N) {
  const int q = idx[blockIdx.y];
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  const double s = nrm[q].x > 0.0 ? 1.0 / nrm[q].x : 0.0;
  const double2 w = W[(long long)q * wr + e];
  V[(long long)q * vr + e] = make_double2(w.x * s, w.y * s);
}

// ||w''|| = sqrt(|w'|^2 - |h2|^2) for w'' = w' - V h2, h2 = V^H w' (V orthonormal; w' is
// orthogonal to V up to rounding after the first projection, so there is no cancellation):
// |w'|^2 sits at h2[K], after the K coefficients.  A negative difference (breakdown, w' = 0 up
// to rounding) gives 0, NaN stays NaN.
__global__ void k_norm_after(const double2* __restrict__ h2, int hstride, int K, double2* __restrict__ nrm,
                             const int* __restrict__ idx, int na) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= na) return;
  const int q = idx[a];
  const double2* h = h2 + (long long)q * hstride;
  double s = h[K].x;
  for (int k = 0; k < K; ++k) s -= h[k].x * h[k].x + h[k].y * h[k].y;
  nrm[q] = make_double2(s > 0.0 ? sqrt(s) : (s == s ? 0.0 : s), 0.0);
}

// V_q = (W_q - sum_{k < K} h2[q][k] X_{q,k}) / nrm_q (0 if the norm vanished)
template <typename TX>
__global__ void __launch_bounds__(256) k_update_scale(double2* __restrict__ V, long long vr,
                                                      const double2* __restrict__ W, long long wr,
                                                      Basis<TX> X, const double2* __restrict__ coef,
                                                      int cstride, int K, const double2* __restrict__ nrm,
                                                      const int* __restrict__ idx, long long N) {
  __shared__ double2 c[kFuse];
  const int q = idx[blockIdx.y];
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const double2 v = coef[(long long)q * cstride + k];
    c[k] = make_double2(-v.x, -v.y);
  }
  __syncthreads();
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N) return;
  double2 acc = W[(long long)q * wr + e];
#pragma unroll
  for (int k = 0; k < kFuse; ++k)
    if (k < K) acc = cfma(acc, c[k], cvt<double2>(X.at(k, q)[e]));
  const double sc = nrm[q].x > 0.0 ? 1.0 / nrm[q].x : 0.0;
  V[(long long)q * vr + e] = make_double2(acc.x * sc, acc.y * sc);
}

// start of a cycle: g = (beta, 0, ..., 0)
__global__ void k_cycle_init(double2* g, int gstride, const double2* beta, const int* idx, int na) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= na) return;
  const int q = idx[a];
  for (int i = 0; i < gstride; ++i) g[(long long)q * gstride + i] = make_double2(0.0, 0.0);
  g[(long long)q * gstride] = beta[q];
}

// column j of the Hessenberg matrix: h = h1 + h2 (two Gram-Schmidt passes), h_{j+1,j} = ||w||;
// apply the previous rotations, make and apply a new one, update g, residual estimate |g_{j+1}|
__global__ void k_givens(int j, int m, const double2* h1, const double2* h2, const double2* hn,
                         double2* H, double* cs, double2* sn, double2* g, double* resid,
                         const int* idx, int na) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= na) return;
  const int q = idx[a];
  double2 col[kMaxRestart + 1];
  for (int i = 0; i <= j; ++i)
    col[i] = cadd(h1[(long long)q * (m + 1) + i], h2[(long long)q * (m + 1) + i]);
  col[j + 1] = make_double2(hn[q].x, 0.0);
  double* c = cs + (long long)q * m;
  double2* s = sn + (long long)q * m;
  for (int i = 0; i < j; ++i) {
    const double2 t = cadd(cscale(col[i], c[i]), cmul(s[i], col[i + 1]));
    col[i + 1] = csub(cscale(col[i + 1], c[i]), cmul(cconj(s[i]), col[i]));
    col[i] = t;
  }
  // [[c, s], [-conj(s), c]] (a, b) = (rho, 0), c real
  const double2 av = col[j];
  const double bv = col[j + 1].x;
  const double aa = sqrt(cabs2(av));
  double cj;
  double2 sj, rho;
  if (bv == 0.0) {
    cj = 1.0;
    sj = make_double2(0.0, 0.0);
    rho = av;
  } else if (aa == 0.0) {
    cj = 0.0;
    sj = make_double2(1.0, 0.0);
    rho = make_double2(bv, 0.0);
  } else {
    const double r = hypot(aa, bv);
    cj = aa / r;
    sj = make_double2(av.x / aa * bv / r, av.y / aa * bv / r);
    rho = make_double2(av.x / aa * r, av.y / aa * r);
  }
  c[j] = cj;
  s[j] = sj;
  col[j] = rho;
  double2* gq = g + (long long)q * (m + 1);
  const double2 gj = gq[j];
  gq[j + 1] = cmul(make_double2(-sj.x, sj.y), gj);   // -conj(s) g_j
  gq[j] = cscale(gj, cj);
  double2* Hq = H + (long long)q * (m + 1) * m;
  for (int i = 0; i <= j; ++i) Hq[(long long)i * m + j] = col[i];
  resid[q] = sqrt(cabs2(gq[j + 1]));
}

// y = R^{-1} g for the leading k_q x k_q triangle
__global__ void k_trisolve(int m, const double2* H, const double2* g, const int* kq, double2* y,
                           const int* idx, int na) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= na) return;
  const int q = idx[a];
  const int k = kq[q];
  const double2* Hq = H + (long long)q * (m + 1) * m;
  const double2* gq = g + (long long)q * (m + 1);
  double2* yq = y + (long long)q * m;
  for (int i = k - 1; i >= 0; --i) {
    double2 s = gq[i];
    for (int l = i + 1; l < k; ++l) s = csub(s, cmul(Hq[(long long)i * m + l], yq[l]));
    yq[i] = cmul(s, cinv(Hq[(long long)i * m + i]));
  }
}

// Device workspace of one solve, taken from the library's pool (pool.cpp) and returned to it
// at the end, so that consecutive solves of the same size reuse the same memory.
struct Workspace {
  hipStream_t s = nullptr;
  double2 *W = nullptr, *partial = nullptr, *H = nullptr, *sn = nullptr, *g = nullptr;
  double2 *h1 = nullptr, *h2 = nullptr, *nrm = nullptr, *ycoef = nullptr, *fnrm = nullptr;
  double *cs = nullptr, *resid = nullptr;
  int *idx = nullptr, *kq = nullptr;
  Basis<double2> V{};
  Basis<float2> Z64{};     // mixed mode: the preconditioned directions in complex64
  Basis<double2> Z128{};
  int nv = 0, nz = 0;      // chunks held
  std::vector<void*> all;
  ~Workspace() {
    for (void* p : all) pool_free(p, s);
  }
  template <typename T> hipError_t get(T** p, size_t count) {
    void* q = nullptr;
    hipError_t e = pool_alloc(&q, std::max<size_t>(count, 1) * sizeof(T), s);
    if (e == hipSuccess) {
      all.push_back(q);
      *p = (T*)q;
    }
    return e;
  }
  // makes V hold vectors 0..kv and Z vectors 0..kz - 1
  hipError_t grow(int kv, int kz, bool c64) {
    while (nv * kChunk <= kv) {
      hipError_t e = get(&V.c[nv], (size_t)kChunk * V.R * V.N);
      if (e != hipSuccess) return e;
      ++nv;
    }
    while (nz * kChunk < kz) {
      hipError_t e = c64 ? get(&Z64.c[nz], (size_t)kChunk * Z64.R * Z64.N)
                         : get(&Z128.c[nz], (size_t)kChunk * Z128.R * Z128.N);
      if (e != hipSuccess) return e;
      ++nz;
    }
    return hipSuccess;
  }
};

// chunks of kChunk vectors that hold k vectors
inline long long chunks_for(long long k) { return (k + kChunk - 1) / kChunk; }

}  // namespace

#define HIP_MSG(expr)                                                   \
  do {                                                                  \
    hipError_t e__ = (expr);                                            \
    if (e__ != hipSuccess) {                                            \
      msg = std::string(#expr) + ": " + hipGetErrorString(e__);         \
      return HELM_EHIP;                                                 \
    }                                                                   \
  } while (0)

size_t fgmres_bytes(const helm_handle* h, int R, int restart, int maxit) {
  const long long N = (long long)h->n * h->n * h->n;
  const long long kmax = std::max(0, std::min(restart, maxit));
  const size_t zsz = h->prec == HELM_C64 ? sizeof(float2) : sizeof(double2);
  const long long nchunk = (N + kDotChunk - 1) / kDotChunk;
  size_t b = (size_t)chunks_for(kmax + 1) * kChunk * R * N * sizeof(double2) +   // V
             (size_t)chunks_for(kmax) * kChunk * R * N * zsz +                      // Z
             (size_t)R * N * sizeof(double2) +                                       // W
             (size_t)R * (restart + 1) * nchunk * sizeof(double2);                   // partial sums
  // Hessenberg matrices, rotations and the per-right-hand-side scalars
  b += (size_t)R * ((restart + 1) * (restart + 4) + 3 * restart + 4) * sizeof(double2);
  return b;
}

int fgmres_solve(helm_handle* h, const double2* f, double2* u, int R, double tol, int restart,
                 int maxit, bool adjoint, int* iters, double* relres, hipStream_t s,
                 std::string& msg) {
  const int m = restart;
  if (m < 1 || m > kMaxRestart) {
    msg = "restart must be in [1, 200]";
    return HELM_EINVAL;
  }
  const long long N = (long long)h->n * h->n * h->n;
  const bool c64 = h->prec == HELM_C64;
  const int nchunk = (int)((N + kDotChunk - 1) / kDotChunk);
  const unsigned nb = (unsigned)((N + 255) / 256);
  // planned before anything is allocated: the bases of the longest cycle maxit allows
  {
    size_t avail = 0;
    HIP_MSG(device_free_bytes(&avail));
    const size_t need = fgmres_bytes(h, R, restart, maxit);
    if (need > avail) {
      msg = "the solve needs up to " + std::to_string(need) + " bytes of device memory (Krylov "
            "bases of min(restart, maxit) iterations for " + std::to_string(R) +
            " right-hand sides), " + std::to_string(avail) + " available";
      return HELM_ENOMEM;
    }
  }
  Workspace ws;
  ws.s = s;
  ws.V.N = ws.Z64.N = ws.Z128.N = N;
  ws.V.R = ws.Z64.R = ws.Z128.R = R;
#define WS_GET(ptr, count)                                                           \
  do {                                                                               \
    if (ws.get(&(ptr), (count)) != hipSuccess) {                                     \
      msg = "device allocation failed for the Krylov workspace";                     \
      return HELM_ENOMEM;                                                            \
    }                                                                                \
  } while (0)
  WS_GET(ws.W, (size_t)R * N);
  WS_GET(ws.partial, (size_t)R * (m + 1) * nchunk);
  WS_GET(ws.H, (size_t)R * (m + 1) * m);
  WS_GET(ws.sn, (size_t)R * m);
  WS_GET(ws.cs, (size_t)R * m);
  WS_GET(ws.g, (size_t)R * (m + 1));
  WS_GET(ws.h1, (size_t)R * (m + 1));
  WS_GET(ws.h2, (size_t)R * (m + 1));
  WS_GET(ws.nrm, (size_t)R);
  WS_GET(ws.fnrm, (size_t)R);
  WS_GET(ws.ycoef, (size_t)R * m);
  WS_GET(ws.resid, (size_t)R);
  WS_GET(ws.idx, (size_t)R);
  WS_GET(ws.kq, (size_t)R);
#undef WS_GET

  std::vector<int> its(R, 0), kq(R, 0);
  std::vector<double> fn(R), beta(R), res(R);
  std::vector<char> done(R, 0);
  std::vector<int> act;

  auto upload = [&](const std::vector<int>& v) -> hipError_t {
    return hipMemcpyAsync(ws.idx, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice, s);
  };
  // norms of the batch w (R vectors of N values)
  auto norms = [&](const double2* w, const std::vector<int>& a, double2* out) -> hipError_t {
    dim3 gd(nchunk, (unsigned)a.size());
    k_dots<double2><<<gd, kDotThreads, 0, s>>>(single(const_cast<double2*>(w), R, N), 1, w, N, ws.idx,
                                               ws.partial, nchunk, N);
    k_dots_final<<<dim3(1, (unsigned)a.size()), kDotThreads, 0, s>>>(ws.partial, 1, nchunk, ws.idx, out, 1, 1);
    return hipGetLastError();
  };

  std::vector<int> all(R);
  for (int q = 0; q < R; ++q) all[q] = q;
  HIP_MSG(upload(all));
  HIP_MSG(norms(f, all, ws.fnrm));
  std::vector<double2> tmp(R);
  HIP_MSG(hipMemcpyAsync(tmp.data(), ws.fnrm, R * sizeof(double2), hipMemcpyDeviceToHost, s));
  HIP_MSG(hipStreamSynchronize(s));
  for (int q = 0; q < R; ++q) {
    fn[q] = tmp[q].x;
    if (!std::isfinite(fn[q])) {
      msg = "right-hand side " + std::to_string(q) + " is not finite";
      return HELM_EINVAL;
    }
  }

  int status = HELM_OK;
  const bool verbose = std::getenv("HELM_VERBOSE") != nullptr;
  while (true) {
    // ---- true residual of every unfinished right-hand side ----
    std::vector<int> cyc;
    for (int q = 0; q < R; ++q)
      if (!done[q]) cyc.push_back(q);
    if (cyc.empty()) break;
    HIP_MSG(upload(cyc));
    HIP_MSG(launch_matvec(h, u, true, f, ws.W, (int)cyc.size(), ws.idx, N, N, adjoint, 1, s));
    HIP_MSG(norms(ws.W, cyc, ws.nrm));
    HIP_MSG(hipMemcpyAsync(tmp.data(), ws.nrm, R * sizeof(double2), hipMemcpyDeviceToHost, s));
    HIP_MSG(hipStreamSynchronize(s));
    std::vector<int> next;
    for (int q : cyc) {
      beta[q] = tmp[q].x;
      res[q] = fn[q] > 0 ? beta[q] / fn[q] : 0.0;
      if (!std::isfinite(beta[q])) {
        // the residual overflowed or became NaN (a preconditioner out of range): give up on
        // this right-hand side and report it
        done[q] = 1;
        res[q] = beta[q];
        status = HELM_ENOTCONV;
        msg = "right-hand side " + std::to_string(q) + ": residual not finite";
      } else if (beta[q] <= tol * fn[q]) {
        done[q] = 1;
      } else if (its[q] >= maxit) {
        done[q] = 1;
        status = HELM_ENOTCONV;
      } else {
        next.push_back(q);
      }
    }
    if (next.empty()) break;
    act = next;
    HIP_MSG(upload(act));
    const unsigned na = (unsigned)act.size();
    if (ws.grow(0, 0, c64) != hipSuccess) {
      msg = "device allocation failed for the Krylov basis";
      return HELM_ENOMEM;
    }
    // V_0 = r / beta, g = (beta, 0, ...)
    k_scale<<<dim3(nb, na), 256, 0, s>>>(ws.V.at(0, 0), N, ws.W, N, ws.nrm, ws.idx, N);
    k_cycle_init<<<(na + 63) / 64, 64, 0, s>>>(ws.g, m + 1, ws.nrm, ws.idx, (int)na);
    HIP_MSG(hipGetLastError());
    std::vector<int> cycle_set = act;
    for (int q : cycle_set) kq[q] = 0;
    for (int j = 0; j < m && !act.empty(); ++j) {
      const unsigned a = (unsigned)act.size();
      if (ws.grow(j + 1, j + 1, c64) != hipSuccess) {
        msg = "device allocation failed for the Krylov basis";
        return HELM_ENOMEM;
      }
      void* zj = c64 ? (void*)ws.Z64.at(j, 0) : (void*)ws.Z128.at(j, 0);
      // z_j = M^{-1} v_j
      HIP_MSG(launch_apply(h, ws.V.at(j, 0), true, N, zj, !c64, N, (int)a, ws.idx, adjoint, s));
      // w = A z_j
      HIP_MSG(launch_matvec(h, zj, !c64, nullptr, ws.W, (int)a, ws.idx, N, N, adjoint, 0, s));
      // two classical Gram-Schmidt passes: h1 = V^H w; w -= V h1 and h2 = V^H w in one pass;
      // w -= V h2 and ||w||^2 in one pass
      k_dots<double2><<<dim3(nchunk, a), kDotThreads, 0, s>>>(ws.V, j + 1, ws.W, N, ws.idx,
                                                              ws.partial, nchunk, N);
      k_dots_final<<<dim3(j + 1, a), kDotThreads, 0, s>>>(ws.partial, j + 1, nchunk, ws.idx, ws.h1, m + 1, 0);
      k_update_dots<double2, false><<<dim3(nchunk, a), kDotThreads, 0, s>>>(
          ws.W, N, ws.V, ws.h1, m + 1, j + 1, ws.idx, ws.partial, nchunk, N);
      if (j + 1 <= kFuse) {
        // h2 and |w'|^2 (at h2[j + 1]); then w'' and its normalisation in one pass
        k_dots_final<<<dim3(j + 2, a), kDotThreads, 0, s>>>(ws.partial, j + 2, nchunk, ws.idx, ws.h2, m + 1, 0);
        k_norm_after<<<(a + 63) / 64, 64, 0, s>>>(ws.h2, m + 1, j + 1, ws.nrm, ws.idx, (int)a);
        k_update_scale<double2><<<dim3(nb, a), 256, 0, s>>>(ws.V.at(j + 1, 0), N, ws.W, N, ws.V, ws.h2, m + 1,
                                                           j + 1, ws.nrm, ws.idx, N);
      } else {
        k_dots_final<<<dim3(j + 1, a), kDotThreads, 0, s>>>(ws.partial, j + 1, nchunk, ws.idx, ws.h2, m + 1, 0);
        k_update_dots<double2, true><<<dim3(nchunk, a), kDotThreads, 0, s>>>(
            ws.W, N, ws.V, ws.h2, m + 1, j + 1, ws.idx, ws.partial, nchunk, N);
        k_dots_final<<<dim3(1, a), kDotThreads, 0, s>>>(ws.partial, 1, nchunk, ws.idx, ws.nrm, 1, 1);
        k_scale<<<dim3(nb, a), 256, 0, s>>>(ws.V.at(j + 1, 0), N, ws.W, N, ws.nrm, ws.idx, N);
      }
      k_givens<<<(a + 63) / 64, 64, 0, s>>>(j, m, ws.h1, ws.h2, ws.nrm, ws.H, ws.cs, ws.sn, ws.g,
                                           ws.resid, ws.idx, (int)a);
      HIP_MSG(hipGetLastError());
      std::vector<double> rr(R);
      HIP_MSG(hipMemcpyAsync(rr.data(), ws.resid, R * sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_MSG(hipStreamSynchronize(s));
      std::vector<int> keep;
      double worst = 0.0;
      for (int q : act) {
        its[q] += 1;
        kq[q] = j + 1;
        res[q] = fn[q] > 0 ? rr[q] / fn[q] : 0.0;
        worst = std::max(worst, res[q]);
        // (a NaN estimate leaves the cycle; the true residual after it decides)
        if (rr[q] > tol * fn[q] && its[q] < maxit) keep.push_back(q);
      }
      if (verbose)
        std::fprintf(stderr, "[helm fgmres] iteration %d: %zu active, worst estimate %.3e\n",
                     j + 1, act.size(), worst);
      if (keep.size() != act.size()) {
        act = keep;
        if (!act.empty()) HIP_MSG(upload(act));
      }
    }
    // ---- x += Z y for every right-hand side of this cycle ----
    HIP_MSG(upload(cycle_set));
    HIP_MSG(hipMemcpyAsync(ws.kq, kq.data(), R * sizeof(int), hipMemcpyHostToDevice, s));
    const unsigned nc = (unsigned)cycle_set.size();
    k_trisolve<<<(nc + 63) / 64, 64, 0, s>>>(m, ws.H, ws.g, ws.kq, ws.ycoef, ws.idx, (int)nc);
    if (c64)
      k_axpy_multi<float2><<<dim3(nb, nc), 256, 0, s>>>(u, N, ws.Z64, ws.ycoef, m, m, ws.kq, 1.0,
                                                        ws.idx, N);
    else
      k_axpy_multi<double2><<<dim3(nb, nc), 256, 0, s>>>(u, N, ws.Z128, ws.ycoef, m, m, ws.kq, 1.0,
                                                         ws.idx, N);
    HIP_MSG(hipGetLastError());
  }
  for (int q = 0; q < R; ++q) {
    if (iters) iters[q] = its[q];
    if (relres) relres[q] = res[q];
  }
  HIP_MSG(hipStreamSynchronize(s));
  return status;
}

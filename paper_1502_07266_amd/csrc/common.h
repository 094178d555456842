// Internal declarations shared by the HIP sources of libhelm (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "helm.h"

// ---------------------------------------------------------------------------------------
// complex arithmetic on float2 / double2 (interleaved re, im)
// ---------------------------------------------------------------------------------------
template <typename R> struct cx;
template <> struct cx<float> { using type = float2; };
template <> struct cx<double> { using type = double2; };

__host__ __device__ inline float2 mk(float r, float i) { return make_float2(r, i); }
__host__ __device__ inline double2 mk(double r, double i) { return make_double2(r, i); }

template <typename C> __host__ __device__ inline C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __host__ __device__ inline C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __host__ __device__ inline C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C> __host__ __device__ inline C cconj(C a) { return C{a.x, -a.y}; }
// a + b * c
template <typename C> __host__ __device__ inline C cfma(C a, C b, C c) {
  return C{a.x + b.x * c.x - b.y * c.y, a.y + b.x * c.y + b.y * c.x};
}
// a + conj(b) * c
template <typename C> __host__ __device__ inline C cfma_conj(C a, C b, C c) {
  return C{a.x + b.x * c.x + b.y * c.y, a.y + b.x * c.y - b.y * c.x};
}
template <typename C> __host__ __device__ inline auto cabs2(C a) { return a.x * a.x + a.y * a.y; }
template <typename C> __host__ __device__ inline C cinv(C a) {
  auto d = a.x * a.x + a.y * a.y;
  return C{a.x / d, -a.y / d};
}
template <typename C> __host__ __device__ inline C cscale(C a, decltype(a.x) s) { return C{a.x * s, a.y * s}; }

// conversions between storage and compute types
template <typename D, typename S> __host__ __device__ inline D cvt(S s);
template <> __host__ __device__ inline float2 cvt<float2, float2>(float2 s) { return s; }
template <> __host__ __device__ inline double2 cvt<double2, double2>(double2 s) { return s; }
template <> __host__ __device__ inline float2 cvt<float2, double2>(double2 s) {
  return make_float2((float)s.x, (float)s.y);
}
template <> __host__ __device__ inline double2 cvt<double2, float2>(float2 s) {
  return make_double2((double)s.x, (double)s.y);
}

// ---------------------------------------------------------------------------------------
// LDS of the sweep kernels
// ---------------------------------------------------------------------------------------
// largest NC * CW of the sweep's launch shapes and largest block B (the one-chain shapes of
// the two-front middle slab reach 8 x 16 columns); sizes the published vectors and the zero
// and junk rows
constexpr int kZMax = 128;

// LDS layout of the sweep kernels, in complex elements from the base (the step table follows
// at a 16-byte boundary): line vector, published vectors, zero and junk rows, couplings, the
// per-step couplings and the per-step table (2 (n + 3) entries each: two chains of at most
// n + 3, or one chain of at most 2n + 1).
struct LdsLayout {
  int ybuf, zb, zeros, junk, cf, cb, ctab;
  size_t tab_byte, bytes;
  __host__ __device__ LdsLayout(int n, int maxB, int csz) {
    ybuf = 0;
    zb = n * maxB;
    zeros = zb + 4 * kZMax;
    junk = zeros + kZMax;
    cf = junk + kZMax;
    cb = cf + (n + 2);
    ctab = cb + (n + 2);
    tab_byte = ((size_t)(ctab + 2 * (n + 3)) * csz + 15) / 16 * 16;
    bytes = tab_byte + 2 * (size_t)(n + 3) * 16;
  }
};

// largest block of the two-chain sweep shapes (two chains of B rows x NC lanes per workgroup):
// 8 x 8 or 4 x 16.  (A 4 x 20 shape for blocks up to 80 was measured: at 640 threads it
// spills registers and keeps a ring of only 2 blocks, and its lines took as long as one
// chain over twice the steps.)
constexpr int kTwoChainMaxB64 = 64;
constexpr int kTwoChainMaxB128 = 64;

// ---------------------------------------------------------------------------------------
// partition of an axis into groups and their auxiliary windows
// ---------------------------------------------------------------------------------------
struct GroupInfo {
  int first;  // first physical node (1-based)
  int last;   // last physical node
  int w0;     // first node of the auxiliary window (= first - p for moving groups)
  int W;      // window length
};

struct Plan {
  int n = 0, b = 0, p = 0, d = 0;
  int fronts = 1;                     // outer sweep from one face (Algorithm 6) or from both
  int fronts_inner = 1;               // the same for the inner sweep over x2 (Algorithm 4)
  int Gz = 0, Gy = 0;                 // x3-groups (outer sweep), x2-groups (inner sweep)
  int zmid = -1;                      // two fronts: the middle x3-group (eliminated last)
  int ymid = -1;                      // two inner fronts: the middle x2-group
  std::vector<GroupInfo> groups;      // [Gz] x3-groups, then [Gy] x2-groups
  std::vector<long long> line_off;    // [Gz*Gy] offset (complex elements) of line (g, l) = g*Gy + l
  std::vector<int> line_B;            // [Gz*Gy]
  long long total_elems = 0;          // sum over lines of n * B^2
  int maxB = 0, maxW = 0;             // over all lines / windows
  int maxB_front = 0, maxB_mid = 0;   // largest block of the two-chain / one-chain lines
  int two_cap = 0;                    // largest block two chains per workgroup can solve
  std::vector<unsigned char> one;     // [Gz*Gy] line solved by one chain (see build_plan)
  const GroupInfo& zg(int g) const { return groups[g]; }
  const GroupInfo& yg(int l) const { return groups[Gz + l]; }
  // lines whose launch holds a block too large for two chains per workgroup are eliminated
  // in x1 order and solved by one chain spanning the workgroup (see build_plan)
  bool one_chain(int g, int l) const { return one[(size_t)g * Gy + l] != 0; }
  // middle block of line (g, l)'s elimination order: both ends towards n/2, or n - 1 (x1 order)
  int line_mid(int g, int l) const { return one_chain(g, l) ? n - 1 : n / 2; }
};

// builds the plan; returns HELM_OK or HELM_EINVAL (with a message)
int build_plan(int n, int b, int p, int d, int fronts, int fronts_inner, int prec, Plan& plan,
               std::string& msg);

// what a workgroup does with one group (an x3-group of the outer sweep or an x2-group of the
// inner sweep): forward from below / from above / the middle group with both couplings;
// backward with the coupling from above / from below
enum SweepKind { kFwdLow = 0, kFwdHigh = 1, kFwdMid = 2, kBwdLow = 3, kBwdHigh = 4 };

// The groups a front visits in one pass over an axis of G groups (middle group mid):
//   pass 0 (one front): 0..G-1 forward from below, then G-2..0 backward
//   pass 1 (two fronts forward): front 0 takes 0..mid-1 from below, front 1 G-1..mid+1 from above
//   pass 2: the middle group with both couplings
//   pass 3 (two fronts backward): front 0 mid-1..0, front 1 mid+1..G-1
__host__ __device__ inline int sweep_count(int pass, int G, int mid, int front) {
  switch (pass) {
    case 0: return 2 * G - 1;
    case 2: return 1;
    default: return front == 0 ? mid : G - 1 - mid;
  }
}
__host__ __device__ inline int2 sweep_at(int pass, int G, int mid, int front, int s) {
  switch (pass) {
    case 0: return s < G ? make_int2(s, kFwdLow) : make_int2(2 * G - 2 - s, kBwdLow);
    case 1: return front == 0 ? make_int2(s, kFwdLow) : make_int2(G - 1 - s, kFwdHigh);
    case 2: return make_int2(mid, kFwdMid);
    default: return front == 0 ? make_int2(mid - 1 - s, kBwdLow) : make_int2(mid + 1 + s, kBwdHigh);
  }
}

// one launch of the sweep: outer pass and its fronts, the range of the pass's slab steps,
// inner pass and its fronts, line chains per workgroup, largest block, and whether it is a
// launch of the dominant (two-chain) kernel
struct SweepLaunch {
  int pass, nfront, slab_lo, slab_hi, ipass, ninner, chains, maxB;
  bool timed;
};
std::vector<SweepLaunch> sweep_schedule(const Plan& P);

// ---------------------------------------------------------------------------------------
// device-time accounting: event pairs recorded around launches, resolved lazily
// ---------------------------------------------------------------------------------------
struct LaunchTimer {
  struct Pending {
    hipEvent_t a, b;
    long long rhs;
  };
  std::vector<Pending> pending;
  long long launches = 0, rhs = 0;
  double ms = 0.0;
  // records the start event; returns it for end()
  hipEvent_t begin(hipStream_t s) {
    hipEvent_t a = nullptr;
    if (hipEventCreate(&a) != hipSuccess) return nullptr;
    if (hipEventRecord(a, s) != hipSuccess) {
      (void)hipEventDestroy(a);
      return nullptr;
    }
    return a;
  }
  void end(hipEvent_t a, hipStream_t s, long long nrhs) {
    if (!a) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) != hipSuccess || hipEventRecord(b, s) != hipSuccess) {
      (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
      return;
    }
    pending.push_back({a, b, nrhs});
    if (pending.size() >= 2048) flush();   // bounds the events alive between reads
  }
  void flush() {
    for (auto& p : pending) {
      float t = 0.f;
      if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
        ms += t;
        launches += 1;
        rhs += p.rhs;
      }
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    pending.clear();
  }
  void reset() {
    flush();
    launches = rhs = 0;
    ms = 0.0;
  }
};

// ---------------------------------------------------------------------------------------
// the opaque handle
// ---------------------------------------------------------------------------------------
struct helm_handle {
  Plan plan;
  int n = 0, prec = HELM_C64, device = 0;
  double omega = 0, h = 0, C = 0, C_mv = 0;
  int lanes_override = 0;

  // device data
  double* kappa = nullptr;         // n^3, omega^2 / c^2
  double2* sbd = nullptr;          // boundary profile s at half-steps t = 0 .. 2(n+1)
  double2* smv = nullptr;          // moving profile s at half-steps u = 0 .. 2p+1 from its plane
  double2* coef = nullptr;         // [4][n+2]: A[m,m-1], A[m,m+1], A^H[m,m-1], A^H[m,m+1]
  double2* diag = nullptr;         // [n+2]: -s_m (s_{m+1/2} + s_{m-1/2}) / h^2
  GroupInfo* d_groups = nullptr;   // [Gz + Gy]
  unsigned char* d_line_one = nullptr;   // [Gz*Gy] Plan::one
  int* d_setup_lines = nullptr;    // [Gz*Gy] line indices in setup_classes order
  long long* d_line_off = nullptr; // [Gz*Gy]
  void* factors = nullptr;         // total_elems complex64 or complex128
  int* d_err = nullptr;            // [2]: error flag, first failing line

  // timing
  LaunchTimer t_apply, t_matvec;
  LaunchTimer t_kernel;            // the sweep's dominant kernel (see helm_stats)
  double setup_ms = 0.0;
  double apply_bytes_per_rhs = 0.0;
  double kernel_bytes_per_rhs = 0.0;
  double kernel_factor_bytes = 0.0, kernel_vector_bytes_per_rhs = 0.0, kernel_flops_per_rhs = 0.0;

  // apply workspace (grown on demand)
  void* slab_scratch = nullptr;
  size_t slab_scratch_bytes = 0;
  // paired two-chain launches (helm_set_split): error word and exchange slots for xpairs
  // workgroup pairs; xseq numbers the lines across launches
  int split = 1;
  void* xbuf = nullptr;
  size_t xpairs = 0;
  unsigned long long xseq = 0;
  bool pairs_used = false;         // a paired launch ran since the error word was last taken
  int* d_rhs_idx = nullptr;
  int rhs_idx_cap = 0;
  // the stream of the last call: the handle's buffers go back to the pool on it
  hipStream_t last_stream = nullptr;
};

// layout of helm_handle::xbuf: an error word (padded), then per pair, chain and line parity a
// slot of kZMax values of up to four 32-bit pieces, one tagged 64-bit word each
constexpr size_t kXHead = 256;
constexpr size_t kXSlot = (size_t)kZMax * 4;
// waits for stream s, then *bad = nonzero if a paired line solve gave up waiting for its
// partner since the flag was last taken (and clears it)
hipError_t take_exchange_error(helm_handle* h, hipStream_t s, int* bad);

// ---------------------------------------------------------------------------------------
// internal launchers (all asynchronous on `stream`)
// ---------------------------------------------------------------------------------------
hipError_t launch_coefficients(helm_handle* h, const double* c_dev, bool tables, hipStream_t s);
hipError_t launch_setup(helm_handle* h, hipStream_t s);
// the setup's launches: lines in class order (small two-chain blocks, other two-chain
// blocks, one-chain lines), the count and largest block of each class
struct SetupClasses {
  std::vector<int> order;
  int count[3];
  int maxB[3];
};
SetupClasses setup_classes(const Plan& P, int csz, const std::vector<int>* subset);
// the setup of the lines listed at d_lines (device copy of c.order)
hipError_t launch_setup_lines(helm_handle* h, const int* d_lines, const SetupClasses& c,
                              hipStream_t s);
// z = M^{-1} r (or M^{-H}) for `R` right-hand sides; r in complex128 or complex64, z likewise;
// rhs_idx (device, may be null = identity) selects which vectors to process: workgroup a
// reads r + idx[a]*r_stride and writes z + idx[a]*z_stride (strides in complex elements).
hipError_t launch_apply(helm_handle* h, const void* r, bool r64, long long r_stride, void* z,
                        bool z64, long long z_stride, int R, const int* rhs_idx, bool adjoint,
                        hipStream_t s);
// device scratch of an apply of R right-hand sides (slab iterates and exchange slots)
size_t apply_scratch_bytes(const helm_handle* h, int R);
hipError_t launch_line_solve(helm_handle* h, int zg, int yg, const double2* r, double2* x, int R,
                             bool adjoint, hipStream_t s);
// y = A u (mode 0) or y = f - A u (mode 1); u complex128 or complex64 (u64 = false)
hipError_t launch_matvec(helm_handle* h, const void* u, bool u64, const double2* f, double2* y,
                         int R, const int* rhs_idx, long long u_stride, long long y_stride,
                         bool adjoint, int mode, hipStream_t s);
hipError_t launch_grad(helm_handle* h, const double2* u, const double2* lam, int R, double* grad,
                       hipStream_t s);
hipError_t launch_misfit(helm_handle* h, const double2* u, const double2* d, int R, int plane_k,
                        double* J_dev, double2* g, hipStream_t s);
// device bytes a solve of R right-hand sides may take at most (its Krylov bases are grown as
// the iterations need them, up to min(restart, maxit) vectors)
size_t fgmres_bytes(const helm_handle* h, int R, int restart, int maxit);
int fgmres_solve(helm_handle* h, const double2* f, double2* u, int R, double tol, int restart,
                 int maxit, bool adjoint, int* iters, double* relres, hipStream_t s, std::string& msg);

void set_error(const std::string& msg);

// device memory of the library (pool.cpp): a process-wide cache of blocks keyed by size,
// stream-ordered (a block returned on one stream and reused on another waits for the first)
hipError_t pool_alloc(void** out, size_t bytes, hipStream_t s);
void pool_free(void* p, hipStream_t s);
// free device memory plus the pool's cached bytes on the current device
hipError_t device_free_bytes(size_t* avail);

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e__ = (expr);                                                           \
    if (e__ != hipSuccess) {                                                           \
      set_error(std::string(#expr) + ": " + hipGetErrorString(e__));                  \
      return HELM_EHIP;                                                                \
    }                                                                                  \
  } while (0)

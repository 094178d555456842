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

// largest block B of a line and largest published vector of the sweep's launch shapes
constexpr int kZMax = 128;

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
  int maxB_front = 0;                 // over the lines on no middle group
  const GroupInfo& zg(int g) const { return groups[g]; }
  const GroupInfo& yg(int l) const { return groups[Gz + l]; }
  // every line is eliminated from both ends towards its middle block n/2 (Sec. 3, that order)
  int line_mid() const { return n / 2; }
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

// ---------------------------------------------------------------------------------------
// device-time accounting: event pairs recorded around launches, resolved lazily
// ---------------------------------------------------------------------------------------
struct LaunchTimer {
  struct Pending {
    hipEvent_t a, b;
    long long rhs;
    double bytes, flops;
  };
  std::vector<Pending> pending;
  long long launches = 0, rhs = 0;
  double ms = 0.0, bytes = 0.0, flops = 0.0;
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
  void end(hipEvent_t a, hipStream_t s, long long nrhs, double nbytes = 0.0, double nflops = 0.0) {
    if (!a) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) != hipSuccess || hipEventRecord(b, s) != hipSuccess) {
      (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
      return;
    }
    pending.push_back({a, b, nrhs, nbytes, nflops});
    if (pending.size() >= 2048) flush();   // bounds the events alive between reads
  }
  void flush() {
    for (auto& p : pending) {
      float t = 0.f;
      if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
        ms += t;
        launches += 1;
        rhs += p.rhs;
        bytes += p.bytes;
        flops += p.flops;
      }
      (void)hipEventDestroy(p.a);
      (void)hipEventDestroy(p.b);
    }
    pending.clear();
  }
  void reset() {
    flush();
    launches = rhs = 0;
    ms = bytes = flops = 0.0;
  }
};

// ---------------------------------------------------------------------------------------
// the opaque handle
// ---------------------------------------------------------------------------------------
// Polls of a partner's exchange word before a sweep's wait gives up (each poll a device-memory
// round trip and a short sleep; 2^28 of them take tens of seconds).  A wait is only as long as
// the partner's work before it: at most one slab of the other outer front (the middle slab,
// for the front that waits for it after its own forward slabs), which at 255^3 with blocks of
// 126 unknowns is beyond 2^20 polls.
constexpr unsigned kSpinDefault = 1u << 28;

struct helm_handle {
  Plan plan;
  int n = 0, prec = HELM_C64, device = 0;
  double omega = 0, h = 0, C = 0, C_mv = 0;
  int variant = -1;                // sweep launch shape (sweep_variants.h); -1: automatic

  // device data
  double* kappa = nullptr;         // n^3, omega^2 / c^2
  double2* sbd = nullptr;          // boundary profile s at half-steps t = 0 .. 2(n+1)
  double2* smv = nullptr;          // moving profile s at half-steps u = 0 .. 2p+1 from its plane
  double2* coef = nullptr;         // [4][n+2]: A[m,m-1], A[m,m+1], A^H[m,m-1], A^H[m,m+1]
  double2* diag = nullptr;         // [n+2]: -s_m (s_{m+1/2} + s_{m-1/2}) / h^2
  GroupInfo* d_groups = nullptr;   // [Gz + Gy]
  int* d_setup_lines = nullptr;    // [Gz*Gy] line indices in setup_classes order
  long long* d_line_off = nullptr; // [Gz*Gy]
  void* factors = nullptr;         // total_elems complex64 or complex128
  // nested-dissection line solver (complex64 forward sweeps): its factors, per-line offsets,
  // levels k (n = 2^k - 1); used by the forward sweeps while nd_on
  void* nd = nullptr;
  long long* d_nd_off = nullptr;
  int nd_k = 0;
  bool nd_on = false;
  size_t nd_bytes = 0;
  double nd_setup_ms = 0.0;
  int* d_err = nullptr;            // [2]: error flag, first failing line

  // timing
  LaunchTimer t_apply, t_matvec;
  LaunchTimer t_kernel;            // the sweep kernel's launches (see helm_stats)
  double setup_ms = 0.0;
  double apply_bytes_per_rhs = 0.0;
  double sweep_factor_bytes = 0.0;    // factor bytes one sweep reads (every block visit once)
  double sweep_factor_entries = 0.0;  // factor entries one sweep visits

  // sweep workspace (grown on demand): slab iterates, received layers, exchange words (an
  // error word, then the words of every launch slot); xseq numbers exchange events across
  // launches; spin_limit and drop_publish are the exchange's bound and failure-injection hook
  void* slab_scratch = nullptr;
  size_t slab_scratch_bytes = 0;
  void* layer = nullptr;
  size_t layer_bytes = 0;
  void* xbuf = nullptr;
  size_t xbytes = 0;
  unsigned long long xseq = 0;
  bool pairs_used = false;         // a sweep ran since the error word was last taken
  unsigned spin_limit = kSpinDefault;
  int drop_publish = 0;
  int* d_rhs_idx = nullptr;
  int rhs_idx_cap = 0;
  // the stream of the last call: the handle's buffers go back to the pool on it
  hipStream_t last_stream = nullptr;
};

// bytes before the exchange words in helm_handle::xbuf (the error word, padded)
constexpr size_t kXHead = 256;
// waits for stream s, then *bad = nonzero if a paired line solve gave up waiting for its
// partner since the flag was last taken (and clears it)
hipError_t take_exchange_error(helm_handle* h, hipStream_t s, int* bad);

// ---------------------------------------------------------------------------------------
// internal launchers (all asynchronous on `stream`)
// ---------------------------------------------------------------------------------------
hipError_t launch_coefficients(helm_handle* h, const double* c_dev, bool tables, hipStream_t s);
hipError_t launch_setup(helm_handle* h, hipStream_t s);
// nested-dissection line solver: support of a plan, entries per line (times B^2), and the
// factorisation of every line into h->nd (HELM_OK or an error code with msg)
bool nd_supported(const Plan& P, int prec, std::string& why);
long long nd_line_blocks(int n);
int nd_build(helm_handle* h, hipStream_t s, std::string& msg);
// the setup's launches: lines in class order (blocks whose two B x B copies fit a quarter of
// the LDS, other blocks up to 64, larger blocks), the count and largest block of each class
// dynamic LDS a setup workgroup takes for blocks up to maxB (complex element size csz), and
// whether the setup supports such blocks
size_t setup_lds_bytes(int maxB, int csz);
bool setup_fits(int maxB, int csz);
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
// caller-provided device scratch of a sweep: `bytes` at `base`, and the counter its exchange
// tags are drawn from (shared by every user of that scratch)
struct FixedScratch {
  char* base;
  size_t bytes;
  unsigned long long* seq;
};
// z = M^{-1} r (or M^{-H}) for R right-hand sides, complex128 in and out, with every buffer
// of the sweep in fx (the right-hand sides are launched in chunks that fit)
hipError_t launch_apply_fixed(helm_handle* h, const void* r, void* z, int R, bool adjoint,
                              const FixedScratch& fx, hipStream_t s);
// device scratch of an apply of R right-hand sides (slab iterates, layers, exchange words)
size_t apply_scratch_bytes(const helm_handle* h, int R);
// the sweep's launch shape for R right-hand sides: the handle's, the autotuner's or the default
int sweep_variant_for(const helm_handle* h, int R);
bool sweep_variant_valid(const helm_handle* h, int k);
std::string sweep_variant_name(bool c64, int k);
std::string tune_key(const helm_handle* h, int R);
int tuned_variant(const std::string& key);
void remember_variant(const std::string& key, int k);
std::vector<int> tune_candidates(const helm_handle* h);
// times a sweep of R right-hand sides with every candidate variant; the fastest and its time
hipError_t autotune_sweep(helm_handle* h, int R, int* best, double* best_ms, hipStream_t s);
// x[0..count) = 1 + 0i
hipError_t fill_ones(double2* x, long long count, hipStream_t s);
// the autotuner's choice for key (from the file at path when it holds one, else measured and
// appended there), remembered for the process; *out and *ms_out may be null
int tune_and_remember(helm_handle* h, int R, const std::string& key, const char* path, int* out,
                      double* ms_out, hipStream_t s);
// whether the sweep kernel has a launch shape and LDS room for the plan's blocks (else why)
bool sweep_plan_supported(const Plan& P, int prec, std::string& why);
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

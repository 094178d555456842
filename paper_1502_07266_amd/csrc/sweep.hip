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
//       line solve: y_i = T_i (q_i - l_i y_{i-1}),  x_i = y_i - u_i T_i x_{i+1}  (lines with
//       g + l odd eliminate downwards: y_i = T_i (q_i - u_i y_{i+1}), x_i = y_i - l_i T_i x_{i-1})
// where v is the slab iterate (n x n x window layers, in global scratch), the line vector
// (n blocks of B = Wy*Wz) lives in LDS, and the T_i stream from HBM.  The adjoint uses the
// couplings of A^H and T_i^H (the same pass order).
//
// Block step: thread t owns output row t / NC of the B x B block and CW consecutive columns;
// the NC partial sums of a row are adjacent lanes of one wavefront and are combined with DPP
// row operations.  The vector a step multiplies (z_i = q_i - l_i y_{i-1} forward, x_{i+1}
// backward) is formed once per row by the row's owner lane and published through a
// double-buffered LDS slot, so one barrier separates consecutive steps.  The factor blocks do
// not depend on the data: each thread keeps its slice of the next D blocks in registers
// (a ring refilled D steps ahead), which hides the HBM latency behind D dependent steps.
#include "common.h"

namespace {

constexpr int kZMax = 64;   // largest NC * CW of the instantiated shapes

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

// sum over groups of NC adjacent lanes (NC in {4, 8, 16}), result in every lane of the group
template <int CTRL> __device__ __forceinline__ float dpp_mov(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <int CTRL> __device__ __forceinline__ double dpp_mov(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int NC, typename T> __device__ __forceinline__ T lane_sum(T v) {
  static_assert(NC == 4 || NC == 8 || NC == 16, "lanes per row must be 4, 8 or 16");
  v += dpp_mov<0xB1>(v);                             // quad_perm [1,0,3,2]: pairs
  v += dpp_mov<0x4E>(v);                             // quad_perm [2,3,0,1]: quads
  if constexpr (NC >= 8) v += dpp_mov<0x141>(v);     // row_half_mirror: the other quad of 8
  if constexpr (NC == 16) v += dpp_mov<0x140>(v);    // row_mirror: the other 8 of each 16
  return v;
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations, then
// s_barrier.  Unlike __syncthreads() it does not wait for outstanding global loads, so the
// factor ring stays in flight across block steps.  Global scratch written around a line
// solve is published with full __syncthreads() by the caller.
__device__ __forceinline__ void lds_barrier() {
  __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <typename R, int NC, int CW, int D, bool ADJ>
struct LineSolver {
  using C = typename cx<R>::type;
  static constexpr int ZS = NC * CW;   // stride of one published vector (>= B, zero-padded)
  static constexpr int NA = CW < 3 ? CW : 3;   // independent accumulators in a block row
  C ring[D][CW];
  unsigned off[CW];                    // this thread's byte offsets inside a B x B block
  int row, c0;
  bool owner_lane;
  // Elimination order of the current line: block f0 + fs * t is eliminated at step t
  // (f0 = 0, fs = 1 upwards; f0 = n - 1, fs = -1 downwards).  The back-substitution visits
  // the blocks in the opposite order, starting from the second to last one eliminated.
  int n_, f0, fs;

  __device__ __forceinline__ LineSolver() {
    row = threadIdx.x / NC;
    const int lc = threadIdx.x - row * NC;
    c0 = lc * CW;
    owner_lane = lc == 0;
  }

  // per-line set-up: offsets and elimination order (dir 0 upwards, 1 downwards, as the
  // factors were computed).  Rows past B are clamped to a valid row (their sums are never
  // published).  Columns past B meet zero padding of the published vector: in the row-major
  // (non-adjoint) walk they run into the next row, or past the last block into the padding
  // that follows the factor array, so they read finite values; the adjoint walk clamps them.
  __device__ __forceinline__ void begin_line(int B, int n, int dir) {
    n_ = n;
    f0 = dir ? n - 1 : 0;
    fs = dir ? -1 : 1;
    const int r = row < B ? row : B - 1;
#pragma unroll
    for (int cc = 0; cc < CW; ++cc) {
      const int col = (ADJ && c0 + cc >= B) ? B - 1 : c0 + cc;
      off[cc] = (unsigned)(ADJ ? col * B + r : r * B + col) * (unsigned)sizeof(C);
    }
  }
  // block of forward step t and of backward step t (t clamped to the last step)
  __device__ __forceinline__ int fblk(int t) const { return f0 + fs * (t < n_ ? t : n_ - 1); }
  __device__ __forceinline__ int bblk(int t) const {
    return f0 + fs * (n_ - 2 - (t < n_ - 1 ? t : n_ - 2));
  }

  // slot S <- this thread's slice of the block at element offset blk_off of the line T.  The
  // byte offset is formed in 32 bits (a line's factors are far below 4 GiB) on a uniform base,
  // which maps to scalar-base + 32-bit vector-offset addressing.
  template <int S> __device__ __forceinline__ void load(const C* __restrict__ T, unsigned blk_off) {
    const char* base = reinterpret_cast<const char*>(T);
    const unsigned b0 = blk_off * (unsigned)sizeof(C);
    if constexpr (ADJ) {
#pragma unroll
      for (int cc = 0; cc < CW; ++cc)
        ring[S][cc] = *reinterpret_cast<const C*>(base + (b0 + off[cc]));
    } else {
      const C* p = reinterpret_cast<const C*>(base + (b0 + off[0]));   // contiguous columns
#pragma unroll
      for (int cc = 0; cc < CW; ++cc) ring[S][cc] = p[cc];
    }
  }

  // Ring refills are unconditional: past either end of the line the step is clamped (a
  // re-read of a block of the same line, never used), which keeps the load stream free of
  // branches so the wait counts before each use stay exact.
  template <int S = 0> __device__ __forceinline__ void fill_forward(const C* T, int BB) {
    if constexpr (S < D) {
      load<S>(T, (unsigned)(fblk(S) * BB));
      fill_forward<S + 1>(T, BB);
    }
  }
  template <int S = 0> __device__ __forceinline__ void fill_backward(const C* T, int BB) {
    if constexpr (S < D) {
      load<S>(T, (unsigned)(bblk(S) * BB));
      fill_backward<S + 1>(T, BB);
    }
  }

  // row sum of ring[S] . z over this thread's columns, reduced over the row's NC lanes
  template <int S> __device__ __forceinline__ C dot(const C* z) const {
    C zr[CW];
#pragma unroll
    for (int cc = 0; cc < CW; ++cc) zr[cc] = z[c0 + cc];
    C acc[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = mk((R)0, (R)0);
#pragma unroll
    for (int cc = 0; cc < CW; ++cc)
      acc[cc % NA] = ADJ ? cfma_conj(acc[cc % NA], ring[S][cc], zr[cc])
                         : cfma(acc[cc % NA], ring[S][cc], zr[cc]);
#pragma unroll
    for (int a = 1; a < NA; ++a) acc[0] = cadd(acc[0], acc[a]);
    acc[0].x = lane_sum<NC>(acc[0].x);
    acc[0].y = lane_sum<NC>(acc[0].y);
    return acc[0];
  }

  // Forward step t with ring slot S on block i = fblk(t): y_i = T_i z_i, then the next
  // block's z = q - (coupling to block i) y_i; refills the slot with the block of step t + D.
  // cfw[m] is the coupling of node m to its predecessor in elimination order.  The owner's
  // operands are read before the reduction.
  template <int S> __device__ __forceinline__ void fwd_step(int t, const C* T, int B, int BB,
                                                            C* ybuf, C* zb, const C* cfw) {
    const bool own = owner_lane && row < B;
    const int i = fblk(t), inext = fblk(t + 1);
    C qn = mk((R)0, (R)0), cn = mk((R)0, (R)0);
    if (own) {
      qn = ybuf[inext * B + row];
      cn = cfw[inext + 1];
    }
    const C acc = dot<S>(zb + (t & 1) * ZS);
    load<S>(T, (unsigned)(fblk(t + D) * BB));
    if (own) {
      ybuf[i * B + row] = acc;
      zb[((t + 1) & 1) * ZS + row] = csub(qn, cmul(cn, acc));
    }
    lds_barrier();
  }

  // Backward step t on block i = bblk(t): x_i = y_i - c_i T_i x_prev, with cbw[m] the coupling
  // of node m to its successor in elimination order; refills the slot with step t + D.
  template <int S>
  __device__ __forceinline__ void bwd_step(int t, const C* T, int B, int BB, C* ybuf, C* zb,
                                           const C* cbw) {
    const bool own = owner_lane && row < B;
    const int i = bblk(t);
    C yi = mk((R)0, (R)0), ci = mk((R)0, (R)0);
    if (own) {
      yi = ybuf[i * B + row];
      ci = cbw[i + 1];
    }
    const C acc = dot<S>(zb + (t & 1) * ZS);
    load<S>(T, (unsigned)(bblk(t + D) * BB));
    if (own) {
      const C x = csub(yi, cmul(ci, acc));
      ybuf[i * B + row] = x;
      zb[((t + 1) & 1) * ZS + row] = x;
    }
    lds_barrier();
  }

  template <int S = 0> __device__ __forceinline__ void fwd_group(int t0, const C* T, int B, int BB,
                                                                 C* ybuf, C* zb, const C* cfw) {
    if constexpr (S < D) {
      if (t0 + S < n_) {
        fwd_step<S>(t0 + S, T, B, BB, ybuf, zb, cfw);
        fwd_group<S + 1>(t0, T, B, BB, ybuf, zb, cfw);
      }
    }
  }
  template <int S = 0>
  __device__ __forceinline__ void bwd_group(int t0, const C* T, int B, int BB, C* ybuf, C* zb,
                                            const C* cbw) {
    if constexpr (S < D) {
      if (t0 + S < n_ - 1) {
        bwd_step<S>(t0 + S, T, B, BB, ybuf, zb, cbw);
        bwd_group<S + 1>(t0, T, B, BB, ybuf, zb, cbw);
      }
    }
  }

  // Solve with the factors T (n blocks) on the right-hand side in ybuf[i*B + q]; begin_line
  // and fill_forward must have run, and ybuf must be complete (barrier).  cf[m] / cb[m] are
  // the couplings of x1-node m to m-1 / m+1.  zb holds 2 * ZS values.  On return ybuf holds
  // the solution (visible to the whole workgroup).  No global memory is touched besides the
  // factor stream, so the wait before each ring slot is exact.
  __device__ __forceinline__ void run(const C* T, int B, C* ybuf, C* zb, const C* cf, const C* cb) {
    const int BB = B * B;
    const C* cfw = fs > 0 ? cf : cb;
    const C* cbw = fs > 0 ? cb : cf;
    for (int e = threadIdx.x; e < 2 * ZS; e += blockDim.x) {
      const int q = e < ZS ? e : e - ZS;
      if (q >= B) zb[e] = mk((R)0, (R)0);
    }
    if (owner_lane && row < B) zb[row] = ybuf[fblk(0) * B + row];   // first z = its q
    lds_barrier();
    for (int t0 = 0; t0 < n_; t0 += D)
      fwd_group(__builtin_amdgcn_readfirstlane(t0), T, B, BB, ybuf, zb, cfw);
    fill_backward(T, BB);
    // the last block eliminated: x = y
    if (owner_lane && row < B) zb[row] = ybuf[fblk(n_ - 1) * B + row];
    lds_barrier();
    for (int t0 = 0; t0 < n_ - 1; t0 += D)
      bwd_group(__builtin_amdgcn_readfirstlane(t0), T, B, BB, ybuf, zb, cbw);
  }
};

template <typename R, typename TI, typename TO, int NC, int CW, int D, bool ADJ>
__global__ void __launch_bounds__((NC * NC * CW + 63) / 64 * 64) k_sweep(SweepArgs a) {
  using C = typename cx<R>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = a.n, G = a.G;
  C* ybuf = reinterpret_cast<C*>(smem_raw);
  C* zb = ybuf + (size_t)n * a.maxB;    // [2][NC*CW], zero-padded past B
  C* cf = zb + 2 * kZMax;               // A'[m, m-1], m = 0..n+1
  C* cb = cf + (n + 2);                 // A'[m, m+1]
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
  LineSolver<R, NC, CW, D, ADJ> ls;

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
        const C* T = reinterpret_cast<const C*>(a.factors) + a.line_off[(size_t)g * G + l];
        ls.begin_line(B, n, (g + l) & 1);
        ls.fill_forward(T, B * B);   // in flight while the line input is gathered
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
        ls.run(T, B, ybuf, zb, cf, cb);
        // ---- line output on the group's rows: v = x (inner forward) or v -= x (backward) ----
        const int npy = j1 - j0 + 1;
        for (int e = tid; e < n * Wz * npy; e += NT) {
          const int i = e % n, kk = (e / n) % Wz, jp = e / (n * Wz);
          const int qq = (Wy - npy + jp) * Wz + kk;
          C* p = v + ((long long)kk * n + (j0 + jp - 1)) * n + i;
          *p = ifwd ? ybuf[i * B + qq] : csub(*p, ybuf[i * B + qq]);
        }
        __syncthreads();
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

// Exact solve of a single line problem on its own grid (exposes the building block).
template <typename R, int NC, int CW, int D, bool ADJ>
__global__ void __launch_bounds__((NC * NC * CW + 63) / 64 * 64) k_line_solve(SweepArgs a, int g, int l) {
  using C = typename cx<R>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = a.n, G = a.G;
  C* ybuf = reinterpret_cast<C*>(smem_raw);
  C* zb = ybuf + (size_t)n * a.maxB;
  C* cf = zb + 2 * kZMax;
  C* cb = cf + (n + 2);
  const int tid = threadIdx.x, NT = blockDim.x;
  for (int m = tid; m < n + 2; m += NT) {
    cf[m] = cvt<C>(a.coef[(ADJ ? 2 : 0) * (n + 2) + m]);
    cb[m] = cvt<C>(a.coef[(ADJ ? 3 : 1) * (n + 2) + m]);
  }
  const int Wz = a.groups[g].W, Wy = a.groups[l].W, B = Wy * Wz;
  const double2* r = reinterpret_cast<const double2*>(a.in) + (long long)blockIdx.x * n * B;
  double2* x = reinterpret_cast<double2*>(a.out) + (long long)blockIdx.x * n * B;
  const C* T = reinterpret_cast<const C*>(a.factors) + a.line_off[(size_t)g * G + l];
  LineSolver<R, NC, CW, D, ADJ> ls;
  ls.begin_line(B, n, (g + l) & 1);
  ls.fill_forward(T, B * B);
  for (int e = tid; e < n * B; e += NT) {   // line grid: x1 fastest, then window row, then layer
    const int i = e % n, jj = (e / n) % Wy, kk = e / (n * Wy);
    ybuf[i * B + jj * Wz + kk] = cvt<C>(r[e]);
  }
  __syncthreads();
  ls.run(T, B, ybuf, zb, cf, cb);
  for (int e = tid; e < n * B; e += NT) {
    const int i = e % n, jj = (e / n) % Wy, kk = e / (n * Wy);
    x[e] = cvt<double2>(ybuf[i * B + jj * Wz + kk]);
  }
}

// ------------------------------------------------------------------------------------------
// launch shapes: NC lanes per block row, CW columns per lane (NC * CW >= B), ring depth D
// (registers: D * CW complex values per thread)
// ------------------------------------------------------------------------------------------
struct Shape {
  int nc, cw;
};

Shape choose_shape(int maxB, int lanes) {
  // default: 16 lanes per block row up to B = 48 (measured fastest at B = 36 in both
  // precisions), 4 lanes beyond (16 x 4 columns would not fit the register budget); CW is
  // the smallest instantiated column count covering B
  const int nc = lanes ? lanes : (maxB <= 48 ? 16 : 4);
  const int need = (maxB + nc - 1) / nc;
  static const int cw4[] = {4, 7, 9, 13, 16}, cw8[] = {4, 8}, cw16[] = {1, 2, 3, 4};
  const int* t = nc == 4 ? cw4 : (nc == 8 ? cw8 : cw16);
  const int cnt = nc == 4 ? 5 : (nc == 8 ? 2 : 4);
  for (int k = 0; k < cnt; ++k)
    if (t[k] >= need) return {nc, t[k]};
  return {nc, -1};
}

inline int block_threads(int maxB, int nc) { return ((maxB * nc + 63) / 64) * 64; }

template <typename K, typename... Args>
hipError_t launch_k(K kern, int grid, int threads, size_t sm, hipStream_t s, Args... args) {
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)sm);
  if (e != hipSuccess) return e;
  kern<<<grid, threads, sm, s>>>(args...);
  return hipGetLastError();
}

// the instantiated shapes: (NC, CW, ring depth for complex64, ring depth for complex128)
#define HELM_SHAPES(X)                                                             \
  X(4, 4, 16, 12) X(4, 7, 10, 6) X(4, 9, 8, 4) X(4, 13, 5, 3) X(4, 16, 4, 2)       \
  X(8, 4, 12, 6) X(8, 8, 6, 4) X(16, 1, 16, 16) X(16, 2, 16, 12) X(16, 3, 12, 6)

template <typename R, typename TI, typename TO, bool ADJ>
hipError_t dispatch_sweep(Shape sh, int maxB, int grid, size_t sm, hipStream_t s, SweepArgs a) {
  const int t = block_threads(maxB, sh.nc);
  constexpr bool c64 = sizeof(R) == 4;
#define X(NC, CW, D64, D128)                                                              \
  if (sh.nc == NC && sh.cw == CW)                                                         \
    return launch_k(k_sweep<R, TI, TO, NC, CW, (c64 ? D64 : D128), ADJ>, grid, t, sm, s, a);
  HELM_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
}

template <typename R, bool ADJ>
hipError_t dispatch_line(Shape sh, int maxB, int grid, size_t sm, hipStream_t s, SweepArgs a, int g,
                         int l) {
  const int t = block_threads(maxB, sh.nc);
  constexpr bool c64 = sizeof(R) == 4;
#define X(NC, CW, D64, D128)                                                              \
  if (sh.nc == NC && sh.cw == CW)                                                         \
    return launch_k(k_line_solve<R, NC, CW, (c64 ? D64 : D128), ADJ>, grid, t, sm, s, a, g, l);
  HELM_SHAPES(X)
#undef X
  return hipErrorInvalidValue;
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

size_t sweep_lds(const helm_handle* h, size_t csz) {
  return ((size_t)h->n * h->plan.maxB + 2 * (size_t)kZMax + 2 * (size_t)(h->n + 2)) * csz;
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
  const size_t sm = sweep_lds(h, csz);
  const int mb = h->plan.maxB;
  const Shape sh = choose_shape(mb, h->lanes_override);
  if (sh.cw < 0) return hipErrorInvalidValue;
  if (!r64) return hipErrorInvalidValue;  // inputs are always complex128
  if (!c64 && !z64) return hipErrorInvalidValue;
  hipEvent_t ev = h->t_apply.begin(s);
  hipError_t e;
  if (!c64)
    e = adjoint ? dispatch_sweep<double, double2, double2, true>(sh, mb, R, sm, s, a)
                : dispatch_sweep<double, double2, double2, false>(sh, mb, R, sm, s, a);
  else if (z64)
    e = adjoint ? dispatch_sweep<float, double2, double2, true>(sh, mb, R, sm, s, a)
                : dispatch_sweep<float, double2, double2, false>(sh, mb, R, sm, s, a);
  else
    e = adjoint ? dispatch_sweep<float, double2, float2, true>(sh, mb, R, sm, s, a)
                : dispatch_sweep<float, double2, float2, false>(sh, mb, R, sm, s, a);
  h->t_apply.end(ev, s, R);
  return e;
}

hipError_t launch_line_solve(helm_handle* h, int zg, int yg, const double2* r, double2* x, int R,
                             bool adjoint, hipStream_t s) {
  const bool c64 = h->prec == HELM_C64;
  const size_t csz = c64 ? sizeof(float2) : sizeof(double2);
  SweepArgs a = base_args(h);
  a.in = r;
  a.out = x;
  const size_t sm = sweep_lds(h, csz);
  const int mb = h->plan.maxB;
  const Shape sh = choose_shape(mb, h->lanes_override);
  if (sh.cw < 0) return hipErrorInvalidValue;
  if (c64)
    return adjoint ? dispatch_line<float, true>(sh, mb, R, sm, s, a, zg, yg)
                   : dispatch_line<float, false>(sh, mb, R, sm, s, a, zg, yg);
  return adjoint ? dispatch_line<double, true>(sh, mb, R, sm, s, a, zg, yg)
                 : dispatch_line<double, false>(sh, mb, R, sm, s, a, zg, yg);
}

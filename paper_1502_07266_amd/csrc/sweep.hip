// Application of the recursive sweeping preconditioner, z = M^{-1} r (Algorithm 6 with
// Algorithm 4 inside, each line block solved exactly by its block LDU), and its adjoint.
//
// One workgroup runs the whole sweep for one right-hand side; a launch covers a batch of
// right-hand sides ("persistent": the workgroup loops over every slab and line itself, so the
// sweep's long chain of dependent block steps never returns to the host).  Workgroups of
// different right-hand sides are independent and read the same factor stream.  In the
// two-chain launches a workgroup pair (one per chain of the two-sided line solves) takes the
// place of that workgroup: each member holds the grid points of its half of every line in x1,
// and the two meet once per line solve, at the middle block (SPLIT below).
//
// Data flow for one right-hand side (one front; the two-front outer sweep is below):
//   outer forward  g = 0..G-1 : slab input  f on the group's layers, minus A[k0,k0-1] u[k0-1]
//   outer backward g = G-2..0 : slab input  A[k1,k1+1] u[k1+1] on the group's last layer
//     inner forward  l = 0..G-1 : line input  slab input on the group's rows, minus
//                                              Ht[j0,j0-1] v[j0-1]   (all window layers)
//     inner backward l = G-2..0 : line input  Ht[j1,j1+1] v[j1+1]
//       line solve: two-sided block LDU, y_i = T_i (q_i - l_i y_{i-1}) for the blocks below the
//       middle, y_i = T_i (q_i - u_i y_{i+1}) above it, the middle block last, then
//       x_i = y_i - u_i T_i x_{i+1} below and x_i = y_i - l_i T_i x_{i-1} above
// where v is the slab iterate (n x n x window layers, in global scratch), the line vector
// (n blocks of B = Wy*Wz) lives in LDS, and the T_i stream from HBM.  The adjoint uses the
// couplings of A^H and T_i^H (the same pass order).
//
// Block step: in each of the line's two chains, thread t owns output row t / NC of the B x B
// block and CW consecutive columns;
// the NC partial sums of a row are adjacent lanes of one wavefront and are combined with DPP
// row operations.  The vector a step multiplies (z_i = q_i - l_i y_{i-1} forward, x_{i+1}
// backward) is formed once per row by the row's owner lane and published through a
// double-buffered LDS slot, so one barrier separates consecutive steps.  The factor blocks do
// not depend on the data: each thread keeps its slice of the next D blocks in registers
// (a ring refilled D steps ahead), which hides the HBM latency behind D dependent steps.
//
// Two fronts in x3 (Sec. 4.2 note 3, Sec. 5): three launches.  (1) Two workgroups per
// right-hand side run the fronts concurrently: the lower one x3-groups 0..mid-1 upwards
// (input f - A[k0,k0-1] u[k0-1]), the upper one groups G-1..mid+1 downwards (input
// f - A[k1,k1+1] u[k1+1]).  (2) One workgroup per right-hand side solves the middle slab
// (input f minus both couplings).  (3) The fronts run backwards: the lower one groups
// mid-1..0 (input A[k1,k1+1] u[k1+1], subtracted), the upper one groups mid+1..G-1 (input
// A[k0,k0-1] u[k0-1]).  The launch boundaries order the fronts and the middle slab; inside a
// launch only the members of a workgroup pair wait for each other.  The middle slab's line problems have moving PML on
// both sides in x3 and larger blocks; their factors are in x1 order and each is solved by one
// chain spanning the whole workgroup.
#include <algorithm>

#include "common.h"

namespace {


struct SweepArgs {
  int n, Gz, Gy, maxW, maxB;
  int fronts, zmid, fronts_inner, ymid;
  int pass;              // outer pass over the x3-groups (sweep_count / sweep_at)
  int nfront;            // outer fronts in this launch: workgroups per right-hand side (1, 2)
  int slab_lo, slab_hi;  // the range of the pass's slabs this launch handles
  int ipass;             // inner pass over the x2-groups of each slab
  int ninner;            // inner fronts in this launch (workgroups per outer front: 1, 2)
  int tpc;               // threads per line chain (two chains, or one spanning the workgroup)
  long long N, in_stride, out_stride;
  const GroupInfo* groups;
  const long long* line_off;
  const double2* coef;   // [4][n+2]
  const void* factors;
  const void* in;
  void* out;
  const int* rhs_idx;
  void* scratch;
  // paired workgroups (the SPLIT kernels): workgroups b and b + 8 (xcd_pair, the same XCD under
  // the dispatcher's round-robin) or 2p and 2p + 1 form a pair; per pair and chain an exchange
  // slot of two vectors (by line parity) of kZMax x kXWords tagged words; err is set when a
  // wait times out
  int xcd_pair;
  unsigned long long seq0, seq_span;   // line k of the launch has sequence number seq0 + k + 1
  unsigned long long* xdata;
  int* xerr;
};

// middle-block exchange of a paired line solve: this chain's slot, the other chain's, the
// line's sequence number
struct Xchg {
  unsigned long long* mine;
  const unsigned long long* other;
  unsigned long long seq;
  int* err;
};

// polls of a partner's word before a paired line solve gives up (each poll a device-memory
// round trip and a short sleep: on the order of a second): the pair is co-resident
// (cooperative launch), so only a fault elsewhere can exhaust it
constexpr unsigned kSpinLimit = 1u << 20;

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

// Loads from the factor array through an explicitly global pointer (global_load, counted by
// vmcnt only; a generic pointer would give flat loads, which also count against lgkmcnt and
// would make every LDS wait drain the factor ring).
#define HELM_GLOBAL __attribute__((address_space(1)))
template <typename R> struct vec2 { using type = R __attribute__((ext_vector_type(2))); };
template <typename R>
__device__ __forceinline__ typename cx<R>::type load_global(const HELM_GLOBAL char* base, unsigned off) {
  using V = typename vec2<R>::type;
  const V v = *reinterpret_cast<const HELM_GLOBAL V*>(base + off);
  return mk(v.x, v.y);
}

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations, then
// s_barrier.  Unlike __syncthreads() it does not wait for outstanding global loads, so the
// factor ring stays in flight across block steps.  Global scratch written around a line
// solve is published with full __syncthreads() by the caller.
__device__ __forceinline__ void lds_barrier() {
  __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Two-sided line solve.  The factors eliminate the blocks of a line from both ends towards the
// middle block mid = n/2 (integer division).  Step t (t = 0..2 mid) of a chain handles block
//     upper chain (threads [0, tpc))      : i = mid - |mid - t|
//     lower chain (threads [tpc, 2 tpc))  : i = mid + |mid - t|
// forward elimination for t < mid, the middle block at t = mid (both chains compute it, from
// the sum of their two partial right-hand sides), back-substitution for t > mid.  The lower
// chain has no block when i > n - 1 (t = 0 and t = 2 mid for even n).  One barrier per step:
// a line takes 2 mid + 1 steps (n for odd n) instead of the 2n - 1 of a one-sided sweep.
//
// A wave issues one instruction every few cycles and the scalar unit is shared by all waves of
// the compute unit, so the step is kept free of per-step bookkeeping: a per-line table gives,
// for each chain and step, the LDS rows to read and write and the factor block to prefetch,
// and every lane of a block row writes the row's (identical) result, so no lane masking is
// needed.  Steps without a destination write to a junk row.
template <typename R, int NC, int CW, int D, bool ADJ, int CH, bool SPLIT = false>
struct LineSolver {
  static_assert(!SPLIT || CH == 2, "only two-chain line solves are split over a workgroup pair");
  using C = typename cx<R>::type;
  static constexpr int ZS = NC * CW;   // stride of one published vector (>= B, zero-padded)
  static_assert(D % 2 == 0, "the ring depth must be even (published-vector parity per slot)");
  static_assert(ZS <= kZMax, "published vector longer than its LDS slot");
  C ring[D][CW];
  unsigned off0;                       // this thread's byte offset inside a B x B block
  unsigned offa[ADJ ? CW : 1];         // adjoint walk: one offset per column
  int row, rowc, c0;
  int lower;                           // 0 upper chain, 1 lower chain (uniform in a wave)
  // per line (uniform)
  int n_, mid, B_, steps;
  unsigned BBb;                        // bytes of one factor block
  const HELM_GLOBAL char* Tb;          // factors of the line
  // per step, carried one step ahead: table entry of this and the next step, the owner
  // operand and the coupling of this step
  int4 ecur, enext;
  C Acur, ccur;

  // tpc: threads per chain, a multiple of the wavefront size; half: the chain of a paired
  // workgroup (SPLIT: the workgroup is that one chain)
  __device__ __forceinline__ LineSolver(int tpc, int half) {
    lower = SPLIT ? half : __builtin_amdgcn_readfirstlane((int)threadIdx.x >= tpc ? 1 : 0);
    const int lt = SPLIT ? (int)threadIdx.x : (int)threadIdx.x - lower * tpc;
    row = lt / NC;
    c0 = (lt - row * NC) * CW;
  }

  // per-line set-up.  Rows past B are clamped to row B - 1 (they compute and write that row's
  // values again).  Columns past B meet zero padding of the published vector: in the
  // row-major (non-adjoint) walk they run into the next row, or past the last block into the
  // padding that follows the factor array, so they read finite values; the adjoint walk
  // clamps them.
  __device__ __forceinline__ void begin_line(const C* T, int B, int n, int line_mid) {
    n_ = n;
    B_ = B;
    mid = line_mid;
    steps = 2 * mid + 1;
    BBb = (unsigned)(B * B) * (unsigned)sizeof(C);
    const unsigned long long tp = reinterpret_cast<unsigned long long>(T);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)tp);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(tp >> 32));
    Tb = (const HELM_GLOBAL char*)(((unsigned long long)hi << 32) | lo);
    rowc = row < B ? row : B - 1;
    off0 = (unsigned)(rowc * B + c0) * (unsigned)sizeof(C);
    if constexpr (ADJ) {
#pragma unroll
      for (int cc = 0; cc < CW; ++cc) {
        const int col = c0 + cc >= B ? B - 1 : c0 + cc;
        offa[cc] = (unsigned)(col * B + rowc) * (unsigned)sizeof(C);
      }
    }
  }

  // block of step t of chain ch, clamped to the line
  __device__ __forceinline__ int blk(int ch, int t) const {
    const int d = mid > t ? mid - t : t - mid;
    const int i = ch ? mid + d : mid - d;
    return i < 0 ? 0 : (i > n_ - 1 ? n_ - 1 : i);
  }

  // slot S <- this thread's slice of the factor block at byte offset b0 of the line: a uniform
  // base plus 32-bit vector offsets (a line's factors are far below 4 GiB); the non-adjoint
  // columns are contiguous and share one offset register.
  template <int S> __device__ __forceinline__ void load(unsigned b0) {
    if constexpr (ADJ) {
#pragma unroll
      for (int cc = 0; cc < CW; ++cc) ring[S][cc] = load_global<R>(Tb, b0 + offa[cc]);
    } else {
      using V = typename vec2<R>::type;
      const HELM_GLOBAL V* p = reinterpret_cast<const HELM_GLOBAL V*>(Tb + (b0 + off0));
#pragma unroll
      for (int cc = 0; cc < CW; ++cc) {
        const V w = p[cc];
        ring[S][cc] = mk(w.x, w.y);
      }
    }
  }

  template <int S = 0> __device__ __forceinline__ void fill() {
    if constexpr (S < D) {
      load<S>((unsigned)blk(lower, S) * BBb);
      fill<S + 1>();
    }
  }

  // row sum of ring[S] . z over this thread's columns, reduced over the row's NC lanes; even
  // and odd columns go to two accumulators, which halves the dependent FMA chain of the wide
  // shapes
  template <int S> __device__ __forceinline__ C first(int cc, const C (&zr)[CW]) const {
    return ADJ ? mk(ring[S][cc].x * zr[cc].x + ring[S][cc].y * zr[cc].y,
                    ring[S][cc].x * zr[cc].y - ring[S][cc].y * zr[cc].x)
               : cmul(ring[S][cc], zr[cc]);
  }
  template <int S> __device__ __forceinline__ C dot(const C (&zr)[CW]) const {
    C acc = first<S>(0, zr);
    if constexpr (CW >= 4) {
      C acc1 = first<S>(1, zr);
#pragma unroll
      for (int cc = 2; cc < CW; ++cc) {
        C& a = (cc & 1) ? acc1 : acc;
        a = ADJ ? cfma_conj(a, ring[S][cc], zr[cc]) : cfma(a, ring[S][cc], zr[cc]);
      }
      acc = cadd(acc, acc1);
    } else {
#pragma unroll
      for (int cc = 1; cc < CW; ++cc)
        acc = ADJ ? cfma_conj(acc, ring[S][cc], zr[cc]) : cfma(acc, ring[S][cc], zr[cc]);
    }
    acc.x = lane_sum<NC>(acc.x);
    acc.y = lane_sum<NC>(acc.y);
    return acc;
  }

  // Step t with ring slot S (parity of t = parity of S):
  //   forward  y_i = T_i z_i; the next published vector is q_next - c y_i (the lower chain
  //            leaves q_mid out: the upper chain's partial right-hand side of the middle block
  //            has it)
  //   middle   x_mid = T_mid (z_upper + z_lower), published by both chains
  //   backward x_i = y_i - c T_i x_prev, published
  // i.e. P = A - c acc with the table's operand row A and coupling c (A = 0, c = -1 in the
  // middle); the block row gets acc (forward) or P.  sb is the LDS base the table indexes.
  template <int S>
  __device__ __forceinline__ void step(int t, C* sb, const C* zme, const C* zot, const int4* tab,
                                       const C* ctab) {
    constexpr int par = (S & 1) * ZS;
    C zr[CW];
#pragma unroll
    for (int cc = 0; cc < CW; ++cc) zr[cc] = zme[par + c0 + cc];
    if (t == mid) {
#pragma unroll
      for (int cc = 0; cc < CW; ++cc) zr[cc] = cadd(zr[cc], zot[par + c0 + cc]);
    }
    const int4 e2 = tab[t + 2];
    const C cn = ctab[t + 1];
    const C acc = dot<S>(zr);
    load<S>((unsigned)ecur.w);
    const C P = csub(Acur, cmul(ccur, acc));
    // component-wise select (a select of whole complex128 values is lowered through scratch)
    const bool fwd = t < mid;
    C out;
    out.x = fwd ? acc.x : P.x;
    out.y = fwd ? acc.y : P.y;
    sb[ecur.y + rowc] = out;
    sb[ecur.z + rowc] = P;
    Acur = sb[enext.x + rowc];   // operand of step t + 1 (never written by step t)
    ccur = cn;
    ecur = enext;
    enext = e2;
    lds_barrier();
  }

  // D consecutive steps, one per ring slot, with no branch between them: the loop over such
  // groups has a single path, so the wait before each slot's use covers exactly the loads
  // issued D steps earlier (with early exits between the steps, the merged paths would make
  // the first step of every group wait for the whole ring)
  template <int S = 0>
  __device__ __forceinline__ void group(int t0, C* sb, const C* zme, const C* zot, const int4* tab,
                                        const C* ctab) {
    if constexpr (S < D) {
      step<S>(t0 + S, sb, zme, zot, tab, ctab);
      group<S + 1>(t0, sb, zme, zot, tab, ctab);
    }
  }
  // steps t0 + S .. end - 1 of a group that ends early (end - t0 < D)
  template <int S = 0>
  __device__ __forceinline__ void tail(int t0, int end, C* sb, const C* zme, const C* zot,
                                       const int4* tab, const C* ctab) {
    if constexpr (S < D) {
      if (t0 + S < end) {
        step<S>(t0 + S, sb, zme, zot, tab, ctab);
        tail<S + 1>(t0, end, sb, zme, zot, tab, ctab);
      }
    }
  }
  // steps t0 + s0 .. min(t0 + D, end) - 1 of a group entered at slot s0 (after the exchange)
  template <int S = 0>
  __device__ __forceinline__ void head(int t0, int s0, int end, C* sb, const C* zme,
                                       const C* zot, const int4* tab, const C* ctab) {
    if constexpr (S < D) {
      if (S >= s0) {
        if (t0 + S >= end) return;
        step<S>(t0 + S, sb, zme, zot, tab, ctab);
      }
      head<S + 1>(t0, s0, end, sb, zme, zot, tab, ctab);
    }
  }

  // Paired line solve, before the middle step: publish this chain's partial right-hand side of
  // the middle block (its published vector of step mid) to the partner and take the partner's
  // into the LDS slot the middle step reads.  Each 32-bit piece of a value travels in one
  // 64-bit word together with the line's sequence number (a relaxed device-scope atomic store
  // and load), so a word read with the expected tag holds this line's piece and no fence is
  // needed (a device-scope fence would write back and invalidate the L2 that the right-hand
  // sides' workgroups share the factor stream through).  A piece whose tag never arrives (a
  // fault elsewhere) is replaced by NaN, so the solution is NaN rather than silently wrong,
  // and err is raised.
  __device__ __forceinline__ void exchange(C* sb, int zb, const Xchg& x) {
    using W = unsigned long long;
    constexpr int np = sizeof(C) / 4;                  // 32-bit pieces per value
    const int par = (mid & 1) * ZS;
    const C* mine = sb + zb + lower * 2 * ZS + par;
    C* other = sb + zb + (1 - lower) * 2 * ZS + par;
    const W tag = (x.seq & 0xffffffffull) << 32;
    for (int e = threadIdx.x; e < B_ * np; e += blockDim.x) {
      const unsigned* src = reinterpret_cast<const unsigned*>(mine);
      __hip_atomic_store(x.mine + e, tag | src[e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    unsigned* dst = reinterpret_cast<unsigned*>(other);
    for (int e = threadIdx.x; e < B_ * np; e += blockDim.x) {
      unsigned spins = 0;
      W w = __hip_atomic_load(x.other + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      while ((w & 0xffffffff00000000ull) != tag) {
        if (++spins > kSpinLimit) {
          __hip_atomic_store(x.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          w = 0x7fc00000u;   // a quiet NaN in either half of a value
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        w = __hip_atomic_load(x.other + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      dst[e] = (unsigned)w;
    }
    lds_barrier();
  }

  // Solve on the right-hand side in ybuf[i*B + q]; begin_line and fill must have run, and
  // ybuf must be complete (barrier).  All LDS regions are given as element offsets from sb:
  // zb (4 ZS values: two double-buffered published vectors per chain), zeros and junk (kZMax
  // values each), ctab (2 (n + 2) couplings), tab (2 (n + 3) entries, 16 bytes each).  On
  // return ybuf holds the solution (visible to the whole workgroup).  No global memory is
  // touched besides the factor stream, so the wait before each ring slot is exact.
  __device__ __forceinline__ void run(C* sb, int ybuf, int zb, int zeros, int junk, C* ctab,
                                      int4* tab, const C* cf, const C* cb,
                                      const Xchg* xc = nullptr) {
    const C zero = mk((R)0, (R)0);
    const int B = B_, ts = steps + 2;   // table entries per chain (CH * ts <= 2 (n + 3))
    for (int e = threadIdx.x; e < 4 * ZS; e += blockDim.x)
      if (e % ZS >= B) sb[zb + e] = zero;
    // per chain and step: couplings (forward upper l_{i+1}, lower u_{i-1}; backward upper u_i,
    // lower l_i; middle -1; block i is x1-node i + 1: l_i = cf[i + 1], u_i = cb[i + 1]) and
    // the table {operand row, result row, published-vector row, prefetch offset}
    for (int e = threadIdx.x; e < CH * ts; e += blockDim.x) {
      const int ch = e >= ts, t = e - ch * ts;
      const int d = mid > t ? mid - t : t - mid;
      const int i = ch ? mid + d : mid - d;
      const bool valid = t < steps && i >= 0 && i < n_;
      const int znext = zb + (2 * ch + ((t + 1) & 1)) * ZS;
      C c = mk((R)-1, (R)0);
      int4 en = make_int4(zeros, junk, junk, (int)((unsigned)blk(ch, t + D) * BBb));
      if (t < mid) {
        c = ch ? cb[i] : cf[i + 2];
        const bool last_lower = ch && t == mid - 1;
        if (valid) {
          en.x = last_lower ? zeros : ybuf + (ch ? i - 1 : i + 1) * B;
          en.y = ybuf + i * B;
          en.z = znext;
        } else if (ch && i == n_) {
          en.x = ybuf + (n_ - 1) * B;   // (even n, t = 0: the lower chain has no block yet)
        }
      } else if (t == mid) {
        en.y = ch ? junk : ybuf + mid * B;
        en.z = znext;
      } else if (valid) {
        c = ch ? cf[i + 1] : cb[i + 1];
        en.x = ybuf + i * B;
        en.y = ybuf + i * B;
        en.z = znext;
      }
      ctab[e] = c;
      tab[e] = en;
    }
    // each chain starts from the q of its first block; without lower blocks (mid = n - 1) the
    // lower chain's published vectors stay zero, so the middle step adds nothing
    if (mid == n_ - 1)
      for (int e = threadIdx.x; e < 2 * ZS; e += blockDim.x) sb[zb + 2 * ZS + e] = zero;
    lds_barrier();
    if (row < B) {
      if (!lower) sb[zb + row] = sb[ybuf + row];
      else if (mid < n_ - 1) sb[zb + (2 + ((2 * mid - n_ + 1) & 1)) * ZS + row] = sb[ybuf + (n_ - 1) * B + row];
    }
    lds_barrier();
    const int4* tb = tab + lower * ts;
    const C* ct = ctab + lower * ts;
    ecur = tb[0];
    enext = tb[1];
    ccur = ct[0];
    Acur = sb[ecur.x + rowc];
    const C* zme = sb + zb + lower * 2 * ZS;
    const C* zot = sb + zb + (1 - lower) * 2 * ZS;
    if constexpr (!SPLIT) {
      const int full = steps - steps % D;
      int t0 = 0;
      for (; t0 < full; t0 += D) group(__builtin_amdgcn_readfirstlane(t0), sb, zme, zot, tb, ct);
      if (t0 < steps) tail(__builtin_amdgcn_readfirstlane(t0), steps, sb, zme, zot, tb, ct);
    } else {
      // forward steps 0 .. mid - 1, the exchange, then mid .. steps - 1 continuing the ring
      // slots where the forward steps left them (step t always uses slot t % D)
      int t0 = 0;
      for (; t0 + D <= mid; t0 += D) group(__builtin_amdgcn_readfirstlane(t0), sb, zme, zot, tb, ct);
      if (t0 < mid) tail(__builtin_amdgcn_readfirstlane(t0), mid, sb, zme, zot, tb, ct);
      exchange(sb, zb, *xc);
      t0 = mid - mid % D;
      if (t0 < mid) {
        head(__builtin_amdgcn_readfirstlane(t0), mid - t0, steps, sb, zme, zot, tb, ct);
        t0 += D;
      }
      for (; t0 + D <= steps; t0 += D) group(__builtin_amdgcn_readfirstlane(t0), sb, zme, zot, tb, ct);
      if (t0 < steps) tail(__builtin_amdgcn_readfirstlane(t0), steps, sb, zme, zot, tb, ct);
    }
  }
};

// threads of a launch: CH chains (2, or 1 spanning the workgroup) of round-up-to-64(B * NC)
template <int NC, int CW, int CH> constexpr int max_threads() { return CH * ((NC * NC * CW + 63) / 64 * 64); }

// SPLIT: each line's two chains run in a pair of workgroups, one chain each, on the grid
// points of their own half of the line in x1 (blocks 0..mid and mid+1..n-1); the pair
// exchanges one B-vector per line solve (the middle block's partial right-hand sides) and is
// otherwise independent, since every coupling outside a line solve joins points of the same x1
template <typename R, typename TI, typename TO, int NC, int CW, int D, bool ADJ, int CH,
          bool SPLIT = false>
__global__ void __launch_bounds__((max_threads<NC, CW, SPLIT ? 1 : CH>())) k_sweep(SweepArgs a) {
  using C = typename cx<R>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = a.n, Gz = a.Gz, Gy = a.Gy;
  const LdsLayout L(n, a.maxB, (int)sizeof(C));
  C* sb = reinterpret_cast<C*>(smem_raw);
  C* ybuf = sb + L.ybuf;
  C* zeros = sb + L.zeros;
  C* cf = sb + L.cf;                    // A'[m, m-1], m = 0..n+1
  C* cb = sb + L.cb;                    // A'[m, m+1]
  C* ctab = sb + L.ctab;
  int4* tab = reinterpret_cast<int4*>(smem_raw + L.tab_byte);
  const int tid = threadIdx.x, NT = blockDim.x;
  // workgroup = (right-hand side, outer front, inner front); the inner fronts of one outer
  // front share its slab iterate and write disjoint rows of it
  int half = 0, bid = (int)blockIdx.x;
  if constexpr (SPLIT) {
    const int b = (int)blockIdx.x;
    half = a.xcd_pair ? (b >> 3) & 1 : b & 1;
    bid = a.xcd_pair ? ((b >> 4) << 3) | (b & 7) : b >> 1;
  }
  const int fw = bid / a.ninner, ifront = bid - fw * a.ninner;
  // the x1 range of this workgroup's grid points: the whole line, or its chain's half
  const int ilo = SPLIT && half ? n / 2 + 1 : 0;
  const int ni = SPLIT ? (half ? n - (n / 2 + 1) : n / 2 + 1) : n;
  const int slot = fw / a.nfront, front = fw - slot * a.nfront;
  const int q = a.rhs_idx ? a.rhs_idx[slot] : slot;
  const TI* __restrict__ f = reinterpret_cast<const TI*>(a.in) + (long long)q * a.in_stride;
  TO* u = reinterpret_cast<TO*>(a.out) + (long long)q * a.out_stride;
  C* v = reinterpret_cast<C*>(a.scratch) + (long long)fw * n * n * a.maxW;
  const C zero = mk((R)0, (R)0);
  for (int m = tid; m < n + 2; m += NT) {
    cf[m] = cvt<C>(a.coef[(ADJ ? 2 : 0) * (n + 2) + m]);
    cb[m] = cvt<C>(a.coef[(ADJ ? 3 : 1) * (n + 2) + m]);
  }
  for (int m = tid; m < kZMax; m += NT) zeros[m] = mk((R)0, (R)0);
  __syncthreads();
  auto gidx = [&](int i, int j, int k) -> long long {  // i 0-based, j, k 1-based
    return ((long long)(k - 1) * n + (j - 1)) * n + i;
  };
  LineSolver<R, NC, CW, D, ADJ, CH, SPLIT> ls(a.tpc, half);
  Xchg xc{};
  if constexpr (SPLIT) {
    xc.err = a.xerr;
    xc.mine = a.xdata + (size_t)(2 * bid + half) * 2 * kXSlot;
    xc.other = a.xdata + (size_t)(2 * bid + 1 - half) * 2 * kXSlot;
  }
  unsigned long long lcount = 0;   // lines solved so far in this launch

  const int nslab = min(a.slab_hi, sweep_count(a.pass, Gz, a.zmid, front));
  const int nline = sweep_count(a.ipass, Gy, a.ymid, ifront);
  for (int si = a.slab_lo; si < nslab; ++si) {
    {
      const int2 gk = sweep_at(a.pass, Gz, a.zmid, front, si);
      const int g = gk.x, kind = gk.y;
      const bool ofwd = kind <= kFwdMid;
      // couplings of the slab input: from the layer below (k0 - 1) and/or above (k1 + 1)
      const bool from_below = (kind == kFwdLow && g > 0) || kind == kFwdMid || kind == kBwdHigh;
      const bool from_above = (kind == kFwdHigh && g < Gz - 1) || kind == kFwdMid || kind == kBwdLow;
      const GroupInfo gz = a.groups[g];
      const int Wz = gz.W, k0 = gz.first, k1 = gz.last, zw0 = gz.w0;
      for (int lp = 0; lp < nline; ++lp) {
        const int2 lk = sweep_at(a.ipass, Gy, a.ymid, ifront, lp);
        const int l = lk.x, lkind = lk.y;
        const bool ifwd = lkind <= kFwdMid;
        // couplings of the line input: forward, the new iterate on the row below (j0 - 1)
        // and/or above (j1 + 1) is subtracted; backward, the input is the coupling to the row
        // above (lower front) or below (upper front)
        const bool in_below = (lkind == kFwdLow && l > 0) || lkind == kFwdMid;
        const bool in_above = (lkind == kFwdHigh && l < Gy - 1) || lkind == kFwdMid;
        const GroupInfo gy = a.groups[Gz + l];
        const int Wy = gy.W, B = Wy * Wz, j0 = gy.first, j1 = gy.last, yw0 = gy.w0;
        const C* T = reinterpret_cast<const C*>(a.factors) + a.line_off[(size_t)g * Gy + l];
        // every line of a launch has the elimination order of the launch's chain count (the
        // plan makes the lines of a launch agree): x1 order with one chain, two-sided with two
        ls.begin_line(T, B, n, CH == 1 ? n - 1 : n / 2);
        ls.fill();   // in flight while the line input is gathered
        for (int e = tid; e < ni * B; e += NT) {
          const int qq = e / ni, i = ilo + e - qq * ni;
          const int jj = qq / Wz, kk = qq - jj * Wz;
          const int j = yw0 + jj, k = zw0 + kk;
          C val = zero;
          if (ifwd) {
            if (j >= j0 && j <= j1) {
              if (ofwd) {
                if (k >= k0 && k <= k1) {
                  val = cvt<C>(f[gidx(i, j, k)]);
                  if (from_below && k == k0) val = csub(val, cmul(cf[k0], cvt<C>(u[gidx(i, j, k0 - 1)])));
                  if (from_above && k == k1) val = csub(val, cmul(cb[k1], cvt<C>(u[gidx(i, j, k1 + 1)])));
                }
              } else if (from_above && k == k1) {
                val = cmul(cb[k1], cvt<C>(u[gidx(i, j, k1 + 1)]));
              } else if (from_below && k == k0) {
                val = cmul(cf[k0], cvt<C>(u[gidx(i, j, k0 - 1)]));
              }
              if (in_below && j == j0) val = csub(val, cmul(cf[j0], v[((long long)kk * n + (j0 - 2)) * n + i]));
              if (in_above && j == j1) val = csub(val, cmul(cb[j1], v[((long long)kk * n + j1) * n + i]));
            }
          } else if (lkind == kBwdLow && j == j1) {
            val = cmul(cb[j1], v[((long long)kk * n + j1) * n + i]);
          } else if (lkind == kBwdHigh && j == j0) {
            val = cmul(cf[j0], v[((long long)kk * n + (j0 - 2)) * n + i]);
          }
          ybuf[i * B + qq] = val;
        }
        __syncthreads();
        if constexpr (SPLIT) {
          Xchg x = xc;
          const int par = (int)(lcount & 1);
          x.mine += par * kXSlot;
          x.other += par * kXSlot;
          x.seq = a.seq0 + lcount + 1;
          // (a launch past its span would share tags with the next launch: reported)
          if (lcount + 1 > a.seq_span && tid == 0)
            __hip_atomic_store(a.xerr, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ls.run(sb, L.ybuf, L.zb, L.zeros, L.junk, ctab, tab, cf, cb, &x);
        } else {
          ls.run(sb, L.ybuf, L.zb, L.zeros, L.junk, ctab, tab, cf, cb);
        }
        ++lcount;
        // ---- line output on the group's rows: v = x (inner forward) or v -= x (backward) ----
        const int npy = j1 - j0 + 1;
        for (int e = tid; e < ni * Wz * npy; e += NT) {
          const int i = ilo + e % ni, kk = (e / ni) % Wz, jp = e / (ni * Wz);
          const int qq = (j0 - yw0 + jp) * Wz + kk;
          C* p = v + ((long long)kk * n + (j0 + jp - 1)) * n + i;
          *p = ifwd ? ybuf[i * B + qq] : csub(*p, ybuf[i * B + qq]);
        }
        __syncthreads();
      }
      // ---- slab output on the group's layers, on the rows final after this inner pass: all
      // of them (one inner front), the middle x2-group's (middle line), the rows of the lines
      // this workgroup swept backwards (two inner fronts) ----
      int r0 = 1, r1 = n;
      if (a.ipass == 1) {
        r1 = 0;
      } else if (a.ipass == 2) {
        r0 = a.groups[Gz + a.ymid].first;
        r1 = a.groups[Gz + a.ymid].last;
      } else if (a.ipass == 3) {
        if (ifront == 0) r1 = a.groups[Gz + a.ymid - 1].last;
        else r0 = a.groups[Gz + a.ymid + 1].first;
      }
      const int nph = k1 - k0 + 1, nr = r1 - r0 + 1;
      for (int e = tid; e < ni * nr * nph; e += NT) {
        const int i = ilo + e % ni, jm = r0 - 1 + (e / ni) % nr, kp = e / (ni * nr);
        const int kk = k0 - zw0 + kp;
        const C val = v[((long long)kk * n + jm) * n + i];
        const long long id = gidx(i, jm + 1, k0 + kp);
        u[id] = ofwd ? cvt<TO>(val) : cvt<TO>(csub(cvt<C>(u[id]), val));
      }
      __syncthreads();
    }
  }
}

// Exact solve of a single line problem on its own grid (exposes the building block).
template <typename R, int NC, int CW, int D, bool ADJ, int CH>
__global__ void __launch_bounds__((max_threads<NC, CW, CH>())) k_line_solve(SweepArgs a, int g, int l) {
  using C = typename cx<R>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = a.n, Gy = a.Gy;
  const LdsLayout L(n, a.maxB, (int)sizeof(C));
  C* sb = reinterpret_cast<C*>(smem_raw);
  C* ybuf = sb + L.ybuf;
  C* zeros = sb + L.zeros;
  C* cf = sb + L.cf;                    // A'[m, m-1], m = 0..n+1
  C* cb = sb + L.cb;                    // A'[m, m+1]
  C* ctab = sb + L.ctab;
  int4* tab = reinterpret_cast<int4*>(smem_raw + L.tab_byte);
  const int tid = threadIdx.x, NT = blockDim.x;
  for (int m = tid; m < n + 2; m += NT) {
    cf[m] = cvt<C>(a.coef[(ADJ ? 2 : 0) * (n + 2) + m]);
    cb[m] = cvt<C>(a.coef[(ADJ ? 3 : 1) * (n + 2) + m]);
  }
  for (int m = tid; m < kZMax; m += NT) zeros[m] = mk((R)0, (R)0);
  const int Wz = a.groups[g].W, Wy = a.groups[a.Gz + l].W, B = Wy * Wz;
  const double2* r = reinterpret_cast<const double2*>(a.in) + (long long)blockIdx.x * n * B;
  double2* x = reinterpret_cast<double2*>(a.out) + (long long)blockIdx.x * n * B;
  const C* T = reinterpret_cast<const C*>(a.factors) + a.line_off[(size_t)g * Gy + l];
  LineSolver<R, NC, CW, D, ADJ, CH> ls(a.tpc, 0);
  ls.begin_line(T, B, n, CH == 1 ? n - 1 : n / 2);   // the host picks CH from the line
  ls.fill();
  for (int e = tid; e < n * B; e += NT) {   // line grid: x1 fastest, then window row, then layer
    const int i = e % n, jj = (e / n) % Wy, kk = e / (n * Wy);
    ybuf[i * B + jj * Wz + kk] = cvt<C>(r[e]);
  }
  __syncthreads();
  ls.run(sb, L.ybuf, L.zb, L.zeros, L.junk, ctab, tab, cf, cb);
  for (int e = tid; e < n * B; e += NT) {
    const int i = e % n, jj = (e / n) % Wy, kk = e / (n * Wy);
    x[e] = cvt<double2>(ybuf[i * B + jj * Wz + kk]);
  }
}

// ------------------------------------------------------------------------------------------
// launch shapes: NC lanes per block row, CW columns per lane (NC * CW >= B), ring depth D
// (registers: D * CW complex values per thread); two chains of round-up-to-64(B * NC) threads
// ------------------------------------------------------------------------------------------
struct Shape {
  int nc, cw;
};

// the instantiated shapes: (NC, CW, ring depth for complex64, ring depth for complex128),
// depths sized so that the ring fits the register budget of the shape's largest launch; depth
// 0: not built (complex128 with 8 x 7 or 8 x 8 columns leaves no registers for a ring)
#define HELM_SHAPES(X)                                                                  \
  X(4, 5, 16, 12) X(4, 7, 16, 12) X(4, 9, 8, 4) X(4, 13, 6, 2) X(4, 16, 4, 2)          \
  X(8, 3, 16, 12) X(8, 4, 16, 10) X(8, 5, 8, 4) X(8, 7, 4, 0) X(8, 8, 2, 0)            \
  X(16, 1, 16, 16) X(16, 2, 16, 8)
// the shape is instantiated for this precision
bool shape_built(Shape sh, bool c64) {
#define X(NC, CW, D64, D128) \
  if (sh.nc == NC && sh.cw == CW) return (c64 ? D64 : D128) > 0;
  HELM_SHAPES(X)
#undef X
  return false;
}

Shape choose_shape(int maxB, int lanes, bool c64) {
  // default: 8 lanes per block row (measured fastest for two chains at B = 36, 49 and 64 in
  // complex64, although 8 x 7 and 8 x 8 columns leave registers for a ring of only 4 and 2
  // blocks; in complex128 they leave none, so 4 lanes beyond B = 40); 16 lanes only fit two
  // chains in one workgroup up to B = 32.  CW is the smallest instantiated column count
  // covering B.
  if (maxB > kTwoChainMaxB64) return Shape{4, -1};
  const int nc = lanes ? lanes : ((c64 || maxB <= 40) ? 8 : 4);
  if (lanes) {   // an override without a shape for this block and precision: automatic
    const Shape sh = choose_shape(maxB, 0, c64);
    const int need = (maxB + nc - 1) / nc;
    for (int cw = need; cw <= 20; ++cw)
      if (shape_built(Shape{nc, cw}, c64)) return Shape{nc, cw};
    return sh;
  }
  const int need = (maxB + nc - 1) / nc;
  static const int cw4[] = {5, 7, 9, 13, 16}, cw8[] = {3, 4, 5, 7, 8}, cw16[] = {1, 2};
  const int* t = nc == 4 ? cw4 : (nc == 8 ? cw8 : cw16);
  const int cnt = nc == 16 ? 2 : 5;
  for (int k = 0; k < cnt; ++k)
    if (t[k] >= need) return {nc, t[k]};
  return {nc, -1};
}

inline int chain_threads(int maxB, int nc) { return ((maxB * nc + 63) / 64) * 64; }

template <typename K, typename... Args>
hipError_t launch_k(K kern, int grid, int threads, size_t sm, hipStream_t s, Args... args) {
  hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)sm);
  if (e != hipSuccess) return e;
  kern<<<grid, threads, sm, s>>>(args...);
  return hipGetLastError();
}

// one chain spanning the workgroup (lines on a middle group, blocks up to 128): 8 lanes per
// row
#define HELM_SHAPES_ONE(X) \
  X(8, 3, 16, 12) X(8, 6, 8, 6) X(8, 9, 4, 2) X(8, 10, 4, 2) X(8, 11, 4, 2) X(8, 12, 2, 2)    \
  X(8, 16, 2, 0)

Shape choose_shape_one(int maxB) {
  static const int cw[] = {3, 6, 9, 10, 11, 12, 16};
  for (int c : cw)
    if (8 * c >= maxB) return {8, c};
  return {8, -1};
}

// A two-chain launch of `grid` line-solving workgroups.  With exchange buffers (a.xdata) and
// room for every pair to be resident at once, the SPLIT kernel runs on 2 grid workgroups of
// one chain each, launched cooperatively (the runtime refuses a cooperative grid that cannot
// be co-resident, so no workgroup waits for a partner that is not running); otherwise one
// workgroup runs both chains of a line.
template <typename K1, typename K2>
hipError_t launch_two(K1 pair_kern, K2 kern, int grid, int tpc, size_t sm, hipStream_t s,
                      SweepArgs a) {
  if (a.xdata) {
    int dev = 0, coop = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)pair_kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e == hipSuccess)
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)pair_kern, tpc, sm);
    if (e != hipSuccess) return e;
    if (coop && (long long)per_cu * cus >= 2LL * grid) {
      a.xcd_pair = grid % 8 == 0;
      void* args[] = {&a};
      e = hipLaunchCooperativeKernel((const void*)pair_kern, dim3(2 * grid), dim3(tpc), args,
                                     (unsigned)sm, s);
      if (e != hipErrorCooperativeLaunchTooLarge) return e != hipSuccess ? e : hipGetLastError();
      (void)hipGetLastError();   // refused (not all resident): run unpaired
    }
  }
  return launch_k(kern, grid, 2 * tpc, sm, s, a);
}

template <typename R, typename TI, typename TO, bool ADJ>
hipError_t dispatch_sweep(Shape sh, int chains, int grid, size_t sm, hipStream_t s, SweepArgs a) {
  constexpr bool c64 = sizeof(R) == 4;
  if (chains == 2) {
#define X(NC, CW, D64, D128)                                                              \
    if (sh.nc == NC && sh.cw == CW) {                                                     \
      if constexpr ((c64 ? D64 : D128) > 0)                                               \
        return launch_two(k_sweep<R, TI, TO, NC, CW, (c64 ? D64 : D128), ADJ, 2, true>,    \
                          k_sweep<R, TI, TO, NC, CW, (c64 ? D64 : D128), ADJ, 2, false>,   \
                          grid, a.tpc, sm, s, a);                                         \
      return hipErrorInvalidValue;                                                        \
    }
    HELM_SHAPES(X)
#undef X
  } else {
    const int t = a.tpc;
#define X(NC, CW, D64, D128)                                                              \
    if (sh.nc == NC && sh.cw == CW) {                                                     \
      if constexpr ((c64 ? D64 : D128) > 0)                                               \
        return launch_k(k_sweep<R, TI, TO, NC, CW, (c64 ? D64 : D128), ADJ, 1>, grid, t, sm, s, a); \
      return hipErrorInvalidValue;                                                        \
    }
    HELM_SHAPES_ONE(X)
#undef X
  }
  return hipErrorInvalidValue;
}

template <typename R, bool ADJ>
hipError_t dispatch_line(Shape sh, int chains, int grid, size_t sm, hipStream_t s, SweepArgs a,
                         int g, int l) {
  constexpr bool c64 = sizeof(R) == 4;
  if (chains == 2) {
    const int t = 2 * a.tpc;
#define X(NC, CW, D64, D128)                                                              \
    if (sh.nc == NC && sh.cw == CW) {                                                     \
      if constexpr ((c64 ? D64 : D128) > 0)                                               \
        return launch_k(k_line_solve<R, NC, CW, (c64 ? D64 : D128), ADJ, 2>, grid, t, sm, s, a, g, l); \
      return hipErrorInvalidValue;                                                        \
    }
    HELM_SHAPES(X)
#undef X
  } else {
    const int t = a.tpc;
#define X(NC, CW, D64, D128)                                                              \
    if (sh.nc == NC && sh.cw == CW) {                                                     \
      if constexpr ((c64 ? D64 : D128) > 0)                                               \
        return launch_k(k_line_solve<R, NC, CW, (c64 ? D64 : D128), ADJ, 1>, grid, t, sm, s, a, g, l); \
      return hipErrorInvalidValue;                                                        \
    }
    HELM_SHAPES_ONE(X)
#undef X
  }
  return hipErrorInvalidValue;
}

// the LDS regions of LdsLayout hold what a launch of this shape touches: published vectors of
// NC*CW, zero/junk rows of B, and the step tables of its chains (2 (n/2) + 3 entries each with
// two chains, 2n + 1 with one)
bool lds_fits(int n, int maxB, Shape sh, int chains) {
  const int ts = chains == 2 ? 2 * (n / 2) + 3 : 2 * n + 1;
  return sh.nc * sh.cw <= kZMax && maxB <= kZMax && maxB <= sh.nc * sh.cw && chains * ts <= 2 * (n + 3);
}

SweepArgs base_args(helm_handle* h) {
  SweepArgs a;
  const Plan& P = h->plan;
  a.n = h->n;
  a.Gz = P.Gz;
  a.Gy = P.Gy;
  a.maxW = P.maxW;
  a.maxB = P.maxB;
  a.fronts = P.fronts;
  a.zmid = P.zmid;
  a.fronts_inner = P.fronts_inner;
  a.ymid = P.ymid;
  a.pass = 0;
  a.nfront = 1;
  a.slab_lo = 0;
  a.slab_hi = 1 << 30;
  a.ipass = 0;
  a.ninner = 1;
  a.tpc = 0;
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
  a.xcd_pair = 0;
  a.seq0 = 0;
  a.seq_span = 0;
  a.xdata = nullptr;
  a.xerr = nullptr;
  return a;
}

// one launch of the sweep (fields of SweepArgs: pass, nfront, slab range, ipass, ninner), blocks
// up to maxB, two chains (shape from the lanes override) or one chain spanning the workgroup
template <typename R, typename TI, typename TO>
hipError_t sweep_launch(helm_handle* h, SweepArgs a, const SweepLaunch& L, int R_, bool adjoint,
                        hipStream_t s) {
  a.pass = L.pass;
  a.nfront = L.nfront;
  a.slab_lo = L.slab_lo;
  a.slab_hi = L.slab_hi;
  a.ipass = L.ipass;
  a.ninner = L.ninner;
  a.maxB = L.maxB;
  const Shape sh = L.chains == 2 ? choose_shape(L.maxB, h->lanes_override, sizeof(R) == 4)
                                 : choose_shape_one(L.maxB);
  if (sh.cw < 0 || !lds_fits(h->n, L.maxB, sh, L.chains)) return hipErrorInvalidValue;
  a.tpc = chain_threads(L.maxB, sh.nc);
  const size_t sm = LdsLayout(h->n, L.maxB, (int)sizeof(typename cx<R>::type)).bytes;
  const int grid = R_ * L.nfront * L.ninner;
  a.xdata = nullptr;
  if (L.chains == 2 && h->split && h->xbuf && (size_t)grid <= h->xpairs) {
    char* base = static_cast<char*>(h->xbuf);
    a.xerr = reinterpret_cast<int*>(base);
    a.xdata = reinterpret_cast<unsigned long long*>(base + kXHead);
    // every line solve of the launch takes the next sequence number: a workgroup solves at
    // most (2 Gz - 1) (2 Gy - 1) lines (both passes of both loops)
    a.seq0 = h->xseq;
    a.seq_span = (unsigned long long)(2 * h->plan.Gz) * (2 * h->plan.Gy);
    h->xseq += a.seq_span;
    h->pairs_used = true;
  }
  return adjoint ? dispatch_sweep<R, TI, TO, true>(sh, L.chains, grid, sm, s, a)
                 : dispatch_sweep<R, TI, TO, false>(sh, L.chains, grid, sm, s, a);
}

// the whole sweep; launches of the dominant kernel (the two-chain launches) are timed on
// their own as well
template <typename R, typename TI, typename TO>
hipError_t sweep_all(helm_handle* h, SweepArgs a, int R_, bool adjoint, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (const SweepLaunch& L : sweep_schedule(h->plan)) {
    if (L.timed) {
      hipEvent_t ev = h->t_kernel.begin(s);
      e = sweep_launch<R, TI, TO>(h, a, L, R_, adjoint, s);
      h->t_kernel.end(ev, s, R_);
    } else {
      e = sweep_launch<R, TI, TO>(h, a, L, R_, adjoint, s);
    }
    if (e != hipSuccess) return e;
  }
  return e;
}

}  // namespace


// one slab iterate per outer front of every right-hand side (shared by its inner fronts)
static size_t slab_bytes(const helm_handle* h, int R) {
  const size_t csz = h->prec == HELM_C64 ? sizeof(float2) : sizeof(double2);
  return (size_t)R * h->plan.fronts * h->n * h->n * h->plan.maxW * csz;
}

// exchange slots of the paired two-chain launches: a pair per workgroup of a launch
static size_t exchange_bytes(const helm_handle* h, int R) {
  const size_t pairs = (size_t)R * h->plan.fronts * h->plan.fronts_inner;
  return kXHead + pairs * 2 * 2 * kXSlot * sizeof(unsigned long long);
}

size_t apply_scratch_bytes(const helm_handle* h, int R) {
  return slab_bytes(h, R) + (h->split ? exchange_bytes(h, R) : 0);
}

hipError_t launch_apply(helm_handle* h, const void* r, bool r64, long long r_stride, void* z,
                        bool z64, long long z_stride, int R, const int* rhs_idx, bool adjoint,
                        hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const bool c64 = h->prec == HELM_C64;
  const size_t need = slab_bytes(h, R);
  if (need > h->slab_scratch_bytes) {
    if (h->slab_scratch) {
      pool_free(h->slab_scratch, s);
      h->slab_scratch = nullptr;
      h->slab_scratch_bytes = 0;
    }
    hipError_t e = pool_alloc(&h->slab_scratch, need, s);
    if (e != hipSuccess) return e;
    h->slab_scratch_bytes = need;
  }
  // exchange buffers of the paired two-chain launches: one pair per workgroup of a launch
  const size_t pairs = (size_t)R * h->plan.fronts * h->plan.fronts_inner;
  if (h->split && pairs > h->xpairs) {
    if (h->xbuf) {
      pool_free(h->xbuf, s);
      h->xbuf = nullptr;
      h->xpairs = 0;
    }
    // (cleared whole: tags left in reused memory by another handle must not match)
    const size_t bytes = exchange_bytes(h, R);
    hipError_t e = pool_alloc(&h->xbuf, bytes, s);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(h->xbuf, 0, bytes, s);
    if (e != hipSuccess) return e;
    h->xpairs = pairs;
  }
  SweepArgs a = base_args(h);
  a.in = r;
  a.out = z;
  a.in_stride = r_stride;
  a.out_stride = z_stride;
  a.rhs_idx = rhs_idx;
  a.scratch = h->slab_scratch;
  if (!r64) return hipErrorInvalidValue;  // inputs are always complex128
  if (!c64 && !z64) return hipErrorInvalidValue;
  hipEvent_t ev = h->t_apply.begin(s);
  hipError_t e;
  if (!c64)
    e = sweep_all<double, double2, double2>(h, a, R, adjoint, s);
  else if (z64)
    e = sweep_all<float, double2, double2>(h, a, R, adjoint, s);
  else
    e = sweep_all<float, double2, float2>(h, a, R, adjoint, s);
  h->t_apply.end(ev, s, R);
  return e;
}

hipError_t take_exchange_error(helm_handle* h, hipStream_t s, int* bad) {
  *bad = 0;
  h->pairs_used = false;
  if (!h->xbuf) return hipSuccess;
  hipError_t e = hipMemcpyAsync(bad, h->xbuf, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess && *bad) {
    e = hipMemsetAsync(h->xbuf, 0, sizeof(int), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  return e;
}

hipError_t launch_line_solve(helm_handle* h, int zg, int yg, const double2* r, double2* x, int R,
                             bool adjoint, hipStream_t s) {
  const bool c64 = h->prec == HELM_C64;
  const size_t csz = c64 ? sizeof(float2) : sizeof(double2);
  const Plan& P = h->plan;
  SweepArgs a = base_args(h);
  a.in = r;
  a.out = x;
  // lines on a middle group: one chain over the workgroup, x1-order factors
  const bool one = P.one_chain(zg, yg);
  const int mb = one ? P.maxB_mid : P.maxB_front;
  a.maxB = mb;
  const size_t sm = LdsLayout(h->n, mb, (int)csz).bytes;
  const Shape sh = one ? choose_shape_one(mb) : choose_shape(mb, h->lanes_override, c64);
  if (sh.cw < 0 || !lds_fits(h->n, mb, sh, one ? 1 : 2)) return hipErrorInvalidValue;
  a.tpc = chain_threads(mb, sh.nc);
  const int chains = one ? 1 : 2;
  if (c64)
    return adjoint ? dispatch_line<float, true>(sh, chains, R, sm, s, a, zg, yg)
                   : dispatch_line<float, false>(sh, chains, R, sm, s, a, zg, yg);
  return adjoint ? dispatch_line<double, true>(sh, chains, R, sm, s, a, zg, yg)
                 : dispatch_line<double, false>(sh, chains, R, sm, s, a, zg, yg);
}

// The sweep kernel: z = M^{-1} r (Algorithm 6 with Algorithm 4 inside, each line block solved
// exactly by its block LDU) or z = M^{-H} r, for a batch of right-hand sides in ONE persistent
// cooperative launch.  Included by the sweep_*.hip sources, each of which instantiates it for
// one precision and direction.
//
// Workgroups.  Every line solve is the two-sided block LDU of the line (the x1-blocks
// eliminated from both ends towards the middle block m = n/2, Sec. 3 with that block order):
// two chains of dependent block steps that meet once, at the middle block.  Each chain runs
// in a workgroup of its own ("member" 0: blocks 0..m, member 1: blocks m+1..n-1) and holds
// only the grid points of its half of the line in x1; every coupling outside a line solve
// joins grid points of the same x1, so the two members are independent except for the
// middle block, whose right-hand side is the sum of both chains' partial ones.  A right-hand
// side takes 2 x (outer fronts) x (inner fronts) members:
//   outer front o (two fronts in x3: o = 0 sweeps the x3-groups upwards from x3 = 0, o = 1
//   downwards from x3 = 1; the middle x3-group is solved by o = 0), inner front f (the same
//   over the x2-groups of every slab; the middle x2-line is solved by f = 0), half h.
// Three placements over the 8 XCDs (k_sweep): all members of a right-hand side on one XCD, so
// their exchanges stay in one L2; each member on its own XCD, so that one XCD's L2 serves one
// part of the factor stream to every right-hand side; or the two members of each line solve on
// one XCD, between the two.
//
// Exchanges.  Members wait for each other only for data, never on a barrier: a value travels
// in 64-bit words, each holding one 32-bit piece beside a tag (the sequence number of the
// event), written and read with relaxed device-scope atomics; a reader polls until every
// word it needs carries the expected tag.  No fence is needed (data and flag are the same
// word), and none is wanted: a device-scope release or acquire writes back or invalidates the
// XCD's L2, through which the right-hand sides' members share the factor stream.
//   E1  the two chains of a line solve: the middle block's partial right-hand side;
//   E2  inner front 1 -> 0, once per slab: the slab iterate on the first row of x2-group
//       ymid + 1 (the middle line's coupling from above);
//   E3  inner front 0 -> 1, once per slab: the middle line's solution on its last row (the
//       first backward line's coupling of front 1);
//   E4  outer front 1 -> 0, once: u on the first layer of x3-group zmid + 1 after the
//       forward sweep (the middle slab's coupling from above);
//   E5  outer front 0 -> 1, once: u on the last layer of the middle x3-group (the first
//       backward slab's coupling of front 1).
// Each pairing joins members of equal half (and, for E4/E5, equal inner front), which own
// the same grid points.  The launch is cooperative: the runtime refuses a grid whose
// workgroups cannot all be resident (the host then launches the right-hand sides in chunks),
// so a member never waits for one that is not running.  Waits are bounded (spin_limit polls,
// each a device-memory round trip and a short sleep); a member that gives up writes NaN into
// the value it waited for and raises the launch's error word.
//
// Block step.  In a chain, thread t owns output row t / NC of the B x B block and CW
// consecutive columns; the NC partial sums of a row are adjacent lanes of one wavefront and
// are combined with DPP row operations.  The vector a step multiplies (z_i = q_i - l_i y_{i-1}
// forward, x_{i+1} backward) is formed once per row and published through a double-buffered
// LDS slot, so one barrier separates consecutive steps.  The factor blocks do not depend on
// the data: each thread keeps its slice of the next D blocks in registers (a ring refilled D
// steps ahead), which hides the HBM latency behind D dependent steps.  A kernel carries two
// shapes: lines with B <= NCA * CWA use shape A, larger blocks (the lines on a middle group)
// shape B; waves with no row of the current line only take part in the barriers.
#pragma once

#include "common.h"

namespace sweepk {

struct SweepArgs {
  int n, Gz, Gy, maxW, maxB;
  int fronts, zmid, fronts_inner, ymid;
  int wpr;               // members per right-hand side: 2 * fronts * fronts_inner
  int R;                 // right-hand sides of this launch
  int mode;              // 0: the whole sweep; 1: the single line (line_g, line_l) on its grid
  int line_g, line_l;
  long long N, in_stride, out_stride;
  const GroupInfo* groups;
  const long long* line_off;
  const double2* coef;   // [4][n+2]: A[m,m-1], A[m,m+1], A^H[m,m-1], A^H[m,m+1]
  const void* factors;
  const void* in;
  void* out;
  const int* rhs_idx;    // launch slot -> right-hand side (null: identity)
  void* slab;            // per slot and outer front: the slab iterate, n x n x maxW
  void* layer;           // per slot and outer front: a received layer of u, n x n
  unsigned long long* xw;  // exchange words (layout: XLayout)
  int* xerr;
  unsigned long long seq0;
  unsigned spin_limit;
  int drop_publish;      // failure injection: member 0 of every pair skips publishing E1
  int xmap;              // workgroup placement over the XCDs (see k_sweep)
  const void* nd;        // nested-dissection factors (k_sweep_nd), per line at nd_off[line]
  const long long* nd_off;
  int nd_k;              // levels: n = 2^nd_k - 1
};

// exchange words per launch slot (all counts in 64-bit words; np = 32-bit pieces per value)
struct XLayout {
  long long e1, e23, e45, per_slot;
  __host__ __device__ XLayout(int n, int maxW, int np, int wpr) {
    const int ni = n / 2 + 1;
    e1 = 2LL * kZMax * np;                    // per member: two parities of B values
    e23 = 2LL * ni * maxW * np;               // per (outer front, half), per kind: two parities
    e45 = (long long)ni * n * np;             // per (inner front, half), per kind
    per_slot = wpr * e1 + 2 * 2 * 2 * e23 + 2 * 2 * 2 * e45;
  }
};

// ------------------------------------------------------------------------------------------
// small device helpers
// ------------------------------------------------------------------------------------------
template <int CTRL> __device__ __forceinline__ float dpp_mov(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}
template <int CTRL> __device__ __forceinline__ double dpp_mov(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
// sum over groups of NC adjacent lanes (NC in {4, 8, 16}), result in every lane of the group
template <int NC, typename T> __device__ __forceinline__ T lane_sum(T v) {
  static_assert(NC == 4 || NC == 8 || NC == 16, "lanes per row must be 4, 8 or 16");
  v += dpp_mov<0xB1>(v);                             // quad_perm [1,0,3,2]: pairs
  v += dpp_mov<0x4E>(v);                             // quad_perm [2,3,0,1]: quads
  if constexpr (NC >= 8) v += dpp_mov<0x141>(v);     // row_half_mirror: the other quad of 8
  if constexpr (NC == 16) v += dpp_mov<0x140>(v);    // row_mirror: the other 8 of each 16
  return v;
}

// Walk over e = tid, tid + NT, ... of a (hi, lo, ii) index space, e = (hi W + lo) ni + ii,
// with ii < ni and lo < W: the three indices are kept by additions (a division per element
// would cost more than the element's own work).
struct Walk {
  int ii, lo, hi;          // current element
  int di, dlo, dhi;        // step of NT elements
  int ni, W;
  __device__ __forceinline__ Walk(int tid, int NT, int ni_, int W_) : ni(ni_), W(W_) {
    const int ro = tid / ni, dq = NT / ni;
    ii = tid - ro * ni;
    hi = ro / W;
    lo = ro - hi * W;
    di = NT - dq * ni;
    dhi = dq / W;
    dlo = dq - dhi * W;
  }
  __device__ __forceinline__ void next() {
    ii += di;
    lo += dlo;
    hi += dhi;
    if (ii >= ni) {
      ii -= ni;
      ++lo;
    }
    if (lo >= W) {
      lo -= W;
      ++hi;
    }
  }
};

// elements per thread whose input loads a line's gather issues together
constexpr int kGatherU = 4;

// Loads from the factor array through an explicitly global pointer (global_load, counted by
// vmcnt only; a generic pointer would give flat loads, which also count against lgkmcnt and
// would make every LDS wait drain the factor ring).
#define HELM_GLOBAL __attribute__((address_space(1)))
template <typename R> struct vec2 { using type = R __attribute__((ext_vector_type(2))); };

// Workgroup barrier for LDS traffic only: waits for this wave's LDS operations, then
// s_barrier.  Unlike __syncthreads() it does not wait for outstanding global loads, so the
// factor ring stays in flight across block steps.
__device__ __forceinline__ void lds_barrier() {
  __asm__ volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// tagged words: piece | (tag << 32)
__device__ __forceinline__ void put_word(unsigned long long* w, unsigned long long tag, unsigned piece) {
  __hip_atomic_store(w, tag | piece, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// the piece of word w once it carries tag (NaN and the error word raised after spin polls)
__device__ __forceinline__ unsigned get_word(const unsigned long long* w, unsigned long long tag,
                                             unsigned spin, int* err) {
  unsigned spins = 0;
  unsigned long long v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // once a wait has given up, later waits do not poll: a broken exchange costs one bound
  if ((v & 0xffffffff00000000ull) != tag && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    return 0x7fc00000u;
  while ((v & 0xffffffff00000000ull) != tag) {
    if (++spins > spin) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return 0x7fc00000u;   // a quiet NaN in either half of a value
    }
    __builtin_amdgcn_s_sleep(1);
    v = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return (unsigned)v;
}

// ------------------------------------------------------------------------------------------
// LDS layout of a member, in complex elements from the base (tables at a 16-byte boundary):
// its half of the line vector (n/2 + 1 blocks of up to maxB), the published vectors (two
// chains x two parities), zero and junk rows, the couplings, a received row (E2/E3), the
// per-step couplings and the per-step table of its chain (at most n + 3 entries each)
// ------------------------------------------------------------------------------------------
struct MemberLds {
  int ybuf, zb, zeros, junk, cf, cb, xrow, ctab;
  size_t tab_byte, bytes;
  __host__ __device__ MemberLds(int n, int maxB, int maxW, int csz) {
    ybuf = 0;
    zb = (n / 2 + 1) * maxB;
    zeros = zb + 4 * kZMax;
    junk = zeros + kZMax;
    cf = junk + kZMax;
    cb = cf + (n + 2);
    xrow = cb + (n + 2);
    ctab = xrow + (n / 2 + 1) * maxW;
    tab_byte = ((size_t)(ctab + (n + 3)) * csz + 15) / 16 * 16;
    bytes = tab_byte + (size_t)(n + 3) * 16;
  }
};

// ------------------------------------------------------------------------------------------
// One chain of a two-sided line solve, on one workgroup.  Chain 0 (member half 0) takes the
// blocks i = mid - |mid - t| at steps t = 0..2 mid, chain 1 the blocks i = mid + |mid - t|
// (none when i > n - 1): forward elimination for t < mid, the middle block at t = mid (both
// chains compute it, from the sum of their partial right-hand sides), back-substitution for
// t > mid.  Block i of the member's half sits at LDS row (i - base) * B.
// ------------------------------------------------------------------------------------------
template <typename R, int NC, int CW, int D, bool ADJ>
struct Chain {
  using C = typename cx<R>::type;
  static constexpr int ZS = NC * CW;   // stride of one published vector (>= B, zero-padded)
  static_assert(D % 2 == 0, "the ring depth must be even (published-vector parity per slot)");
  static_assert(ZS <= kZMax, "published vector longer than its LDS slot");
  C ring[D][CW];
  unsigned off0;                       // this thread's byte offset inside a B x B block
  unsigned offa[ADJ ? CW : 1];         // adjoint walk: one offset per column
  int row, rowc, c0;
  int lower;                           // chain (member half)
  int n_, mid, B_, steps, base;
  unsigned BBb;                        // bytes of one factor block
  const HELM_GLOBAL char* Tb;          // factors of the line
  int4 ecur, enext;
  C Acur, ccur;

  __device__ __forceinline__ Chain(int half) {
    lower = half;
    row = (int)threadIdx.x / NC;
    c0 = ((int)threadIdx.x - row * NC) * CW;
  }

  // Rows past B are clamped to row B - 1 (they compute and write that row's values again).
  // Columns past B meet zero padding of the published vector: in the row-major
  // (non-adjoint) walk they run into the next row, or past the last block into the padding
  // that follows the factor array, so they read finite values; the adjoint walk clamps them.
  __device__ __forceinline__ void begin_line(const C* T, int B, int n) {
    n_ = n;
    B_ = B;
    mid = n / 2;
    steps = 2 * mid + 1;
    base = lower ? mid + 1 : 0;
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

  // block of step t, clamped to the line
  __device__ __forceinline__ int blk(int t) const {
    const int d = mid > t ? mid - t : t - mid;
    const int i = lower ? mid + d : mid - d;
    return i < 0 ? 0 : (i > n_ - 1 ? n_ - 1 : i);
  }

  template <int S> __device__ __forceinline__ void load(unsigned b0) {
    if constexpr (ADJ) {
#pragma unroll
      for (int cc = 0; cc < CW; ++cc) {
        using V = typename vec2<R>::type;
        const V v = *reinterpret_cast<const HELM_GLOBAL V*>(Tb + b0 + offa[cc]);
        ring[S][cc] = mk(v.x, v.y);
      }
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
      load<S>((unsigned)blk(S) * BBb);
      fill<S + 1>();
    }
  }

  template <int S> __device__ __forceinline__ C first(int cc, const C (&zr)[CW]) const {
    return ADJ ? mk(ring[S][cc].x * zr[cc].x + ring[S][cc].y * zr[cc].y,
                    ring[S][cc].x * zr[cc].y - ring[S][cc].y * zr[cc].x)
               : cmul(ring[S][cc], zr[cc]);
  }
  // row sum of ring[S] . z over this thread's columns, reduced over the row's NC lanes; even
  // and odd columns go to two accumulators (a shorter dependent FMA chain)
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

  // Step t with ring slot S (parity of t = parity of S): P = A - c acc with the table's
  // operand row A and coupling c (A = 0, c = -1 in the middle); the block row gets acc
  // (forward steps, t < mid: FWD) or P, and P is published for the next step.
  template <int S, bool FWD>
  __device__ __forceinline__ void step(int t, C* sb, const C* zme, const C* zot, const int4* tab,
                                       const C* ctab) {
    constexpr int par = (S & 1) * ZS;
    C zr[CW];
#pragma unroll
    for (int cc = 0; cc < CW; ++cc) zr[cc] = zme[par + c0 + cc];
    if constexpr (!FWD) {
      if (t == mid) {
#pragma unroll
        for (int cc = 0; cc < CW; ++cc) zr[cc] = cadd(zr[cc], zot[par + c0 + cc]);
      }
    }
    const int4 e2 = tab[t + 2];
    const C cn = ctab[t + 1];
    const C acc = dot<S>(zr);
    load<S>((unsigned)ecur.w);
    const C P = csub(Acur, cmul(ccur, acc));
    sb[ecur.y + rowc] = FWD ? acc : P;
    sb[ecur.z + rowc] = P;
    Acur = sb[enext.x + rowc];   // operand of step t + 1 (never written by step t)
    ccur = cn;
    ecur = enext;
    enext = e2;
    lds_barrier();
  }

  // D consecutive steps, one per ring slot, with no branch between them (the wait before
  // each slot's use then covers exactly the loads issued D steps earlier)
  template <bool FWD, int S = 0>
  __device__ __forceinline__ void group(int t0, C* sb, const C* zme, const C* zot, const int4* tab,
                                        const C* ctab) {
    if constexpr (S < D) {
      step<S, FWD>(t0 + S, sb, zme, zot, tab, ctab);
      group<FWD, S + 1>(t0, sb, zme, zot, tab, ctab);
    }
  }
  template <bool FWD, int S = 0>
  __device__ __forceinline__ void tail(int t0, int end, C* sb, const C* zme, const C* zot,
                                       const int4* tab, const C* ctab) {
    if constexpr (S < D) {
      if (t0 + S < end) {
        step<S, FWD>(t0 + S, sb, zme, zot, tab, ctab);
        tail<FWD, S + 1>(t0, end, sb, zme, zot, tab, ctab);
      }
    }
  }
  // backward steps from t0 + s0 (t0 a multiple of D)
  template <int S = 0>
  __device__ __forceinline__ void head(int t0, int s0, int end, C* sb, const C* zme,
                                       const C* zot, const int4* tab, const C* ctab) {
    if constexpr (S < D) {
      if (S >= s0) {
        if (t0 + S >= end) return;
        step<S, false>(t0 + S, sb, zme, zot, tab, ctab);
      }
      head<S + 1>(t0, s0, end, sb, zme, zot, tab, ctab);
    }
  }

  // E1: publish this chain's partial right-hand side of the middle block (its published
  // vector of step mid) to the partner and take the partner's into the slot the middle step
  // reads (a word whose tag never arrives gives NaN and raises err)
  __device__ __forceinline__ void exchange(C* sb, int zb, unsigned long long* mine,
                                           const unsigned long long* other, unsigned long long seq,
                                           unsigned spin, int* err, bool publish) {
    constexpr int np = sizeof(C) / 4;
    const int par = (mid & 1) * ZS;
    const unsigned* src = reinterpret_cast<const unsigned*>(sb + zb + lower * 2 * ZS + par);
    unsigned* dst = reinterpret_cast<unsigned*>(sb + zb + (1 - lower) * 2 * ZS + par);
    const unsigned long long tag = (seq & 0xffffffffull) << 32;
    if (publish)
      for (int e = threadIdx.x; e < B_ * np; e += blockDim.x) put_word(mine + e, tag, src[e]);
    for (int e = threadIdx.x; e < B_ * np; e += blockDim.x) dst[e] = get_word(other + e, tag, spin, err);
    lds_barrier();
  }

  // Solve on the right-hand side in the member's half of ybuf (complete, after a barrier).
  // LDS regions as element offsets from sb.  On return ybuf holds the solution on the
  // member's blocks (visible to the whole workgroup).  The step table and the zero padding of
  // the published vectors depend on B and the shape only: with fresh false they are those of
  // the member's previous line and are kept.
  __device__ __forceinline__ void run(C* sb, int ybuf, int zb, int zeros, int junk, C* ctab,
                                      int4* tab, const C* cf, const C* cb, bool idle, bool fresh,
                                      unsigned long long* xmine, const unsigned long long* xother,
                                      unsigned long long seq, unsigned spin, int* err, bool publish) {
    if (fresh) tables(sb, ybuf, zb, zeros, junk, ctab, tab, cf, cb);
    start(sb, ybuf, zb, ctab, tab, idle, xmine, xother, seq, spin, err, publish);
  }
  __device__ __forceinline__ void tables(C* sb, int ybuf, int zb, int zeros, int junk, C* ctab,
                                         int4* tab, const C* cf, const C* cb) {
    const C zero = mk((R)0, (R)0);
    const int B = B_, ts = steps + 2;   // table entries (<= n + 3)
    for (int e = threadIdx.x; e < 4 * ZS; e += blockDim.x)
      if (e % ZS >= B) sb[zb + e] = zero;
    // per step: coupling (forward chain 0 l_{i+1}, chain 1 u_{i-1}; backward chain 0 u_i,
    // chain 1 l_i; middle -1; block i is x1-node i + 1: l_i = cf[i + 1], u_i = cb[i + 1])
    // and the table {operand row, result row, published-vector row, prefetch offset}
    const int ch = lower;
    for (int t = threadIdx.x; t < ts; t += blockDim.x) {
      const int d = mid > t ? mid - t : t - mid;
      const int i = ch ? mid + d : mid - d;
      const bool valid = t < steps && i >= 0 && i < n_;
      const int znext = zb + (2 * ch + ((t + 1) & 1)) * ZS;
      C c = mk((R)-1, (R)0);
      int4 en = make_int4(zeros, junk, junk, (int)((unsigned)blk(t + D) * BBb));
      if (t < mid) {
        c = ch ? cb[i] : cf[i + 2];
        const bool last_lower = ch && t == mid - 1;
        if (valid) {
          en.x = last_lower ? zeros : ybuf + ((ch ? i - 1 : i + 1) - base) * B;
          en.y = ybuf + (i - base) * B;
          en.z = znext;
        } else if (ch && i == n_) {
          en.x = ybuf + (n_ - 1 - base) * B;   // (even n, t = 0: chain 1 has no block yet)
        }
      } else if (t == mid) {
        en.y = ch ? junk : ybuf + (mid - base) * B;
        en.z = znext;
      } else if (valid) {
        c = ch ? cf[i + 1] : cb[i + 1];
        en.x = ybuf + (i - base) * B;
        en.y = ybuf + (i - base) * B;
        en.z = znext;
      }
      ctab[t] = c;
      tab[t] = en;
    }
    lds_barrier();
  }
  __device__ __forceinline__ void start(C* sb, int ybuf, int zb, const C* ctab, const int4* tab,
                                        bool idle, unsigned long long* xmine,
                                        const unsigned long long* xother, unsigned long long seq,
                                        unsigned spin, int* err, bool publish) {
    const int B = B_;
    // each chain starts from the q of its first block (chain 1: block n - 1 at step 2 mid - n + 1)
    if (row < B) {
      if (!lower) sb[zb + row] = sb[ybuf + row];
      else sb[zb + (2 + ((2 * mid - n_ + 1) & 1)) * ZS + row] = sb[ybuf + (n_ - 1 - base) * B + row];
    }
    lds_barrier();
    const C* zme = sb + zb + lower * 2 * ZS;
    const C* zot = sb + zb + (1 - lower) * 2 * ZS;
    if (idle) {
      // no row of this line: the barriers of every step, the exchange, nothing else
      for (int t = 0; t < mid; ++t) lds_barrier();
      exchange(sb, zb, xmine, xother, seq, spin, err, publish);
      for (int t = mid; t < steps; ++t) lds_barrier();
      return;
    }
    ecur = tab[0];
    enext = tab[1];
    ccur = ctab[0];
    Acur = sb[ecur.x + rowc];
    // forward steps 0 .. mid - 1, the exchange, then mid .. steps - 1 continuing the ring
    // slots where the forward steps left them (step t always uses slot t % D)
    int t0 = 0;
    for (; t0 + D <= mid; t0 += D) group<true>(__builtin_amdgcn_readfirstlane(t0), sb, zme, zot, tab, ctab);
    if (t0 < mid) tail<true>(__builtin_amdgcn_readfirstlane(t0), mid, sb, zme, zot, tab, ctab);
    exchange(sb, zb, xmine, xother, seq, spin, err, publish);
    t0 = mid - mid % D;
    if (t0 < mid) {
      head(__builtin_amdgcn_readfirstlane(t0), mid - t0, steps, sb, zme, zot, tab, ctab);
      t0 += D;
    }
    for (; t0 + D <= steps; t0 += D) group<false>(__builtin_amdgcn_readfirstlane(t0), sb, zme, zot, tab, ctab);
    if (t0 < steps) tail<false>(__builtin_amdgcn_readfirstlane(t0), steps, sb, zme, zot, tab, ctab);
  }
};


// threads of a chain of blocks up to NC * CW rows
template <int NC, int CW> constexpr int chain_threads_max() { return (NC * CW * NC + 63) / 64 * 64; }
template <int NCA, int CWA, int NCB, int CWB> constexpr int kernel_threads_max() {
  return chain_threads_max<NCA, CWA>() > chain_threads_max<NCB, CWB>() ? chain_threads_max<NCA, CWA>()
                                                                         : chain_threads_max<NCB, CWB>();
}

// One member's part of the sweep (see the top of this file).  Everything is inlined into the
// kernel (each step of the program is reached from a single call site), so the member's
// state stays in registers: a call taking the object's address would put it in scratch.
// first of block i's nested-dissection matrices, in B^2 units from the line's start
__device__ __forceinline__ long long nd_first(int i) { return 3LL * i - 2LL * __popc((unsigned)i); }

template <typename R, typename TI, typename TO, int NCA, int CWA, int DA, int NCB, int CWB, int DB,
          bool ADJ, bool ND = false>
struct Sweeper {
  using C = typename cx<R>::type;
  static constexpr int np = sizeof(C) / 4;   // 32-bit pieces per value
  MemberLds L;
  C* sb;
  int4* tab;
  C *cf, *cb, *xrow;
  const TI* f;
  TO* u;
  C* v;      // slab iterate of the outer front (rows of all its inner fronts)
  C* lay;    // received layer of u (E4 / E5)
  const GroupInfo* groups;
  const long long* line_off;
  const C* factors;
  const C* ndf;               // nested-dissection factors (ND)
  const long long* nd_off;
  int nd_k;
  unsigned long long *x1mine, *x1other, *xs;
  int* xerr;
  long long e23, e45;
  unsigned long long seq0;
  unsigned spin;
  int n, Gz, Gy, zmid, ymid, fronts, fronts_inner, ofront, ifront, half, ilo, ni, tid, NT;
  bool publish;
  unsigned long long lcount, sstep;           // lines solved, slab steps done (tags)
  int tab_key;                                // block size and shape of the step table in LDS

  __device__ __forceinline__ Sweeper(const SweepArgs& a, unsigned char* smem, int slot, int member)
      : L(a.n, a.maxB, a.maxW, (int)sizeof(C)) {
    n = a.n;
    Gz = a.Gz;
    Gy = a.Gy;
    zmid = a.zmid;
    ymid = a.ymid;
    fronts = a.fronts;
    fronts_inner = a.fronts_inner;
    groups = a.groups;
    line_off = a.line_off;
    factors = reinterpret_cast<const C*>(a.factors);
    ndf = reinterpret_cast<const C*>(a.nd);
    nd_off = a.nd_off;
    nd_k = a.nd_k;
    xerr = a.xerr;
    seq0 = a.seq0;
    spin = a.spin_limit;
    lcount = 0;
    sstep = 0;
    tab_key = -1;
    tid = (int)threadIdx.x;
    NT = (int)blockDim.x;
    half = member & 1;
    publish = !(a.drop_publish && half == 0);
    ifront = (member >> 1) % fronts_inner;
    ofront = (member >> 1) / fronts_inner;
    ilo = half ? n / 2 + 1 : 0;
    ni = half ? n - n / 2 - 1 : n / 2 + 1;
    sb = reinterpret_cast<C*>(smem);
    tab = reinterpret_cast<int4*>(smem + L.tab_byte);
    cf = sb + L.cf;
    cb = sb + L.cb;
    xrow = sb + L.xrow;
    const int q = a.rhs_idx ? a.rhs_idx[slot] : slot;
    f = reinterpret_cast<const TI*>(a.in) + (long long)q * a.in_stride;
    u = reinterpret_cast<TO*>(a.out) + (long long)q * a.out_stride;
    const long long sf = (long long)slot * fronts + ofront;
    v = reinterpret_cast<C*>(a.slab) + sf * n * n * a.maxW;
    lay = reinterpret_cast<C*>(a.layer) + sf * n * n;
    const XLayout X(n, a.maxW, np, a.wpr);
    unsigned long long* base = a.xw + (long long)slot * X.per_slot;
    x1mine = base + member * X.e1;
    x1other = base + (member ^ 1) * X.e1;
    xs = base + a.wpr * X.e1;
    e23 = X.e23;
    e45 = X.e45;
    for (int m = tid; m < n + 2; m += NT) {
      cf[m] = cvt<C>(a.coef[(ADJ ? 2 : 0) * (n + 2) + m]);
      cb[m] = cvt<C>(a.coef[(ADJ ? 3 : 1) * (n + 2) + m]);
    }
    for (int m = tid; m < kZMax; m += NT) sb[L.zeros + m] = mk((R)0, (R)0);
    __syncthreads();
  }

  __device__ __forceinline__ long long gidx(int i, int j, int k) const {   // i 0-based, j, k 1-based
    return ((long long)(k - 1) * n + (j - 1)) * n + i;
  }


  // gather (into this member's half of the line vector), solve, with the shape B takes
  template <int NC, int CW, int D, typename G>
  __device__ __forceinline__ void solve(const C* T, int B, G& gather) {
    Chain<R, NC, CW, D, ADJ> ch(half);
    ch.begin_line(T, B, n);
    const bool idle = (tid >> 6) * (64 / NC) >= B;   // no row of this line in the wave
    if (!idle) ch.fill();                             // in flight while the input is gathered
    gather();
    lds_barrier();   // the gather writes LDS only (its global loads are consumed by then)
    const int par = (int)(lcount & 1);
    const int key = B * 2 + (NC == NCA && CW == CWA && D == DA ? 0 : 1);
    const bool fresh = key != tab_key;
    tab_key = key;
    ch.run(sb, L.ybuf, L.zb, L.zeros, L.junk, sb + L.ctab, tab, cf, cb, idle, fresh,
           x1mine + par * kZMax * np, x1other + par * kZMax * np, seq0 + lcount + 1, spin, xerr, publish);
    lcount += 1;
  }
  template <typename G> __device__ __forceinline__ void solve_any(const C* T, int B, G& gather) {
    if constexpr (ND) {
      gather();
      __syncthreads();
      if (B <= 64) nd_solve<1>(T, B);
      else nd_solve<2>(T, B);
      lcount += 1;
    } else {
      if (B <= NCA * CWA) solve<NCA, CWA, DA>(T, B, gather);
      else solve<NCB, CWB, DB>(T, B, gather);
    }
  }
  // the factors of line (g, l): its block LDU factors, or its nested-dissection matrices
  __device__ __forceinline__ const C* line_factors(int g, int l) const {
    const size_t line = (size_t)g * Gy + l;
    return ND ? ndf + nd_off[line] : factors + line_off[line];
  }

  // ---- nested-dissection line solve (block cyclic reduction; the factor layout is described
  // with the setup).  acc[rr] (row lane + 64 rr) += sc (M v), M column-major B x B in HBM, v
  // in LDS: a wave per product, 16 (8 with two rows per lane) columns' loads in flight
  template <int RPL>
  __device__ __forceinline__ void nd_mv(C (&acc)[RPL], const C* M, C sc, const C* v, int B) const {
    const int lane = tid & 63;
    int rows[RPL];
    C t[RPL];
#pragma unroll
    for (int rr = 0; rr < RPL; ++rr) {
      rows[rr] = lane + 64 * rr < B ? lane + 64 * rr : B - 1;
      t[rr] = mk((R)0, (R)0);
    }
    constexpr int U = RPL == 1 ? 16 : 8;
    for (int j0 = 0; j0 < B; j0 += U) {
      C mv[U][RPL], xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u < B ? j0 + u : B - 1;
        xv[u] = v[j];
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) mv[u][rr] = M[(long long)j * B + rows[rr]];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (j0 + u < B)
#pragma unroll
          for (int rr = 0; rr < RPL; ++rr) t[rr] = cfma(t[rr], mv[u][rr], xv[u]);
    }
#pragma unroll
    for (int rr = 0; rr < RPL; ++rr) acc[rr] = cfma(acc[rr], sc, t[rr]);
  }
  // acc[rr] = M (b - c1 x1 - c2 x2), or M (b + x1) with sum (the two halves' middle parts)
  template <int RPL>
  __device__ __forceinline__ void nd_mv3(C (&acc)[RPL], const C* M, const C* b, const C* x1, C c1,
                                         const C* x2, C c2, int B) const {
    const int lane = tid & 63;
    int rows[RPL];
#pragma unroll
    for (int rr = 0; rr < RPL; ++rr) {
      rows[rr] = lane + 64 * rr < B ? lane + 64 * rr : B - 1;
      acc[rr] = mk((R)0, (R)0);
    }
    constexpr int U = RPL == 1 ? 16 : 8;
    for (int j0 = 0; j0 < B; j0 += U) {
      C mv[U][RPL], xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u < B ? j0 + u : B - 1;
        xv[u] = csub(csub(b[j], cmul(c1, x1[j])), cmul(c2, x2[j]));
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) mv[u][rr] = M[(long long)j * B + rows[rr]];
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (j0 + u < B)
#pragma unroll
          for (int rr = 0; rr < RPL; ++rr) acc[rr] = cfma(acc[rr], mv[u][rr], xv[u]);
    }
  }
  template <int RPL> __device__ __forceinline__ void nd_load(C (&acc)[RPL], const C* v, int B) const {
    const int lane = tid & 63;
#pragma unroll
    for (int rr = 0; rr < RPL; ++rr) acc[rr] = v[lane + 64 * rr < B ? lane + 64 * rr : B - 1];
  }
  template <int RPL> __device__ __forceinline__ void nd_store(C* v, const C (&acc)[RPL], int B) const {
    const int lane = tid & 63;
#pragma unroll
    for (int rr = 0; rr < RPL; ++rr)
      if (lane + 64 * rr < B) v[lane + 64 * rr] = acc[rr];
  }

  // Solve on the right-hand side in the member's half of ybuf (complete, after a barrier); on
  // return ybuf holds the solution on the member's blocks.  Half 0 takes blocks 0 .. mid - 1
  // and the middle block's reduction from below, half 1 blocks mid + 1 .. n - 1 and the
  // reduction from above (its copy of the middle block in the first published-vector slot);
  // the two partial right-hand sides of the middle block are summed through E1, and both
  // halves solve the middle block.  Every level is one phase: its products spread over the
  // waves, one barrier after it.
  template <int RPL> __device__ void nd_solve(const C* F, int B) {
    const int k = nd_k, mid = n / 2, wv = tid >> 6, NW = NT >> 6;
    const long long BB = (long long)B * B;
    C* yb = sb + L.ybuf;
    C* own = half ? sb + L.zb : yb + (mid - ilo) * B;   // this half's copy of the middle block
    C* oth = sb + L.zb + kZMax;                         // the partner's partial
    const C* zv = sb + L.zeros;
    const C zero = mk((R)0, (R)0), one = mk((R)1, (R)0), mone = mk((R)-1, (R)0);
    auto vec = [&](int i) -> C* { return i == mid ? own : yb + (i - ilo) * B; };
    auto mat = [&](int i, int q) -> const C* { return F + (nd_first(i) + q) * BB; };
    if (half)
      for (int x = tid; x < B; x += NT) own[x] = zero;
    __syncthreads();
    // forward: level l reduces the right-hand sides of the blocks above it (r = m 2^{l+1} - 1)
    // and, for l >= 2, turns those of level l - 1 into y = Inv b
    for (int l = 0; l <= k - 2; ++l) {
      const int s = 1 << l, mh = 1 << (k - 2 - l);
      const int m0 = half ? mh : 1, ny = l >= 2 ? 2 * mh : 0, o0 = half ? 4 * mh + 1 : 1;
      for (int t = wv; t < mh + ny; t += NW) {
        C acc[RPL];
        if (t < mh) {
          const int r = (m0 + t) * 2 * s - 1;
          nd_load<RPL>(acc, vec(r), B);
          if (r != mid || !half)
            nd_mv<RPL>(acc, l == 0 ? mat(r - 1, 0) : mat(r, 3 + 2 * (l - 1)), l == 0 ? csub(zero, cf[r + 1]) : mone,
                       vec(r - s), B);
          if (r != mid || half)
            nd_mv<RPL>(acc, l == 0 ? mat(r + 1, 0) : mat(r, 4 + 2 * (l - 1)), l == 0 ? csub(zero, cb[r + 1]) : mone,
                       vec(r + s), B);
          nd_store<RPL>(vec(r), acc, B);
        } else {
          const int e = (o0 + 2 * (t - mh)) * (s >> 1) - 1;
          nd_mv3<RPL>(acc, mat(e, 0), vec(e), zv, zero, zv, zero, B);
          nd_store<RPL>(vec(e), acc, B);
        }
      }
      __syncthreads();
    }
    // E1: the partial right-hand side of the middle block to the partner, the partner's in
    {
      const int par = (int)(lcount & 1);
      unsigned long long* mine = x1mine + par * kZMax * np;
      const unsigned long long* other = x1other + par * kZMax * np;
      const unsigned long long tag = ((seq0 + lcount + 1) & 0xffffffffull) << 32;
      const unsigned* src = reinterpret_cast<const unsigned*>(own);
      unsigned* dst = reinterpret_cast<unsigned*>(oth);
      if (publish)
        for (int e = tid; e < B * np; e += NT) put_word(mine + e, tag, src[e]);
      for (int e = tid; e < B * np; e += NT) dst[e] = get_word(other + e, tag, spin, xerr);
      __syncthreads();
    }
    // the middle block, and y of this half's level k - 2 block
    for (int t = wv; t < 2; t += NW) {
      C acc[RPL];
      if (t == 0) {
        nd_mv3<RPL>(acc, mat(mid, 0), own, oth, mone, zv, zero, B);
        nd_store<RPL>(own, acc, B);
      } else if (k >= 3) {
        const int e = (half ? 3 : 1) * (1 << (k - 2)) - 1;
        nd_mv3<RPL>(acc, mat(e, 0), vec(e), zv, zero, zv, zero, B);
        nd_store<RPL>(vec(e), acc, B);
      }
    }
    __syncthreads();
    // backward: level l's blocks e = odd 2^l - 1 from the solution of the levels above
    for (int l = k - 2; l >= 0; --l) {
      const int s = 1 << l, ne = 1 << (k - 2 - l), o0 = half ? 2 * ne + 1 : 1;
      for (int t = wv; t < ne; t += NW) {
        const int e = (o0 + 2 * t) * s - 1;
        const bool hl = e - s >= 0, hu = e + s <= n - 1;
        C acc[RPL];
        if (l >= 1) {
          nd_load<RPL>(acc, vec(e), B);
          if (hl) nd_mv<RPL>(acc, mat(e, 1), mone, vec(e - s), B);
          if (hu) nd_mv<RPL>(acc, mat(e, 2), mone, vec(e + s), B);
        } else {
          nd_mv3<RPL>(acc, mat(e, 0), vec(e), hl ? vec(e - 1) : zv, hl ? cf[e + 1] : zero,
                      hu ? vec(e + 1) : zv, hu ? cb[e + 1] : zero, B);
        }
        nd_store<RPL>(vec(e), acc, B);
      }
      __syncthreads();
    }
  }

  // Line (g, l) of slab g.  Input: forward, the slab input on the line's rows minus the
  // couplings to the new iterate on the row below (j0 - 1) and/or above (j1 + 1); backward,
  // the coupling to the row above (lower front) or below (upper front).  The slab input is f
  // on the group's layers minus the couplings to u on the layer below (k0 - 1) and/or above
  // (k1 + 1) forward, or those couplings alone backward.  Couplings that another member
  // produced are read from what it sent: the layer buffer (lay_above: the layer above, in
  // the middle slab; lay_below: the layer below, in front 1's first backward slab) and the
  // received row (x_above: the row above, in the middle line; x_below: the row below, in
  // front 1's first backward line).  Output: v = x (forward) or v -= x on the line's rows.
  __device__ __forceinline__ void line(int g, int kind, int l, int lkind, bool lay_above, bool lay_below,
                                       bool x_above, bool x_below) {
    const GroupInfo gz = groups[g], gy = groups[Gz + l];
    const int Wz = gz.W, k0 = gz.first, k1 = gz.last, zw0 = gz.w0;
    const int Wy = gy.W, B = Wy * Wz, j0 = gy.first, j1 = gy.last, yw0 = gy.w0;
    const bool ofwd = kind <= kFwdMid, ifwd = lkind <= kFwdMid;
    const bool from_below = (kind == kFwdLow && g > 0) || kind == kFwdMid || kind == kBwdHigh;
    const bool from_above = (kind == kFwdHigh && g < Gz - 1) || kind == kFwdMid || kind == kBwdLow;
    const bool in_below = (lkind == kFwdLow && l > 0) || lkind == kFwdMid;
    const bool in_above = (lkind == kFwdHigh && l < Gy - 1) || lkind == kFwdMid;
    const C* T = line_factors(g, l);
    C* yb = sb + L.ybuf;
    // The elements are taken kGatherU per thread at a time: the loads of f (the bulk of the
    // gather) for the whole batch are issued first, so a batch waits for one memory latency.
    auto gather = [&]() {
      const C zero = mk((R)0, (R)0);
      const bool need_f = ifwd && ofwd;
      Walk wk(tid, NT, ni, Wz);
      for (int e0 = tid; e0 < ni * B; e0 += kGatherU * NT) {
        Walk w2 = wk;
        TI fr[kGatherU];
#pragma unroll
        for (int r = 0; r < kGatherU; ++r) {
          const int e = e0 + r * NT;
          fr[r] = TI{};
          if (e < ni * B && need_f) {
            const int j = yw0 + wk.hi, k = zw0 + wk.lo;
            if (j >= j0 && j <= j1 && k >= k0 && k <= k1) fr[r] = f[gidx(ilo + wk.ii, j, k)];
          }
          wk.next();
        }
#pragma unroll
        for (int r = 0; r < kGatherU; ++r) {
        const int e = e0 + r * NT;
        if (e >= ni * B) break;
        const int jj = w2.hi, kk = w2.lo, qq = jj * Wz + kk, i = ilo + w2.ii;
        w2.next();
        const int j = yw0 + jj, k = zw0 + kk;
        C val = zero;
        if (ifwd) {
          if (j >= j0 && j <= j1) {
            const C ub = (from_below && k == k0)
                             ? (lay_below ? lay[(long long)(j - 1) * n + i] : cvt<C>(u[gidx(i, j, k0 - 1)]))
                             : zero;
            const C ua = (from_above && k == k1)
                             ? (lay_above ? lay[(long long)(j - 1) * n + i] : cvt<C>(u[gidx(i, j, k1 + 1)]))
                             : zero;
            if (ofwd) {
              if (k >= k0 && k <= k1) {
                val = cvt<C>(fr[r]);
                val = csub(val, cmul(cf[k0], ub));
                val = csub(val, cmul(cb[k1], ua));
              }
            } else {
              val = cadd(cmul(cb[k1], ua), cmul(cf[k0], ub));
            }
            if (in_below && j == j0) val = csub(val, cmul(cf[j0], v[((long long)kk * n + (j0 - 2)) * n + i]));
            if (in_above && j == j1)
              val = csub(val, cmul(cb[j1], x_above ? xrow[kk * ni + (i - ilo)]
                                                   : v[((long long)kk * n + j1) * n + i]));
          }
        } else if (lkind == kBwdLow && j == j1) {
          val = cmul(cb[j1], v[((long long)kk * n + j1) * n + i]);
        } else if (lkind == kBwdHigh && j == j0) {
          val = cmul(cf[j0], x_below ? xrow[kk * ni + (i - ilo)] : v[((long long)kk * n + (j0 - 2)) * n + i]);
        }
        yb[(i - ilo) * B + qq] = val;
        }
      }
    };
    solve_any(T, B, gather);
    const int npy = j1 - j0 + 1;
    Walk wk(tid, NT, ni, Wz);
    for (int e = tid; e < ni * Wz * npy; e += NT, wk.next()) {
      const int i = ilo + wk.ii, kk = wk.lo, jp = wk.hi;
      const int qq = (j0 - yw0 + jp) * Wz + kk;
      C* p = v + ((long long)kk * n + (j0 + jp - 1)) * n + i;
      *p = ifwd ? yb[(i - ilo) * B + qq] : csub(*p, yb[(i - ilo) * B + qq]);
    }
    __syncthreads();
  }

  // E2 / E3 words of this slab step (kind 0: E2, 1: E3) of this member's outer front and half
  __device__ __forceinline__ unsigned long long* w23(int kind) const {
    return xs + ((kind * 2 + ofront) * 2 + half) * e23 + (long long)(sstep & 1) * (e23 / 2);
  }
  // row r (1-based) of the slab iterate on Wz layers and this half: send / receive into xrow
  __device__ __forceinline__ void send_row(unsigned long long* w, int r, int Wz, unsigned long long tag) {
    for (int e = tid; e < Wz * ni * np; e += NT) {
      const int val = e / np, kk = val / ni, ii = val - kk * ni;
      const C x = v[((long long)kk * n + (r - 1)) * n + ilo + ii];
      const unsigned* pc = reinterpret_cast<const unsigned*>(&x);
      unsigned piece = pc[0];
#pragma unroll
      for (int k = 1; k < np; ++k)
        if (e - val * np == k) piece = pc[k];
      put_word(w + e, tag, piece);
    }
  }
  __device__ __forceinline__ void recv_row(const unsigned long long* w, int Wz, unsigned long long tag) {
    for (int e = tid; e < Wz * ni; e += NT) {
      unsigned pc[np];
#pragma unroll
      for (int k = 0; k < np; ++k) pc[k] = get_word(w + (long long)e * np + k, tag, spin, xerr);
      xrow[e] = *reinterpret_cast<const C*>(pc);   // e = kk * ni + ii
    }
    lds_barrier();
  }

  // slab step: the inner sweep (Algorithm 4) of x3-group g (kind: how its input couples), then
  // the slab output on this member's rows.  The lines in order: one inner front, all of them
  // forward then backward; two inner fronts, front 0 its lines forward, the middle line
  // (after E2 arrives), E3 out, its lines backward; front 1 its lines forward, E2 out, E3 in,
  // its lines backward.
  __device__ __forceinline__ void slab(int g, int kind) {
    const bool lay_above = fronts == 2 && kind == kFwdMid;
    const bool lay_below = fronts == 2 && kind == kBwdHigh && g == zmid + 1;
    const GroupInfo gz = groups[g];
    const int Wz = gz.W;
    const int ym = ymid;
    const int rA = fronts_inner == 2 ? groups[Gz + ym + 1].first : 1;
    const int rB = fronts_inner == 2 ? groups[Gz + ym].last : n;
    const unsigned long long tag = ((seq0 + 1 + sstep) & 0xffffffffull) << 32;
    const int c1 = Gy - 1 - ym;
    const int nl = fronts_inner == 1 ? 2 * Gy - 1 : (ifront == 0 ? 2 * ym + 1 : 2 * c1);
    for (int lp = 0; lp < nl; ++lp) {
      int l, lkind;
      bool x_above = false, x_below = false;
      if (fronts_inner == 1) {
        const int2 lk = sweep_at(0, Gy, ym, 0, lp);
        l = lk.x;
        lkind = lk.y;
      } else if (ifront == 0) {
        if (lp < ym) {
          l = lp;
          lkind = kFwdLow;
        } else if (lp == ym) {
          recv_row(w23(0), Wz, tag);                            // E2
          l = ym;
          lkind = kFwdMid;
          x_above = true;
        } else {
          l = 2 * ym - lp;
          lkind = kBwdLow;
        }
      } else {
        if (lp < c1) {
          l = Gy - 1 - lp;
          lkind = kFwdHigh;
        } else {
          if (lp == c1) {
            send_row(w23(0), rA, Wz, tag);                      // E2
            recv_row(w23(1), Wz, tag);                          // E3
          }
          l = ym + 1 + (lp - c1);
          lkind = kBwdHigh;
          x_below = lp == c1;
        }
      }
      line(g, kind, l, lkind, lay_above, lay_below, x_above, x_below);
      if (fronts_inner == 2 && ifront == 0 && lp == ym) send_row(w23(1), rB, Wz, tag);   // E3
    }
    const int r0 = fronts_inner == 2 && ifront == 1 ? rA : 1;
    const int r1 = fronts_inner == 2 && ifront == 0 ? rB : n;
    const bool ofwd = kind <= kFwdMid;
    const int k0 = gz.first, k1 = gz.last, zw0 = gz.w0;
    const int nph = k1 - k0 + 1, nr = r1 - r0 + 1;
    Walk wk(tid, NT, ni, nr);
    for (int e = tid; e < ni * nr * nph; e += NT, wk.next()) {
      const int i = ilo + wk.ii, jm = r0 - 1 + wk.lo, kp = wk.hi;
      const int kk = k0 - zw0 + kp;
      const C val = v[((long long)kk * n + jm) * n + i];
      const long long id = gidx(i, jm + 1, k0 + kp);
      u[id] = ofwd ? cvt<TO>(val) : cvt<TO>(csub(cvt<C>(u[id]), val));
    }
    __syncthreads();
    sstep += 1;
  }

  // rows of this member's inner front (the middle x2-group belongs to front 0)
  __device__ __forceinline__ int2 my_rows() const {
    if (fronts_inner == 1) return make_int2(1, n);
    const int rB = groups[Gz + ymid].last;
    return ifront == 0 ? make_int2(1, rB) : make_int2(rB + 1, n);
  }
  // E4 / E5: layer k of u on this member's rows and half
  __device__ __forceinline__ void send_layer(unsigned long long* w, int k, unsigned long long tag) {
    const int2 rr = my_rows();
    const int nr = rr.y - rr.x + 1;
    for (int e = tid; e < nr * ni * np; e += NT) {
      const int val = e / np, jr = val / ni, ii = val - jr * ni;
      const C x = cvt<C>(u[gidx(ilo + ii, rr.x + jr, k)]);
      const unsigned* pc = reinterpret_cast<const unsigned*>(&x);
      unsigned piece = pc[0];
#pragma unroll
      for (int q = 1; q < np; ++q)
        if (e - val * np == q) piece = pc[q];
      put_word(w + e, tag, piece);
    }
  }
  __device__ __forceinline__ void recv_layer(const unsigned long long* w, unsigned long long tag) {
    const int2 rr = my_rows();
    const int nr = rr.y - rr.x + 1;
    for (int e = tid; e < nr * ni; e += NT) {
      unsigned pc[np];
#pragma unroll
      for (int k = 0; k < np; ++k) pc[k] = get_word(w + (long long)e * np + k, tag, spin, xerr);
      const int jr = e / ni, ii = e - jr * ni;
      lay[(long long)(rr.x + jr - 1) * n + ilo + ii] = *reinterpret_cast<const C*>(pc);
    }
    __syncthreads();
  }

  // The whole sweep of this member, one slab step at a time.  One front: slabs 0..G-1 forward
  // and G-2..0 backward.  Two fronts: outer front 0 its slabs forward, the middle slab (after
  // E4 arrives), E5 out, its slabs backward; outer front 1 its slabs forward, E4 out, E5 in,
  // its slabs backward.
  __device__ __forceinline__ void sweep() {
    const int zm = zmid, c1 = Gz - 1 - zm;
    const unsigned long long tag = ((seq0 + 1) & 0xffffffffull) << 32;   // E4 / E5: once
    unsigned long long* w4 = xs + 8 * e23 + ((0 * 2 + ifront) * 2 + half) * e45;
    unsigned long long* w5 = xs + 8 * e23 + ((1 * 2 + ifront) * 2 + half) * e45;
    const int ns = fronts == 1 ? 2 * Gz - 1 : (ofront == 0 ? 2 * zm + 1 : 2 * c1);
    for (int si = 0; si < ns; ++si) {
      int g, kind;
      if (fronts == 1) {
        const int2 gk = sweep_at(0, Gz, zm, 0, si);
        g = gk.x;
        kind = gk.y;
      } else if (ofront == 0) {
        if (si < zm) {
          g = si;
          kind = kFwdLow;
        } else if (si == zm) {
          recv_layer(w4, tag);                                  // E4
          g = zm;
          kind = kFwdMid;
        } else {
          g = 2 * zm - si;
          kind = kBwdLow;
        }
      } else {
        if (si < c1) {
          g = Gz - 1 - si;
          kind = kFwdHigh;
        } else {
          if (si == c1) {
            send_layer(w4, groups[zm + 1].first, tag);          // E4
            recv_layer(w5, tag);                                // E5
          }
          g = zm + 1 + (si - c1);
          kind = kBwdHigh;
        }
      }
      slab(g, kind);
      if (fronts == 2 && ofront == 0 && si == zm) send_layer(w5, groups[zm].last, tag);   // E5
    }
  }

  // exact solve of the single line (line_g, line_l) on its own grid (x1 fastest, then the x2
  // window row, then the x3 window layer), input and output complex128
  __device__ __forceinline__ void single_line(int g, int l) {
    const int Wz = groups[g].W, Wy = groups[Gz + l].W, B = Wy * Wz;
    const C* T = line_factors(g, l);
    C* yb = sb + L.ybuf;
    const double2* r = reinterpret_cast<const double2*>(f);
    auto gather = [&]() {
      for (int e = tid; e < ni * B; e += NT) {
        const int qq = e / ni, i = ilo + e - qq * ni;
        const int jj = qq / Wz, kk = qq - jj * Wz;
        yb[(i - ilo) * B + qq] = cvt<C>(r[i + (long long)n * (jj + (long long)Wy * kk)]);
      }
    };
    solve_any(T, B, gather);
    double2* x = reinterpret_cast<double2*>(u);
    for (int e = tid; e < ni * B; e += NT) {
      const int qq = e / ni, i = ilo + e - qq * ni;
      const int jj = qq / Wz, kk = qq - jj * Wz;
      x[i + (long long)n * (jj + (long long)Wy * kk)] = cvt<double2>(yb[(i - ilo) * B + qq]);
    }
  }
};

// Workgroup b sits on XCD b mod 8 (the dispatcher's round-robin).  Placement 0: right-hand
// side slot 8 (b / 8 / wpr) + b mod 8, member (b / 8) mod wpr, so the members of a right-hand
// side share one XCD's L2 for their exchanges.  Placement 1: slot b / wpr, member b mod wpr,
// so with eight members every XCD runs one member of each right-hand side: one part of the
// factor stream (a member's fronts and half of every line) read by all right-hand sides
// through one L2, the exchanges crossing XCDs.  Placement 2: the two halves of a line solve
// (members 2q and 2q + 1) on one XCD, XCD q (8 / P) + slot mod (8 / P) for the P = wpr / 2
// pairs of a right-hand side, so the exchange inside a line solve stays in one L2 and each
// XCD reads 1 / P of the factor stream.  Slots past R (the grid is rounded up) exit at once.
__device__ __forceinline__ void member_of(const SweepArgs& a, int b, int& slot, int& member) {
  if (a.xmap == 1) {
    slot = b / a.wpr;
    member = b - slot * a.wpr;
  } else if (a.xmap == 2) {
    const int per = 16 / a.wpr;                    // right-hand sides sharing an XCD's pair type
    const int x = b & 7, k = b >> 3, q = x / per;  // k: (slot / per, half)
    slot = (k >> 1) * per + (x - q * per);
    member = 2 * q + (k & 1);
  } else {
    const int k8 = b >> 3, grp = k8 / a.wpr;
    member = k8 - grp * a.wpr;
    slot = grp * 8 + (b & 7);
  }
}

template <typename R, typename TI, typename TO, int NCA, int CWA, int DA, int NCB, int CWB, int DB,
          bool ADJ>
__global__ void __launch_bounds__((kernel_threads_max<NCA, CWA, NCB, CWB>())) k_sweep(SweepArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int slot, member;
  member_of(a, (int)blockIdx.x, slot, member);
  if (slot >= a.R) return;
  Sweeper<R, TI, TO, NCA, CWA, DA, NCB, CWB, DB, ADJ> s(a, smem_raw, slot, member);
  if (a.mode == 1) s.single_line(a.line_g, a.line_l);
  else s.sweep();
}

// The same sweep with every line solved by nested dissection (complex64, forward sweeps):
// the members, their exchanges and the placements are those of k_sweep
constexpr int kNdThreads = 512;
template <typename TI, typename TO>
__global__ void __launch_bounds__(kNdThreads) k_sweep_nd(SweepArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int slot, member;
  member_of(a, (int)blockIdx.x, slot, member);
  if (slot >= a.R) return;
  Sweeper<float, TI, TO, 8, 7, 2, 8, 11, 2, false, true> s(a, smem_raw, slot, member);
  if (a.mode == 1) s.single_line(a.line_g, a.line_l);
  else s.sweep();
}

}  // namespace sweepk

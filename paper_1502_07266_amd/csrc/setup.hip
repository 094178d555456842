// Setup of the recursive sweep (Algorithm 5, with Algorithm 3 per slab): every quasi-1D
// auxiliary problem is factored by the block LDU of Sec. 3 with x1 as the block index
// (Sec. 4.1: dimensions 3 and 2 grouped first, dimension 1 last).
//
// For line (g, l) the window grid is x1 = 1..n times the x2-window of group l times the
// x3-window of group g.  In eq. (3) the stretching s_d depends on x_d only, so the coupling
// between x1-neighbour blocks is a multiple of the identity:
//     K_{i,i-1} = l_i I,  l_i = s1_i s1_{i-1/2} / h^2,   K_{i,i+1} = u_i I,  u_i = s1_i s1_{i+1/2} / h^2,
// and the block recursion S_1 = D_1, S_i = D_i - K_{i,i-1} S_{i-1}^{-1} K_{i-1,i} becomes the
// scaled update S_i = D_i - (l_i u_{i-1}) T_{i-1} (and its mirror image from the other end):
// the only dense work is inverting S_i.
// D_i is the 5-point (x2, x3) operator of the window plus the x1 diagonal and kappa.
//
// One workgroup owns a line, or one half of a two-sided line: it forms S_i in LDS, inverts it
// by Gauss-Jordan elimination with partial pivoting in panels (the eliminations outside each
// panel as one complex matrix product on the matrix cores), stores T_i = S_i^{-1} and keeps
// it in registers for the next Schur update.  The blocks are eliminated
// from both ends towards the middle (see the order below), which halves the dependent chain
// of the line solve; the two halves do not meet before the middle block, so they are factored
// by two workgroups and the middle blocks by a launch of their own.  All
// lines are independent (Sec. 6 notes that the setup is O(n^2) independent quasi-1D
// problems).  The LDS of a launch is sized by its largest block, so the lines on a middle
// group (few, with blocks up to 128) get a launch of their own, on a side stream beside the
// launches of the other lines (split again by block size, so that the many small ones share
// CUs several at a time).
#include <algorithm>

#include "common.h"

namespace {

constexpr int kMaxW = 64;
constexpr int kMaxB = 128;
constexpr int kSetupThreads = 256;        // lines with two-chain blocks (B <= 64)
constexpr int kSetupThreadsBig = 1024;    // lines on a middle group (B up to 128)
constexpr size_t kSetupLdsBytes = 152 * 1024;   // dynamic LDS the setup may take (of 160 KiB)
constexpr size_t kSmallLds = 20 * 1024;         // a block within this: several workgroups per CU

struct SetupArgs {
  int n, Gz, Gy, p;
  int fronts, zmid, fronts_inner, ymid;
  int part;          // 0: whole lines; 1: the two halves of two-sided lines, one workgroup
                     // each (workgroup 2w + h takes half h of line lines[w]); 2: their middle
                     // blocks, after part 1
  const int* lines;  // the lines of this launch (workgroup w takes line lines[w])
  double h;
  const GroupInfo* groups;
  const long long* line_off;
  const double2* sbd;
  const double2* smv;
  const double* kappa;
  void* factors;
  int* err;
};

// s at half-step t of the window of group gi: the moving profile replaces the boundary one
// strictly below the group's first node when the window extends below it, and (mirrored,
// measured from the plane p+1 spacings above the last node) strictly above the group's last
// node when the window extends above it
__device__ inline double2 window_s(const SetupArgs& a, const GroupInfo& gi, int t) {
  if (gi.w0 < gi.first && t < 2 * gi.first) return a.smv[t - 2 * (gi.first - a.p - 1)];
  if (gi.w0 + gi.W - 1 > gi.last && t > 2 * gi.last) return a.smv[2 * (gi.last + a.p + 1) - t];
  return a.sbd[t];
}

// ---- matrix-core helpers: one 16 x 16 x 4 real product per call, D = A B + C.  Lane l
// supplies A[l mod 16][l / 16] and B[l / 16][l mod 16] and holds four elements of column
// l mod 16 of D: rows 4 (l / 16) + i (fp32) or l / 16 + 4 i (fp64), i = 0..3.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <typename R> struct Mfma;
template <> struct Mfma<float> {
  using acc = f32x4;
  static __device__ __forceinline__ acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int i) { return 4 * (l >> 4) + i; }
};
template <> struct Mfma<double> {
  using acc = f64x4;
  static __device__ __forceinline__ acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int i) { return (l >> 4) + 4 * i; }
};

// ---- wave-level helpers of the pivot search (one wavefront of 64 lanes)
__device__ __forceinline__ unsigned umax(unsigned a, unsigned b) { return a > b ? a : b; }
// maximum over the wave: prefix maxima inside each row of 16 lanes (row_shr 1, 2, 4, 8; a
// lane without a source keeps 0), so lane 15 of each row holds the row's maximum; the four
// are combined as scalars
__device__ __forceinline__ unsigned wave_max(unsigned v) {
  v = umax(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, false));
  v = umax(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, false));
  v = umax(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, false));
  v = umax(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, false));
  const unsigned a = (unsigned)__builtin_amdgcn_readlane((int)v, 15);
  const unsigned b = (unsigned)__builtin_amdgcn_readlane((int)v, 31);
  const unsigned c = (unsigned)__builtin_amdgcn_readlane((int)v, 47);
  const unsigned d = (unsigned)__builtin_amdgcn_readlane((int)v, 63);
  return umax(umax(a, b), umax(c, d));
}
// 1 / a: fp32 with the hardware reciprocal of |a|^2 (one ulp), fp64 exact
__device__ __forceinline__ float2 cinv_fast(float2 a) {
  const float r = __builtin_amdgcn_rcpf(a.x * a.x + a.y * a.y);
  return make_float2(a.x * r, -a.y * r);
}
__device__ __forceinline__ double2 cinv_fast(double2 a) { return cinv(a); }
// order-preserving 32-bit key of a magnitude m >= 0 (NaN above every finite value)
__device__ __forceinline__ unsigned mag_key(float m) { return __float_as_uint(m); }
__device__ __forceinline__ unsigned mag_key(double m) { return (unsigned)__double2hiint(m); }
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}
template <typename C> __device__ __forceinline__ C lane_value(C v, int l) {
  return C{lane_value(v.x, l), lane_value(v.y, l)};
}

// Line setup: per block, S_i = D_i - (coupling) T_prev is formed in LDS and inverted in place
// by Gauss-Jordan elimination in panels of NB columns:
//  * the panel: wavefront 0 holds the panel's columns of every row in registers (lane l rows
//    l and l + 64), chooses each pivot as the largest magnitude in the column among the rows
//    not yet used (a wave maximum, no barrier), broadcasts the pivot row with readlane and
//    eliminates the column from all other rows.  Rows are not moved: the pivot of column k is
//    recorded as piv[k].  The pivot row's scaling is kept as a per-row factor until the panel
//    is written back;
//  * the columns outside the panel: every Gauss-Jordan step of the panel is the same left
//    multiplication of all columns, so they take it at once, A[:, rest] = Z + F G with F the
//    finished panel (B x NB), G the panel's pivot rows of A[:, rest] before it and Z that
//    matrix with those rows zero: a complex product on the matrix cores (four real 16 x 16 x
//    4 products per complex one), tiles spread over all waves.
// After the last panel, T = S^{-1} is the stored array R read as T[r][piv[k]] = R[piv[r]][k].
// RPL: rows per lane of the panel wave (B <= 64 RPL); NB: panel width.  LDS: the block
// (B x B) and the panel's pivot rows (NB x B).
template <typename R, int NTB, int RPL>
__global__ void __launch_bounds__(NTB) __attribute__((amdgpu_waves_per_eu(NTB == 256 && sizeof(R) == 4 ? 5 : 1)))
k_line_setup(SetupArgs a) {
  using C = typename cx<R>::type;
  using M = Mfma<R>;
  constexpr int NB = sizeof(R) == 8 && RPL == 2 ? 4 : 8;
  constexpr int NW = NTB / 64;
  constexpr int BMAX = 64 * RPL;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double2 syn[kMaxW], syh[kMaxW + 1], szn[kMaxW], szh[kMaxW + 1];
  __shared__ int piv[kMaxB], qinv[kMaxB], pnl[kMaxB];
  // storage maps: logical row u of the current block is LDS row rmap[u], logical column v
  // LDS column cmap[v] (rinv, cinv_ the inverses)
  __shared__ int rmap[kMaxB], cmap[kMaxB], rinv[kMaxB], cinv_[kMaxB];
  __shared__ int bad_s;

  const int w = a.part == 1 ? (int)blockIdx.x >> 1 : (int)blockIdx.x;
  const int half = a.part == 1 ? (int)blockIdx.x & 1 : 0;
  const int line = a.lines[w];
  const int g = line / a.Gy, l = line % a.Gy;
  const GroupInfo gz = a.groups[g], gy = a.groups[a.Gz + l];
  const int Wz = gz.W, Wy = gy.W, B = Wy * Wz;
  const int n = a.n;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  for (int u = tid; u < kMaxB; u += NTB) rmap[u] = cmap[u] = rinv[u] = cinv_[u] = u;
  C* S = reinterpret_cast<C*>(smem_raw);
  C* Gp = S + B * B;   // the current panel's pivot rows, as they were before the panel
  C* out = reinterpret_cast<C*>(a.factors) + a.line_off[line];
  const double ih2 = 1.0 / (a.h * a.h);
  const C zero = mk((R)0, (R)0);

  if (tid < Wy) syn[tid] = window_s(a, gy, 2 * (gy.w0 + tid));
  if (tid <= Wy) syh[tid] = window_s(a, gy, 2 * (gy.w0 + tid) - 1);
  if (tid < Wz) szn[tid] = window_s(a, gz, 2 * (gz.w0 + tid));
  if (tid <= Wz) szh[tid] = window_s(a, gz, 2 * (gz.w0 + tid) - 1);
  if (tid == 0) bad_s = 0;
  __syncthreads();

  // Two-sided elimination order: blocks 0..m-1 upwards, blocks n-1..m+1 downwards, and the
  // middle block m = n/2 (integer division) last, whose Schur complement takes the update
  // from both sides.  It is the block LDU of Sec. 3 with the blocks in that order (every
  // block eliminated is an end of the remaining chain, so there is no fill); the sweep runs
  // the two halves of each line solve as two concurrent chains.
  const int mid = n / 2;
  const bool has_lower = mid + 1 <= n - 1;
  const C* T_mid_minus1 = out + (long long)(mid - 1) * B * B;   // T_{m-1}, stored at t = m - 1
  // steps t0..t1-1 of the order: all, one half (the halves do not meet before the middle
  // block, so they run in two workgroups), or the middle block alone, which then reads both
  // neighbours' factors from HBM
  int t0 = 0, t1 = n;
  if (a.part == 1) {
    t0 = half ? mid : 0;
    t1 = half ? n - 1 : mid;
  } else if (a.part == 2) {
    t0 = n - 1;
  }
  // The factor of the previous block of this workgroup's order stays in LDS where the
  // inversion left it: T[u][v] at row rmap[u], column cmap[v].  The next Schur complement is
  // formed in place, element by element, so the storage order is carried along.
  for (int t = t0; t < t1; ++t) {
    const int i = t < mid ? t : (t < n - 1 ? n - 1 - (t - mid) : mid);
    const int m = i + 1;  // global x1 node of block i
    const double2 sxn = a.sbd[2 * m], sxd = a.sbd[2 * m - 1], sxu = a.sbd[2 * m + 1];
    const double2 dx = cscale(cmul(sxn, cadd(sxu, sxd)), -ih2);
    // update from the block below: l_i u_{i-1} = (s_m s_{m-1/2} / h^2)(s_{m-1} s_{m-1/2} / h^2)
    // update from the block above: u_i l_{i+1} = (s_m s_{m+1/2} / h^2)(s_{m+1} s_{m+1/2} / h^2)
    const C sc_below = cvt<C>(cmul(cscale(cmul(sxn, sxd), ih2), cscale(cmul(a.sbd[2 * m - 2], sxd), ih2)));
    const C sc_above = cvt<C>(cmul(cscale(cmul(sxn, sxu), ih2), cscale(cmul(a.sbd[2 * m + 2], sxu), ih2)));
    const bool is_mid = t == n - 1;
    const bool use_a = (t > 0 && t < mid) || (t > mid && t < n - 1) || is_mid;
    const C scA = (t < mid || is_mid) ? sc_below : sc_above;
    // The previous block of this workgroup's order is in LDS (a workgroup's first block has
    // none); the middle block of a two-sided line is a launch's first block and reads both
    // neighbours' factors from HBM (T_{m-1} and T_{m+1}, or only T_{m-1} when nothing lies
    // above it), as does the whole-line order for T_{m-1}.
    const bool prev_lds = use_a && t > t0;
    const C* TA = is_mid ? T_mid_minus1 : nullptr;                      // scale sc_below
    const C* TB = (is_mid && has_lower && t == t0) ? out + (long long)(mid + 1) * B * B : nullptr;
    const C scL = is_mid ? sc_above : scA;   // scale of the factor in LDS
    for (int sr_ = wv; sr_ < B; sr_ += NW) {   // LDS row, logical row r
      const int r = rinv[sr_];
      const int jr = r / Wz, kr = r - jr * Wz;
      for (int sc_ = lane; sc_ < B; sc_ += 64) {   // LDS column, logical column c
        const int c = cinv_[sc_];
        const int e = r * B + c, se = sr_ * B + sc_;
        const int jc = c / Wz, kc = c - jc * Wz;
        double2 val = make_double2(0.0, 0.0);
        if (r == c) {
          const int k = gz.w0 + kr, jj = gy.w0 + jr;
          const double kap = a.kappa[((long long)(k - 1) * n + (jj - 1)) * n + i];
          double2 dy = cscale(cmul(syn[jr], cadd(syh[jr + 1], syh[jr])), -ih2);
          double2 dz = cscale(cmul(szn[kr], cadd(szh[kr + 1], szh[kr])), -ih2);
          val = cadd(cadd(dx, dy), dz);
          val.x += kap;
        } else if (jr == jc) {
          if (kc == kr + 1) val = cscale(cmul(szn[kr], szh[kr + 1]), ih2);
          else if (kc == kr - 1) val = cscale(cmul(szn[kr], szh[kr]), ih2);
        } else if (kr == kc) {
          if (jc == jr + 1) val = cscale(cmul(syn[jr], syh[jr + 1]), ih2);
          else if (jc == jr - 1) val = cscale(cmul(syn[jr], syh[jr]), ih2);
        }
        C v = cvt<C>(val);
        if (prev_lds) v = csub(v, cmul(scL, S[se]));
        if (TA) v = csub(v, cmul(sc_below, TA[e]));
        if (TB) v = csub(v, cmul(sc_above, TB[e]));
        S[se] = v;
      }
    }
    for (int r = tid; r < B; r += NTB) pnl[r] = -1;
    __syncthreads();

    // ---- Gauss-Jordan in panels
    for (int K = 0; K < B; K += NB) {
      const int nbp = B - K < NB ? B - K : NB;
      // the panel wave changes from panel to panel and between workgroups, so that the
      // workgroups sharing a CU do not all load the same SIMD with their serial parts
      if (wv == ((int)blockIdx.x + K / NB) % NW) {
        C x[RPL][NB], sr[RPL];
        bool done[RPL];   // pivot row of an earlier column
        int prs[NB];      // the panel's pivot rows
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
          const int row = lane + 64 * rr;
          done[rr] = row >= B || pnl[row] >= 0;
          sr[rr] = mk((R)1, (R)0);
#pragma unroll
          for (int c = 0; c < NB; ++c) x[rr][c] = (row < B && c < nbp) ? S[row * B + K + c] : zero;
        }
#pragma unroll
        for (int kk = 0; kk < NB; ++kk) {
          if (kk < nbp) {
            // pivot: the largest |s x| in column kk among this lane's rows not yet used
            unsigned key = 0;
            int sel = 0;
            bool any = false;
  #pragma unroll
            for (int rr = 0; rr < RPL; ++rr) {
              if (done[rr]) continue;
              const unsigned kb = mag_key(cabs2(sr[rr]) * cabs2(x[rr][kk]));
              if (!any || kb > key) {
                key = kb;
                sel = rr;
              }
              any = true;
            }
            const unsigned mk_ = wave_max(any ? key : 0u);
            unsigned long long bal = __ballot(any && key == mk_);
            if (bal == 0) bal = __ballot(any);   // (not reached: some lane holds the maximum)
            const int p = __builtin_amdgcn_readfirstlane((int)__builtin_ctzll(bal));
            const int rsel = __builtin_amdgcn_readlane(sel, p);
            const int pr = p + 64 * rsel;
            C prow[NB];
  #pragma unroll
            for (int c = 0; c < NB; ++c) {
              C v = x[0][c];
  #pragma unroll
              for (int rr = 1; rr < RPL; ++rr)
                if (rsel == rr) v = x[rr][c];
              prow[c] = lane_value(v, p);
            }
            C sv = sr[0];
  #pragma unroll
            for (int rr = 1; rr < RPL; ++rr)
              if (rsel == rr) sv = sr[rr];
            const C sp = lane_value(sv, p);
            C pv = cmul(sp, prow[kk]);
            const R pm = cabs2(pv);
            if (!(pm > (R)0) || !isfinite(pm)) {   // singular block: flagged, finished with a unit pivot
              if (lane == 0) bad_s = 1;
              pv = mk((R)1, (R)0);
            }
            const C pinv = cinv_fast(pv);
            const C spn = cmul(pinv, sp);   // the pivot row's scale after the step
            const C isp = cmul(pinv, prow[kk]);   // 1 / sp
  #pragma unroll
            for (int rr = 0; rr < RPL; ++rr) {
              if (lane == p && rr == rsel) {
                // stored * scale is the row's value: column kk becomes pinv
                sr[rr] = spn;
                x[rr][kk] = isp;
                done[rr] = true;
              } else {
                const C f = x[rr][kk];
                const C gg = cmul(f, spn);
  #pragma unroll
                for (int c = 0; c < NB; ++c) x[rr][c] = csub(x[rr][c], cmul(gg, prow[c]));
                x[rr][kk] = C{-(f.x * pinv.x - f.y * pinv.y), -(f.x * pinv.y + f.y * pinv.x)};
              }
            }
            prs[kk] = pr;
            if (lane == 0) {
              piv[K + kk] = pr;
              pnl[pr] = K;
            }
          }
        }
        // the panel's pivot rows as they were before it (the columns outside the panel)
#pragma unroll
        for (int kk = 0; kk < NB; ++kk)
          if (kk < nbp)
            for (int c = lane; c < B; c += 64) Gp[kk * B + c] = S[prs[kk] * B + c];
        // the finished panel, with each row's scale applied
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
          const int row = lane + 64 * rr;
          if (row >= B) continue;
#pragma unroll
          for (int c = 0; c < NB; ++c)
            if (c < nbp) S[row * B + K + c] = cmul(sr[rr], x[rr][c]);
        }
      }
      __syncthreads();
      // A[:, rest] = Z + F G on the matrix cores, tile by tile (16 x 16, K steps of 4): G
      // comes from the copy of the pivot rows, so a tile's result can go straight back
      const int RT = (B + 15) >> 4, ntile = RT * RT;
      for (int tile = wv; tile < ntile; tile += NW) {
        const int ti = tile / RT, tj = tile - ti * RT;
        const int col = tj * 16 + (lane & 15);
        if (tj * 16 >= K && tj * 16 + 15 < K + nbp) continue;   // all inside the panel
        typename M::acc are, aim;
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int row = ti * 16 + M::row(lane, ii);
          const C z = (row < B && col < B && pnl[row] != K) ? S[row * B + col] : zero;
          are[ii] = z.x;
          aim[ii] = z.y;
        }
        const int frow = ti * 16 + (lane & 15);
        for (int k0 = 0; k0 < nbp; k0 += 4) {
          const int k = k0 + (lane >> 4);
          const C f = (frow < B && k < nbp) ? S[frow * B + K + k] : zero;
          const C gv = (k < nbp && col < B) ? Gp[k * B + col] : zero;
          are = M::mac(f.x, gv.x, are);
          are = M::mac(-f.y, gv.y, are);
          aim = M::mac(f.x, gv.y, aim);
          aim = M::mac(f.y, gv.x, aim);
        }
        if (col < B && (col < K || col >= K + nbp)) {
#pragma unroll
          for (int ii = 0; ii < 4; ++ii) {
            const int row = ti * 16 + M::row(lane, ii);
            if (row < B) S[row * B + col] = mk(are[ii], aim[ii]);
          }
        }
      }
      __syncthreads();
    }
    // The LDS array X (= the block with rows and columns in storage order) now holds R with
    // X^{-1}[a][b] = R[piv[a]][qinv[b]], qinv the inverse of piv; the block's inverse is
    // T[u][v] = X^{-1}[cmap[u]][rmap[v]], so T sits at row piv[cmap[u]], column
    // qinv[rmap[v]]: the storage maps of the next block
    for (int k = tid; k < B; k += NTB) qinv[piv[k]] = k;
    __syncthreads();
    int nr = 0, nc = 0;
    if (tid < B) {
      nr = piv[cmap[tid]];
      nc = qinv[rmap[tid]];
    }
    __syncthreads();
    if (tid < B) {
      rmap[tid] = nr;
      cmap[tid] = nc;
      rinv[nr] = tid;
      cinv_[nc] = tid;
    }
    __syncthreads();
    C* dst = out + (long long)i * B * B;
    for (int u = wv; u < B; u += NW) {
      const int ru = rmap[u];
      for (int v = lane; v < B; v += 64) dst[u * B + v] = S[ru * B + cmap[v]];
    }
    __syncthreads();   // the whole-line order's middle block reads T_{m-1} back from HBM
  }
  if (tid == 0 && bad_s) {
    atomicOr(&a.err[0], 1);
    atomicExch(&a.err[1], line);
  }
}

// one launch over `count` lines listed at d_lines, LDS sized for blocks up to maxB; two-sided
// lines take two launches, their halves on two workgroups each, then their middle blocks
template <int NTB>
hipError_t setup_launch(const helm_handle* h, SetupArgs a, const int* d_lines, int count, int maxB,
                        hipStream_t s, bool two_sided) {
  if (count <= 0) return hipSuccess;
  if (two_sided) {
    a.part = 1;
    hipError_t e = setup_launch<NTB>(h, a, d_lines, 2 * count, maxB, s, false);
    if (e != hipSuccess) return e;
    a.part = 2;
    return setup_launch<NTB>(h, a, d_lines, count, maxB, s, false);
  }
  a.lines = d_lines;
  const size_t csz = h->prec == HELM_C64 ? sizeof(float2) : sizeof(double2);
  // the block being inverted and the panel's pivot rows (the previous factor stays in the
  // block's array)
  constexpr int RPL = NTB == kSetupThreads ? 1 : 2;
  const size_t sm = setup_lds_bytes(maxB, (int)csz);
  if (sm > kSetupLdsBytes) return hipErrorInvalidValue;
  if (maxB > 64 * RPL) return hipErrorInvalidValue;
  if (h->prec == HELM_C64) {
    hipError_t e = hipFuncSetAttribute((const void*)k_line_setup<float, NTB, RPL>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    k_line_setup<float, NTB, RPL><<<count, NTB, sm, s>>>(a);
  } else {
    hipError_t e = hipFuncSetAttribute((const void*)k_line_setup<double, NTB, RPL>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    k_line_setup<double, NTB, RPL><<<count, NTB, sm, s>>>(a);
  }
  return hipGetLastError();
}

}  // namespace

// dynamic LDS of a setup workgroup: the block and the pivot rows of one panel
size_t setup_lds_bytes(int maxB, int csz) { return ((size_t)maxB * maxB + (size_t)8 * maxB) * csz; }
bool setup_fits(int maxB, int csz) { return maxB <= 128 && setup_lds_bytes(maxB, csz) <= kSetupLdsBytes; }

// The setup's line classes, each with LDS for its own largest block: lines whose B x B block
// takes at most kSmallLds (several workgroups share a CU), the other lines with blocks up to
// 64, and the larger blocks (those of the lines on a middle group; 1024 threads, two rows per
// lane in the panel wave).
SetupClasses setup_classes(const Plan& P, int csz, const std::vector<int>* subset) {
  SetupClasses c;
  std::vector<int> all;
  if (!subset) {
    for (int line = 0; line < P.Gz * P.Gy; ++line) all.push_back(line);
    subset = &all;
  }
  for (int k = 0; k < 3; ++k) {
    c.count[k] = 0;
    c.maxB[k] = 0;
  }
  for (int k = 0; k < 3; ++k)
    for (int line : *subset) {
      const int B = P.line_B[line];
      const int cls = B > 64 ? 2 : ((size_t)B * B * csz <= kSmallLds ? 0 : 1);
      if (cls != k) continue;
      c.order.push_back(line);
      c.count[k] += 1;
      c.maxB[k] = std::max(c.maxB[k], B);
    }
  return c;
}

hipError_t launch_setup(helm_handle* h, hipStream_t s) {
  const int csz = h->prec == HELM_C64 ? (int)sizeof(float2) : (int)sizeof(double2);
  return launch_setup_lines(h, h->d_setup_lines, setup_classes(h->plan, csz, nullptr), s);
}

hipError_t launch_setup_lines(helm_handle* h, const int* d_lines, const SetupClasses& c,
                              hipStream_t s) {
  const Plan& P = h->plan;
  SetupArgs a;
  a.n = h->n;
  a.Gz = P.Gz;
  a.Gy = P.Gy;
  a.p = P.p;
  a.fronts = P.fronts;
  a.zmid = P.zmid;
  a.fronts_inner = P.fronts_inner;
  a.ymid = P.ymid;
  a.h = h->h;
  a.groups = h->d_groups;
  a.line_off = h->d_line_off;
  a.sbd = h->sbd;
  a.smv = h->smv;
  a.kappa = h->kappa;
  a.factors = h->factors;
  a.err = h->d_err;
  a.lines = nullptr;
  a.part = 0;
  // class 0 on s, classes 1 and 2 on side streams that start after the work already queued
  // on s; s continues only after both are done
  hipStream_t side[2] = {nullptr, nullptr};
  hipEvent_t start = nullptr, done[2] = {nullptr, nullptr};
  hipError_t e = hipSuccess;
  const bool need_side = c.count[1] > 0 || c.count[2] > 0;
  if (need_side) {
    e = hipEventCreateWithFlags(&start, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(start, s);
  }
  int first = c.count[0];
  for (int k = 1; k < 3 && e == hipSuccess; ++k) {
    if (c.count[k] == 0) continue;
    e = hipStreamCreateWithFlags(&side[k - 1], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&done[k - 1], hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamWaitEvent(side[k - 1], start, 0);
    if (e == hipSuccess)
      e = k == 2 ? setup_launch<kSetupThreadsBig>(h, a, d_lines + first, c.count[k], c.maxB[k], side[k - 1], true)
                 : setup_launch<kSetupThreads>(h, a, d_lines + first, c.count[k], c.maxB[k], side[k - 1], true);
    if (e == hipSuccess) e = hipEventRecord(done[k - 1], side[k - 1]);
    first += c.count[k];
  }
  if (e == hipSuccess) e = setup_launch<kSetupThreads>(h, a, d_lines, c.count[0], c.maxB[0], s, true);
  for (int k = 0; k < 2 && e == hipSuccess; ++k)
    if (done[k]) e = hipStreamWaitEvent(s, done[k], 0);
  // destroying a stream or event with work pending is allowed: it is released once done
  for (int k = 0; k < 2; ++k) {
    if (done[k]) (void)hipEventDestroy(done[k]);
    if (side[k]) (void)hipStreamDestroy(side[k]);
  }
  if (start) (void)hipEventDestroy(start);
  return e;
}

// ==========================================================================================
// Nested-dissection factors of the line problems (complex64): block cyclic reduction in x1.
//
// Sec. 6 suggests replacing the line's block LDU by a 1D nested dissection, whose halves are
// independent at every level.  With n = 2^k - 1 blocks, block i belongs to level
// l_i = (trailing zeros of i + 1); level 0 are the even blocks, level k - 1 the middle block
// n / 2 alone.  Eliminating level 0, then 1, ... is Gaussian elimination of the line in the
// nested-dissection order (each level's separators after the halves they split).  Before
// level l the reduced system couples block i only to i - 2^l (L_i) and i + 2^l (U_i); at
// level 0 these are the scalar x1-couplings l_i I and u_i I.  Eliminating the level-l blocks
// e (s = 2^l) with Inv_e = D_e^{-1}, G_e = Inv_e L_e, H_e = Inv_e U_e leaves, for each
// remaining block r with e1 = r - s, e2 = r + s,
//     D_r <- D_r - L_r H_e1 - U_r G_e2,   L_r <- -L_r G_e1,   U_r <- -U_r H_e2,
// and a solve reduces the right-hand sides level by level (b_r -= P_r b_e1 + Q_r b_e2 with
// P_r = L_r Inv_e1, Q_r = U_r Inv_e2), solves the middle block, and substitutes back
// (x_e = Inv_e b_e - G_e x_{e-s} - H_e x_{e+s}).
//
// Stored per line, blocks B x B column-major (element (r, c) at c B + r), block i's matrices
// from (3 i - 2 popcount(i)) B^2 on: Inv_i, and for l_i >= 1 also G_i, H_i and P_i, Q_i of
// the levels 1 .. l_i - 1 (at level 0, P and Q are the neighbours' Inv times a scalar).  A
// line takes (3 n - 2 popcount(n)) B^2 entries, about 2.9 times its block LDU factors.
// ==========================================================================================
namespace {

constexpr size_t kNdPad = 64;   // complex zeros after the factors (the solve's row clamp reads stay inside)

__host__ __device__ inline long long nd_first(int i) { return 3LL * i - 2LL * __builtin_popcount((unsigned)i); }

struct NdArgs {
  int n, k, Gz, Gy, level;
  double h;
  const GroupInfo* groups;
  const long long* woff;   // per line: offset of its n dense work blocks (the block LDU layout)
  const long long* foff;   // per line: offset of its nested-dissection factors
  const int* lines;        // lines of this launch (blockIdx.y)
  const double2* sbd;
  float2* F;
  float2 *Wd, *Wl, *Wu, *Wl2, *Wu2;
  int* err;
};

__device__ inline float2 nd_l(const NdArgs& a, int i) {   // K_{i,i-1} = l_i I
  const int m = i + 1;
  return cvt<float2>(cscale(cmul(a.sbd[2 * m], a.sbd[2 * m - 1]), 1.0 / (a.h * a.h)));
}
__device__ inline float2 nd_u(const NdArgs& a, int i) {   // K_{i,i+1} = u_i I
  const int m = i + 1;
  return cvt<float2>(cscale(cmul(a.sbd[2 * m], a.sbd[2 * m + 1]), 1.0 / (a.h * a.h)));
}

// D_i of every block of the launch's lines, dense, column-major into Wd (workgroup: block
// blockIdx.x of line lines[blockIdx.y]); the entries are those of the block LDU's D_i
__global__ void __launch_bounds__(256) k_nd_form(SetupArgs s, NdArgs a) {
  __shared__ double2 syn[kMaxW], syh[kMaxW + 1], szn[kMaxW], szh[kMaxW + 1];
  const int line = a.lines[blockIdx.y], i = blockIdx.x;
  const int g = line / a.Gy, l = line % a.Gy;
  const GroupInfo gz = a.groups[g], gy = a.groups[a.Gz + l];
  const int Wz = gz.W, Wy = gy.W, B = Wy * Wz, n = a.n, tid = threadIdx.x;
  if (tid < Wy) syn[tid] = window_s(s, gy, 2 * (gy.w0 + tid));
  if (tid <= Wy) syh[tid] = window_s(s, gy, 2 * (gy.w0 + tid) - 1);
  if (tid < Wz) szn[tid] = window_s(s, gz, 2 * (gz.w0 + tid));
  if (tid <= Wz) szh[tid] = window_s(s, gz, 2 * (gz.w0 + tid) - 1);
  __syncthreads();
  const double ih2 = 1.0 / (a.h * a.h);
  const int m = i + 1;
  const double2 dx = cscale(cmul(a.sbd[2 * m], cadd(a.sbd[2 * m + 1], a.sbd[2 * m - 1])), -ih2);
  float2* out = a.Wd + a.woff[line] + (long long)i * B * B;
  for (int e = tid; e < B * B; e += blockDim.x) {
    const int c = e / B, r = e - c * B;   // column-major
    const int jr = r / Wz, kr = r - jr * Wz, jc = c / Wz, kc = c - jc * Wz;
    double2 val = make_double2(0.0, 0.0);
    if (r == c) {
      const int k = gz.w0 + kr, jj = gy.w0 + jr;
      const double kap = s.kappa[((long long)(k - 1) * n + (jj - 1)) * n + i];
      const double2 dy = cscale(cmul(syn[jr], cadd(syh[jr + 1], syh[jr])), -ih2);
      const double2 dz = cscale(cmul(szn[kr], cadd(szh[kr + 1], szh[kr])), -ih2);
      val = cadd(cadd(dx, dy), dz);
      val.x += kap;
    } else if (jr == jc) {
      if (kc == kr + 1) val = cscale(cmul(szn[kr], szh[kr + 1]), ih2);
      else if (kc == kr - 1) val = cscale(cmul(szn[kr], szh[kr]), ih2);
    } else if (kr == kc) {
      if (jc == jr + 1) val = cscale(cmul(syn[jr], syh[jr + 1]), ih2);
      else if (jc == jr - 1) val = cscale(cmul(syn[jr], syh[jr]), ih2);
    }
    out[e] = cvt<float2>(val);
  }
}

// Inv_e = D_e^{-1} for the level's blocks e = (2 j + 1) 2^level - 1 (j = blockIdx.x):
// Gauss-Jordan elimination with partial pivoting (row exchanges) on [D_e | I] in LDS
__global__ void __launch_bounds__(256) k_nd_invert(NdArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ float2 fcol[kMaxB];
  __shared__ int piv_s;
  const int line = a.lines[blockIdx.y];
  const int e = (2 * (int)blockIdx.x + 1) * (1 << a.level) - 1;
  const int g = line / a.Gy, l = line % a.Gy;
  const int B = a.groups[g].W * a.groups[a.Gz + l].W, W2 = 2 * B;
  const int tid = threadIdx.x, NT = blockDim.x;
  float2* M = reinterpret_cast<float2*>(smem_raw);   // B rows of 2B: row r at M + r 2B
  const float2* src = a.Wd + a.woff[line] + (long long)e * B * B;
  for (int x = tid; x < B * W2; x += NT) {
    const int r = x / W2, c = x - r * W2;
    M[x] = c < B ? src[(long long)c * B + r] : make_float2(c - B == r ? 1.f : 0.f, 0.f);
  }
  __syncthreads();
  bool bad = false;
  for (int k = 0; k < B; ++k) {
    if (tid < 64) {
      float best = -1.f;
      int br = k;
      for (int r = k + tid; r < B; r += 64) {
        const float m = cabs2(M[r * W2 + k]);
        if (m > best || m != m) {
          best = m != m ? __builtin_huge_valf() : m;
          br = r;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const float ob = __shfl_xor(best, off);
        const int orr = __shfl_xor(br, off);
        if (ob > best || (ob == best && orr < br)) {
          best = ob;
          br = orr;
        }
      }
      if (tid == 0) piv_s = br;
    }
    __syncthreads();
    const int p = piv_s;
    if (p != k)
      for (int c = k + tid; c < W2; c += NT) {
        const float2 t = M[k * W2 + c];
        M[k * W2 + c] = M[p * W2 + c];
        M[p * W2 + c] = t;
      }
    __syncthreads();
    const float2 pv = M[k * W2 + k];
    const float pm = cabs2(pv);
    if (!(pm > 0.f) || !(pm < __builtin_huge_valf())) bad = true;
    const float2 pinv = (pm > 0.f && pm < __builtin_huge_valf()) ? cinv(pv) : make_float2(1.f, 0.f);
    for (int r = tid; r < B; r += NT) fcol[r] = M[r * W2 + k];
    __syncthreads();
    for (int c = k + tid; c < W2; c += NT) M[k * W2 + c] = cmul(M[k * W2 + c], pinv);
    __syncthreads();
    const int span = W2 - k;
    for (int x = tid; x < B * span; x += NT) {
      const int r = x / span, c = k + (x - r * span);
      if (r != k) M[r * W2 + c] = csub(M[r * W2 + c], cmul(fcol[r], M[k * W2 + c]));
    }
    __syncthreads();
  }
  if (bad && tid == 0) {
    atomicOr(&a.err[0], 1);
    atomicExch(&a.err[1], line);
  }
  float2* dst = a.F + a.foff[line] + nd_first(e) * B * B;
  for (int x = tid; x < B * B; x += NT) {
    const int c = x / B, r = x - c * B;
    dst[x] = M[r * W2 + B + c];
  }
}

// after level 0: for the odd blocks r, D_r -= l_r u_{r-1} Inv_{r-1} + u_r l_{r+1} Inv_{r+1},
// L_r = -l_r l_{r-1} Inv_{r-1} (0 when r - 2 < 0), U_r = -u_r u_{r+1} Inv_{r+1} (0 past the end)
__global__ void __launch_bounds__(256) k_nd_level0(NdArgs a) {
  const int line = a.lines[blockIdx.y];
  const int r = 2 * (int)blockIdx.x + 1;
  const int g = line / a.Gy, l = line % a.Gy;
  const int B = a.groups[g].W * a.groups[a.Gz + l].W;
  const long long BB = (long long)B * B;
  const float2 lr = nd_l(a, r), ur = nd_u(a, r);
  const float2 c1 = cmul(lr, nd_u(a, r - 1)), c2 = cmul(ur, nd_l(a, r + 1));
  const float2 cl = r - 2 >= 0 ? cmul(make_float2(-lr.x, -lr.y), nd_l(a, r - 1)) : make_float2(0.f, 0.f);
  const float2 cu = r + 2 <= a.n - 1 ? cmul(make_float2(-ur.x, -ur.y), nd_u(a, r + 1)) : make_float2(0.f, 0.f);
  const float2* I1 = a.F + a.foff[line] + nd_first(r - 1) * BB;
  const float2* I2 = a.F + a.foff[line] + nd_first(r + 1) * BB;
  const long long w = a.woff[line] + r * BB;
  for (int x = threadIdx.x; x < B * B; x += blockDim.x) {
    const float2 i1 = I1[x], i2 = I2[x];
    a.Wd[w + x] = csub(csub(a.Wd[w + x], cmul(c1, i1)), cmul(c2, i2));
    a.Wl[w + x] = cmul(cl, i1);
    a.Wu[w + x] = cmul(cu, i2);
  }
}

// one output C (B x B, column-major) = beta C + s1 A1 B1 + s2 A2 B2 on the matrix cores:
// 16 x 16 tiles over the four waves, complex products as four real 16 x 16 x 4 products
__device__ inline void nd_gemm(float2* C, bool beta, const float2* A1, const float2* B1, float2 s1,
                               const float2* A2, const float2* B2, float2 s2, int B) {
  using M = Mfma<float>;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, NW = blockDim.x >> 6;
  const int RT = (B + 15) >> 4;
  for (int tile = wv; tile < RT * RT; tile += NW) {
    const int ti = tile / RT, tj = tile - ti * RT;
    const int col = tj * 16 + (lane & 15), arow = ti * 16 + (lane & 15);
    f32x4 cre = {0.f, 0.f, 0.f, 0.f}, cim = {0.f, 0.f, 0.f, 0.f};
    for (int t = 0; t < 2; ++t) {
      const float2* A = t ? A2 : A1;
      const float2* Bm = t ? B2 : B1;
      if (!A) continue;
      const float2 sc = t ? s2 : s1;
      f32x4 pre = {0.f, 0.f, 0.f, 0.f}, pim = {0.f, 0.f, 0.f, 0.f};
      for (int k0 = 0; k0 < B; k0 += 4) {
        const int kk = k0 + (lane >> 4);
        const float2 av = (arow < B && kk < B) ? A[(long long)kk * B + arow] : make_float2(0.f, 0.f);
        const float2 bv = (kk < B && col < B) ? Bm[(long long)col * B + kk] : make_float2(0.f, 0.f);
        pre = M::mac(av.x, bv.x, pre);
        pre = M::mac(-av.y, bv.y, pre);
        pim = M::mac(av.x, bv.y, pim);
        pim = M::mac(av.y, bv.x, pim);
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        cre[q] += sc.x * pre[q] - sc.y * pim[q];
        cim[q] += sc.x * pim[q] + sc.y * pre[q];
      }
    }
    if (col < B) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = ti * 16 + M::row(lane, q);
        if (row < B) {
          float2 v = make_float2(cre[q], cim[q]);
          if (beta) v = cadd(v, C[(long long)col * B + row]);
          C[(long long)col * B + row] = v;
        }
      }
    }
  }
}

// level >= 1, after the inversions: G_e, H_e of the level's blocks (blockIdx.x = 2 j + kind)
__global__ void __launch_bounds__(256) k_nd_gh(NdArgs a) {
  const int line = a.lines[blockIdx.y];
  const int j = (int)blockIdx.x >> 1, kind = (int)blockIdx.x & 1;
  const int e = (2 * j + 1) * (1 << a.level) - 1;
  const int g = line / a.Gy, l = line % a.Gy;
  const int B = a.groups[g].W * a.groups[a.Gz + l].W;
  const long long BB = (long long)B * B;
  float2* f = a.F + a.foff[line] + nd_first(e) * BB;
  const float2* W = (kind ? a.Wu : a.Wl) + a.woff[line] + e * BB;
  nd_gemm(f + (1 + kind) * BB, false, f, W, make_float2(1.f, 0.f), nullptr, nullptr, make_float2(0.f, 0.f), B);
}

// level >= 1: for the remaining blocks r = 2 (m + 1) 2^level - 1 (blockIdx.x = 5 m + kind):
// P_r, Q_r (kinds 0, 1), the new D_r (2), L_r and U_r into the second buffers (3, 4)
__global__ void __launch_bounds__(256) k_nd_reduce(NdArgs a) {
  const int line = a.lines[blockIdx.y];
  const int m = (int)blockIdx.x / 5, kind = (int)blockIdx.x - 5 * m;
  const int s = 1 << a.level, r = 2 * (m + 1) * s - 1, e1 = r - s, e2 = r + s;
  const int g = line / a.Gy, l = line % a.Gy;
  const int B = a.groups[g].W * a.groups[a.Gz + l].W;
  const long long BB = (long long)B * B, wo = a.woff[line];
  const float2* Fl = a.F + a.foff[line];
  const float2* I1 = Fl + nd_first(e1) * BB;
  const float2* I2 = Fl + nd_first(e2) * BB;
  const float2* Lr = a.Wl + wo + r * BB;
  const float2* Ur = a.Wu + wo + r * BB;
  const float2 one = make_float2(1.f, 0.f), mone = make_float2(-1.f, 0.f), zero = make_float2(0.f, 0.f);
  float2* Pr = a.F + a.foff[line] + (nd_first(r) + 3 + 2 * (a.level - 1)) * BB;
  switch (kind) {
    case 0: nd_gemm(Pr, false, Lr, I1, one, nullptr, nullptr, zero, B); break;
    case 1: nd_gemm(Pr + BB, false, Ur, I2, one, nullptr, nullptr, zero, B); break;
    case 2: nd_gemm(a.Wd + wo + r * BB, true, Lr, I1 + 2 * BB, mone, Ur, I2 + BB, mone, B); break;
    case 3: nd_gemm(a.Wl2 + wo + r * BB, false, Lr, I1 + BB, mone, nullptr, nullptr, zero, B); break;
    default: nd_gemm(a.Wu2 + wo + r * BB, false, Ur, I2 + 2 * BB, mone, nullptr, nullptr, zero, B); break;
  }
}

}  // namespace

long long nd_line_blocks(int n) { return nd_first(n); }

bool nd_supported(const Plan& P, int prec, std::string& why) {
  if (prec != HELM_C64) {
    why = "the nested-dissection line solver is built for complex64 factors";
    return false;
  }
  if (P.n < 3 || ((P.n + 1) & P.n) != 0) {
    why = "the nested-dissection line solver needs n = 2^k - 1 blocks per line";
    return false;
  }
  if (P.maxB > 96) {
    why = "the nested-dissection setup inverts blocks of at most 96 unknowns";
    return false;
  }
  return true;
}

// the factors of every line (see above) into h->nd; the work arrays come from the pool and go
// back to it
int nd_build(helm_handle* h, hipStream_t s, std::string& msg) {
  const Plan& P = h->plan;
  if (!nd_supported(P, h->prec, msg)) return HELM_EINVAL;
  const int n = P.n, lines = P.Gz * P.Gy;
  int k = 0;
  while ((1 << k) < n + 1) ++k;
  std::vector<long long> foff(lines);
  long long total = 0;
  for (int line = 0; line < lines; ++line) {
    foff[line] = total;
    total += nd_line_blocks(n) * (long long)P.line_B[line] * P.line_B[line];
  }
  // lines by block size: each launch of the inversion sized by its largest block
  std::vector<int> order(lines);
  for (int i = 0; i < lines; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return P.line_B[x] < P.line_B[y]; });
  std::vector<std::pair<int, int>> cls;   // [first, count) ranges of `order` with maxB <= 48, 64, 96
  for (int lim : {48, 64, 96}) {
    int first = cls.empty() ? 0 : cls.back().first + cls.back().second, cnt = 0;
    while (first + cnt < lines && P.line_B[order[first + cnt]] <= lim) ++cnt;
    if (cnt) cls.push_back({first, cnt});
  }
  const size_t W = (size_t)P.total_elems * sizeof(float2);
  const size_t fbytes = ((size_t)total + kNdPad) * sizeof(float2);
  void *F = nullptr, *Wd = nullptr, *Wl = nullptr, *Wu = nullptr, *Wl2 = nullptr, *Wu2 = nullptr;
  long long* d_foff = nullptr;
  int* d_order = nullptr;
  auto cleanup = [&]() {
    for (void* p : {Wd, Wl, Wu, Wl2, Wu2, (void*)d_order})
      if (p) pool_free(p, s);
  };
  if (h->nd) {
    pool_free(h->nd, s);
    h->nd = nullptr;
  }
  if (h->d_nd_off) {
    pool_free(h->d_nd_off, s);
    h->d_nd_off = nullptr;
  }
  if (pool_alloc(&F, fbytes, s) != hipSuccess || pool_alloc((void**)&d_foff, lines * sizeof(long long), s) != hipSuccess ||
      pool_alloc(&Wd, W, s) != hipSuccess || pool_alloc(&Wl, W, s) != hipSuccess ||
      pool_alloc(&Wu, W, s) != hipSuccess || pool_alloc(&Wl2, W, s) != hipSuccess ||
      pool_alloc(&Wu2, W, s) != hipSuccess || pool_alloc((void**)&d_order, lines * sizeof(int), s) != hipSuccess) {
    cleanup();
    if (F) pool_free(F, s);
    if (d_foff) pool_free(d_foff, s);
    msg = "device allocation failed for the nested-dissection factors (" + std::to_string(fbytes) +
          " bytes) and their work arrays (5 x " + std::to_string(W) + " bytes)";
    return HELM_ENOMEM;
  }
  h->nd = F;
  h->d_nd_off = d_foff;
  h->nd_k = k;
  h->nd_bytes = fbytes;
  hipError_t e = hipMemsetAsync((char*)F + (size_t)total * sizeof(float2), 0, kNdPad * sizeof(float2), s);
  if (e == hipSuccess) e = hipMemsetAsync(h->d_err, 0, 2 * sizeof(int), s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_foff, foff.data(), lines * sizeof(long long), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(d_order, order.data(), lines * sizeof(int), hipMemcpyHostToDevice, s);
  SetupArgs sa{};
  sa.n = n;
  sa.Gz = P.Gz;
  sa.Gy = P.Gy;
  sa.p = P.p;
  sa.h = h->h;
  sa.groups = h->d_groups;
  sa.sbd = h->sbd;
  sa.smv = h->smv;
  sa.kappa = h->kappa;
  NdArgs a{};
  a.n = n;
  a.k = k;
  a.Gz = P.Gz;
  a.Gy = P.Gy;
  a.h = h->h;
  a.groups = h->d_groups;
  a.woff = h->d_line_off;
  a.foff = d_foff;
  a.lines = d_order;
  a.sbd = h->sbd;
  a.F = static_cast<float2*>(F);
  a.Wd = static_cast<float2*>(Wd);
  a.Wl = static_cast<float2*>(Wl);
  a.Wu = static_cast<float2*>(Wu);
  a.Wl2 = static_cast<float2*>(Wl2);
  a.Wu2 = static_cast<float2*>(Wu2);
  a.err = h->d_err;
  if (e == hipSuccess) {
    k_nd_form<<<dim3(n, lines), 256, 0, s>>>(sa, a);
    e = hipGetLastError();
  }
  for (int lev = 0; lev < k && e == hipSuccess; ++lev) {
    a.level = lev;
    const int nelim = 1 << (k - 1 - lev);   // blocks of this level
    for (const auto& c : cls) {
      const int maxB = P.line_B[order[c.first + c.second - 1]];
      const size_t sm = (size_t)2 * maxB * maxB * sizeof(float2);
      NdArgs ac = a;
      ac.lines = d_order + c.first;
      e = hipFuncSetAttribute((const void*)k_nd_invert, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
      if (e != hipSuccess) break;
      k_nd_invert<<<dim3(nelim, c.second), 256, sm, s>>>(ac);
      e = hipGetLastError();
      if (e != hipSuccess) break;
    }
    if (e != hipSuccess || lev == k - 1) break;
    const int nrem = nelim - 1;   // blocks above this level
    if (lev == 0) {
      k_nd_level0<<<dim3(nrem, lines), 256, 0, s>>>(a);
    } else {
      k_nd_gh<<<dim3(2 * nelim, lines), 256, 0, s>>>(a);
      k_nd_reduce<<<dim3(5 * nrem, lines), 256, 0, s>>>(a);
      std::swap(a.Wl, a.Wl2);
      std::swap(a.Wu, a.Wu2);
    }
    e = hipGetLastError();
  }
  int err[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(err, h->d_err, sizeof(err), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  cleanup();
  if (e != hipSuccess) {
    msg = std::string("nested-dissection setup: ") + hipGetErrorString(e);
    return HELM_EHIP;
  }
  if (err[0]) {
    msg = "singular reduced block in line " + std::to_string(err[1]) + " (nested-dissection setup)";
    return HELM_ESINGULAR;
  }
  return HELM_OK;
}

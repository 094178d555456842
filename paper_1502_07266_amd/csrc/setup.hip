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
// by Gauss-Jordan elimination with partial pivoting (row interchanges inside the block only),
// stores T_i = S_i^{-1} and reuses it for the next Schur update.  The blocks are eliminated
// from both ends towards the middle (see the order below), which halves the dependent chain
// of the line solve; the two halves do not meet before the middle block, so they are factored
// by two workgroups and the middle blocks by a launch of their own.  All
// lines are independent (Sec. 6 notes that the setup is O(n^2) independent quasi-1D
// problems).  The LDS of a launch is sized by its largest block, so the lines on a middle
// group (few, with blocks up to 128) get a launch of their own, on a side stream beside the
// launches of the other lines (split again by block size, so that the many small ones share
// CUs four at a time).
#include <algorithm>

#include "common.h"

namespace {

constexpr int kMaxW = 64;
constexpr int kMaxB = 128;
constexpr int kSetupThreads = 256;        // lines with two-chain blocks (B <= 64)
constexpr int kSetupThreadsBig = 1024;    // lines on a middle group (B up to 128)
constexpr size_t kSetupLdsBytes = 144 * 1024;   // dynamic LDS the setup may take (of 160 KiB)
constexpr size_t kSmallLds = 40 * 1024;         // two blocks within this: four workgroups per CU

struct SetupArgs {
  int n, Gz, Gy, p;
  int fronts, zmid, fronts_inner, ymid;
  int prev_in_lds;   // the previous block's factor is kept in LDS (else re-read from HBM)
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

// The B x B loops run rows across waves and columns across lanes (c and c + 64), so no
// element index is divided by B.
template <typename R, int NTB>
__global__ void __launch_bounds__(NTB) k_line_setup(SetupArgs a) {
  using C = typename cx<R>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ double2 syn[kMaxW], syh[kMaxW + 1], szn[kMaxW], szh[kMaxW + 1];
  __shared__ int perm[kMaxB], rho[kMaxB];
  __shared__ C fcol[kMaxB];
  __shared__ C pinv_s;
  __shared__ int piv_s, bad_s;

  const int w = a.part == 1 ? (int)blockIdx.x >> 1 : (int)blockIdx.x;
  const int half = a.part == 1 ? (int)blockIdx.x & 1 : 0;
  const int line = a.lines[w];
  const int g = line / a.Gy, l = line % a.Gy;
  const GroupInfo gz = a.groups[g], gy = a.groups[a.Gz + l];
  const int Wz = gz.W, Wy = gy.W, B = Wy * Wz;
  const int n = a.n;
  const int tid = threadIdx.x, NT = blockDim.x;
  const int lane = tid & 63, wv = tid >> 6, nw = NT >> 6;
  C* S = reinterpret_cast<C*>(smem_raw);
  C* out = reinterpret_cast<C*>(a.factors) + a.line_off[line];
  const double ih2 = 1.0 / (a.h * a.h);

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
  // the factor of the block eliminated last: an LDS copy, or the block just written to HBM
  C* Tlds = S + B * B;
  const C* Tprev = Tlds;
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
    Tprev = has_lower ? out + (long long)(mid + 1) * B * B : T_mid_minus1;
  }
  for (int t = t0; t < t1; ++t) {
    const int i = t < mid ? t : (t < n - 1 ? n - 1 - (t - mid) : mid);
    const int m = i + 1;  // global x1 node of block i
    const double2 sxn = a.sbd[2 * m], sxd = a.sbd[2 * m - 1], sxu = a.sbd[2 * m + 1];
    const double2 dx = cscale(cmul(sxn, cadd(sxu, sxd)), -ih2);
    // update from the block below: l_i u_{i-1} = (s_m s_{m-1/2} / h^2)(s_{m-1} s_{m-1/2} / h^2)
    // update from the block above: u_i l_{i+1} = (s_m s_{m+1/2} / h^2)(s_{m+1} s_{m+1/2} / h^2)
    const C sc_below = cvt<C>(cmul(cscale(cmul(sxn, sxd), ih2), cscale(cmul(a.sbd[2 * m - 2], sxd), ih2)));
    const C sc_above = cvt<C>(cmul(cscale(cmul(sxn, sxu), ih2), cscale(cmul(a.sbd[2 * m + 2], sxu), ih2)));
    // (scale, factor) pairs of the Schur update; Tprev holds the factor computed last
    const bool is_mid = t == n - 1;
    const bool use_a = (t > 0 && t < mid) || (t > mid && t < n - 1) || is_mid;
    const C scA = (t < mid || is_mid) ? sc_below : sc_above;
    const C* TA = (is_mid && has_lower) ? T_mid_minus1 : Tprev;
    const bool use_b = is_mid && has_lower;
    for (int r = wv; r < B; r += nw) {
      const int jr = r / Wz, kr = r - jr * Wz;
      for (int c = lane; c < B; c += 64) {
      const int e = r * B + c;
      const int jc = c / Wz, kc = c - jc * Wz;
      double2 val = make_double2(0.0, 0.0);
      if (r == c) {
        const int k = gz.w0 + kr, j = gy.w0 + jr;
        const double kap = a.kappa[((long long)(k - 1) * n + (j - 1)) * n + i];
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
      if (use_a) v = csub(v, cmul(scA, TA[e]));
      if (use_b) v = csub(v, cmul(sc_above, Tprev[e]));
      S[e] = v;
      }
    }
    __syncthreads();

    // ---- in-place Gauss-Jordan inversion with partial pivoting ----
    for (int k = 0; k < B; ++k) {
      if (tid < 64) {
        R best = (R)-1;
        int bi = B;
        for (int r = k + tid; r < B; r += 64) {
          R mg = cabs2(S[r * B + k]);
          if (mg > best) { best = mg; bi = r; }
        }
        for (int off = 32; off > 0; off >>= 1) {
          R ob = __shfl_xor(best, off);
          int oi = __shfl_xor(bi, off);
          if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        if (tid == 0) {
          C pv = S[bi * B + k];
          if (!(best > (R)0) || !isfinite(best)) { bad_s = 1; pv = mk((R)1, (R)0); }
          piv_s = bi;
          perm[k] = bi;
          pinv_s = cinv(pv);
        }
      }
      __syncthreads();
      const int pr = piv_s;
      if (pr != k) {
        for (int c = tid; c < B; c += NT) {
          C tmp = S[k * B + c];
          S[k * B + c] = S[pr * B + c];
          S[pr * B + c] = tmp;
        }
      }
      __syncthreads();
      const C pinv = pinv_s;
      for (int c = tid; c < B; c += NT) S[k * B + c] = (c == k) ? pinv : cmul(S[k * B + c], pinv);
      for (int r = tid; r < B; r += NT)
        if (r != k) fcol[r] = S[r * B + k];
      __syncthreads();
      for (int r = wv; r < B; r += nw) {
        if (r == k) continue;
        const C fr = fcol[r];
        for (int c = lane; c < B; c += 64) {
          const int e = r * B + c;
          const C old = (c == k) ? mk((R)0, (R)0) : S[e];
          S[e] = csub(old, cmul(fr, S[k * B + c]));
        }
      }
      __syncthreads();
    }
    // column order of the inverse: (PS)^{-1} P = S^{-1}, i.e. T[r][rho(m)] = X[r][m]
    if (tid == 0) {
      for (int q = 0; q < B; ++q) rho[q] = q;
      for (int k = 0; k < B; ++k) {
        int tmp = rho[k];
        rho[k] = rho[perm[k]];
        rho[perm[k]] = tmp;
      }
    }
    __syncthreads();
    C* dst = out + (long long)i * B * B;
    if (a.prev_in_lds) {
      for (int r = wv; r < B; r += nw)
        for (int q = lane; q < B; q += 64) Tlds[r * B + rho[q]] = S[r * B + q];
      __syncthreads();
      for (int e = tid; e < B * B; e += NT) dst[e] = Tlds[e];
    } else {
      for (int r = wv; r < B; r += nw)
        for (int q = lane; q < B; q += 64) dst[r * B + rho[q]] = S[r * B + q];
      __syncthreads();   // the next block's Schur update reads dst (workgroup-scope fence)
      Tprev = dst;
    }
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
  // keep the previous factor in LDS when two B x B blocks fit, else re-read it from HBM
  a.prev_in_lds = 2 * (size_t)maxB * maxB * csz <= kSetupLdsBytes;
  const size_t sm = (a.prev_in_lds ? 2 : 1) * (size_t)maxB * maxB * csz;
  if (h->prec == HELM_C64) {
    hipError_t e = hipFuncSetAttribute((const void*)k_line_setup<float, NTB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    k_line_setup<float, NTB><<<count, NTB, sm, s>>>(a);
  } else {
    hipError_t e = hipFuncSetAttribute((const void*)k_line_setup<double, NTB>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    k_line_setup<double, NTB><<<count, NTB, sm, s>>>(a);
  }
  return hipGetLastError();
}

}  // namespace

// The setup's line classes, each with LDS for its own largest block: lines whose two B x B
// blocks take at most kSmallLds (several workgroups share a CU), the other lines with blocks
// up to 64, and the larger blocks (those of the lines on a middle group; 1024 threads).
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
      const int cls = B > 64 ? 2 : (2 * (size_t)B * B * csz <= kSmallLds ? 0 : 1);
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

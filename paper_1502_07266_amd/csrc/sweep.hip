// Application of the recursive sweeping preconditioner, z = M^{-1} r (Algorithm 6 with
// Algorithm 4 inside, each line block solved exactly by its block LDU), and its adjoint: the
// host side of the sweep kernel (sweep_kernel.h).
//
// A sweep of R right-hand sides is ONE cooperative launch of 2 x (outer fronts) x (inner
// fronts) workgroups per right-hand side, each running its part of Algorithm 6 / Algorithm 4
// from the first slab to the last and meeting the others only through tagged exchange words.
// When the workgroups of all right-hand sides cannot be resident at once, the right-hand
// sides are launched in chunks that can (the chunks are independent).  The launch shape (a
// variant of sweep_variants.h) is the handle's choice (helm_set_launch), the autotuner's for
// the configuration (helm_autotune, run on the first solve of a configuration), or the first
// listed variant that covers the blocks.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

#include "common.h"
#include "sweep_kernel.h"
#include "sweep_variants.h"

const std::vector<SweepVariant>& sweep_variants(bool c64) {
#define X(A, B, C, D, E, F) SweepVariant{A, B, C, D, E, F},
  static const std::vector<SweepVariant> v64 = {HELM_SWEEP_VARIANTS_C64(X)};
  static const std::vector<SweepVariant> v128 = {HELM_SWEEP_VARIANTS_C128(X)};
#undef X
  return c64 ? v64 : v128;
}

const void* sweep_kernel(bool c64, bool z64, bool adj, int k) {
  if (!c64) return sweep_kernel_c128(adj, k);
  return adj ? sweep_kernel_c64_adj(z64, k) : sweep_kernel_c64_fwd(z64, k);
}

namespace {

using sweepk::MemberLds;
using sweepk::SweepArgs;
using sweepk::XLayout;

constexpr size_t kLdsBytes = 160 * 1024;   // LDS per workgroup on gfx950
constexpr int kMaxThreads = 1024;

size_t csize(const helm_handle* h) { return h->prec == HELM_C64 ? sizeof(float2) : sizeof(double2); }
int pieces(const helm_handle* h) { return (int)(csize(h) / 4); }

// threads of a launch: every line's chain of B rows x NC lanes (its shape's), rounded up to
// whole wavefronts; 0 if a line does not fit the variant
int variant_threads(const Plan& P, const SweepVariant& v) {
  int t = 0;
  for (int B : P.line_B) {
    if (B > v.capB()) return 0;
    const int nc = B <= v.capA() ? v.nca : v.ncb;
    t = std::max(t, (B * nc + 63) / 64 * 64);
  }
  return t <= kMaxThreads ? t : 0;
}

bool plan_variant_valid(const Plan& P, int prec, int k) {
  const auto& vs = sweep_variants(prec == HELM_C64);
  if (k < 0 || k >= (int)vs.size()) return false;
  const int cs = prec == HELM_C64 ? (int)sizeof(float2) : (int)sizeof(double2);
  return variant_threads(P, vs[k]) > 0 && MemberLds(P.n, P.maxB, P.maxW, cs).bytes <= kLdsBytes;
}

bool variant_valid(const helm_handle* h, int k) { return plan_variant_valid(h->plan, h->prec, k); }

__global__ void k_fill_ones(double2* x, long long count) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) x[e] = make_double2(1.0, 0.0);
}

// the first listed variant whose shape A covers the blocks off the middle groups and whose
// shape B covers all, with the smallest shape A, then the smallest shape B
int default_variant(const helm_handle* h) {
  const auto& vs = sweep_variants(h->prec == HELM_C64);
  int best = -1;
  for (int k = 0; k < (int)vs.size(); ++k) {
    if (!variant_valid(h, k) || vs[k].capA() < h->plan.maxB_front) continue;
    if (best < 0 || vs[k].capA() < vs[best].capA() ||
        (vs[k].capA() == vs[best].capA() && vs[k].capB() < vs[best].capB()))
      best = k;
  }
  if (best < 0)   // no shape A covers the blocks off the middle groups: any that covers all
    for (int k = 0; k < (int)vs.size() && best < 0; ++k)
      if (variant_valid(h, k)) best = k;
  return best;
}

// process-wide choices of the autotuner, keyed by configuration and batch size
std::mutex g_tune_mu;
std::map<std::string, int> g_tuned;

}  // namespace

bool sweep_plan_supported(const Plan& P, int prec, std::string& why) {
  const int cs = prec == HELM_C64 ? (int)sizeof(float2) : (int)sizeof(double2);
  if (MemberLds(P.n, P.maxB, P.maxW, cs).bytes > kLdsBytes) {
    why = "half a line vector ((n/2 + 1) x B values) does not fit in LDS";
    return false;
  }
  for (int k = 0; k < (int)sweep_variants(prec == HELM_C64).size(); ++k)
    if (plan_variant_valid(P, prec, k)) return true;
  why = std::string("block size (window width in x2 times in x3) ") + std::to_string(P.maxB) +
        " exceeds the sweep's launch shapes (" + (prec == HELM_C64 ? "128" : "96") + " unknowns)";
  return false;
}

hipError_t fill_ones(double2* x, long long count, hipStream_t s) {
  k_fill_ones<<<(unsigned)((count + 255) / 256), 256, 0, s>>>(x, count);
  return hipGetLastError();
}

std::string tune_key(const helm_handle* h, int R) {
  const Plan& P = h->plan;
  return "n=" + std::to_string(P.n) + ",front=" + std::to_string(P.maxB_front) + ",maxB=" +
         std::to_string(P.maxB) + ",maxW=" + std::to_string(P.maxW) + ",fronts=" +
         std::to_string(P.fronts) + std::to_string(P.fronts_inner) + ",prec=" +
         (h->prec == HELM_C64 ? "c64" : "c128") + ",R=" + std::to_string((R + 7) / 8 * 8) +
         (h->nd_on ? ",nd" : "");
}

int tuned_variant(const std::string& key) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tuned.find(key);
  return it == g_tuned.end() ? -1 : it->second;
}

void remember_variant(const std::string& key, int k) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tuned[key] = k;
}

std::vector<int> tune_candidates(const helm_handle* h) {
  // the valid variants whose shapes A and B are each among the two smallest that cover the
  // blocks (and every ring depth listed for them)
  const auto& vs = sweep_variants(h->prec == HELM_C64);
  std::vector<int> capA, capB;
  for (int k = 0; k < (int)vs.size(); ++k) {
    if (!variant_valid(h, k) || vs[k].capA() < h->plan.maxB_front) continue;
    capA.push_back(vs[k].capA());
    capB.push_back(vs[k].capB());
  }
  std::sort(capA.begin(), capA.end());
  capA.erase(std::unique(capA.begin(), capA.end()), capA.end());
  std::sort(capB.begin(), capB.end());
  capB.erase(std::unique(capB.begin(), capB.end()), capB.end());
  std::vector<int> out;
  if (h->nd_on) {   // the nested-dissection kernel has one shape: only its placement varies
    for (int m = 0; m < 3; ++m) out.push_back(4 * default_variant(h) + m);
    return out;
  }
  for (int k = 0; k < (int)vs.size(); ++k) {
    if (!variant_valid(h, k) || vs[k].capA() < h->plan.maxB_front) continue;
    const bool a = vs[k].capA() == capA[0] || (capA.size() > 1 && vs[k].capA() == capA[1]);
    const bool b = vs[k].capB() == capB[0] || (capB.size() > 1 && vs[k].capB() == capB[1]);
    if (a && b)
      for (int m = 0; m < 3; ++m) out.push_back(4 * k + m);
  }
  return out;
}

// A launch choice c is variant c / 4 of sweep_variants with workgroup placement c % 4
// (sweep_kernel.h, k_sweep): 0 a right-hand side's members on one XCD, 1 one member per XCD,
// 2 one line-solve pair per XCD (3 is unused).
int sweep_variant_for(const helm_handle* h, int R) {
  if (h->variant >= 0) return h->variant;
  // a batch size the tuner has not timed (a solve's last sweeps, once some right-hand sides
  // have converged) takes the choice tuned for the nearest larger batch of the configuration:
  // a sweep's time is set by its chain, not by its batch
  for (int r = (R + 7) / 8 * 8; r <= 4096; r += 8) {
    const int t = tuned_variant(tune_key(h, r));
    if (t >= 0) return t;
  }
  return 4 * default_variant(h) + 1;
}

bool sweep_variant_valid(const helm_handle* h, int c) {
  return c >= 0 && c % 4 != 3 && variant_valid(h, c / 4);
}

std::string sweep_variant_name(bool c64, int c) {
  const auto& vs = sweep_variants(c64);
  const int k = c / 4;
  if (c < 0 || c % 4 == 3 || k >= (int)vs.size()) return "none";
  const SweepVariant& v = vs[k];
  static const char* place[] = {", one right-hand side per XCD", ", one member per XCD",
                                ", one line-solve pair per XCD"};
  return std::to_string(v.nca) + "x" + std::to_string(v.cwa) + "/ring" + std::to_string(v.da) + " + " +
         std::to_string(v.ncb) + "x" + std::to_string(v.cwb) + "/ring" + std::to_string(v.db) + place[c % 4];
}

namespace {

// right-hand side slots one cooperative launch of this kernel can hold (whole groups of 8)
hipError_t slots_per_launch(const helm_handle* h, const void* kern, int tpc, size_t sm, int wpr,
                            int* slots) {
  int dev = 0, cus = 0, per_cu = 0, coop = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
  if (e == hipSuccess) e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, tpc, sm);
  if (e != hipSuccess) return e;
  if (!coop) return hipErrorNotSupported;
  *slots = (int)(((long long)per_cu * cus) / (8LL * wpr)) * 8;
  return *slots > 0 ? hipSuccess : hipErrorInvalidConfiguration;
}

// device buffers of a sweep of `slots` right-hand side slots (grown on demand)
hipError_t ensure_buffers(helm_handle* h, int slots, int wpr, bool need_slab, hipStream_t s) {
  const Plan& P = h->plan;
  const size_t cs = csize(h);
  if (need_slab) {
    const size_t slab = (size_t)slots * P.fronts * P.n * P.n * P.maxW * cs;
    const size_t layer = (size_t)slots * P.fronts * P.n * P.n * cs;
    if (slab > h->slab_scratch_bytes) {
      if (h->slab_scratch) pool_free(h->slab_scratch, s);
      h->slab_scratch = nullptr;
      h->slab_scratch_bytes = 0;
      hipError_t e = pool_alloc(&h->slab_scratch, slab, s);
      if (e != hipSuccess) return e;
      h->slab_scratch_bytes = slab;
    }
    if (layer > h->layer_bytes) {
      if (h->layer) pool_free(h->layer, s);
      h->layer = nullptr;
      h->layer_bytes = 0;
      hipError_t e = pool_alloc(&h->layer, layer, s);
      if (e != hipSuccess) return e;
      h->layer_bytes = layer;
    }
  }
  const size_t words = (size_t)slots * XLayout(P.n, P.maxW, pieces(h), wpr).per_slot;
  const size_t bytes = kXHead + words * sizeof(unsigned long long);
  if (bytes > h->xbytes) {
    if (h->xbuf) pool_free(h->xbuf, s);
    h->xbuf = nullptr;
    h->xbytes = 0;
    hipError_t e = pool_alloc(&h->xbuf, bytes, s);
    if (e != hipSuccess) return e;
    // cleared whole: tags left in reused memory must not match (sequence numbers start at 1)
    e = hipMemsetAsync(h->xbuf, 0, bytes, s);
    if (e != hipSuccess) return e;
    h->xbytes = bytes;
  }
  return hipSuccess;
}

SweepArgs base_args(helm_handle* h) {
  SweepArgs a{};
  const Plan& P = h->plan;
  a.n = P.n;
  a.Gz = P.Gz;
  a.Gy = P.Gy;
  a.maxW = P.maxW;
  a.maxB = P.maxB;
  a.fronts = P.fronts;
  a.zmid = P.zmid;
  a.fronts_inner = P.fronts_inner;
  a.ymid = P.ymid;
  a.wpr = 2 * P.fronts * P.fronts_inner;
  a.N = (long long)P.n * P.n * P.n;
  a.groups = h->d_groups;
  a.line_off = h->d_line_off;
  a.coef = h->coef;
  a.factors = h->factors;
  a.spin_limit = h->spin_limit;
  a.drop_publish = h->drop_publish;
  return a;
}

__global__ void k_zero_word(int* w) { *w = 0; }

// one sweep (or line solve) of R right-hand sides with variant k: cooperative launches of as
// many right-hand sides as can be resident at once (and, with fixed scratch, as fit in it).
// Input / output of launch slot s: in + idx(s) in_stride, out + idx(s) out_stride, idx =
// rhs_idx or the identity.  Without fixed scratch the handle's buffers are grown from the
// pool and its own sequence numbers tag the exchanges.
hipError_t run_launches(helm_handle* h, SweepArgs a, int choice, bool z64, bool adj, int R, hipStream_t s,
                        bool timed, double bytes_per_launch_base, double vec_bytes_per_rhs,
                        double flops_per_rhs, const FixedScratch* fx = nullptr) {
  const Plan& P = h->plan;
  const bool c64 = h->prec == HELM_C64;
  if (!sweep_variant_valid(h, choice)) return hipErrorInvalidValue;
  const int k = choice / 4;
  a.xmap = choice % 4;
  const SweepVariant v = sweep_variants(c64)[k];
  // line solves by nested dissection (forward complex64 sweeps, once its factors exist)
  const bool nd = h->nd_on && h->nd && c64 && !adj;
  const void* kern = nd ? sweep_kernel_c64_nd(z64) : sweep_kernel(c64, z64, adj, k);
  if (!kern) return hipErrorInvalidValue;
  const int tpc = nd ? sweepk::kNdThreads : variant_threads(P, v);
  a.nd = nd ? h->nd : nullptr;
  a.nd_off = nd ? h->d_nd_off : nullptr;
  a.nd_k = nd ? h->nd_k : 0;
  const size_t sm = MemberLds(P.n, P.maxB, P.maxW, (int)csize(h)).bytes;
  int slots = 0;
  hipError_t e = slots_per_launch(h, kern, tpc, sm, a.wpr, &slots);
  if (e != hipSuccess) return e;
  slots = std::min(slots, (R + 7) / 8 * 8);
  unsigned long long* seq = &h->xseq;
  if (fx) {
    // [error word][exchange words][slab iterates][layers] for as many slots as fit
    const size_t cs = csize(h);
    const size_t wslot = (size_t)XLayout(P.n, P.maxW, pieces(h), a.wpr).per_slot * sizeof(unsigned long long);
    const size_t sslot = a.mode == 0 ? (size_t)P.fronts * P.n * P.n * P.maxW * cs : 0;
    const size_t lslot = a.mode == 0 ? (size_t)P.fronts * P.n * P.n * cs : 0;
    const size_t per = wslot + sslot + lslot;
    const long long fit = fx->bytes > kXHead + 3 * 256 ? (long long)((fx->bytes - kXHead - 3 * 256) / per) : 0;
    if (fit < 1) return hipErrorOutOfMemory;
    slots = (int)std::min<long long>(slots, fit);
    char* xb = fx->base;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    a.xerr = reinterpret_cast<int*>(xb);
    a.xw = reinterpret_cast<unsigned long long*>(xb + kXHead);
    a.slab = xb + up(kXHead + slots * wslot);
    a.layer = xb + up(kXHead + slots * wslot) + up(slots * sslot);
    seq = fx->seq;
    k_zero_word<<<1, 1, 0, s>>>(a.xerr);
    e = hipGetLastError();
  } else {
    e = ensure_buffers(h, slots, a.wpr, a.mode == 0, s);
    char* xb = static_cast<char*>(h->xbuf);
    a.xerr = reinterpret_cast<int*>(xb);
    a.xw = reinterpret_cast<unsigned long long*>(xb + kXHead);
    a.slab = h->slab_scratch;
    a.layer = h->layer;
  }
  if (e != hipSuccess) return e;
  // sequence numbers: every member's lines and slab steps in a launch stay below the span
  const unsigned long long span = (unsigned long long)(2 * P.Gz) * (2 * P.Gy) + 2 * P.Gz + 8;
  const int* idx = a.rhs_idx;
  const char* in0 = static_cast<const char*>(a.in);
  char* out0 = static_cast<char*>(a.out);
  const size_t isz = sizeof(double2), osz = z64 ? sizeof(double2) : (c64 ? sizeof(float2) : sizeof(double2));
  for (int r0 = 0; r0 < R; r0 += slots) {
    const int Rc = std::min(slots, R - r0);
    SweepArgs c = a;
    c.R = Rc;
    if (idx) {
      c.rhs_idx = idx + r0;
    } else {
      c.in = in0 + (size_t)r0 * a.in_stride * isz;
      c.out = out0 + (size_t)r0 * a.out_stride * osz;
    }
    c.seq0 = *seq;
    *seq += span;
    // placement 0: whole groups of 8 slots; 1: wpr per slot; 2: whole groups of 16 / wpr slots
    const int per = 16 / a.wpr;
    const unsigned grid = (unsigned)(a.xmap == 1 ? a.wpr * Rc
                                     : a.xmap == 2 ? 16 * ((Rc + per - 1) / per)
                                                   : 8 * a.wpr * ((Rc + 7) / 8));
    void* args[] = {&c};
    hipEvent_t ev = timed ? h->t_kernel.begin(s) : nullptr;
    e = hipLaunchCooperativeKernel(kern, dim3(grid), dim3(tpc), args, (unsigned)sm, s);
    if (e == hipSuccess) e = hipGetLastError();
    if (timed)
      h->t_kernel.end(ev, s, Rc, bytes_per_launch_base + vec_bytes_per_rhs * Rc, flops_per_rhs * Rc);
    if (e != hipSuccess) return e;
  }
  if (!fx) h->pairs_used = true;
  return hipSuccess;
}

}  // namespace

size_t apply_scratch_bytes(const helm_handle* h, int R) {
  const Plan& P = h->plan;
  const int wpr = 2 * P.fronts * P.fronts_inner;
  const size_t slots = (size_t)(R + 7) / 8 * 8;
  const size_t cs = csize(h);
  return slots * P.fronts * P.n * P.n * (P.maxW + 1) * cs + kXHead +
         slots * XLayout(P.n, P.maxW, pieces(h), wpr).per_slot * sizeof(unsigned long long);
}

hipError_t launch_apply(helm_handle* h, const void* r, bool r64, long long r_stride, void* z,
                        bool z64, long long z_stride, int R, const int* rhs_idx, bool adjoint,
                        hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const bool c64 = h->prec == HELM_C64;
  if (!r64) return hipErrorInvalidValue;   // inputs are always complex128
  if (!c64 && !z64) return hipErrorInvalidValue;
  SweepArgs a = base_args(h);
  a.mode = 0;
  a.in = r;
  a.out = z;
  a.in_stride = r_stride;
  a.out_stride = z_stride;
  a.rhs_idx = rhs_idx;
  const int k = sweep_variant_for(h, R);
  // algorithmic work of a launch: the sweep's factor blocks once per visit (its right-hand
  // sides share them), and per right-hand side its input read and output written
  const double N = (double)a.N;
  const double vec = N * (sizeof(double2) + (z64 ? sizeof(double2) : sizeof(float2)));
  hipEvent_t ev = h->t_apply.begin(s);
  hipError_t e = run_launches(h, a, k, z64, adjoint, R, s, true, h->sweep_factor_bytes, vec,
                              8.0 * h->sweep_factor_entries);
  h->t_apply.end(ev, s, R, 0.0, 0.0);
  return e;
}

hipError_t launch_apply_fixed(helm_handle* h, const void* r, void* z, int R, bool adjoint,
                              const FixedScratch& fx, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const long long N = (long long)h->n * h->n * h->n;
  SweepArgs a = base_args(h);
  a.mode = 0;
  a.in = r;
  a.out = z;
  a.in_stride = a.out_stride = N;
  a.rhs_idx = nullptr;
  return run_launches(h, a, sweep_variant_for(h, R), true, adjoint, R, s, false, 0.0, 0.0, 0.0, &fx);
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
  const Plan& P = h->plan;
  SweepArgs a = base_args(h);
  a.mode = 1;
  a.line_g = zg;
  a.line_l = yg;
  a.fronts = 1;
  a.fronts_inner = 1;
  a.wpr = 2;
  const long long LB = (long long)P.n * P.line_B[(size_t)zg * P.Gy + yg];
  a.in = r;
  a.out = x;
  a.in_stride = a.out_stride = LB;
  a.rhs_idx = nullptr;
  return run_launches(h, a, sweep_variant_for(h, R), true, adjoint, R, s, false, 0.0, 0.0, 0.0);
}

// time sweeps of R right-hand sides with each candidate variant, keep the fastest
hipError_t autotune_sweep(helm_handle* h, int R, int* best_out, double* best_ms, hipStream_t s) {
  std::vector<int> cand = tune_candidates(h);
  *best_out = -1;
  *best_ms = 0.0;
  if (cand.empty()) cand.push_back(4 * default_variant(h) + 1);
  if (cand[0] < 0) return hipErrorInvalidValue;
  const long long N = (long long)h->n * h->n * h->n;
  const bool c64 = h->prec == HELM_C64;
  void *in = nullptr, *out = nullptr;
  hipError_t e = pool_alloc(&in, (size_t)R * N * sizeof(double2), s);
  if (e != hipSuccess) return e;
  e = pool_alloc(&out, (size_t)R * N * (c64 ? sizeof(float2) : sizeof(double2)), s);
  if (e != hipSuccess) {
    pool_free(in, s);
    return e;
  }
  // a right-hand side of ones (the time of a sweep does not depend on the values)
  e = fill_ones(static_cast<double2*>(in), (long long)R * N, s);
  const int saved = h->variant;
  for (int k : cand) {
    if (e != hipSuccess) break;
    h->variant = k;
    SweepArgs a = base_args(h);
    a.mode = 0;
    a.in = in;
    a.out = out;
    a.in_stride = a.out_stride = N;
    e = run_launches(h, a, k, !c64, false, R, s, false, 0, 0, 0);   // warm-up
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    if (e == hipSuccess) e = hipEventRecord(t0, s);
    for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) e = run_launches(h, a, k, !c64, false, R, s, false, 0, 0, 0);
    if (e == hipSuccess) e = hipEventRecord(t1, s);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    if (e == hipSuccess && (*best_out < 0 || ms / 2 < *best_ms)) {
      *best_out = k;
      *best_ms = ms / 2;
    }
    if (e == hipSuccess && std::getenv("HELM_VERBOSE")) {
      std::fprintf(stderr, "[helm tune] R=%d candidate %d (%s): %.2f ms per sweep\n", R, k,
                   sweep_variant_name(c64, k).c_str(), ms / 2);
      std::fflush(stderr);
    }
  }
  h->variant = saved;
  pool_free(in, s);
  pool_free(out, s);
  return e;
}

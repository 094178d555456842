// C ABI of libhelm: argument validation, memory planning and ownership, error codes.
// Every numerical step runs in the HIP kernels of this library; the host only plans,
// allocates, launches and reads the scalars GMRES needs to decide.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "common.h"

namespace {
thread_local std::string g_last_error;

constexpr size_t kFactorPad = 64;        // complex entries of zeros after the factor array

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

size_t csize(int prec) { return prec == HELM_C64 ? sizeof(float2) : sizeof(double2); }

int validate(const helm_grid* grid, const helm_pml* pml, int d, int prec, Plan& plan) {
  if (!grid || !pml) return fail(HELM_EINVAL, "grid and pml must not be NULL");
  if (prec != HELM_C64 && prec != HELM_C128) return fail(HELM_EINVAL, "prec must be HELM_C64 or HELM_C128");
  if (!(pml->C > 0.0) || !std::isfinite(pml->C)) return fail(HELM_EINVAL, "PML constant C must be finite and > 0");
  if (!(pml->C_moving >= 0.0) || !std::isfinite(pml->C_moving))
    return fail(HELM_EINVAL, "moving-PML constant C_moving must be finite and >= 0");
  std::string msg;
  const int fronts = pml->fronts == 0 ? 1 : pml->fronts;
  const int fronts_inner = pml->fronts_inner == 0 ? 1 : pml->fronts_inner;
  int rc = build_plan(grid->n, pml->b, pml->p, d, fronts, fronts_inner, prec, plan, msg);
  if (rc != HELM_OK) return fail(rc, msg);
  if (!setup_fits(plan.maxB, (int)csize(prec)))
    return fail(HELM_EINVAL, "a B x B block does not fit in LDS for the setup");
  if (!sweep_plan_supported(plan, prec, msg)) return fail(HELM_EINVAL, msg);
  return HELM_OK;
}

size_t planned_bytes(const Plan& p, int prec) {
  const size_t N = (size_t)p.n * p.n * p.n;
  return ((size_t)p.total_elems + kFactorPad) * csize(prec) + N * sizeof(double) +
         (size_t)(2 * (p.n + 1) + 1 + 2 * p.p + 2 + 5 * (p.n + 2)) * sizeof(double2) +
         (size_t)(p.Gz + p.Gy) * sizeof(GroupInfo) +
         (size_t)p.Gz * p.Gy * (sizeof(long long) + sizeof(int) + 1);
}

// factor entries one sweep visits: line (g, l) is solved once per inner pass it takes part
// in (twice unless l is the last x2-group with one inner front, or the middle one with two)
// and once per outer pass (twice unless g is the last x3-group with one front, or the middle
// one with two fronts); each solve visits its n blocks twice (forward and backward
// substitution) and reads B*B entries per visit.  Algorithmic bytes of one sweep of one
// right-hand side: these entries plus the input read and the output written (complex128).
double sweep_entries(const Plan& p) {
  double acc = 0.0;
  for (int g = 0; g < p.Gz; ++g)
    for (int l = 0; l < p.Gy; ++l) {
      const bool once = p.fronts == 2 ? g == p.zmid : g == p.Gz - 1;
      const bool ionce = p.fronts_inner == 2 ? l == p.ymid : l == p.Gy - 1;
      const double mult = (once ? 1.0 : 2.0) * (ionce ? 1.0 : 2.0);
      const double B = p.line_B[(size_t)g * p.Gy + l];
      acc += mult * 2.0 * p.n * B * B;
    }
  return acc;
}

void release(helm_handle* h) {
  h->t_apply.reset();
  h->t_matvec.reset();
  h->t_kernel.reset();
  void* ptrs[] = {h->kappa, h->sbd, h->smv, h->coef, h->diag, h->d_groups, h->d_line_off,
                  h->d_setup_lines, h->factors, h->d_err, h->slab_scratch, h->layer,
                  h->d_rhs_idx, h->xbuf, h->nd, h->d_nd_off};
  for (void* p : ptrs)
    if (p) pool_free(p, h->last_stream);
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

// the nested-dissection factors of every line (timed); on failure none are kept
int nd_factor(helm_handle* h, hipStream_t s, std::string& why) {
  LaunchTimer t;
  hipEvent_t ev = t.begin(s);
  const int rc = nd_build(h, s, why);
  t.end(ev, s, 1);
  t.flush();
  h->nd_setup_ms = t.ms;
  if (rc != HELM_OK) {
    if (h->nd) pool_free(h->nd, s);
    if (h->d_nd_off) pool_free(h->d_nd_off, s);
    h->nd = nullptr;
    h->d_nd_off = nullptr;
    h->nd_on = false;
  }
  return rc;
}
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

extern "C" {

const char* helm_last_error(void) { return g_last_error.c_str(); }

const char* helm_error_string(int code) {
  switch (code) {
    case HELM_OK: return "HELM_OK";
    case HELM_ENOTCONV: return "HELM_ENOTCONV: GMRES reached maxit before tol, or a residual was not finite";
    case HELM_EINVAL: return "HELM_EINVAL: invalid argument";
    case HELM_ENOMEM: return "HELM_ENOMEM: not enough device memory";
    case HELM_ESINGULAR: return "HELM_ESINGULAR: singular block in the line factorisation";
    case HELM_EHIP: return "HELM_EHIP: HIP runtime error";
    default: return "unknown helm status";
  }
}

int helm_plan_bytes(const helm_grid* grid, const helm_pml* pml, int slab_layers, int prec,
                    size_t* bytes, int* n_lines, int* max_block) {
  Plan plan;
  int rc = validate(grid, pml, slab_layers, prec, plan);
  if (rc != HELM_OK) return rc;
  if (bytes) *bytes = planned_bytes(plan, prec);
  if (n_lines) *n_lines = plan.Gz * plan.Gy;
  if (max_block) *max_block = plan.maxB;
  return HELM_OK;
}

int helm_setup(const helm_grid* grid, const double* c_dev, double omega, const helm_pml* pml,
               int slab_layers, int prec, void* stream, helm_handle** out) {
  if (!out) return fail(HELM_EINVAL, "out must not be NULL");
  *out = nullptr;
  if (!c_dev) return fail(HELM_EINVAL, "c_dev must not be NULL");
  if (!(omega > 0.0) || !std::isfinite(omega)) return fail(HELM_EINVAL, "omega must be finite and > 0");
  Plan plan;
  int rc = validate(grid, pml, slab_layers, prec, plan);
  if (rc != HELM_OK) return rc;
  size_t free_b = 0;
  if (device_free_bytes(&free_b) != hipSuccess) return fail(HELM_EHIP, "hipMemGetInfo failed");
  const size_t need = planned_bytes(plan, prec);
  if (need > free_b)
    return fail(HELM_ENOMEM, "setup needs " + std::to_string(need) + " bytes, " +
                                 std::to_string(free_b) + " free");
  helm_handle* h = new helm_handle();
  h->plan = plan;
  h->n = plan.n;
  h->prec = prec;
  h->omega = omega;
  h->h = 1.0 / (plan.n + 1);
  h->C = pml->C;
  h->C_mv = pml->C_moving > 0.0 ? pml->C_moving : pml->C;
  (void)hipGetDevice(&h->device);
  const size_t N = (size_t)plan.n * plan.n * plan.n;
  hipStream_t s = S(stream);
  h->last_stream = s;
  auto bail = [&](int code, const std::string& m) {
    release(h);
    delete h;
    return fail(code, m);
  };
#define ALLOC(ptr, bytes)                                                             \
  if (pool_alloc((void**)&(ptr), (bytes), s) != hipSuccess)                           \
    return bail(HELM_ENOMEM, std::string("device allocation failed for ") + #ptr);
  ALLOC(h->kappa, N * sizeof(double));
  ALLOC(h->sbd, (size_t)(2 * (plan.n + 1) + 1) * sizeof(double2));
  ALLOC(h->smv, (size_t)(2 * plan.p + 2) * sizeof(double2));
  ALLOC(h->coef, (size_t)4 * (plan.n + 2) * sizeof(double2));
  ALLOC(h->diag, (size_t)(plan.n + 2) * sizeof(double2));
  ALLOC(h->d_groups, plan.groups.size() * sizeof(GroupInfo));
  ALLOC(h->d_line_off, plan.line_off.size() * sizeof(long long));
  ALLOC(h->d_setup_lines, plan.line_off.size() * sizeof(int));
  // the sweep's row-major block walk may read up to 64 entries past the last block
  ALLOC(h->factors, ((size_t)plan.total_elems + kFactorPad) * csize(prec));
  ALLOC(h->d_err, 2 * sizeof(int));
#undef ALLOC
  if (hipMemsetAsync((char*)h->factors + (size_t)plan.total_elems * csize(prec), 0,
                     kFactorPad * csize(prec), s) != hipSuccess)
    return bail(HELM_EHIP, "clearing the factor padding failed");
  if (hipMemcpyAsync(h->d_groups, plan.groups.data(), plan.groups.size() * sizeof(GroupInfo),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(h->d_line_off, plan.line_off.data(), plan.line_off.size() * sizeof(long long),
                     hipMemcpyHostToDevice, s) != hipSuccess)
    return bail(HELM_EHIP, "copying the plan failed");
  const std::vector<int> setup_lines = setup_classes(plan, (int)csize(prec), nullptr).order;
  if (hipMemcpyAsync(h->d_setup_lines, setup_lines.data(), setup_lines.size() * sizeof(int),
                     hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)   // the host vector goes out of scope
    return bail(HELM_EHIP, "copying the plan failed");
  h->sweep_factor_entries = sweep_entries(plan);
  h->sweep_factor_bytes = h->sweep_factor_entries * csize(prec);
  h->apply_bytes_per_rhs = h->sweep_factor_bytes + 32.0 * N;
  LaunchTimer t_setup;
  hipEvent_t ev = t_setup.begin(s);
  if (launch_coefficients(h, c_dev, true, s) != hipSuccess) return bail(HELM_EHIP, "coefficient kernels failed");
  int err[2] = {0, 0};
  if (hipMemcpyAsync(err, h->d_err, sizeof(err), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return bail(HELM_EHIP, "coefficient kernels failed");
  if (err[0]) return bail(HELM_EINVAL, "c must be finite and > 0 at every node");
  hipError_t e = launch_setup(h, s);
  if (e != hipSuccess) return bail(HELM_EHIP, std::string("setup kernel: ") + hipGetErrorString(e));
  t_setup.end(ev, s, 1);
  if (hipMemcpyAsync(err, h->d_err, sizeof(err), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return bail(HELM_EHIP, "setup kernel failed");
  t_setup.flush();
  h->setup_ms = t_setup.ms;
  if (err[0]) return bail(HELM_ESINGULAR, "singular block in line " + std::to_string(err[1]));
  *out = h;
  return HELM_OK;
}

static int check_batch(helm_handle* h, const void* a, const void* b, int R) {
  if (!h) return fail(HELM_EINVAL, "handle is NULL");
  if (!a || !b) return fail(HELM_EINVAL, "vector pointers must not be NULL");
  if (a == b) return fail(HELM_EINVAL, "input and output must not alias");
  if (R < 1) return fail(HELM_EINVAL, "R must be >= 1");
  return HELM_OK;
}

// the error word of the paired line solves: a member that gave up waiting for its partner
// (possible only after a fault elsewhere) has written NaN into its line solution
static int check_exchange(helm_handle* h, hipStream_t s) {
  int bad = 0;
  HIP_TRY(take_exchange_error(h, s, &bad));
  if (bad) return fail(HELM_EHIP, "a paired line solve of the sweep timed out waiting for its partner");
  return HELM_OK;
}

// the first sweep of a configuration (and batch size) in the process times the candidate
// launch shapes and keeps the fastest (HELM_AUTOTUNE=0 turns this off; HELM_TUNE_CACHE names
// a file of earlier choices, read and appended)
static int first_use_tune(helm_handle* h, int R, hipStream_t s) {
  if (h->variant >= 0) return HELM_OK;
  const char* env = std::getenv("HELM_AUTOTUNE");
  if (env && env[0] == '0') return HELM_OK;
  const std::string key = tune_key(h, R);
  if (tuned_variant(key) >= 0) return HELM_OK;
  const char* path = std::getenv("HELM_TUNE_CACHE");
  return tune_and_remember(h, R, key, path, nullptr, nullptr, s);
}

static int apply_impl(helm_handle* h, const void* r, void* z, int R, bool adjoint, void* stream) {
  int rc = check_batch(h, r, z, R);
  if (rc != HELM_OK) return rc;
  const long long N = (long long)h->n * h->n * h->n;
  hipStream_t s = S(stream);
  h->last_stream = s;
  rc = first_use_tune(h, R, s);
  if (rc != HELM_OK) return rc;
  HIP_TRY(launch_apply(h, r, true, N, z, true, N, R, nullptr, adjoint, s));
  if (h->pairs_used) return check_exchange(h, s);
  return HELM_OK;
}

int helm_apply(helm_handle* h, const void* r_dev, void* z_dev, int R, void* stream) {
  return apply_impl(h, r_dev, z_dev, R, false, stream);
}

int helm_apply_adjoint(helm_handle* h, const void* r_dev, void* z_dev, int R, void* stream) {
  return apply_impl(h, r_dev, z_dev, R, true, stream);
}

int helm_matvec(helm_handle* h, const void* u_dev, void* y_dev, int R, int adjoint, void* stream) {
  int rc = check_batch(h, u_dev, y_dev, R);
  if (rc != HELM_OK) return rc;
  const long long N = (long long)h->n * h->n * h->n;
  HIP_TRY(launch_matvec(h, u_dev, true, nullptr, (double2*)y_dev, R, nullptr, N, N, adjoint != 0, 0,
                        S(stream)));
  return HELM_OK;
}

int helm_solve(helm_handle* h, const void* f_dev, void* u_dev, int R, double tol, int restart,
               int maxit, int adjoint, int* iters_host, double* relres_host, void* stream) {
  int rc = check_batch(h, f_dev, u_dev, R);
  if (rc != HELM_OK) return rc;
  if (!(tol > 0.0)) return fail(HELM_EINVAL, "tol must be > 0");
  if (maxit < 0) return fail(HELM_EINVAL, "maxit must be >= 0");
  hipStream_t s = S(stream);
  h->last_stream = s;
  rc = first_use_tune(h, R, s);
  if (rc != HELM_OK) return rc;
  std::string msg;
  rc = fgmres_solve(h, (const double2*)f_dev, (double2*)u_dev, R, tol, restart, maxit, adjoint != 0,
                    iters_host, relres_host, s, msg);
  // the error word is taken (and cleared) on every exit: a timed-out exchange is reported by
  // the call whose sweeps it spoiled, and never by a later one
  const int xrc = check_exchange(h, s);
  if (rc < 0) return fail(rc, msg);
  if (xrc != HELM_OK) return xrc;
  if (rc != HELM_OK && !msg.empty()) g_last_error = msg;
  return rc;
}

int helm_grad_c(helm_handle* h, const void* u_dev, const void* lam_dev, int R, double* grad_dev,
                void* stream) {
  int rc = check_batch(h, u_dev, lam_dev, R);
  if (rc != HELM_OK) return rc;
  if (!grad_dev) return fail(HELM_EINVAL, "grad_dev must not be NULL");
  HIP_TRY(launch_grad(h, (const double2*)u_dev, (const double2*)lam_dev, R, grad_dev, S(stream)));
  return HELM_OK;
}

int helm_misfit(helm_handle* h, const void* u_dev, const void* d_dev, int R, int plane_k,
                double* J_host, void* g_dev, void* stream) {
  int rc = check_batch(h, u_dev, d_dev, R);
  if (rc != HELM_OK) return rc;
  if (plane_k < 1 || plane_k > h->n) return fail(HELM_EINVAL, "plane_k must be in [1, n]");
  hipStream_t s = S(stream);
  double* J_dev = nullptr;
  h->last_stream = s;
  HIP_TRY(pool_alloc((void**)&J_dev, sizeof(double), s));
  hipError_t e = launch_misfit(h, (const double2*)u_dev, (const double2*)d_dev, R, plane_k, J_dev,
                               (double2*)g_dev, s);
  if (e == hipSuccess && J_host) {
    e = hipMemcpyAsync(J_host, J_dev, sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
  }
  pool_free(J_dev, s);
  HIP_TRY(e);
  return HELM_OK;
}

int helm_set_line_solver(helm_handle* h, int solver, void* stream) {
  if (!h) return fail(HELM_EINVAL, "handle must not be NULL");
  if (solver == HELM_LINE_LDU) {
    h->nd_on = false;
    return HELM_OK;
  }
  if (solver != HELM_LINE_ND) return fail(HELM_EINVAL, "solver must be HELM_LINE_LDU or HELM_LINE_ND");
  std::string why;
  if (!nd_supported(h->plan, h->prec, why)) return fail(HELM_EINVAL, why);
  hipStream_t s = S(stream);
  h->last_stream = s;
  if (!h->nd) {
    const int rc = nd_factor(h, s, why);
    if (rc != HELM_OK) return fail(rc, why);
  }
  h->nd_on = true;
  return HELM_OK;
}

int helm_set_medium(helm_handle* h, const double* c_dev, void* stream) {
  if (!h || !c_dev) return fail(HELM_EINVAL, "handle and c_dev must not be NULL");
  hipStream_t s = S(stream);
  HIP_TRY(launch_coefficients(h, c_dev, false, s));
  int err[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(err, h->d_err, sizeof(err), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (err[0]) return fail(HELM_EINVAL, "c must be finite and > 0 at every node");
  return HELM_OK;
}

int helm_update_medium(helm_handle* h, const double* c_dev, const int* box_host, int* n_refactored,
                       void* stream) {
  if (n_refactored) *n_refactored = 0;
  if (!h || !c_dev || !box_host) return fail(HELM_EINVAL, "handle, c_dev and box must not be NULL");
  const int n = h->n;
  const int i0 = box_host[0], i1 = box_host[1], j0 = box_host[2], j1 = box_host[3],
            k0 = box_host[4], k1 = box_host[5];
  if (i0 < 1 || i1 < i0 || i1 > n || j0 < 1 || j1 < j0 || j1 > n || k0 < 1 || k1 < k0 || k1 > n)
    return fail(HELM_EINVAL, "box must satisfy 1 <= lo <= hi <= n on every axis");
  hipStream_t s = S(stream);
  HIP_TRY(launch_coefficients(h, c_dev, false, s));
  int err[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(err, h->d_err, sizeof(err), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (err[0]) return fail(HELM_EINVAL, "c must be finite and > 0 at every node");
  // a line's matrix reads omega^2/c^2 on its window only (x3-window x x2-window x all of x1)
  const Plan& P = h->plan;
  auto meets = [](const GroupInfo& gi, int lo, int hi) { return gi.w0 <= hi && gi.w0 + gi.W - 1 >= lo; };
  std::vector<int> lines;
  for (int g = 0; g < P.Gz; ++g) {
    if (!meets(P.zg(g), k0, k1)) continue;
    for (int l = 0; l < P.Gy; ++l)
      if (meets(P.yg(l), j0, j1)) lines.push_back(g * P.Gy + l);
  }
  if (lines.empty()) return HELM_OK;
  const SetupClasses cls = setup_classes(P, (int)csize(h->prec), &lines);
  // the setup's line list is free after helm_setup: it takes this list
  HIP_TRY(hipMemcpyAsync(h->d_setup_lines, cls.order.data(), cls.order.size() * sizeof(int),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(h->d_err, 0, 2 * sizeof(int), s));
  LaunchTimer t;
  hipEvent_t ev = t.begin(s);
  HIP_TRY(launch_setup_lines(h, h->d_setup_lines, cls, s));
  t.end(ev, s, 1);
  HIP_TRY(hipMemcpyAsync(err, h->d_err, sizeof(err), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  t.flush();
  h->setup_ms = t.ms;
  if (n_refactored) *n_refactored = (int)lines.size();
  if (err[0]) return fail(HELM_ESINGULAR, "singular block in line " + std::to_string(err[1]));
  if (h->nd) {   // the nested-dissection factors, all lines again
    std::string why;
    const int rc = nd_factor(h, s, why);
    if (rc != HELM_OK) return fail(rc, why);
  }
  return HELM_OK;
}

int helm_workspace_bytes(const helm_handle* h, int R, int restart, int maxit, size_t* solve_bytes,
                         size_t* apply_bytes) {
  if (!h) return fail(HELM_EINVAL, "handle is NULL");
  if (R < 1 || restart < 1 || restart > 200 || maxit < 0)
    return fail(HELM_EINVAL, "need R >= 1, 1 <= restart <= 200, maxit >= 0");
  const size_t ab = apply_scratch_bytes(h, R);
  if (apply_bytes) *apply_bytes = ab;
  if (solve_bytes) *solve_bytes = fgmres_bytes(h, R, restart, maxit) + ab;
  return HELM_OK;
}

int helm_info(const helm_handle* h, size_t* factor_bytes, int* n_lines, int* max_block) {
  if (!h) return fail(HELM_EINVAL, "handle is NULL");
  if (factor_bytes) *factor_bytes = (size_t)h->plan.total_elems * csize(h->prec);
  if (n_lines) *n_lines = h->plan.Gz * h->plan.Gy;
  if (max_block) *max_block = h->plan.maxB;
  return HELM_OK;
}

int helm_line_factors(const helm_handle* h, int zg, int yg, void* dst_dev, int* B_out,
                      int* mid_out, void* stream) {
  if (!h) return fail(HELM_EINVAL, "handle is NULL");
  if (zg < 0 || zg >= h->plan.Gz || yg < 0 || yg >= h->plan.Gy)
    return fail(HELM_EINVAL, "group index out of range");
  const size_t line = (size_t)zg * h->plan.Gy + yg;
  const int B = h->plan.line_B[line];
  if (B_out) *B_out = B;
  if (mid_out) *mid_out = h->plan.line_mid();
  if (!dst_dev) return HELM_OK;
  const size_t cs = csize(h->prec);
  HIP_TRY(hipMemcpyAsync(dst_dev, (const char*)h->factors + (size_t)h->plan.line_off[line] * cs,
                         (size_t)h->n * B * B * cs, hipMemcpyDeviceToDevice, S(stream)));
  return HELM_OK;
}

int helm_line_solve(helm_handle* h, int zg, int yg, const void* r_dev, void* x_dev, int R,
                    int adjoint, void* stream) {
  int rc = check_batch(h, r_dev, x_dev, R);
  if (rc != HELM_OK) return rc;
  if (zg < 0 || zg >= h->plan.Gz || yg < 0 || yg >= h->plan.Gy)
    return fail(HELM_EINVAL, "group index out of range");
  HIP_TRY(launch_line_solve(h, zg, yg, (const double2*)r_dev, (double2*)x_dev, R, adjoint != 0,
                            S(stream)));
  return HELM_OK;
}

int helm_set_launch(helm_handle* h, int variant) {
  if (!h) return fail(HELM_EINVAL, "handle is NULL");
  if (variant < -1 || (variant >= 0 && !sweep_variant_valid(h, variant)))
    return fail(HELM_EINVAL, "variant " + std::to_string(variant) + " does not cover this handle's blocks");
  h->variant = variant;
  return HELM_OK;
}

int helm_sweep_shape(const helm_handle* h, int R, int* variant, char* name, int name_len) {
  if (!h) return fail(HELM_EINVAL, "handle is NULL");
  if (R < 1) return fail(HELM_EINVAL, "R must be >= 1");
  const int k = sweep_variant_for(h, R);
  if (variant) *variant = k;
  if (name && name_len > 0) {
    const std::string nm = sweep_variant_name(h->prec == HELM_C64, k);
    std::snprintf(name, (size_t)name_len, "%s", nm.c_str());
  }
  return HELM_OK;
}

int helm_set_exchange_test(helm_handle* h, int drop_publish, unsigned spin_limit) {
  if (!h) return fail(HELM_EINVAL, "handle is NULL");
  if (drop_publish != 0 && drop_publish != 1) return fail(HELM_EINVAL, "drop_publish must be 0 or 1");
  h->drop_publish = drop_publish;
  h->spin_limit = spin_limit ? spin_limit : kSpinDefault;
  return HELM_OK;
}

}  // extern "C"

// ---- launch-shape autotuner -------------------------------------------------------------
static int tune_lookup(const char* path, const std::string& key) {
  FILE* fp = std::fopen(path, "r");
  if (!fp) return -1;
  char line[512];
  int found = -1;
  const std::string pat = "\"key\": \"" + key + "\"";
  while (std::fgets(line, sizeof line, fp)) {
    if (std::strstr(line, pat.c_str())) {
      const char* q = std::strstr(line, "\"variant\":");
      int v = -1;
      if (q && std::sscanf(q + 10, "%d", &v) == 1) found = v;
    }
  }
  std::fclose(fp);
  return found;
}

int tune_and_remember(helm_handle* h, int R, const std::string& key, const char* path, int* out,
                      double* ms_out, hipStream_t s) {
  if (path) {
    const int v = tune_lookup(path, key);
    if (v >= 0 && sweep_variant_valid(h, v)) {
      remember_variant(key, v);
      if (out) *out = v;
      if (ms_out) *ms_out = 0.0;
      return HELM_OK;
    }
  }
  int best = -1;
  double ms = 0.0;
  HIP_TRY(autotune_sweep(h, R, &best, &ms, s));
  int bad = 0;
  HIP_TRY(take_exchange_error(h, s, &bad));
  if (bad) return fail(HELM_EHIP, "a sweep exchange timed out while tuning");
  remember_variant(key, best);
  if (out) *out = best;
  if (ms_out) *ms_out = ms;
  if (path) {
    FILE* fp = std::fopen(path, "a");
    if (fp) {
      std::fprintf(fp, "{\"key\": \"%s\", \"variant\": %d, \"shape\": \"%s\", \"ms_per_sweep\": %.3f}\n",
                   key.c_str(), best, sweep_variant_name(h->prec == HELM_C64, best).c_str(), ms);
      std::fclose(fp);
    }
  }
  return HELM_OK;
}

extern "C" {

int helm_autotune(helm_handle* h, int R, const char* cache_path, int* variant_out, double* ms_per_sweep,
                  void* stream) {
  if (!h) return fail(HELM_EINVAL, "handle is NULL");
  if (R < 1) return fail(HELM_EINVAL, "R must be >= 1");
  hipStream_t s = S(stream);
  h->last_stream = s;
  int best = -1;
  double ms = 0.0;
  const int rc = tune_and_remember(h, R, tune_key(h, R), cache_path, &best, &ms, s);
  if (rc != HELM_OK) return rc;
  h->variant = best;
  if (variant_out) *variant_out = best;
  if (ms_per_sweep) *ms_per_sweep = ms;
  return HELM_OK;
}

int helm_get_stats(helm_handle* h, helm_stats* out) {
  if (!h || !out) return fail(HELM_EINVAL, "handle and out must not be NULL");
  h->t_apply.flush();
  h->t_matvec.flush();
  out->setup_ms = h->setup_ms;
  out->apply_launches = h->t_apply.launches;
  out->apply_rhs = h->t_apply.rhs;
  out->apply_ms = h->t_apply.ms;
  out->apply_bytes_per_rhs = h->apply_bytes_per_rhs;
  out->matvec_launches = h->t_matvec.launches;
  out->matvec_rhs = h->t_matvec.rhs;
  out->matvec_ms = h->t_matvec.ms;
  out->matvec_bytes_per_rhs = 40.0 * h->n * h->n * h->n;
  h->t_kernel.flush();
  out->kernel_launches = h->t_kernel.launches;
  out->kernel_rhs = h->t_kernel.rhs;
  out->kernel_ms = h->t_kernel.ms;
  out->kernel_bytes = h->t_kernel.bytes;
  out->kernel_flops = h->t_kernel.flops;
  out->nd_setup_ms = h->nd_setup_ms;
  return HELM_OK;
}

int helm_reset_stats(helm_handle* h) {
  if (!h) return fail(HELM_EINVAL, "handle is NULL");
  h->t_apply.reset();
  h->t_matvec.reset();
  h->t_kernel.reset();
  return HELM_OK;
}

void helm_destroy(helm_handle* h) {
  if (!h) return;
  release(h);
  delete h;
}

}  // extern "C"

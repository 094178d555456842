/*
 * helm.h -- C ABI of the MI355X (gfx950) recursive sweeping preconditioner for the 3D
 * Helmholtz equation (F. Liu, L. Ying, "Recursive Sweeping Preconditioner for the 3D
 * Helmholtz Equation", 2015).
 *
 * Problem (Sec. 2, eq. (2) and its discretisation eq. (3)): on the unit cube with n interior
 * nodes per axis, h = 1/(n+1), node (i,j,k) at (ih, jh, kh),
 *     sum_d (s_d)_p/h [ (s_d)_{p+e_d/2}/h (u_{p+e_d}-u_p) - (s_d)_{p-e_d/2}/h (u_p-u_{p-e_d}) ]
 *     + (omega^2/c^2)_p u_p = f_p ,            u = 0 outside the grid,
 * with s = 1/(1 + i sigma/omega), sigma(x) = (C/eta)((x-eta)/eta)^2 on [0, eta] (Sec. 2),
 * eta = b h, mirrored on all six faces (Sec. 5 puts PMLs on every face).
 *
 * Conventions for every entry point:
 *  - All *_dev pointers are device pointers on the current HIP device, owned by the caller,
 *    contiguous.  Grids are stored with x1 fastest, then x2, then x3 (the column-major order
 *    of Sec. 3); a batch of R vectors is R consecutive grids of n^3 values.
 *  - Complex data is interleaved (re, im) double precision (complex128) unless stated.
 *  - `stream` is a hipStream_t (NULL = default stream).  Work is queued on it; calls that
 *    return host outputs (helm_solve, helm_setup's error check) synchronise it.
 *  - A handle is used by one stream at a time; calls on one handle must not overlap.
 *  - Return value: HELM_OK (0), HELM_ENOTCONV (1, a warning: outputs are valid), or a
 *    negative error code.  Nothing is thrown across the ABI.  helm_error_string() names a
 *    code; helm_last_error() gives the last detailed message of the calling thread.
 */
#ifndef HELM_H
#define HELM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HELM_OK 0
#define HELM_ENOTCONV 1     /* GMRES hit maxit; u, iters and relres are still valid      */
#define HELM_EINVAL (-1)    /* invalid argument (sizes, parameters, non-positive c, ...)  */
#define HELM_ENOMEM (-2)    /* planned device bytes exceed free memory (checked first)    */
#define HELM_ESINGULAR (-3) /* zero or non-finite pivot while inverting a block            */
#define HELM_EHIP (-4)      /* a HIP runtime call failed                                 */

#define HELM_C64 0          /* complex64 factors and sweeps, FP64 GMRES (mixed precision) */
#define HELM_C128 1         /* complex128 everywhere                                     */

typedef struct helm_handle helm_handle; /* opaque: owns kappa, factors and workspaces */

typedef struct {
  int n;                    /* interior nodes per axis, h = 1/(n+1)                       */
} helm_grid;

typedef struct {
  int b;                    /* boundary PML cells, eta = b h (Sec. 2)                      */
  double C;                 /* the constant C of sigma (Sec. 2), > 0                        */
  int p;                    /* moving-PML cells of each auxiliary problem (Sec. 3, 4.2)    */
  int fronts;               /* outer sweep over x3: 1 (or 0) = from x3 = 0 only, as in     */
                            /* Algorithm 6; 2 = from both faces meeting in a middle slab   */
                            /* padded with moving PML on both sides (Sec. 4.2 note 3, the  */
                            /* configuration of Sec. 5)                                    */
  int fronts_inner;         /* the same choice for the inner sweep over x2 (Algorithm 4):  */
                            /* 1 (or 0) from x2 = 0 only; 2 from both faces, meeting in a  */
                            /* middle x2-group                                              */
  double C_moving;          /* the constant C of the auxiliary problems' moving PML (Sec. 3,*/
                            /* 4.2); 0: the same as C.  Changes the preconditioner only.  */
} helm_pml;

/*
 * helm_setup -- Algorithm 5 (with Algorithm 3 per slab, Sec. 4.2): form and block-LDU factor
 * every quasi-1D auxiliary ("line") problem.
 *   grid, pml     : host structs.  Requires n >= 2b+1, b >= 1, 0 <= p <= b, C > 0,
 *                   pml->fronts and pml->fronts_inner in {0, 1, 2}.
 *   c_dev         : n^3 float64 velocities at the nodes, all finite and > 0; may be freed
 *                   after the call (the handle keeps omega^2/c^2).
 *   omega         : angular frequency > 0.
 *   slab_layers   : d >= 1, physical layers per auxiliary problem in x3 and in x2 (Sec. 4.2).
 *   prec          : HELM_C64 or HELM_C128 (precision of factors and sweeps).
 *   out           : receives the handle (NULL on error).
 * Groups along an axis swept from one face: nodes 1..b, then consecutive groups of d nodes
 * (the last may be shorter).  The auxiliary problem of every group but the first is padded
 * with p moving-PML nodes whose zero-Dirichlet plane lies p+1 spacings below the group, with
 * sigma(.; (p+1)h) measured from that plane; above the group's first node the boundary
 * profile is kept.  Along an axis swept from both faces (x3 with fronts = 2, x2 with
 * fronts_inner = 2) the groups are nodes 1..b, groups of d over b+1..n-b (the last may be
 * shorter) and nodes n-b+1..n; with G of them the middle one is group G/2; groups below it
 * are padded below as above, groups above it padded above with the mirror image (plane p+1
 * spacings above the group), the middle group on both sides, and the first and last groups
 * not at all.  Line blocks have B = (x2 window) x (x3 window) unknowns, at most 128
 * (complex64) or 96 (complex128), and half a line's values ((n/2 + 1) x B) must fit in the
 * LDS of a workgroup.  Every line is factored with its x1-blocks eliminated from both ends
 * towards the middle block (helm_line_factors).
 * Errors: HELM_EINVAL, HELM_ENOMEM (the planned bytes of helm_plan_bytes exceed the free
 * device memory plus the pool's cached blocks; checked before anything is allocated),
 * HELM_ESINGULAR, HELM_EHIP.
 * Synchronises `stream`.
 */
int helm_setup(const helm_grid* grid, const double* c_dev, double omega, const helm_pml* pml,
               int slab_layers, int prec, void* stream, helm_handle** out);

/*
 * helm_apply -- Algorithm 6 (outer sweep over x3-groups; each slab block applied by
 * Algorithm 4, the inner sweep over x2-groups; each line block solved exactly by its block
 * LDU): z = M^{-1} r for R right-hand sides in one persistent launch.  With two fronts the
 * outer sweep is the block LDU with the x3-groups eliminated from both faces towards the
 * middle group (forward: each front carries its f - A u coupling, the middle slab takes
 * both; backward: each front subtracts the correction from its neighbour nearer the middle).
 * Two inner fronts do the same over the x2-groups of every slab.  The whole sweep of the R
 * right-hand sides is one cooperative launch (in chunks of right-hand sides when they cannot
 * all be resident): per right-hand side one workgroup for each half of every line solve
 * (the two chains of the two-sided block LDU), each outer front and each inner front; they
 * exchange the few values they share through device memory (a wait gives up after a bounded
 * number of polls, leaving NaN and an error word).
 *   r_dev, z_dev : R*n^3 complex128 each (may not alias).  In HELM_C64 mode r is rounded to
 *                  complex64 on entry and z is widened on exit.
 * Synchronises `stream` to read the sweep's error word; returns HELM_EHIP if an exchange
 * timed out (only possible after a fault elsewhere, or with helm_set_exchange_test).
 * The first sweep of a configuration in the process runs the autotuner (helm_autotune) unless
 * the environment sets HELM_AUTOTUNE=0; HELM_TUNE_CACHE may name a file of earlier choices.
 */
int helm_apply(helm_handle* h, const void* r_dev, void* z_dev, int R, void* stream);

/*
 * helm_apply_static -- helm_apply (adjoint = 0) or helm_apply_adjoint (adjoint = 1) that
 * allocates nothing, for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  The sweep's scratch (slab
 * iterates, received layers, exchange words) lives in a static device array of 128 MiB that
 * each GPU the library runs on holds until the process ends; the right-hand sides are swept
 * in chunks that fit in it (about 3.8 MB per right-hand side at 127^3 with complex64 factors
 * and two fronts in both axes).  The launch shape is the handle's or the autotuner's earlier
 * choice, else the default (this call never tunes).  Does not synchronise `stream` and does
 * not report an exchange timeout (z then holds NaN there).  Every call on a GPU shares that
 * GPU's array: calls that overlap on one GPU (from different streams or threads) race and
 * must not be made.
 *   r_dev, z_dev : R*n^3 complex128 each (may not alias), as for helm_apply.
 * Errors: HELM_EINVAL (NULL or aliasing vectors, R < 1, one right-hand side's scratch larger
 * than the array), HELM_EHIP.
 */
int helm_apply_static(helm_handle* h, const void* r_dev, void* z_dev, int R, int adjoint, void* stream);

/*
 * helm_apply_adjoint -- z = M^{-H} r: the conjugate transpose of helm_apply's operator (the
 * same forward-then-backward passes with the couplings of A^H and conjugate-transposed block
 * inverses).  Same arguments as helm_apply.
 */
int helm_apply_adjoint(helm_handle* h, const void* r_dev, void* z_dev, int R, void* stream);

/*
 * helm_matvec -- y = A u (adjoint = 0) or y = A^H u (adjoint = 1), eq. (3), in FP64.
 *   u_dev, y_dev : R*n^3 complex128 (may not alias).
 */
int helm_matvec(helm_handle* h, const void* u_dev, void* y_dev, int R, int adjoint, void* stream);

/*
 * helm_solve -- right-preconditioned flexible GMRES(restart) in FP64 (Sec. 5 solves eq. (3)
 * with GMRES preconditioned by the recursive sweep), all R right-hand sides batched.
 *   f_dev        : R*n^3 complex128 right-hand sides.
 *   u_dev        : R*n^3 complex128; in: initial guess (zeros for x0 = 0); out: solution.
 *   tol          : stop when ||f - A u||_2 <= tol ||f||_2 (checked with the true residual).
 *   restart      : Krylov basis length (>= 1); maxit: iteration cap per right-hand side.
 *   adjoint      : 0 solves A u = f with M^{-1}; 1 solves A^H u = f with M^{-H}.
 *   iters_host   : [R] iterations used per right-hand side (may be NULL).
 *   relres_host  : [R] final true relative residuals (may be NULL).
 * Returns HELM_ENOTCONV if some right-hand side did not reach tol within maxit, or if its
 * true residual became non-finite (then relres_host holds NaN or inf for it; e.g. a
 * preconditioner whose complex64 values overflow), and HELM_EINVAL for a right-hand side
 * that is not finite.
 * Memory: the Krylov bases (V complex128, Z complex64 in HELM_C64 mode, complex128
 * otherwise) grow with the iterations, up to min(restart, maxit) vectors per right-hand side;
 * their largest size (helm_workspace_bytes) is checked against the free device memory before
 * anything is allocated and gives HELM_ENOMEM if it does not fit.  The workspace comes from
 * the library's memory pool and returns to it (helm_pool_trim).
 * Errors also: HELM_EHIP when an exchange of the sweep timed out (see helm_apply).
 * Synchronises `stream`.
 */
int helm_solve(helm_handle* h, const void* f_dev, void* u_dev, int R, double tol, int restart,
               int maxit, int adjoint, int* iters_host, double* relres_host, void* stream);

/*
 * helm_grad_c -- adjoint-state gradient of J = 1/2 sum_s ||P u_s - d_s||^2 with respect to
 * the velocity: grad_p = (2 omega^2 / c_p^3) Re sum_s conj(lam_s,p) u_s,p, where u_s solves
 * A u = f_s and lam_s solves A^H lam = P^T (P u_s - d_s).  (c enters eq. (3) only through
 * omega^2/c^2 on the diagonal.)  Uses the handle's current medium.
 *   u_dev, lam_dev : R*n^3 complex128.   grad_dev : n^3 float64, overwritten.
 */
int helm_grad_c(helm_handle* h, const void* u_dev, const void* lam_dev, int R, double* grad_dev,
                void* stream);

/*
 * helm_misfit -- receiver misfit J = 1/2 sum_s ||P u_s - d_s||^2, P = restriction to all n^2
 * nodes of the x3-layer plane_k (1-based), and the adjoint source g_s = P^T (P u_s - d_s)
 * (the right-hand side of A^H lam_s = g_s in the adjoint-state gradient).
 *   u_dev   : R*n^3 complex128 solutions.   d_dev : R*n^2 complex128 data (x1 fastest).
 *   J_host  : receives J (may be NULL).     g_dev : R*n^3 complex128, overwritten (may be NULL).
 * Synchronises `stream` when J_host is given.
 */
int helm_misfit(helm_handle* h, const void* u_dev, const void* d_dev, int R, int plane_k,
                double* J_host, void* g_dev, void* stream);

/*
 * helm_set_medium -- replace omega^2/c^2 used by helm_matvec / helm_solve / helm_grad_c with
 * a new c_dev (n^3 float64 > 0); the factors (built for the old medium) are kept.
 */
int helm_set_medium(helm_handle* h, const double* c_dev, void* stream);

/*
 * helm_update_medium -- local update of the setup after a change of the velocity (Sec. 6,
 * future work: re-factor only the auxiliary problems a local change reaches).  c_dev (n^3
 * float64 > 0) replaces the medium; it must differ from the medium of the current factors
 * only inside box_host = {i0, i1, j0, j1, k0, k1} (host array, 1-based, inclusive,
 * 1 <= lo <= hi <= n).  A line problem's matrix reads omega^2/c^2 on its own window only, so
 * line (g, l) is re-factored iff its x3-window meets [k0, k1] and its x2-window meets
 * [j0, j1] (every line spans all of x1); all other factors are kept and are those of the new
 * medium already.  The result equals a fresh helm_setup on the new medium, bit for bit.
 * helm_stats.setup_ms then reports the update's device time.
 *   n_refactored : receives the number of lines re-factored (may be NULL).
 * Errors: HELM_EINVAL (bad box, c not finite and > 0), HELM_ESINGULAR, HELM_EHIP.
 * Synchronises `stream`.
 */
int helm_update_medium(helm_handle* h, const double* c_dev, const int* box_host, int* n_refactored,
                       void* stream);

/*
 * helm_info -- sizes of the setup: factor bytes, number of line problems, largest block.
 * Any output pointer may be NULL.
 */
int helm_info(const helm_handle* h, size_t* factor_bytes, int* n_lines, int* max_block);

/*
 * helm_workspace_bytes -- device memory beyond the handle's own (helm_info) that calls on it
 * may take, computed on the host: *apply_bytes for helm_apply / helm_apply_adjoint of R
 * right-hand sides (slab iterates of the sweep and the exchange slots of paired line solves),
 * *solve_bytes for helm_solve(R, restart, maxit) at most (those plus the Krylov bases of
 * min(restart, maxit) iterations and the Arnoldi scalars).  Either pointer may be NULL.
 * Errors: HELM_EINVAL (h NULL, R < 1, restart outside [1, 200], maxit < 0).
 */
int helm_workspace_bytes(const helm_handle* h, int R, int restart, int maxit, size_t* solve_bytes,
                         size_t* apply_bytes);

/*
 * Device memory pool.  Every device buffer of the library (handles' factors and
 * coefficients, sweep scratch, Krylov bases) is taken from a process-wide pool and returned
 * to it when freed, so repeated setups and solves of similar sizes reuse memory instead of
 * asking the HIP runtime each time.  A block returned on one stream and reused on another
 * waits for the first stream's work.  When the runtime cannot satisfy a request, the cached
 * blocks of that device are released and the request retried.
 * helm_pool_trim -- release every cached (unused) block to the HIP runtime.
 * helm_pool_stats -- bytes cached (free, held by the pool) and in use; NULL pointers skipped.
 */
void helm_pool_trim(void);
void helm_pool_stats(size_t* cached_bytes, size_t* live_bytes);

/*
 * helm_plan_bytes -- device bytes helm_setup would allocate for these parameters (factors +
 * coefficients), computed on the host without touching the GPU.  Returns HELM_EINVAL for
 * invalid parameters.
 */
int helm_plan_bytes(const helm_grid* grid, const helm_pml* pml, int slab_layers, int prec,
                    size_t* bytes, int* n_lines, int* max_block);

/*
 * helm_line_factors -- copy the block inverses of line problem (zg, yg) (0-based x3-group
 * and x2-group) into dst_dev: n blocks of B*B complex values, block i (0-based x1 index)
 * holding the factor of x1-block i, row-major within a block, unknowns of a block ordered
 * (x2 window row, x3 window layer) with x3 fastest.  The blocks are eliminated from both
 * ends towards the middle block m = n/2 (0-based, integer division): block i < m holds the
 * inverse Schur complement after eliminating blocks 0..i-1 (Sec. 3), block i > m the one
 * after blocks i+1..n-1, and block m the one after all others, which equals the (m, m)
 * block of the line matrix's inverse.  The solve is exact for any such order.
 * Element type is complex64 in HELM_C64 mode and complex128 in HELM_C128 mode.
 * *B_out receives B and *mid_out m (either may be NULL).  Pass dst_dev = NULL to query them
 * only.
 */
int helm_line_factors(const helm_handle* h, int zg, int yg, void* dst_dev, int* B_out,
                      int* mid_out, void* stream);

/*
 * helm_line_solve -- x = K^{-1} r (adjoint = 0) or K^{-H} r (adjoint = 1) for the line
 * problem (zg, yg) with its factors, on the line grid (n x Wy x Wz, x1 fastest, then the x2
 * window row, then the x3 window layer).  r_dev, x_dev: R consecutive line vectors of
 * n*B complex128 values.  Exposes the building block of helm_apply for testing.
 */
int helm_line_solve(helm_handle* h, int zg, int yg, const void* r_dev, void* x_dev, int R,
                    int adjoint, void* stream);

/*
 * helm_set_launch -- choose the sweep's launch shape: choice k >= 0 is variant k / 4 of the
 * library's list (two shapes each: lanes per block row, columns per lane and factor-ring
 * depth for the lines on no middle group and for the others) with workgroup placement k % 4
 * (0: the workgroups of a right-hand side on one XCD; 1: each of its workgroups on its own
 * XCD, so that one XCD serves one part of the factor stream to all right-hand sides; 2: the
 * two workgroups of each line solve on one XCD, the pairs of a right-hand side spread; 3 is
 * not a placement);
 * helm_sweep_shape names it.  -1 restores the automatic choice (the autotuner's for this
 * configuration, else the first listed variant that covers the blocks, placement 1).
 * Changes summation order only: results agree to rounding.
 * Errors: HELM_EINVAL (h NULL, k not a variant covering this handle's blocks).
 */
int helm_set_launch(helm_handle* h, int choice);

/*
 * helm_sweep_shape -- the launch choice a sweep of R right-hand sides on this handle uses now
 * (*variant, may be NULL) and its description "NCxCW/ringD + NCxCW/ringD, placement" (written
 * to name, at most name_len bytes with the terminating zero; name may be NULL).
 */
int helm_sweep_shape(const helm_handle* h, int R, int* variant, char* name, int name_len);

/*
 * helm_autotune -- time one sweep of R right-hand sides (after a warm-up sweep) with each
 * candidate launch shape for this handle (the variants whose two shapes are each among the
 * two smallest covering its blocks, with every ring depth listed for them, in both
 * placements) and keep the
 * fastest, for this handle (helm_set_launch) and for the process (handles of the same
 * configuration and batch size, rounded up to a multiple of 8, take it on their first
 * sweep).  If cache_path is not NULL the choice is looked up in / appended to that file (one
 * JSON object per line, keyed by n, block sizes, window, fronts, precision and batch size),
 * so the timing runs once per configuration.  *variant_out (may be NULL) receives the choice
 * and *ms_per_sweep (may be NULL) its time per sweep (0 when taken from the file).  Results
 * of later sweeps change only by rounding.  Synchronises `stream`.
 */
int helm_autotune(helm_handle* h, int R, const char* cache_path, int* variant_out,
                  double* ms_per_sweep, void* stream);

/*
 * helm_set_exchange_test -- failure-injection hook for tests of the sweep's error path:
 * drop_publish = 1 makes the first-half workgroup of every line solve skip publishing its
 * partial middle-block values, so its partner gives up after spin_limit polls (0: the
 * default bound, 2^28 polls, tens of seconds) and the next helm_apply / helm_solve returns
 * HELM_EHIP;
 * drop_publish = 0 restores normal operation.  Every kernel still ends normally.
 * Errors: HELM_EINVAL (h NULL, drop_publish not 0 or 1).
 */
int helm_set_exchange_test(helm_handle* h, int drop_publish, unsigned spin_limit);

/*
 * Device-time statistics of one handle, from HIP events recorded on the launch stream around
 * every sweep (helm_apply / helm_apply_adjoint / inside helm_solve) and every matvec launch.
 */
typedef struct {
  double setup_ms;             /* device time of the last setup (coefficients + factors)      */
  long long apply_launches;    /* sweep launches since the last reset                          */
  long long apply_rhs;         /* right-hand sides those launches processed                    */
  double apply_ms;             /* summed device time of those launches                         */
  double apply_bytes_per_rhs;  /* algorithmic bytes of one sweep of one right-hand side:      */
                               /* every block visit reads B*B factor entries, plus the input  */
                               /* vector read and the output vector written once              */
  long long matvec_launches;   /* 7-point operator launches since the last reset             */
  long long matvec_rhs;
  double matvec_ms;
  double matvec_bytes_per_rhs; /* 40 bytes per grid point (u, kappa read; y written)          */
  /* the sweep kernel: one cooperative launch per sweep (per chunk of right-hand sides when  */
  /* they cannot all be resident at once)                                                     */
  long long kernel_launches;
  long long kernel_rhs;
  double kernel_ms;
  double kernel_bytes;         /* algorithmic bytes of those launches: each launch reads its  */
                               /* sweep's factor blocks once per visit (its right-hand sides  */
                               /* share them), and every right-hand side's input is read and */
                               /* its output written once                                     */
  double kernel_flops;         /* useful real flops: 8 per factor entry visited per           */
                               /* right-hand side (one complex multiply-add)                  */
  double nd_setup_ms;          /* device time of the last nested-dissection factorisation    */
                               /* (helm_set_line_solver, helm_update_medium)                  */
} helm_stats;

/*
 * helm_set_line_solver -- how the forward complex64 sweeps solve their line problems.
 *   HELM_LINE_LDU (default): the block LDU of Algorithm 3 with the x1-blocks eliminated from
 *     both ends towards the middle block, two chains of n/2 dependent block steps.
 *   HELM_LINE_ND: 1D nested dissection in x1 (Sec. 6), done as block cyclic reduction: with
 *     n = 2^k - 1 the line's blocks fall into k levels (block i at the number of trailing
 *     zero bits of i + 1); each level is eliminated at once, the middle block last.  A line
 *     solve then takes 2k - 1 dependent phases of independent block products instead of a
 *     chain; the result is the same solve up to rounding.
 * The first switch to HELM_LINE_ND factors every line in that order (complex64, about 2.9 x
 * the memory of the block LDU factors, kept with them; 5 x that memory of work arrays during
 * the call).  helm_update_medium then refactors both; adjoint sweeps and helm_line_factors
 * keep using the block LDU.  Requires HELM_C64, n = 2^k - 1 and blocks of at most 96
 * unknowns.  Errors: HELM_EINVAL (unsupported plan or solver), HELM_ENOMEM, HELM_ESINGULAR,
 * HELM_EHIP.  Synchronises `stream`.
 */
#define HELM_LINE_LDU 0
#define HELM_LINE_ND 1
int helm_set_line_solver(helm_handle* h, int solver, void* stream);

/* helm_get_stats -- fill *out (waits for the recorded events); helm_reset_stats -- zero them. */
int helm_get_stats(helm_handle* h, helm_stats* out);
int helm_reset_stats(helm_handle* h);

/* helm_destroy -- free the handle and everything it owns (NULL is ignored). */
void helm_destroy(helm_handle* h);

/* helm_error_string -- static name of a return code. */
const char* helm_error_string(int code);

/* helm_last_error -- last detailed error message of the calling thread ("" if none). */
const char* helm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HELM_H */

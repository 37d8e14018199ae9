/*
 * sg.h -- C ABI of the MI355X stochastic-Galerkin KKT solver.
 *
 * The library solves the discrete first-order optimality (KKT) systems of
 * optimal control problems constrained by a diffusion (steady) or heat
 * (time-dependent) equation with a random coefficient, discretised by Q1 finite
 * elements in space and a stochastic Galerkin (generalised polynomial chaos)
 * expansion in the random variables, following
 *   Z. Li, A. Onwunta, B. Sousedik, "Stochastic Galerkin method and
 *   hierarchical preconditioning for PDE-constrained optimization",
 *   arXiv 2512.23804:
 *   - steady problem: Section 2.1, eq. (problem-stoch), eq. (pde-stoch);
 *     KKT system eq. (stoch-system);
 *   - time-dependent problem: Section 3, eq. (obj:stoch-time-dependent),
 *     eq. (constraint:stochastic-time-dependent); backward Euler all-at-once
 *     KKT system eq. (KKT:stoch-time-dependent);
 *   - preconditioner: block-diagonal Schur preconditioner eq. (stoch-prec) /
 *     eq. (precon for time) with Chebyshev (or exact) mass solves and the
 *     hierarchical Gauss-Seidel sweep of Algorithm 1 inside the Schur block
 *     (Algorithm 5 with N steps, N = 1 by default), or the coupled sweep of
 *     Algorithms 2-3 (hGSoc); Krylov solver: flexible GMRES (Section 5).
 *
 * Problem data.  Domain [0,1]^2 split into n x n square elements (n a power of
 * two, 4 <= n <= 4096), homogeneous Dirichlet data (g = 0).  Two coefficient
 * models (sg_problem.field): the affine field, random input xi ~ U(-1,1)^M
 * with orthonormal Legendre chaos of total degree P and a(x, xi) = kappa_0(x)
 * + sum_k kappa_k(x) psi_{e_k}(xi), each kappa_k constant per element (by
 * default a = 1 + sigma sum_{k=1}^{M} k^-2 cos(k pi x1) cos(k pi x2) xi_k);
 * or the log-normal field of Section 5, Gaussian xi with orthonormal Hermite
 * chaos of total degree P for the solution and 2P for the coefficient.
 *
 * Vector layout ("canonical layout").  One field block (state y, control u or
 * adjoint lambda) is an array [t][j][node] of n_t * n_xi * (n+1)^2 values:
 * t = time step (n_t = 1 for steady problems), j = chaos index in graded order
 * (degree ascending; inside a degree descending lexicographic on the
 * multi-index), node = iy*(n+1)+ix on the full grid.  Boundary nodes are zero
 * on output and ignored on input.  A KKT vector is [y | u | lambda], three
 * blocks back to back.  Several vectors are stored back to back.  All device
 * pointers are HIP device addresses on the current device; element types are
 * double (SG_FP64) or float (SG_FP32).
 *
 * Status codes.  Every entry point returns 0 (SG_OK), a positive
 * informational code or a negative error code; sg_last_error() gives a
 * thread-local message for the last failure on the calling thread.  No C++
 * exception crosses this boundary.  On error no output is guaranteed.
 *
 * Ownership.  The caller owns every pointer it passes; sg_setup* and sg_submit
 * copy what they need.  A handle owns its device workspace, released by
 * sg_destroy.  One handle must not be used by two threads at once; the server
 * is internally synchronised.
 */
#ifndef SG_H
#define SG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define SG_OK              0
#define SG_PENDING         1   /* sg_poll: request not finished yet */
#define SG_NOT_CONVERGED   2   /* solve stopped at max_iter above rtol */
#define SG_ERR_INVALID    -1   /* bad argument or unsupported size */
#define SG_ERR_NONCOERCIVE -2  /* coefficient can vanish for some xi */
#define SG_ERR_NONFINITE  -3   /* NaN/Inf in the problem data */
#define SG_ERR_NOMEM      -4   /* device memory or admission budget too small */
#define SG_ERR_HIP        -5   /* a HIP runtime call failed */
#define SG_ERR_CANCELLED  -6   /* request cancelled */
#define SG_ERR_UNKNOWN    -7   /* unknown ticket */

/* ---- element types and precision modes ------------------------------- */
#define SG_FP64 0
#define SG_FP32 1
#define SG_PREC_FP64         0  /* operator, preconditioner and Krylov in FP64 */
#define SG_PREC_FP32_REFINE  1  /* FP32 storage for the operator and preconditioner inside
                                   FGMRES (their arithmetic as below), FP64 Arnoldi sums,
                                   FP64 outer residual and refinement */
#define SG_PREC_FP32_PRECOND 2  /* FP32 preconditioner (basis Z in FP32) inside FP64
                                   FGMRES: FP64 operator and Arnoldi; every restart
                                   recomputes the FP64 residual */

/* Problem data (Section 2.1 steady, Section 3 time-dependent), g = 0.
 *   n       elements per side (power of two, 4..4096)
 *   M       number of random variables (1..16)
 *   P       total polynomial degree (1..8)
 *   n_t     <= 1: steady problem; >= 2: number of backward-Euler steps on
 *           (0, T], tau = T/n_t, unknowns at t_k = k tau, k = 1..n_t
 *   T       final time (time-dependent only)
 *   beta    control cost weight (> 0)
 *   gamma   variance weight (>= 0); the objective's variance term
 *   sigma   amplitude of the default cosine field (ignored if kappa != NULL)
 *   kappa   optional host array [(M+1)][n][n] of per-element coefficient
 *           modes, index [k][ey][ex]; kappa_0 must be one positive constant
 *           (the multigrid inner solver assumes a constant mean coefficient)
 *   y_target host array [n_t][(n+1)^2] of nodal target values (n_t = 1 when
 *           steady); the target enters the right-hand side as the full-grid
 *           mass matrix times the target, restricted to interior rows
 *   y0      optional host array [(n+1)^2] initial state (time-dependent);
 *           NULL means zero
 *   field   SG_FIELD_AFFINE (0): the affine coefficient 1 + sigma sum_k
 *           k^-2 cos(k pi x1) cos(k pi x2) xi_k (or kappa) with orthonormal
 *           Legendre chaos in xi ~ U(-1, 1)^M, so G_k couples alpha with
 *           alpha +- e_k; SG_FIELD_LOGNORMAL (1): the log-normal coefficient
 *           of Section 5 with orthonormal Hermite chaos in Gaussian xi: the
 *           exponential of the M-term Karhunen-Loeve expansion of a Gaussian
 *           field with covariance sigma^2 exp(-|x1-y1|/corr_len -
 *           |x2-y2|/corr_len) on [-1, 1]^2 (mapped onto the unit square of
 *           the grid), mean coefficient 1, expanded to total degree 2P
 *           (n_A = C(M+2P, 2P) terms H_l (x) A_l); kappa must be NULL
 *   corr_len correlation length of the log-normal field (Section 5: 1) */
typedef struct sg_problem {
    int32_t n, M, P, n_t;
    double T, beta, gamma, sigma;
    const double* kappa;
    const double* y_target;
    const double* y0;
    int32_t field;
    double corr_len;
} sg_problem;

#define SG_FIELD_AFFINE    0
#define SG_FIELD_LOGNORMAL 1

/* Solver options.  sg_default_options() fills the defaults in brackets.
 *   rtol         relative residual ||b - K x|| / ||b|| to reach [1e-8]
 *   restart      FGMRES restart length [30]
 *   max_iter     total FGMRES iterations over all cycles [600]
 *   cheb_steps   Chebyshev semi-iteration steps for mass solves, or 0 for
 *                exact mass solves by the 2D sine transform (the direct
 *                factorisation variant of Section 5) [5]
 *   truncation_r hGS truncation: coefficient terms k = 1..r-1 are kept in the
 *                off-level products (r = 1 mean-based, r = M+1 all modes of
 *                the affine field, r = n_A all terms of the log-normal field;
 *                Section 5's n_tau) [0 = all]
 *   gmg_pre/post Chebyshev smoothing degree before/after coarse correction [2,2]
 *   precision    SG_PREC_FP64, SG_PREC_FP32_REFINE or SG_PREC_FP32_PRECOND [SG_PREC_FP64]
 *   inner_rtol   FP32 inner solve reduction per refinement step [1e-5]
 *   use_graphs   replay each FGMRES iteration from a cached hipGraph when the
 *                handle has a stream other than the default stream [1]
 *   verbose      print per-cycle residuals to stderr [0]
 *   profile      time one kernel's launches with HIP events during sg_solve
 *                (SG_PROF_* below) and report them in sg_solve_info [0]
 *   arnoldi      FGMRES orthogonalisation: SG_ARNOLDI_DCGS2 (classical
 *                Gram-Schmidt with the reorthogonalisation of each basis
 *                vector delayed to the next iteration: two passes over the
 *                basis per iteration) or SG_ARNOLDI_CGS2 (classical
 *                Gram-Schmidt applied twice: three passes) [SG_ARNOLDI_DCGS2]
 *   sweep_rows   node rows per strip of the SG/KKT/hGS sweep kernels (the
 *                SG apply on FP64 storage uses a paired-node kernel with a
 *                fixed shape and ignores it): 2, 4
 *                or 8, or 0 to let sg_setup time the three on the handle's
 *                shape and keep the fastest (cached per device model and
 *                shape, in memory and in the file SG_TUNE_CACHE names, see
 *                sg_tune_save; every choice gives bit-identical results) [0]
 *   basis_fp32   SG_PREC_FP32_REFINE with DCGS2 only: 1 stores the inner
 *                cycles' Arnoldi basis and operator output in FP32 (every dot
 *                product, projection and Hessenberg entry is still formed in
 *                FP64), 0 stores them in FP64 [1]
 *   mean_solver  solves with the mean block A-tilde_1 (eq. mathcalZ) /
 *                A-hat_1 (eq. A_hat) inside hGS: SG_MEAN_MULTIGRID (one
 *                geometric-multigrid V-cycle) or SG_MEAN_EXACT (exact, by the
 *                2D sine transform on FP64 MFMA; the mean coefficient is
 *                constant, so the block is a K + b M on the uniform grid)
 *                [SG_MEAN_MULTIGRID]
 *   precond      SG_PRECOND_BLOCK_DIAGONAL: the block-diagonal preconditioner
 *                of eq. (stoch-prec) / eq. (precon for time); SG_PRECOND_HGSOC:
 *                the coupled level sweep of Algorithms 2-3 (cheb_steps 1..9;
 *                time-dependent problems take it on every time step at once,
 *                the couplings between steps left out: Algorithm 4, with the
 *                step's blocks tau D_tt h^gamma_j M, beta tau D_tt M and the
 *                mean block A-hat_1), each level solved with the block-diagonal
 *                preconditioner restricted to its chaos columns (the adjoint
 *                by A-tilde_1^{-1} h^gamma_j M A-tilde_1^{-1}: the printed
 *                third block A-tilde_1 does not approximate the adjoint row)
 *                [SG_PRECOND_BLOCK_DIAGONAL]
 *   richardson_steps  N of the preconditioned Richardson iteration of
 *                Algorithm 5 for each Z^{-1} of the Schur block, each step
 *                preconditioned by one hGS sweep (Algorithm 1); N = 1 is one
 *                hGS application, as in the paper's runs [1]
 *
 * Arithmetic precision.  The stiffness sums of the SG operator, KKT apply and
 * hGS right-hand sides are formed in FP64 for FP32 storage too (an FP32
 * vector is widened on load, results rounded on store): summed in FP32, the
 * Q1 stencil's cancellation on fine grids (relative error growing like
 * eps / h^2) would cap what an FP32 refinement step can gain.  The mass,
 * Chebyshev and multigrid kernels compute in the storage precision. */
typedef struct sg_options {
    double rtol;
    int32_t restart, max_iter, cheb_steps, truncation_r;
    int32_t gmg_pre, gmg_post, precision;
    double inner_rtol;
    int32_t use_graphs, verbose, profile;
    int32_t arnoldi;
    int32_t sweep_rows;
    int32_t basis_fp32;
    int32_t mean_solver;
    int32_t richardson_steps;
    int32_t precond;
} sg_options;

#define SG_PRECOND_BLOCK_DIAGONAL 0
#define SG_PRECOND_HGSOC          1

#define SG_MEAN_MULTIGRID 0
#define SG_MEAN_EXACT     1

#define SG_ARNOLDI_DCGS2 0
#define SG_ARNOLDI_CGS2  1

/* Kernels that sg_options.profile can time (HIP events around every launch). */
#define SG_PROF_NONE        0
#define SG_PROF_KKT_APPLY   1   /* fused KKT apply (two SG operator applies + mass terms) */
#define SG_PROF_MG_SMOOTH   2   /* multigrid down kernel (pre-smoothing, stored; residual, restriction), finest level */
#define SG_PROF_MULTIDOT    3   /* Arnoldi dot-product pass (read-only pass over the basis) */
#define SG_PROF_HGS_RHS     4   /* hierarchical Gauss-Seidel off-level right-hand side */
#define SG_PROF_ARNOLDI_UPD 5   /* Arnoldi update pass (DCGS2: finalise V_j, next candidate) */
#define SG_PROF_MG_TAIL     6   /* fused coarse end of the V-cycle (levels <= 64, direct solve) */
#define SG_PROF_MASS_CHEB   7   /* Chebyshev semi-iteration on the mass blocks */
#define SG_PROF_MG_UP       8   /* multigrid up kernel (stored pre-smoothed iterate, correction, post-smoothing), finest level */

/* Per-solve report. */
typedef struct sg_solve_info {
    int32_t iters;              /* FGMRES iterations (all cycles, all refinement steps) */
    int32_t outer_refinements;  /* FP64 refinement steps (0 in SG_PREC_FP64) */
    int32_t converged;          /* 1 if rel_res_true <= rtol */
    int32_t status;             /* SG_OK / SG_NOT_CONVERGED / error of this member */
    double rel_res_true;        /* ||b - K x|| / ||b|| in FP64 at exit */
    double t_setup_ms;          /* handle setup time (host + device) */
    double t_solve_ms;          /* wall time of the solve */
    double latency_ms;          /* serving: submit -> completion */
    double bytes_moved;         /* model of this member's algorithmic HBM bytes: every
                                   launch counted as the streaming passes its kernels
                                   make (each input and output node once) on their
                                   storage types, per FGMRES iteration the KKT apply,
                                   the preconditioner and the Arnoldi passes, per
                                   cycle the true residual, the start vector and the
                                   update of x */
    double prof_ms;             /* profiled kernel: summed launch durations (HIP events) */
    double prof_bytes;          /* profiled kernel: summed algorithmic bytes of those launches */
    int32_t prof_launches;      /* profiled kernel: number of launches */
    int32_t joined_batch;       /* serving: 1 if the request took the slot of a finished member of a
                                   running batch at a restart boundary (0 otherwise, and in sg_solve) */
} sg_solve_info;

/* Sizes of a handle's problems. */
typedef struct sg_sizes {
    int32_t n, M, P, n_t, n_xi, members;
    int64_t nodes;              /* (n+1)^2 */
    int64_t block_elems;        /* n_t * n_xi * nodes (one field) */
    int64_t kkt_elems;          /* 3 * block_elems (one KKT vector) */
    int32_t level_offsets[17];  /* degree d columns: [off[d], off[d+1]), d = 0..P */
    int32_t sweep_rows[2][3];   /* strip rows in use: [FP64, FP32][SG apply, hGS rhs, KKT apply]
                                   ([FP64][SG apply] is unused: paired-node kernel) */
} sg_sizes;

typedef struct sg_handle sg_handle;
typedef struct sg_server sg_server;

/* Fill `opt` with the defaults listed above. */
void sg_default_options(sg_options* opt);

/* Host-only validation of a problem and options (no device work):
 * SG_ERR_INVALID for out-of-range sizes or parameters, SG_ERR_NONFINITE for
 * NaN/Inf data, SG_ERR_NONCOERCIVE when min_e [kappa_0 - sqrt(3) sum_k
 * |kappa_k(e)|] <= 0, i.e. the coefficient can reach zero for some xi in
 * [-1,1]^M (the bounded-coefficient assumption of Section 2.1). */
int sg_validate(const sg_problem* prob, const sg_options* opt);

/* Build a handle for `count` problems of the same shape (n, M, P, n_t equal;
 * beta, gamma, sigma, kappa, targets may differ) that are solved together as
 * one batch ("members").  Builds the multi-index set, triple-product tables
 * (Section 2.1), per-element coefficient modes, multigrid hierarchy and
 * right-hand sides, uploads them to the current device, and binds `stream`
 * (a hipStream_t, NULL = default stream).  On success *out owns the device
 * memory.  Errors: as sg_validate, SG_ERR_NOMEM, SG_ERR_HIP. */
int sg_setup(const sg_problem* probs, int32_t count, const sg_options* opt,
             void* stream, sg_handle** out);

/* Report the sizes of a handle. */
int sg_query(const sg_handle* h, sg_sizes* out);

/* Copy the multi-index set, int32 [n_xi][M] host array (graded order). */
int sg_get_multiindex(const sg_handle* h, int32_t* out);

/* Copy the triple-product neighbour table used by the kernels (Section 2.1,
 * H_l with l = e_k): for chaos index j and mode k = 1..M, slot 0 is the
 * neighbour j - e_k and slot 1 is j + e_k; idx = -1 where the neighbour is not
 * in the set, else its chaos index; val = E[psi_{e_k} psi_j psi_idx].
 * Host arrays idx int32 [n_xi][M][2], val double [n_xi][M][2]. */
int sg_get_gtable(const sg_handle* h, int32_t* idx, double* val);

/* Write the KKT right-hand sides of all members (one KKT vector per member,
 * canonical layout, FP64) to device memory b_dev. */
int sg_get_rhs(sg_handle* h, double* b_dev);

/* SG operator apply, eq. (Zv) with the stiffness modes A_l (Section 2.2):
 * Y = sum_{k=0}^{M} K_k X G_k for every time step, i.e. one field block in,
 * one field block out, per vector.  x_dev, y_dev hold nvec blocks back to
 * back; with members > 1, nvec must equal members and block v uses member v's
 * coefficients; with one member any nvec >= 1 shares it.  dtype SG_FP64 or
 * SG_FP32.  Runs on `stream` (NULL = the handle's stream), asynchronous. */
int sg_apply_operator(sg_handle* h, const void* x_dev, void* y_dev, int32_t nvec,
                      int32_t dtype, void* stream);

/* KKT matrix apply, eq. (stoch-system) (steady) or eq. (KKT:stoch-time-
 * dependent) (time): y = K x for nvec KKT vectors (member rule as above). */
int sg_apply_kkt(sg_handle* h, const void* x_dev, void* y_dev, int32_t nvec,
                 int32_t dtype, void* stream);

/* Preconditioner apply z = P^{-1} r, eq. (stoch-prec) / eq. (precon for
 * time): Chebyshev semi-iteration on the state and control blocks and
 * S^{-1} = Z^{-1} M_gamma Z^{-1} (time: tau Z~^{-1} (D (x) M_gamma) Z~^{-1})
 * on the adjoint block, each Z^{-1} one hGS sweep (Algorithm 1) whose
 * A-tilde_1 solves are one multigrid V-cycle.  r_dev is not modified. */
int sg_precond_apply(sg_handle* h, const void* r_dev, void* z_dev, int32_t nvec,
                     int32_t dtype, void* stream);

/* sg_precond_apply for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same operation and kernels, bit-identical results, but
 * every scratch buffer (iterates of the hGS sweeps, the Schur mass product,
 * multigrid levels) is carved from a fixed 64 MiB device array that the
 * library holds on each device until the process ends; no hipMalloc,
 * hipFree or memset is issued.  The handle must have been set up beforehand
 * (sg_setup allocates; this call does not) and its device must be current.
 * Arguments as sg_precond_apply.  Returns SG_ERR_NOMEM, before launching
 * anything, when the scratch nvec vectors need exceeds the fixed size
 * (about 7 field blocks of the handle's shape per vector).  All calls on one
 * device share the array and it keeps the last call's contents: calls that
 * overlap on one device (other streams, other threads) race and must be
 * serialised by the caller. */
int sg_precond_apply_noalloc(sg_handle* h, const void* r_dev, void* z_dev, int32_t nvec,
                             int32_t dtype, void* stream);

/* Solve K x = b for every member with preconditioned FGMRES(restart) from
 * x = 0.  b_dev: FP64 KKT vectors (NULL = the problems' own right-hand
 * sides); x_dev: FP64 output KKT vectors; info: array of `members` reports
 * (may be NULL).  Synchronous on the handle's stream.  Returns SG_OK when all
 * members converged, SG_NOT_CONVERGED otherwise. */
int sg_solve(sg_handle* h, const double* b_dev, double* x_dev, sg_solve_info* info);

/* Release a handle (NULL is ignored). */
void sg_destroy(sg_handle* h);

/* ---- serving: continuous batching of independent steady requests ------ */

/* Create a server that owns a scheduler thread and its own HIP streams on the
 * current device.  hbm_budget_bytes bounds the summed footprint of admitted
 * requests (0 = 80% of free device memory); max_slots bounds requests in
 * flight.  A request whose footprint exceeds the budget is rejected.
 * Requests of one shape (n, M, P and options) admitted together run as the
 * members of one batch on one worker stream; batches on different workers
 * overlap on the device.  At each restart boundary of a running batch, the
 * slot of a member whose solve has ended is reported and handed to the oldest
 * queued request of the batch's shape, which starts there from x = 0; its
 * arithmetic is that of an alone solve. */
int sg_server_create(size_t hbm_budget_bytes, int32_t max_slots, sg_server** out);

/* Queue one request (problem + options are copied).  x_out: caller-owned host
 * buffer of one FP64 KKT vector, written when the request completes and valid
 * from then until the caller frees it.  *ticket identifies the request. */
int sg_submit(sg_server* s, const sg_problem* prob, const sg_options* opt,
              double* x_out, uint64_t* ticket);

/* SG_PENDING while queued or running; otherwise the request's final status,
 * with *info filled (latency_ms = submit to completion).  A finished ticket
 * stays valid until sg_server_destroy. */
int sg_poll(sg_server* s, uint64_t ticket, sg_solve_info* info);

/* Cancel a queued request (SG_OK) or report that it already started or ended
 * (SG_ERR_INVALID).  A cancelled ticket polls as SG_ERR_CANCELLED. */
int sg_cancel(sg_server* s, uint64_t ticket);

/* Serving statistics since creation: completed count, p50/p99 latency (ms),
 * completions per second of wall time. */
int sg_server_stats(sg_server* s, int64_t* completed, double* p50_ms, double* p99_ms,
                    double* solves_per_s);

/* Block until every submitted request finished, then stop the scheduler and
 * free all device memory (NULL is ignored). */
void sg_server_destroy(sg_server* s);

/* ---- strip-height autotuner cache -------------------------------------- */

/* The choices of sg_options.sweep_rows = 0 are kept per process, keyed by
 * device model (architecture name and compute-unit count), n, M, P, n_t,
 * steady or time-dependent, one member or a batch, and element type.  When
 * the environment variable SG_TUNE_CACHE names a file, the first tuning (or
 * any call below) of the process merges that file if it exists, and every new
 * choice rewrites it (temporary file, then rename).  The file is text: the
 * line "sgkkt-tune 1", then one entry per line, "<arch> <CUs> <n> <M> <P>
 * <n_t> <time 0/1> <batch 1/2> <fp32 0/1> <apply> <hgs> <kkt>" with strip
 * heights in {2, 4, 8}.  These calls touch no device. */

/* Write every cached choice to `path`.  SG_ERR_INVALID: NULL or empty path,
 * or the file cannot be written. */
int sg_tune_save(const char* path);

/* Merge the choices in `path` into the cache (an entry replaces the cached
 * one with the same key); a later sg_setup with sweep_rows = 0 and a matching
 * key uses it without timing.  SG_ERR_INVALID: NULL or empty path, unreadable
 * file, wrong first line or a malformed entry (then nothing is merged). */
int sg_tune_load(const char* path);

/* Number of cached choices (>= 0). */
int sg_tune_count(void);

/* Empty the cache (the SG_TUNE_CACHE file is not read again by this process). */
int sg_tune_clear(void);

/* Thread-local message of the last failure on this thread ("" if none). */
const char* sg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SG_H */

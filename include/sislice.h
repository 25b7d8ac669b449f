/*
 * sislice.h -- C ABI of an MI355X (gfx950) shift-invert spectrum-slicing
 * eigensolver for symmetric-definite pencils (A, B), after
 * "SISLICE: shift-invert spectrum slicing for the SCF eigenvalue problem"
 * (arXiv:1908.06043).
 *
 * Problem (Section 1, eq. seq_gep): A X = B X Lambda with A symmetric and B
 * symmetric positive definite; the n_e wanted eigenpairs are the lowest ones.
 *
 * Conventions shared by every entry point
 *   - Matrices are FP64, column-major, leading dimension >= n.  Symmetric inputs
 *     (A, B) are read from their LOWER triangle only and are never written.
 *   - "device" pointers are HIP device memory on the handle's device; "host"
 *     pointers are ordinary CPU memory.  The caller owns every buffer it passes;
 *     the library never frees caller memory.  Workspace belongs to the handle.
 *   - Work is ordered on the handle's stream.  Entry points that return host
 *     results (inertia, reports, planned shifts) synchronise that stream;
 *     sislice_ldlt_solve is asynchronous.
 *   - All arithmetic is FP64; the inertia is an exact integer count.
 *   - Errors: negative status = usage/runtime error, positive = numerical
 *     outcome.  No exception crosses the ABI.  Calls on one handle must not
 *     overlap (a handle is not thread-safe); separate handles are independent.
 */
#ifndef SISLICE_H
#define SISLICE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SISLICE_OK = 0,
  SISLICE_ERR_ARG = -1,        /* invalid argument (size, pointer, option)              */
  SISLICE_ERR_HIP = -2,        /* a HIP runtime call failed                             */
  SISLICE_ERR_ALLOC = -3,      /* device or host allocation failed                      */
  SISLICE_ERR_NO_DEVICE = -4,  /* no usable gfx950 device                               */
  SISLICE_SINGULAR_SHIFT = 1,  /* exact zero pivot: a shift is an eigenvalue (Sec. 2.1
                                  assumes this never happens)                          */
  SISLICE_NOT_CONVERGED = 2,   /* residual tolerance not met within the iteration cap   */
  SISLICE_MISSING_EIGS = 3     /* a slice holds more eigenvalues than validated
                                  candidates (Sec. 2.2, second case), or fewer than n_e
                                  eigenvalues lie below the top boundary               */
} sislice_status;

typedef struct sislice_handle sislice_handle;

/* Options of the full solve and of the planner.  Fill with sislice_default_opts. */
typedef struct {
  int32_t block;         /* Lanczos block size b (8)                                   */
  int32_t max_basis;     /* active Lanczos basis cap, multiple of block, <= 112 (112)   */
  int32_t max_cycles;    /* restart cycles per probe before NOT_CONVERGED (40)           */
  int32_t kpm_moments;   /* Chebyshev moments of the DOS estimate (64)                   */
  int32_t kpm_vectors;   /* Rademacher probe vectors (20)                                */
  int32_t bounds_steps;  /* Lanczos steps of the spectral-bounds estimate (30)           */
  int32_t nb;            /* factorization panel width (0 = library default)             */
  int32_t profile;       /* time kernel classes with HIP events into the report (0):   */
                         /* 1 every class; 0x100 | m only the classes whose bit is set */
                         /* in m (bit c: class c of t_kern_ms), e.g. to time one class */
                         /* at a few events per step                                   */
  double tol;            /* residual ||Ax - lambda Bx|| / (||A||_2 ||x||) target (1e-10) */
  double top_margin;     /* top boundary at the CDOS root of n_e + top_margin*n_e/n_s (2) */
  uint64_t seed;         /* SplitMix64 seed of every random draw (0)                     */
  int32_t driver;        /* per-probe iteration: 0 block shift-invert Lanczos in the B
                            inner product (block size `block`, thick restart); 1 the
                            paper's shift-invert subspace iteration (Algorithm 2) with
                            k = max(2 need, 16) columns (a multiple of 8, <= 112) for
                            the probe with the largest need, rounds of M iterations,
                            each round restarted from its Ritz vectors (0)            */
  int32_t subspace_iters;/* M of Algorithm 2: applications per round (4)               */
  int32_t max_recovery;  /* rounds of probe insertion into slices that miss
                            eigenvalues (Sec. 3.3) before SISLICE_MISSING_EIGS (2)    */
  int32_t graphs;        /* 1: the factorization's panel/update step sequence is
                            captured once per order, shift count and panel
                            parameters into a HIP graph and replayed (on streams
                            other than the null stream, which cannot be
                            captured); 0: launched directly (1)                      */
} sislice_opts;

/* Per-solve report, host memory owned by the caller.  Array members are optional
 * caller arrays (may be NULL) of the stated length. */
typedef struct {
  int64_t n_shifts;        /* shifts used (n_s)                                        */
  int64_t n_validated;     /* validated eigenpairs below the top boundary              */
  int64_t n_converged;     /* of the returned n_e, how many meet tol                   */
  int64_t nu_top;          /* inertia count at the top boundary                        */
  double omega_top;        /* top boundary used                                        */
  double anorm;            /* ||A||_2 estimate used to normalise residuals             */
  int32_t cycles_max;      /* largest number of Lanczos restart cycles of any probe    */
  int32_t block_steps;     /* block Lanczos steps summed over probes                   */
  double t_factor_ms;      /* shift-form + LDL^T + inertia of every shift and boundary */
  double t_lanczos_ms;     /* block Lanczos incl. restarts                             */
  double t_rr_ms;          /* explicit Rayleigh-Ritz and residuals                     */
  double t_host_ms;        /* host validation                                          */
  double t_total_ms;
  double flops_factor;     /* n^3/3 per factorization, summed                          */
  int64_t *nu;             /* [n_shifts] inertia nu(sigma_j) = #{lambda < sigma_j}      */
  int32_t *slice_case;     /* [n_shifts+1] 0 equal counts, 1 missing, 2 trimmed        */
  int32_t *slice_exact;    /* [n_shifts+1] exact counts from inertia                   */
  int32_t *slice_cand;     /* [n_shifts+1] validation candidates                       */
  /* With opts->profile: summed HIP-event durations and launch counts of the
   * kernel classes 0 Bunch-Kaufman panels, 1 MFMA trailing updates, 2 triangular
   * solves, 3 GEMMs, 4 projected eigensolves, 5 other; and the algorithmic flops
   * of the trailing updates (2 kb per lower-triangle element per panel). */
  double t_kern_ms[6];
  int64_t n_kern[6];
  double flops_update;
  /* Algorithmic bytes of the triangular sweeps: 8 n^2 per shift and
   * forward/backward pair (the packed L read once per direction). */
  double bytes_solve;
  /* Identifies the factorizations of this solve, which the handle keeps until
   * its next sislice_solve, sislice_sisubit or sislice_adjoint (pass to
   * sislice_adjoint); 0 when probes were inserted (the adjoint then refactors). */
  uint64_t factor_id;
  /* Missing eigenvalues (Sec. 3.3): probes inserted into slices that held more
   * eigenvalues than validated candidates, and the rounds of insertion. */
  int32_t probes_inserted;
  int32_t recovery_rounds;
  /* With opts->profile: algorithmic bytes of the Bunch-Kaufman panels, the panel
   * block (n - k0) x kb of every shift read and written once per panel step. */
  double bytes_panel;
} sislice_report;

/* Report of sislice_adjoint, host memory owned by the caller. */
typedef struct {
  int32_t iterations;        /* conjugate-gradient iterations (all columns together)  */
  int32_t reused_factors;    /* 1: the solve's factorizations were reused             */
  int32_t n_groups;          /* groups of at most 8 columns sharing one factorization */
  int32_t breakdowns;        /* columns stopped after repeated non-positive curvature */
  double max_rel_residual;   /* max_i ||r_i|| / ||b_i|| of the projected solves        */
  double t_factor_ms;        /* refactorization (0 when reused)                       */
  double t_solve_ms;         /* preconditioned conjugate gradients                    */
  double t_total_ms;
  double flops_outer;        /* algorithmic flops of the two rank-2k outputs: 4 n^2 n_e */
  double t_outer_ms;         /* device time of the fused rank-2k output kernel         */
} sislice_adjoint_report;

void sislice_default_opts(sislice_opts *opts);
const char *sislice_status_string(sislice_status s);

/* Create a handle on HIP device `device`, ordering work on `stream` (a
 * hipStream_t; NULL = the null stream).  Fails with SISLICE_ERR_NO_DEVICE when
 * the device is absent or is not gfx950. */
sislice_status sislice_create(sislice_handle **h, int device, void *stream);
sislice_status sislice_destroy(sislice_handle *h);
sislice_status sislice_set_stream(sislice_handle *h, void *stream);

/* Bound of the device-side waits.  The triangular solves of the shift-invert
 * step (Algorithm 2, third step) hand row blocks between workgroups, and a
 * workgroup polls for a block it needs; a poll that does not find it after
 * `polls` attempts (about 1 us each; default 2^21, about 2 s) gives up so that
 * the launch still completes, and the call that ran it (or, for the
 * asynchronous sislice_ldlt_solve, the next synchronising call on the handle)
 * returns SISLICE_ERR_HIP.  Correct hand-offs complete in microseconds; the
 * bound only turns a logic fault into an error instead of a hung device.
 * polls in [0, 2^32 - 1]; applies to the handle and its batch workers. */
sislice_status sislice_set_wait_limit(sislice_handle *h, int64_t polls);

/* Bunch-Kaufman LDL^T of C = A - sigma B (Sec. 2.1: the probe's major cost) and
 * the Sylvester inertia of D (Sec. 2.2).
 *   A, B   device, n x n, lower triangle read (lda, ldb >= n).
 *   LD     device, n x n, ldld >= n, written: D on the diagonal and, for a 2x2
 *          pivot block at (k, k+1), D[k+1,k] at LD[k+1,k]; the strictly lower
 *          remainder holds unit-lower L (L[k+1,k] = 0 inside a 2x2 block).
 *   ipiv   device int32[n], written: P C P^T = L D L^T where row i of P C P^T is
 *          row p(i) of C; ipiv[i] = p(i) for a 1x1 pivot row and -(p(i)+1) for
 *          both rows of a 2x2 pivot block.
 *   inertia host int64[3]: (negative, zero, positive) eigenvalue counts of D;
 *          inertia[0] = #{lambda(A,B) < sigma}.
 * Returns SISLICE_SINGULAR_SHIFT (with the factors written) when a pivot is an
 * exact zero.  Synchronises the stream. */
sislice_status sislice_ldlt_factor(sislice_handle *h, int64_t n, const double *A, int64_t lda,
                                   const double *B, int64_t ldb, double sigma, double *LD,
                                   int64_t ldld, int32_t *ipiv, int64_t inertia[3]);

/* The same for n_shifts shifts (host array `sigmas`), factored together (the
 * GPU's share of the probes of Sec. 4.1).  LD and ipiv are HOST arrays of
 * n_shifts DEVICE pointers; inertia is host int64[3*n_shifts]. */
sislice_status sislice_ldlt_factor_multi(sislice_handle *h, int64_t n, const double *A, int64_t lda,
                                         const double *B, int64_t ldb, int64_t n_shifts,
                                         const double *sigmas, double *const *LD, int64_t ldld,
                                         int32_t *const *ipiv, int64_t *inertia);

/* X <- C^{-1} X with the factors of sislice_ldlt_factor (Algorithm 2, third step:
 * L^{-T} D^{-1} L^{-1} applied through P).  X device n x nrhs (ldx >= n),
 * 1 <= nrhs <= 64.  Asynchronous. */
sislice_status sislice_ldlt_solve(sislice_handle *h, int64_t n, const double *LD, int64_t ldld,
                                  const int32_t *ipiv, int64_t nrhs, double *X, int64_t ldx);

/* sislice_ldlt_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same arguments, kernels and results, but no call allocates, frees or
 * synchronises.  Its workspace is one fixed device array of 13 MiB per GPU (held
 * from the first handle created on that GPU until the process ends), so
 * n <= 4096 (SISLICE_ERR_ARG beyond) and 1 <= nrhs <= 64.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams or
 * handles) race.  Asynchronous; an expired hand-off wait (see
 * sislice_set_wait_limit) is reported by the next synchronising call on the
 * handle. */
sislice_status sislice_ldlt_solve_noalloc(sislice_handle *h, int64_t n, const double *LD,
                                          int64_t ldld, const int32_t *ipiv, int64_t nrhs,
                                          double *X, int64_t ldx);

/* Shift placement from a stochastic Chebyshev DOS estimate (Sec. 3.1 with the
 * kernel polynomial method in place of the Lanczos DOS): spectral bounds by a
 * Lanczos run on L_B^{-1} A L_B^{-T}, opts->kpm_moments Jackson-damped moments
 * from opts->kpm_vectors Rademacher vectors, the closed-form CDOS, its roots at
 * equal counts over [a, omega_top] with omega_top the root at
 * n_e + top_margin*n_e/n_s, and one shift at each interval midpoint.
 *   sigmas     host double[n_s] out, ascending.
 *   omega_top  host double out.
 *   moments    host double[kpm_moments] out (may be NULL).
 *   bounds     host double[2] out (a, b) (may be NULL).
 * Synchronises. */
sislice_status sislice_plan_shifts_kpm(sislice_handle *h, int64_t n, const double *A, int64_t lda,
                                       const double *B, int64_t ldb, int64_t n_e, int64_t n_s,
                                       const sislice_opts *opts, double *sigmas, double *omega_top,
                                       double *moments, double *bounds);

/* The paper's own shift selection (Sec. 3.1): nv runs of k-step Lanczos (full
 * reorthogonalisation, Gaussian starts from the SplitMix64 stream of
 * opts->seed) on L_B^{-1} A L_B^{-T}, their Ritz values and the squared first
 * components of the Ritz vectors, then the planning of sislice_dos_plan with
 * mode 0 (equal-count roots of the Lanczos CDOS) or 1 (DOSCluster, refinement,
 * safeguards, DOS-expectation shifts) and opts->top_margin.
 *   k in [2, 112], nv in [1, 32].
 *   sigmas host double[n_s] out ascending, omega_top host double out, bounds
 *   host double[2] out (the extreme Ritz values; may be NULL).  Synchronises. */
sislice_status sislice_plan_shifts_lanczos(sislice_handle *h, int64_t n, const double *A,
                                           int64_t lda, const double *B, int64_t ldb, int64_t n_e,
                                           int64_t n_s, const sislice_opts *opts, int32_t mode,
                                           int32_t k, int32_t nv, double *sigmas, double *omega_top,
                                           double *bounds);

/* The plain per-pencil path (Algorithm 1, one pass on a fixed pencil): factor
 * every shift and the top boundary, read the inertias, run block shift-invert
 * Lanczos in the B inner product per shift (b = opts->block, thick restart with
 * locking), explicit Rayleigh-Ritz with A and B, residuals, slice validation
 * (Sec. 2.2), and return the lowest n_e validated eigenpairs.  A value is
 * reported from the probe whose shift is nearer; when that copy misses the
 * tolerance and the other probe of its slice holds a copy of the same value
 * that meets it, that copy is reported instead.
 *   sigmas     host double[n_s], ascending, or NULL: then the shifts and the top
 *              boundary are planned with sislice_plan_shifts_kpm.
 *   omega_top  host double in/out: the top boundary when sigmas != NULL (must
 *              exceed every shift); the boundary used on return.
 *   evals      device double[n_e] out, ascending.
 *   evecs      device n x n_e (ldx >= n) out, B-orthonormal columns.
 *   resid      device double[n_e] out, ||A x - lambda B x|| / (||A||_2 ||x||).
 *   report     host, may be NULL.
 * Synchronises. */
sislice_status sislice_solve(sislice_handle *h, int64_t n, const double *A, int64_t lda,
                             const double *B, int64_t ldb, int64_t n_e, int64_t n_s,
                             const double *sigmas, double *omega_top, const sislice_opts *opts,
                             double *evals, double *evecs, int64_t ldx, double *resid,
                             sislice_report *report);

/* The paper's shift-invert subspace iteration, SISubIt(A, B, V0, sigma, M)
 * (Algorithm 2): CholeskyQR of V0 in the B inner product, the LDL^T of
 * A - sigma B, M times V <- L^{-T} D^{-1} L^{-1} B V followed by CholeskyQR,
 * then Rayleigh-Ritz with A and B (Sec. 2.1).  CholeskyQR is applied twice
 * per step (the same span; the second pass restores B-orthonormality).
 *   V0      device n x k (ldv >= n), 1 <= k <= min(112, n); M in [1, 64].
 *   evals   device double[k] out, ascending; X device n x k (ldx >= n) out,
 *           B-orthonormal Ritz vectors; resid device double[k] out, the
 *           normalised residuals ||A x - lambda B x|| / (||A||_2 ||x||).
 * The factorization replaces the one that sislice_adjoint could reuse.  Returns
 * SISLICE_SINGULAR_SHIFT when sigma is an eigenvalue.  Synchronises. */
sislice_status sislice_sisubit(sislice_handle *h, int64_t n, const double *A, int64_t lda,
                               const double *B, int64_t ldb, double sigma, int64_t k,
                               const double *V0, int64_t ldv, int32_t M, double *evals,
                               double *X, int64_t ldx, double *resid);

/* Reverse-mode derivative of the eigenpairs that sislice_solve returns (the
 * lowest n_e of the pencil of Sec. 1).  The paper does not differentiate them;
 * this is first-order perturbation theory of the symmetric-definite problem.
 * For a loss L with cotangents g_evals = dL/dlambda and g_evecs = dL/dX it
 * writes symmetric G_A, G_B with dL = tr(G_A dA) + tr(G_B dB) for symmetric
 * dA, dB:
 *   G_A = X M_A X^T + (Z X^T + X Z^T) / 2
 *   G_B = X M_B X^T - (Z Lam X^T + X Lam Z^T) / 2
 * where K = X^T g_evecs, S and T are its symmetric and antisymmetric parts,
 * F_ji = 1 / (lambda_i - lambda_j) off the diagonal,
 *   M_A = diag(g_evals) + T o F
 *   M_B = -diag(lambda g_evals) - S / 2 - (lambda_i + lambda_j) (T o F) / 2,
 * and column z_i of Z solves (A - lambda_i B) z_i = -(I - B X X^T) g_i with
 * X^T B z_i = 0.  Those solves run as flexible (Polak-Ribiere) conjugate
 * gradients, restarted on a non-positive curvature, on the B-orthogonal
 * complement of X (where A - lambda_i B is positive definite), preconditioned
 * by (A - sigma B)^{-1} for the point sigma nearest lambda_i among those shifts
 * and top boundary that lie below lambda_{n_e+1} (inertia <= n_e: positive
 * definite there).  The factorizations are the ones that the last sislice_solve
 * on this handle left behind when factor_id matches them, else they are
 * computed again.  Pairs with |lambda_i - lambda_j| <= 64 eps max|lambda| drop
 * their T o F terms: a loss of the eigenvectors of a degenerate eigenvalue must
 * be invariant under rotations inside it.
 *   evals, evecs     device: the eigenpairs (n_e, and n x n_e with ldx >= n).
 *   g_evals          device double[n_e], or NULL for zero.
 *   g_evecs          device n x n_e (ldg >= n), or NULL for zero (then Z = 0).
 *   sigmas, omega_top host: the shifts (n_s, ascending) and top boundary of that
 *                    solve; at least one point must have inertia <= n_e
 *                    (SISLICE_ERR_ARG otherwise).
 *   factor_id        sislice_report.factor_id of that solve, or 0.
 *   tol, max_iter    relative residual target of the solves (<= 0: 1e-10) and
 *                    iteration cap (<= 0: 500).
 *   GA, GB           device n x n out (ldga, ldgb >= n), both triangles written.
 *   report           host, may be NULL.
 * Returns SISLICE_NOT_CONVERGED when a solve misses tol within max_iter (the
 * gradients are still written).  Synchronises. */
sislice_status sislice_adjoint(sislice_handle *h, int64_t n, const double *A, int64_t lda,
                               const double *B, int64_t ldb, int64_t n_e, const double *evals,
                               const double *evecs, int64_t ldx, const double *g_evals,
                               const double *g_evecs, int64_t ldg, int64_t n_s,
                               const double *sigmas, double omega_top, uint64_t factor_id,
                               double tol, int32_t max_iter, double *GA, int64_t ldga, double *GB,
                               int64_t ldgb, sislice_adjoint_report *report);

/* One pencil of a batched solve: inputs and outputs as in sislice_solve (all
 * device pointers); its n_s shifts and top boundary are planned by KPM. */
typedef struct {
  int64_t n;
  const double *A;
  int64_t lda;
  const double *B;
  int64_t ldb;
  int64_t n_e;
  int64_t n_s;
  double *evals;   /* device double[n_e] out, ascending            */
  double *evecs;   /* device n x n_e (ldx >= n) out, B-orthonormal */
  int64_t ldx;
  double *resid;   /* device double[n_e] out                       */
} sislice_problem;

typedef struct {
  int32_t workers;       /* pencils in flight at a time                          */
  int32_t n_ok;          /* problems that returned SISLICE_OK                    */
  int32_t n_tuned;       /* orders autotuned by this call (0: all were cached)   */
  int64_t n_converged;   /* returned eigenpairs meeting opts->tol, summed        */
  double t_total_ms;
  double t_tune_ms;      /* autotuning time inside t_total_ms                    */
  int64_t graph_replays; /* factorizations run as replays of captured graphs     */
  int64_t graphs_built;  /* graphs captured by this call                          */
} sislice_batch_report;

/* Many independent pencils of possibly different orders (the paper's probes
 * are independent, Sec. 4.1; so are whole pencils): each problem is planned
 * (sislice_plan_shifts_kpm) and solved (sislice_solve) exactly as alone, with
 * `workers` pencils in flight at a time (<= 0: 4; at most 16), each on a
 * worker handle with its own stream and workspaces that the handle keeps, the
 * largest orders first.  Unless opts->nb fixes it, the factorization's
 * parameters are autotuned per order on the first pencil of that order (the
 * lock-step factorization of its planned points timed by coordinate descent
 * over the panel width 32, 48, 64, the pivoting-panel width 16, 32 and the
 * trailing order 512, 1024, 2048 from which the update takes 128x128 tiles)
 * and cached in the handle.  With opts->graphs every worker replays captured
 * factorization sequences (sislice_opts.graphs; the report counts the
 * replays).  status: host int32[count] out, one sislice_status
 * per problem.  Returns SISLICE_OK when every problem did, else the most
 * severe status (negative before positive).  Synchronises; inputs must be
 * complete on the handle's stream. */
sislice_status sislice_solve_batched(sislice_handle *h, int64_t count,
                                     const sislice_problem *problems, const sislice_opts *opts,
                                     int32_t workers, int32_t *status,
                                     sislice_batch_report *report);

/* Panel width the autotuner cached for order n on this handle (0: none). */
int32_t sislice_tuned_nb(sislice_handle *h, int64_t n);
/* All three cached factorization parameters for order n (host int32 out, any
 * may be NULL): returns 1, or 0 when order n has not been tuned. */
int32_t sislice_tuned_factor(sislice_handle *h, int64_t n, int32_t *nb, int32_t *nbpiv,
                             int32_t *wide_min);

/* Shift migration by k-means (Sec. 3.2), host only: Lloyd iterations on the 1-D
 * set `ritz` (host double[n]) from the initial centroids `prev_shifts` (host
 * double[n_s]) or, if use_kmeanspp, from k-means++ seeding drawn from the
 * SplitMix64 stream of `seed`.  Ties go to the lower centroid; an empty cluster
 * keeps its centroid; at most 300 sweeps.  new_shifts: host double[n_s] out,
 * ascending.  labels: host int32[n] out (may be NULL). */
sislice_status sislice_kmeans_shifts(const double *ritz, int64_t n, const double *prev_shifts,
                                     int64_t n_s, int32_t use_kmeanspp, uint64_t seed,
                                     double *new_shifts, int32_t *labels);

/* Probe migration between SCF steps (Sec. 3.2), host only.  The validated values
 * `ritz` (host double[n]) with the probe that validated each (probe_of, host
 * int32[n], in [0, n_s)) are clustered by k-means (Lloyd as in
 * sislice_kmeans_shifts, seeded with prev_shifts or by k-means++); each cluster is
 * mapped to the probe that validated most of its members (ties: the probe whose
 * previous shift is nearest the centroid, then the lower index); clusters mapped
 * to one probe are merged; probes without a cluster are deleted; while fewer than
 * n_s probes remain, the probe holding the most values is split by 2-means (Lloyd
 * from its smallest and largest value) and the half whose centroid is nearer that
 * probe's previous shift stays with it while the other half seeds an inserted
 * probe.  Outputs: new_shifts host double[n_s] (ascending; the first *n_new are
 * set, *n_new < n_s only when no probe holds two values), value_probe host
 * int32[n] (the new probe each value seeds; may be NULL), origin host
 * int32[n_s] (the previous probe each new probe continues, -1 if inserted; may
 * be NULL), stats host int32[3] (merged, deleted, inserted; may be NULL). */
sislice_status sislice_scf_migrate(const double *ritz, const int32_t *probe_of, int64_t n,
                                   const double *prev_shifts, int64_t n_s, int32_t use_kmeanspp,
                                   uint64_t seed, double *new_shifts, int32_t *value_probe,
                                   int32_t *origin, int32_t *n_new, int32_t *stats);

/* SCF sequence (Algorithm 1 over successive pencils; shift migration of
 * Sec. 3.2, missing eigenvalues and the partial-trace monitor of Sec. 3.3).  The
 * state keeps the shifts, top boundary, validated eigenvalues, the probe that
 * validated each, and the eigenvectors (device, owned) of the last step.
 *   sislice_scf_create: for pencils of order n, the lowest n_e pairs, n_s
 *     shifts; opts as for sislice_solve; eta_tol (<= 0: 0.05) the relative change
 *     of the partial trace that sends a step back to the DOS planner.  The state
 *     holds about (2 n_e + n + 8 n_s) n doubles of device memory.
 *   sislice_scf_step: one pencil.  The first step plans the shifts by KPM and
 *     starts every probe from a Gaussian block.  Later steps compare
 *     eta = tr(X^T A X) of the previous eigenvectors under the previous pencil
 *     (the sum of the previous eigenvalues) and the new one; within eta_tol the
 *     shifts migrate (sislice_scf_migrate; k-means++ after a DOS step), the top
 *     boundary moves to two local spacings above the previous lambda_{n_e} (the
 *     solve lifts it when the pencil has moved past it), and every
 *     probe starts from the previous eigenvectors of the values that seed it (a
 *     Gaussian combination of them, or the vectors padded with Gaussian columns
 *     when fewer than the block size); otherwise, or when the migrated shifts
 *     miss eigenvalues, the step uses DOS shifts and Gaussian starts.  Outputs as
 *     for sislice_solve; sigmas host double[n_s] and omega_top host double out
 *     (may be NULL).  The factorizations stay with the handle for
 *     sislice_adjoint (report->factor_id).  Synchronises.
 *   sislice_scf_destroy: frees the state (not the handle). */
typedef struct sislice_scf sislice_scf;
typedef struct {
  int32_t step;          /* 0 for the first pencil                                   */
  int32_t replanned;     /* 0 migrated shifts, 1 DOS shifts (first step or trace jump), */
                         /* 2 DOS shifts after the migrated shifts missed eigenvalues  */
  int32_t merged, deleted, inserted;  /* probe migration counts (sislice_scf_migrate)  */
  int32_t status_solve;  /* status of the solve                                        */
  double eta_prev;       /* sum of the previous eigenvalues                            */
  double eta_new;        /* tr(X_prev^T A X_prev) with the new A                        */
  int64_t block_steps;   /* block Lanczos steps of the step's solves                   */
  uint64_t factor_id;
  double t_solve_ms, t_total_ms;
  int32_t cycles_max;    /* largest number of Lanczos restart cycles of a probe        */
  int32_t probes_inserted; /* probes inserted by the solve into slices that missed
                              eigenvalues (Sec. 3.3)                                 */
  double t_factor_ms;    /* factorizations of the step's solves (shift-form, LDL^T,
                            inertia)                                                   */
  double flops_factor;   /* n^3/3 per factorization, summed                           */
} sislice_scf_report;

sislice_status sislice_scf_create(sislice_handle *h, int64_t n, int64_t n_e, int64_t n_s,
                                  const sislice_opts *opts, double eta_tol, sislice_scf **scf);
sislice_status sislice_scf_step(sislice_scf *scf, const double *A, int64_t lda, const double *B,
                                int64_t ldb, double *evals, double *evecs, int64_t ldx,
                                double *resid, double *sigmas, double *omega_top,
                                sislice_scf_report *report);
sislice_status sislice_scf_destroy(sislice_scf *scf);

/* Slice validation (Sec. 2.2), host only.  Probe j (shift sigmas[j]) reports
 * counts[j] Ritz values and residual norms stored contiguously from
 * offsets[j] in `thetas` / `resids`.  Slices: (-inf, s_1), [s_j, s_{j+1}) split
 * at their midpoint tau (a value at tau belongs to the lower probe),
 * [s_ns, omega_top).  Outputs: slice_case/slice_exact/slice_cand int32[n_s+1];
 * chosen int32[total] flags (1 = validated) aligned with `thetas`.
 * Returns the number of validated values, or a negative status. */
int64_t sislice_validate(int64_t n_s, const double *sigmas, const int64_t *nu, double omega_top,
                         int64_t nu_top, const int64_t *offsets, const int64_t *counts,
                         const double *thetas, const double *resids, int32_t *slice_case,
                         int32_t *slice_exact, int32_t *slice_cand, int32_t *chosen);

/* Host helpers of the planner (Sec. 3.1), exposed for testing:
 * CDOS Phi(omega) of Jackson-damped moments mu[0..M) on [a, b] for order n, and
 * the equal-count placement described at sislice_plan_shifts_kpm. */
double sislice_kpm_cdos(const double *mu, int32_t M, double a, double b, int64_t n, double omega);
sislice_status sislice_kpm_place(const double *mu, int32_t M, double a, double b, int64_t n,
                                 int64_t n_e, int64_t n_s, double top_margin, double *sigmas,
                                 double *omega_top);

/* The paper's DOS shift selection (Sec. 3.1), host part: from n_v runs of
 * k-step Lanczos (host theta[r*k + j] Ritz values ascending per run, zeta2 the
 * squared first components of their eigenvectors), the Gaussian-broadened DOS
 * phi and its closed-form CDOS Phi (eq. dos, eq. cdos; averaged over the runs;
 * widths nu_j = d_j / 3 with d_j the larger neighbour gap, floored at
 * 1e-3 (b - a) / k), the window [a, omega_top] with Phi(omega_top) =
 * n_e + top_margin n_e / n_s, and n_s shifts: mode 0 equal-count roots and
 * interval midpoints (eq. cdos_root); mode 1 DOSCluster on 10 k grid points,
 * merging of intervals with fewer than 2 estimated eigenvalues, refinement of
 * intervals with more than 50, the safeguards that split or merge to exactly n_s
 * intervals, and each shift the DOS expectation over its interval.  sigmas host
 * double[n_s] out ascending, omega_top host double out. */
sislice_status sislice_dos_plan(const double *theta, const double *zeta2, int32_t k, int32_t nv,
                                int64_t n, int64_t n_e, int64_t n_s, int32_t mode,
                                double top_margin, double *sigmas, double *omega_top);

/* SplitMix64 output i of `seed` (counter form): the generator behind every
 * random draw of the library. */
uint64_t sislice_splitmix64(uint64_t seed, uint64_t i);

/* Small dense symmetric eigensolver used for the projected problems of
 * Rayleigh-Ritz (Sec. 2.1): `batch` matrices of order m <= 112, device,
 * column-major with leading dimension lda, lower triangle read.  W device
 * double[batch*m] eigenvalues ascending; V device batch*(m x m) eigenvectors
 * (leading dimension m).  The rotations are recorded in a workspace of the
 * handle (about 4 MB per matrix of order 112, batches of more than 67 such
 * matrices are processed in chunks); it grows on the first call that needs
 * more, and a failed growth returns SISLICE_ERR_ALLOC.  Returns after the work
 * has completed (the host staging of the per-matrix tables is reused). */
sislice_status sislice_sym_eig(sislice_handle *h, int32_t m, int32_t batch, const double *A,
                               int64_t lda, double *W, double *V);

/* The same solver for a batch of matrices of different orders, as the solve
 * path launches it: matrix b, of order m[b] (host int32, 0 <= m[b] <= mmax <=
 * 112; 0 skips it), is the leading m[b] x m[b] block at A + b*lda*mmax (device,
 * column-major, leading dimension lda >= mmax, lower triangle read).  Its
 * eigenvalues go to W + b*mmax (ascending) and its eigenvectors to
 * V + b*mmax*mmax (leading dimension mmax, column j for eigenvalue j); entries
 * past m[b] are not written.  Returns after the work has completed. */
sislice_status sislice_sym_eig_var(sislice_handle *h, int32_t batch, const int32_t *m,
                                   int32_t mmax, const double *A, int64_t lda, double *W,
                                   double *V);

#ifdef __cplusplus
}
#endif

#endif /* SISLICE_H */

/*
 * sgmres.h -- C ABI of the MI355X (gfx950) sketched GMRES library.
 *
 * Method: Y. Nakatsukasa and J. A. Tropp, "Fast & accurate randomized
 * algorithms for linear systems and eigenvalue problems", arXiv:2111.00113,
 * Algorithm 1 (sGMRES + k-truncated Arnoldi) with restarting (Section 3.5).
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers (HIP) unless stated otherwise and are
 *     owned by the caller; the library never frees them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     All device work is enqueued on it.  Entry points that return host-side
 *     results (status codes, info structs, host scalars) synchronise `stream`
 *     before returning.
 *   - Dense matrices are column-major with the stated leading dimension.
 *   - Indices are int32 (n < 2^31, nnz < 2^31).  CSR column indices need not
 *     be sorted within a row.
 *   - Internal workspace is allocated by the library on first use on each
 *     device and cached (grow-only) until sgmres_release_workspace().
 *     Concurrent calls on one device from several host threads are not
 *     supported.
 *   - Return codes: SGMRES_OK (0) on success, SGMRES_NOT_CONVERGED (1) when a
 *     solve ran out of restarts (x then holds the last iterate), or a negative
 *     SGMRES_E* code.  Nothing is written to outputs on SGMRES_EINVAL.
 *
 * Readings of points the paper leaves open (listed with the library design):
 *   sketch columns scaled by 1/sqrt(zeta); real +-1 signs; zeta distinct rows
 *   per column drawn by rejection from Philox4x32-10; classical Gram-Schmidt
 *   twice against the window; unpivoted Householder QR of S A B; the longest
 *   prefix with max|T_ii|/min|T_ii| <= kappa_max is used; x <- x + B y.
 */
#ifndef SGMRES_H
#define SGMRES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SGMRES_OK 0
#define SGMRES_NOT_CONVERGED 1
#define SGMRES_EINVAL (-1)     /* bad argument (null pointer, size out of range) */
#define SGMRES_ECSR (-2)       /* malformed CSR (row_ptr not monotone, column out of range) */
#define SGMRES_ENOMEM (-3)     /* device or pinned-host allocation failed */
#define SGMRES_EHIP (-4)       /* a HIP runtime call failed */
#define SGMRES_ENONFINITE (-5) /* NaN/Inf met in b, x0, A or a residual norm */
#define SGMRES_ETIMEOUT (-6)   /* an in-kernel grid barrier exceeded its wait limit */

#define SGMRES_FLAG_KAPPA_TRUNC 1 /* a cycle used a prefix of its basis (kappa guard) */
#define SGMRES_FLAG_BREAKDOWN 2   /* a cycle's basis ended early (invariant subspace) */

#define SGMRES_BASIS_ARNOLDI 0   /* k-truncated Arnoldi (Algorithm 1) */
#define SGMRES_BASIS_CHEBYSHEV 1 /* shifted-and-scaled Chebyshev recurrence (Section 4.4) */

/* Precision of the basis cycles (the residual b - A x, the sums of partial
 * results, the sketched least squares and x stay FP64 in every mode; restarting
 * from the FP64 residual is the iterative refinement that wins the accuracy
 * back). */
#define SGMRES_PREC_FP64 0       /* everything FP64 */
#define SGMRES_PREC_FP32 1       /* SpMV (on an FP32 copy of A's values), basis and
                                    sketch inputs in FP32, basis stored in FP32 */
#define SGMRES_PREC_BF16_BASIS 2 /* as FP32, with the basis stored in bfloat16 */

/* Square sparse matrix in CSR form; all arrays on the device. */
typedef struct {
    int64_t n;              /* order, 1 <= n < 2^31 */
    int64_t nnz;            /* row_ptr[n] */
    const int32_t *row_ptr; /* n + 1 entries, row_ptr[0] = 0, nondecreasing */
    const int32_t *col_idx; /* nnz entries in [0, n) */
    const double *val;      /* nnz entries */
} sgmres_csr_t;

/* Host-side solve report (pointer may be NULL). */
typedef struct {
    int32_t cycles;     /* basis cycles run (restarts + 1 at most) */
    int32_t steps;      /* basis columns built, summed over cycles */
    int32_t d_eff_last; /* columns used by the last cycle's least-squares solve */
    int32_t flags;      /* OR of SGMRES_FLAG_* over all cycles */
    double relres;      /* final true relative residual |b - A x| / |b| */
    double rest_est;    /* last cycle's sketched residual estimate / |b| (Section 3.2) */
    double kappa_est;   /* last cycle's max|T_ii| / min|T_ii| over the used prefix */
    /* GPU time per kernel class, summed over the solve, measured with HIP events
     * on `stream`; filled only when sgmres_options_t.profile is nonzero. */
    double t_residual_ms; /* residual r = b - A x and its norm */
    double t_basis_ms;    /* basis + sketch kernel (one launch per cycle) */
    double t_lsq_ms;      /* sketched least squares */
    double t_combine_ms;  /* x <- x + B y */
    /* Basis kernel, workgroup 0's wall time per phase summed over all steps
     * (microseconds; profile only): [0] SpMV + dots, [1] sketch scatter,
     * [2] wait after phase 1, [3] first Gram-Schmidt update + dots,
     * [4] barrier after phase 2, [5] second update + new column,
     * [6] sketch column sums, [7] wait after phase 3.  Chebyshev basis:
     * [0] SpMV + recurrence, [1] norm and sketch partials, [2] barrier wait,
     * [7] end-of-cycle reduction. */
    double phase_us[8];
    /* Basis kernel that ran (the last cycle's launch): SGMRES_PATH_*, its
     * workgroup size, rows per thread and grid (0 when no basis cycle ran).
     * SGMRES_PATH_STREAM reports rows per thread as -P when each workgroup
     * parks its rows' m and w in an HBM buffer (P rows per thread and tile). */
    int32_t path;
    int32_t launch_block;
    int32_t launch_rows;
    int32_t launch_grid;
    double t_sketch_ms; /* streaming path: sketch of the finished basis, S A B = (S B) H
                           and g = S r (profile only; included in t_basis_ms) */
    double cheb_box[3]; /* Chebyshev basis: the box (c, dx, dy) used, given or estimated */
} sgmres_info_t;

#define SGMRES_PATH_ARNOLDI_3BAR 1 /* resident truncated Arnoldi, three grid barriers per step */
#define SGMRES_PATH_ARNOLDI_HALO 2 /* resident truncated Arnoldi, two barriers (halo rebuild) */
#define SGMRES_PATH_CHEBYSHEV 3    /* resident Chebyshev basis, one barrier per step */
#define SGMRES_PATH_PART_SPLIT 4   /* part-split kernel of the batched solve */
#define SGMRES_PATH_STREAM 5       /* streaming truncated Arnoldi (n above the resident
                                      capacity): window read back from B, S B formed
                                      from the finished basis and S A B = (S B) H */
#define SGMRES_PATH_MULTI 6        /* batched solve: several systems per resident
                                      truncated-Arnoldi launch, one group of
                                      workgroups each */

/* Options of sgmres_solve_ex; zero-initialise for the defaults. */
typedef struct {
    int32_t zeta;       /* nonzeros per sketch column; 0 -> 8; must be <= s and <= 32 */
    double kappa_max;   /* condition guard on T (Sections 3.4, 5.3); 0 -> 1e14 */
    int32_t transposed; /* nonzero: solve A^T x = b */
    int32_t block_size; /* basis-kernel workgroup size, 256 / 512 / 1024; 0 -> auto */
    int32_t rows_per_thread; /* basis-kernel rows per thread, 1 / 2 / 4 / 8; 0 -> auto */
    int32_t profile;    /* nonzero: fill the t_*_ms fields of sgmres_info_t */
    int32_t barrier_mode; /* basis-kernel grid barrier: 0 one L2 write-back per XCD
                             (default), 1 one per workgroup (reference protocol;
                             results are bit-identical) */
    int32_t spmv_mode;  /* must be 0: the basis kernels read A through a sliced
                           ELL copy (slices of 64 rows, one wavefront each), built
                           per call, summing each row in CSR order */
    int32_t basis;      /* SGMRES_BASIS_ARNOLDI (default) or SGMRES_BASIS_CHEBYSHEV */
    double cheb_c;      /* Chebyshev basis: the spectrum of A lies in the box */
    double cheb_dx;     /* [cheb_c - cheb_dx, cheb_c + cheb_dx] x [-cheb_dy, cheb_dy] */
    double cheb_dy;     /* (Section 4.4); dx, dy >= 0; k is unused.  dx = dy = 0: the box is
                           estimated from a short Arnoldi pass on b (sgmres_chebyshev_box);
                           not for transposed solves without a plan */
    int32_t precision;  /* SGMRES_PREC_* (0 = FP64) */
    int32_t batch_eager; /* sgmres_solve_batched: launch each cycle's kernels directly
                            instead of replaying the captured hipGraph */
    int32_t halo_off;   /* truncated Arnoldi: nonzero keeps three grid barriers per step;
                           0 uses two when at most a quarter of the nonzeros reach outside
                           their row's block of the basis kernel (results are bit-identical) */
    int32_t path;       /* 0 auto: the resident kernels when the system fits them, else
                           SGMRES_PATH_STREAM (k <= 4, s <= 1024, n < 2^26), else the part-split
                           kernel (k <= 4); SGMRES_PATH_STREAM or SGMRES_PATH_PART_SPLIT
                           force that path (truncated Arnoldi only) */
    int32_t stream_state; /* streaming path: 0 auto, 1 keep m and w in registers (fails
                             with SGMRES_EINVAL when the grid cannot hold every row),
                             2 park them in an HBM buffer between phases */
} sgmres_options_t;

/*
 * Restarted sGMRES with k-truncated Arnoldi (Algorithm 1; restarts Section 3.5).
 * Solves A x = b.
 *   A        CSR matrix (struct on the host, arrays on the device)
 *   b        n right-hand side
 *   x        n; in: initial guess x0, out: approximate solution
 *   d        basis columns per cycle, 1 <= d <= min(n, 1024)
 *   k        truncation window (previous columns orthogonalised against), k >= 1;
 *            k >= d-1 gives full Arnoldi
 *   s        sketch rows, d + 1 <= s <= 4096 (the paper recommends s = 2(d+1))
 *   seed     sketch key; cycle c uses Philox counter word 2 = c
 *   tol      stop when |b - A x|_2 / |b|_2 <= tol (true residual), tol >= 0
 *   restarts maximum additional cycles (total cycles <= restarts + 1), >= 0
 *   info     host pointer, may be NULL
 * Returns SGMRES_OK, SGMRES_NOT_CONVERGED or an SGMRES_E* code.  b = 0 gives
 * x = 0 and SGMRES_OK.
 */
int sgmres_solve(const sgmres_csr_t *A, const double *b, double *x, int d, int k, int s,
                 uint64_t seed, double tol, int restarts, sgmres_info_t *info, void *stream);

/* As sgmres_solve, for the transposed system A^T x = b.  CSR(A^T) is built on
 * the device (sgmres_csr_transpose) into library workspace on each call. */
int sgmres_solve_transposed(const sgmres_csr_t *A, const double *b, double *x, int d, int k,
                            int s, uint64_t seed, double tol, int restarts,
                            sgmres_info_t *info, void *stream);

/* As sgmres_solve with options (NULL = defaults). */
int sgmres_solve_ex(const sgmres_csr_t *A, const double *b, double *x, int d, int k, int s,
                    uint64_t seed, double tol, int restarts, const sgmres_options_t *opts,
                    sgmres_info_t *info, void *stream);

/* Plan: a matrix's set-up, done once and reused by many solves.
 * sgmres_plan_create validates A's CSR arrays
 * (SGMRES_ECSR if malformed) and builds on the current device the sliced ELL
 * copy the basis kernels read (FP64 values; also FP32 values with
 * SGMRES_PLAN_FP32) and, with SGMRES_PLAN_TRANSPOSE, CSR(A^T) and its copies,
 * so sgmres_solve_plan with opts->transposed solves A^T x = b without
 * rebuilding the transpose (the adjoint solve of a differentiable step).  The
 * plan keeps pointers to A's arrays, which must stay unchanged while it lives;
 * it owns everything else and frees it in sgmres_plan_destroy.  A plan is used
 * on the device it was created on (SGMRES_EINVAL otherwise).  sgmres_solve_plan
 * takes the arguments of sgmres_solve_ex after the matrix and gives the same
 * bits; it returns SGMRES_EINVAL when the plan lacks the copy the precision or
 * the transposition asks for. */
#define SGMRES_PLAN_TRANSPOSE 1
#define SGMRES_PLAN_FP32 2
typedef struct sgmres_plan sgmres_plan_t;
int sgmres_plan_create(const sgmres_csr_t *A, int flags, sgmres_plan_t **plan, void *stream);
int sgmres_plan_destroy(sgmres_plan_t *plan);
int sgmres_solve_plan(const sgmres_plan_t *plan, const double *b, double *x, int d, int k, int s,
                      uint64_t seed, double tol, int restarts, const sgmres_options_t *opts,
                      sgmres_info_t *info, void *stream);

/* ---------------------------------------------------------------------------
 * Hot-path steps, callable one by one (they compose into sgmres_solve).
 * ------------------------------------------------------------------------- */

/* Sparse sign embedding pattern (Section 2.3.2).  For columns i = i0 .. i0+count-1
 * writes rows[(i-i0)*zeta + t] in [0, s) (distinct within a column) and
 * signs[(i-i0)*zeta + t] in {-1, +1}, t in acceptance order.  Column i uses
 * Philox4x32-10 with key (lo32(seed), hi32(seed)) and counters
 * (lo32(i), hi32(i), cycle, t), t = 0, 1, ...; each 32-bit output word u, in
 * order, proposes row floor(u*s/2^32) with sign -1 iff u is odd; proposals
 * repeating an accepted row are discarded.  1 <= zeta <= min(s, 32). */
int sgmres_sketch_pattern(uint64_t seed, uint32_t cycle, int64_t i0, int64_t count, int s,
                          int zeta, int32_t *rows, int8_t *signs, void *stream);

/* g = S v (Section 2.3.2, scale 1/sqrt(zeta)): v (device) has n >= 0 entries,
 * g (device) has s; requires 1 <= s <= 4096 and 1 <= zeta <= min(s, 32).  The
 * sums run in a fixed order (rows in chunks of 512, each sketch row's terms in
 * ascending input index inside a chunk, chunk totals per workgroup, then the
 * workgroups in order), so the result is the same bits on every call.  Uses
 * the library's workspace (allocated on first use); returns after the work on
 * `stream` has finished.  Errors: SGMRES_EINVAL for a bad size or null
 * pointer, SGMRES_ENOMEM / SGMRES_EHIP from the runtime. */
int sgmres_sketch_apply(int64_t n, const double *v, uint64_t seed, uint32_t cycle, int s,
                        int zeta, double *g, void *stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): sgmres_sketch_apply
 * with the same arguments, limits and bits, but no allocation of any kind.
 * Its block partials (s x G doubles, G = min(512, ceil(n / 512))) live in one
 * fixed 16 MiB device array per GPU, held until the process ends; sizes
 * beyond it cannot occur within s <= 4096 and are rejected with SGMRES_EINVAL
 * all the same.  The work is only enqueued on `stream` (no synchronisation):
 * g is ready when the stream reaches that point.  Every call on one GPU
 * shares that GPU's array, so calls that overlap on one GPU (other streams,
 * other threads) race and must be ordered by the caller.  The array needs no
 * clearing: every partial is written before it is read. */
int sgmres_sketch_apply_noalloc(int64_t n, const double *v, uint64_t seed, uint32_t cycle, int s,
                                int zeta, double *g, void *stream);

/* r = f - A x and its 2-norm (Algorithm 1, residual step).  r has n entries
 * (device); *norm (host) receives |r|_2. */
int sgmres_residual(const sgmres_csr_t *A, const double *f, const double *x, double *r,
                    double *norm, void *stream);

/* One cycle of basis generation and sketching (Algorithm 1, basis loop;
 * truncated-Arnoldi recurrence of Section 1.2.2 with two classical
 * Gram-Schmidt passes).  From the residual r (n, nonzero):
 *   B   n x d, leading dim ldb >= n: columns b_1 .. b_dc (b_1 = r/|r|)
 *   SB  s x d (ld s):  S b_j          SAB s x d (ld s):  S A b_j
 *   H   (k+1) x d (ld k+1): column j holds the summed Gram-Schmidt coefficients
 *       against the window, newest column first, then |w| in row k
 *   g   s: S r
 * *dc (host) receives the number of columns built (< d after breakdown) and
 * *flags (host) ORs in SGMRES_FLAG_BREAKDOWN.  Requires 1 <= d <= 1024,
 * 1 <= k <= 1024, 1 <= s <= 4096, 1 <= zeta <= min(s, 32).  H is cleared first;
 * column d-1 (and columns past a breakdown) stay zero. */
int sgmres_arnoldi_cycle(const sgmres_csr_t *A, const double *r, int d, int k, int s, int zeta,
                         uint64_t seed, uint32_t cycle, double *B, int64_t ldb, double *SB,
                         double *SAB, double *H, double *g, int *dc, int *flags, void *stream);

/* One cycle of the Chebyshev basis (Section 4.4) with sketching.  For the
 * box [c - dx, c + dx] x [-dy, dy] containing the spectrum, rho = max(dx, dy):
 * b_1 = r/|r|, b_2 = (A - cI) b_1 / (2 rho),
 * b_j = [(A - cI) b_{j-1} - (dx^2 - dy^2)/(4 rho) b_{j-2}] / rho, and each
 * column is scaled to unit norm after its use.  Outputs (device):
 *   B        n x d, ld ldb >= n: the unnormalised recurrence vectors
 *            kappa^(j-1) b_j, kappa = 2 rho / (dx + dy) (a constant rescale
 *            per step that normalisation removes)
 *   colnorm  d: |B[:, j]|_2; column j of the normalised basis is B[:, j]/colnorm[j]
 *   SB, SAB  s x d (ld s): S and S A applied to the normalised columns
 *   g        s: S r
 * A column of norm 0 gives zero sketch columns.  1 <= d <= 1024,
 * 1 <= s <= 4096, 1 <= zeta <= min(s, 32); dx, dy >= 0 with max(dx, dy) > 0. */
int sgmres_chebyshev_cycle(const sgmres_csr_t *A, const double *r, int d, int s, int zeta,
                           uint64_t seed, uint32_t cycle, double c, double dx, double dy,
                           double *B, int64_t ldb, double *SB, double *SAB, double *colnorm,
                           double *g, void *stream);

/* Sketched least squares (Algorithm 1 solve step; Section 3.3).  C (s x dc,
 * ld s) is overwritten by its Householder factorisation (T in the upper
 * triangle), g (s) by Q^T g.  y (d_eff entries) solves
 * T[:d_eff,:d_eff] y = (Q^T g)[:d_eff], where d_eff is the longest prefix with
 * max|T_ii|/min|T_ii| <= kappa_max.  Host outputs: *d_eff, *rest = |(Q^T g)[d_eff:]|,
 * *kappa = the ratio at d_eff; *flags ORs in SGMRES_FLAG_KAPPA_TRUNC when
 * d_eff < dc.  0 <= dc <= min(s, 1024), s <= 32767. */
int sgmres_sketched_lsq(int s, int dc, double *C, double *g, double kappa_max, double *y,
                        int *d_eff, double *rest, double *kappa, int *flags, void *stream);

/* x <- x + B[:, :d_eff] y (Section 3.3, solution step).  B n x d_eff, ld ldb. */
int sgmres_basis_combine(int64_t n, int d_eff, const double *B, int64_t ldb, const double *y,
                         double *x, void *stream);

/* CSR(A^T) on the device: t_row_ptr (n+1), t_col_idx (nnz), t_val (nnz) are
 * caller-allocated device arrays; each output row lists its columns in
 * ascending order. */
int sgmres_csr_transpose(const sgmres_csr_t *A, int32_t *t_row_ptr, int32_t *t_col_idx,
                         double *t_val, void *stream);

/* Gradient of a linear solve with respect to the matrix entries, on A's
 * sparsity pattern: dval[q] = alpha * u[i] * v[j] for each stored entry
 * q = (i, j) of A (same order as A->val).  With x = A^{-1} b and the adjoint
 * A^T lambda = dL/dx, alpha = -1, u = lambda, v = x gives dL/dA_ij =
 * -lambda_i x_j (and dL/db = lambda).  u, v: n entries; dval: nnz entries. */
int sgmres_csr_outer_grad(const sgmres_csr_t *A, const double *u, const double *v, double alpha,
                          double *dval, void *stream);

/* ---------------------------------------------------------------------------
 * Batched solve: many independent systems A_i x_i = b_i of uneven sizes.
 * ------------------------------------------------------------------------- */

/* One system of a batch; the struct array is on the host, its arrays on the
 * device.  Several systems may share A (blocks of right-hand sides). */
typedef struct {
    sgmres_csr_t A;
    const double *b; /* n right-hand side */
    double *x;       /* n; in: initial guess, out: approximate solution */
} sgmres_system_t;

/* Host-side result of one system. */
typedef struct {
    int32_t status; /* SGMRES_OK, SGMRES_NOT_CONVERGED or SGMRES_ENONFINITE */
    int32_t cycles; /* basis cycles run */
    int32_t steps;  /* basis columns built, summed */
    int32_t flags;  /* OR of SGMRES_FLAG_* */
    double relres;  /* final true relative residual |b - A x| / |b| */
} sgmres_batch_result_t;

/*
 * Restarted sGMRES (Algorithm 1 with the restarts of Section 3.5) on each
 * system independently, with the method of sgmres_solve_ex for truncated
 * Arnoldi: the same sketch (keyed by seed, cycle and the row within the system)
 * and the same stopping rule per system, so system i gets what sgmres_solve_ex
 * gives for it alone, up to rounding.  Systems that share one matrix (the
 * same three CSR pointers) and have at least 65,536 rows are solved as blocks
 * of up to 32 right-hand sides (Section 1.3.3's setting of many right-hand
 * sides, each with its own basis): one streaming basis launch per cycle builds
 * every basis of the block, reading each nonzero of A once per step for all of
 * them (SGMRES_PATH_STREAM; s <= 1024); opts->path = SGMRES_PATH_PART_SPLIT
 * keeps them on the per-system kernels.  Other systems of at least 2^19 rows
 * fill the chip alone: they are solved one after another by the resident
 * kernels of sgmres_solve_ex.  The rest (SGMRES_PATH_MULTI, the default) run
 * several to a resident truncated-Arnoldi launch, each on its own group of
 * ceil(n / (1024 * rows_per_thread)) workgroups (rows_per_thread 2 or 4,
 * default 4), packed largest first into launches that fit the chip; a system
 * gets what sgmres_solve_ex gives it with that launch shape.  With opts->path
 * = SGMRES_PATH_PART_SPLIT they run instead one persistent launch per cycle
 * of the part-split kernel, each split into parts of at most 16384 rows taken
 * by workgroups from a queue, each cycle's kernels replayed from a captured
 * hipGraph.  opts: zeta, kappa_max, precision (mixed precision with FP64
 * refinement as in sgmres_solve_ex), path, rows_per_thread (multi-system
 * launches: 2 or 4); for the part-split kernel block_size / rows_per_thread
 * (0 = 512 x 4 for batches under 2^20 rows, else chosen by timing the first
 * cycle of each candidate; the choice is kept per problem class) and
 * batch_eager; other fields are ignored.
 *   nsys     number of systems (0 returns SGMRES_OK)
 *   systems  host array of nsys systems; every n >= d, 1 <= k <= 4
 *   results  host array of nsys results, may be NULL
 * Returns SGMRES_OK when every system converged, SGMRES_NOT_CONVERGED when some
 * did not (results[i].status tells which), or an SGMRES_E* code for bad
 * arguments (nothing is solved then).
 */
int sgmres_solve_batched(int nsys, const sgmres_system_t *systems, int d, int k, int s, uint64_t seed,
                         double tol, int restarts, const sgmres_options_t *opts,
                         sgmres_batch_result_t *results, void *stream);

/* Frees the cached workspace of every device. */
void sgmres_release_workspace(void);

/*
 * Spectral box for the Chebyshev basis from a short Arnoldi pass (Section 4.4:
 * a few Arnoldi iterations estimate the spectrum of A, and the shifted and
 * scaled Chebyshev polynomials are fitted to a region containing it).  Runs
 * m + 1 steps of Arnoldi with a full window (two classical Gram-Schmidt
 * passes, FP64) from r on the device, takes the Ritz values (eigenvalues of
 * the leading m x m block of the Hessenberg matrix, computed on the host; the
 * leading dc x dc block when the Krylov space of r is invariant after dc
 * columns) and returns their bounding rectangle with both half-widths widened
 * by 10%.  sgmres_solve_ex does this with m = min(20, d, n - 1) and r = b when
 * the Chebyshev basis is asked for with cheb_dx = cheb_dy = 0.
 *   A      device CSR, n > m
 *   r      n device vector (r = 0 gives the box (0, 1, 0) and no Ritz values)
 *   m      1 <= m <= 64
 *   box    host, 3 doubles out: c, dx, dy
 *   ritz   host, 2m doubles out (nullable): real parts, then imaginary parts
 *   nritz  host out (nullable): Ritz values returned
 * Synchronises the stream.  Returns SGMRES_OK, SGMRES_EINVAL, SGMRES_ECSR,
 * SGMRES_ENONFINITE (non-finite r or Hessenberg entries) or SGMRES_ETIMEOUT.
 */
int sgmres_chebyshev_box(const sgmres_csr_t *A, const double *r, int m, double *box, double *ritz, int *nritz,
                         void *stream);

/*
 * Eigenvalues of an m x m upper Hessenberg matrix (host memory, column-major,
 * leading dimension ldh; entries below the subdiagonal are ignored; H is not
 * modified) by the implicitly double-shifted QR iteration: the step that
 * sgmres_chebyshev_box applies to the Arnoldi Hessenberg matrix.  wr, wi: m
 * doubles out (real and imaginary parts; a complex pair is stored
 * consecutively).  Host code only, no device.  Returns SGMRES_OK, or
 * SGMRES_EINVAL for bad sizes or when the iteration does not converge.
 */
int sgmres_hessenberg_eigenvalues(int m, const double *H, int ldh, double *wr, double *wi);

/* Library version string (static storage). */
const char *sgmres_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SGMRES_H */

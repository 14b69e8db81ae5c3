/*
 * Sketched GMRES oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of what the GPU path
 * computes.  Only the test suite, the package smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header or helper with the
 * HIP implementation; the only common ground is the written specification of
 * the sketch pattern (Philox4x32-10 counter layout, see oracle_sketch_pattern).
 *
 * Source: Y. Nakatsukasa and J. A. Tropp, "Fast & accurate randomized
 * algorithms for linear systems and eigenvalue problems", arXiv:2111.00113.
 *   Algorithm 1        sGMRES + k-truncated Arnoldi (Section 1.2.2)
 *   Section 1.2.2      truncated-Arnoldi recurrence (eq. "partorth")
 *   Section 2.3.2      sparse sign embedding
 *   Section 3.3        sketched LS solve: y = T^{-1} U^* S r0, r_est = |(I-UU^*) S r0|
 *   Section 3.4        reliability threshold kappa_2(AB) <= 1e14 in FP64
 *   Section 3.5        restarting from the current residual
 *   Section 5.3        adaptive restart when kappa(T_j) first exceeds tol
 * Philox4x32-10: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,
 *   "Parallel random numbers: as easy as 1, 2, 3", SC'11.
 *
 * Readings of points the paper leaves open (each repeated where it applies):
 *   R-scale   sparse-map columns are scaled by 1/sqrt(zeta), not 1/sqrt(s), so
 *             that E|Sx|^2 = |x|^2 (Section 2.3.2 prints 1/sqrt(s), which would
 *             contradict the embedding definition of Section 2).
 *   R-field   real Rademacher signs instead of Steinhaus entries (real field).
 *   R-place   "exactly zeta nonzeros in uniformly random coordinates" is read as
 *             zeta distinct rows drawn by rejection from a counter-based stream.
 *   R-cgs2    "double Gram-Schmidt" (Algorithm 1, Implementation) is classical
 *             Gram-Schmidt applied twice against the same window.
 *   R-window  the window for b_{j+1} is b_j, ..., b_{max(1, j-k+1)}.
 *   R-break   if |w| <= 4u|m| the basis stops at that column (invariant space).
 *   R-qr      unpivoted Householder QR (LAPACK dlarfg sign convention).
 *   R-kappa   kappa_est(j) = max_{i<=j}|T_ii| / min_{i<=j}|T_ii|; the solve uses
 *             the longest prefix with kappa_est <= kappa_max (Section 5.3).
 *   R-soln    the solution update is x + B y (Section 3.2 / 3.3); Algorithm 1's
 *             last line, which multiplies y by the reduced matrix, is a typo.
 *   R-tol     the stopping tolerance is the true relative residual |b-Ax|/|b|;
 *             the paper's `tol` (a condition-number bound) is kappa_max.
 *   R-restart a fresh sketch per cycle: Philox counter word 2 = cycle index.
 *   R-cheb    Chebyshev basis (Section 4.4): the recurrence runs on the
 *             unnormalised vectors; each is scaled to unit norm only for B,
 *             S B and S A B.  A vector of norm 0 gives a zero column.
 *
 * Summation order.  Every sum over the n rows (inner products, norms, the
 * sketch S v) is taken in fixed chunks of OR_CHUNK consecutive rows: each
 * chunk is summed in ascending row order, and the chunk sums are added in
 * ascending chunk order.  Row-wise loops (SpMV, vector updates, the basis
 * combination) have no cross-row sums.  The result therefore does not depend
 * on the number of threads: oracle_set_threads(t) only spreads the chunks and
 * rows over t OpenMP threads (default 1), and any t gives the same bits.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_EINVAL (-1)
#define OR_ENOMEM (-3)
#define OR_ENONFINITE (-5)

#define OR_FLAG_KAPPA_TRUNC 1
#define OR_FLAG_BREAKDOWN 2

#define OR_CHUNK 4096 /* rows per fixed reduction chunk */

static int g_threads = 1;

/* Threads used by the row loops and chunk sums (results are identical for any
 * count, see "Summation order" above). */
void oracle_set_threads(int t) { g_threads = t < 1 ? 1 : t; }
int oracle_get_threads(void) { return g_threads; }

static int64_t chunks_of(int64_t n) { return (n + OR_CHUNK - 1) / OR_CHUNK; }

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): a 4x32-bit Feistel-like bijection    */
/* keyed by 2x32 bits; each round multiplies words 0 and 2 by fixed odd        */
/* constants, and the key is bumped by Weyl constants between rounds.         */
/* ------------------------------------------------------------------------ */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    memcpy(out, c, sizeof c);
}

/* ------------------------------------------------------------------------ */
/* Sparse sign embedding, Section 2.3.2 (readings R-place, R-field).           */
/*                                                                            */
/* Column i of S: key = (lo32(seed), hi32(seed)); counter block t (t = 0,1,..) */
/* = (lo32(i), hi32(i), cycle, t).  The 32-bit words of blocks t = 0,1,... are */
/* taken in order; word u proposes row floor(u*s / 2^32) with sign -1 if u is */
/* odd, +1 if even.  A proposal whose row is already taken in this column is   */
/* discarded.  The first zeta accepted proposals are the column's nonzeros, in */
/* acceptance order.                                                          */
/* ------------------------------------------------------------------------ */
void oracle_sketch_pattern(uint64_t seed, uint32_t cycle, int64_t i, int s, int zeta,
                           int32_t *rows, int8_t *signs) {
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int have = 0;
    for (uint32_t t = 0; have < zeta; ++t) {
        const uint32_t ctr[4] = {(uint32_t)(uint64_t)i, (uint32_t)((uint64_t)i >> 32), cycle, t};
        uint32_t w[4];
        oracle_philox4x32_10(ctr, key, w);
        for (int q = 0; q < 4 && have < zeta; ++q) {
            const int32_t row = (int32_t)(((uint64_t)w[q] * (uint64_t)s) >> 32);
            int dup = 0;
            for (int a = 0; a < have; ++a)
                if (rows[a] == row) dup = 1;
            if (dup) continue;
            rows[have] = row;
            signs[have] = (w[q] & 1u) ? (int8_t)-1 : (int8_t)1;
            ++have;
        }
    }
}

/* Unscaled sum over rows [i0, i1) of S[:, i] v[i] into acc (s entries, added
 * to), rows ascending and, inside a column, in acceptance order. */
static void sketch_rows(int64_t i0, int64_t i1, const double *v, uint64_t seed, uint32_t cycle, int s,
                        int zeta, int32_t *rows, int8_t *signs, double *acc) {
    for (int64_t i = i0; i < i1; ++i) {
        oracle_sketch_pattern(seed, cycle, i, s, zeta, rows, signs);
        for (int t = 0; t < zeta; ++t) acc[rows[t]] += (double)signs[t] * v[i];
    }
}

/* g = S v for v of length n, S = (1/sqrt(zeta)) [s_1 ... s_n]  (R-scale).
 * Each chunk of OR_CHUNK rows is accumulated on its own (sketch_rows); the
 * chunk sums are added in chunk order; the scale is applied once at the end. */
int oracle_sketch_apply(int64_t n, const double *v, uint64_t seed, uint32_t cycle, int s, int zeta,
                        double *g) {
    if (n < 0 || s < 1 || zeta < 1 || zeta > s) return OR_EINVAL;
    const int64_t nc = chunks_of(n);
    double *part = (double *)calloc((size_t)(nc > 0 ? nc : 1) * (size_t)s, sizeof(double));
    if (!part) return OR_ENOMEM;
    int bad = 0;
#pragma omp parallel num_threads(g_threads)
    {
        int32_t *rows = (int32_t *)malloc(sizeof(int32_t) * (size_t)zeta);
        int8_t *signs = (int8_t *)malloc((size_t)zeta);
        if (!rows || !signs) {
#pragma omp atomic write
            bad = 1;
        } else {
#pragma omp for schedule(static)
            for (int64_t c = 0; c < nc; ++c) {
                const int64_t i1 = (c + 1) * OR_CHUNK < n ? (c + 1) * OR_CHUNK : n;
                sketch_rows(c * OR_CHUNK, i1, v, seed, cycle, s, zeta, rows, signs, part + (size_t)c * s);
            }
        }
        free(rows);
        free(signs);
    }
    if (bad) {
        free(part);
        return OR_ENOMEM;
    }
    for (int r = 0; r < s; ++r) g[r] = 0.0;
    for (int64_t c = 0; c < nc; ++c)
        for (int r = 0; r < s; ++r) g[r] += part[(size_t)c * s + r];
    const double scale = 1.0 / sqrt((double)zeta);
    for (int r = 0; r < s; ++r) g[r] *= scale;
    free(part);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Matrix access x -> A x (the paper accesses A only through products).        */
/* ------------------------------------------------------------------------ */
void oracle_csr_spmv(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                     const double *x, double *y) {
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) acc += val[p] * x[col_idx[p]];
        y[i] = acc;
    }
}

/* Transpose a CSR matrix; entries of each output row come out in ascending
 * column order (= ascending row of the input). */
int oracle_csr_transpose(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                         const double *val, int32_t *t_row_ptr, int32_t *t_col_idx,
                         double *t_val) {
    const int64_t nnz = row_ptr[n];
    int32_t *fill = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    if (!fill) return OR_ENOMEM;
    for (int64_t i = 0; i <= n; ++i) t_row_ptr[i] = 0;
    for (int64_t p = 0; p < nnz; ++p) t_row_ptr[col_idx[p] + 1] += 1;
    for (int64_t i = 0; i < n; ++i) t_row_ptr[i + 1] += t_row_ptr[i];
    for (int64_t i = 0; i < n; ++i) {
        for (int32_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            const int32_t c = col_idx[p];
            const int32_t dst = t_row_ptr[c] + fill[c]++;
            t_col_idx[dst] = (int32_t)i;
            t_val[dst] = val[p];
        }
    }
    free(fill);
    return OR_OK;
}

/* sum_i a[i] b[i] in the fixed chunk order (chunk sums kept, then added in
 * chunk order; without memory for them the same sums are formed one chunk
 * after another, which gives the same bits). */
static double chunk_dot(int64_t i0, int64_t i1, const double *a, const double *b) {
    double acc = 0.0;
    for (int64_t i = i0; i < i1; ++i) acc += a[i] * b[i];
    return acc;
}

static double dot(int64_t n, const double *a, const double *b) {
    const int64_t nc = chunks_of(n);
    double *part = (double *)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
    double tot = 0.0;
    if (!part) {
        for (int64_t c = 0; c < nc; ++c)
            tot += chunk_dot(c * OR_CHUNK, (c + 1) * OR_CHUNK < n ? (c + 1) * OR_CHUNK : n, a, b);
        return tot;
    }
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (int64_t c = 0; c < nc; ++c)
        part[c] = chunk_dot(c * OR_CHUNK, (c + 1) * OR_CHUNK < n ? (c + 1) * OR_CHUNK : n, a, b);
    for (int64_t c = 0; c < nc; ++c) tot += part[c];
    free(part);
    return tot;
}

static int all_finite(int64_t n, const double *a) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

/* r = f - A x; returns |r|_2. */
double oracle_residual(int64_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                       const double *f, const double *x, double *r) {
    oracle_csr_spmv(n, row_ptr, col_idx, val, x, r);
    #pragma omp parallel for num_threads(g_threads) schedule(static)
    for (int64_t i = 0; i < n; ++i) r[i] = f[i] - r[i];
    return sqrt(dot(n, r, r));
}

/* ------------------------------------------------------------------------ */
/* One cycle of basis generation and sketching (Algorithm 1, lines 2-8).       */
/*                                                                            */
/* Inputs: residual r (|r| > 0), sketch key (seed, cycle).                    */
/* Outputs (column-major, caller-allocated):                                  */
/*   B   n x d   basis columns b_1..b_dc                                       */
/*   SB  s x d   S b_j                                                         */
/*   SAB s x d   S (A b_j)                                                     */
/*   H   (k+1) x d  column j: [h+h'] for the window (newest first), then nu   */
/*   g   s       S r                                                           */
/* Returns dc, the number of basis columns produced (dc < d after breakdown). */
/* passes = number of Gram-Schmidt passes (2 = the method; 1 is a test hook). */
/* ------------------------------------------------------------------------ */
int oracle_arnoldi_cycle(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                         const double *val, const double *r, int d, int k, int s, int zeta,
                         uint64_t seed, uint32_t cycle, int passes, double *B, double *SB,
                         double *SAB, double *H, double *g, int *flags) {
    if (n < 1 || d < 1 || k < 1 || s < 1 || zeta < 1 || zeta > s) return OR_EINVAL;
    const double u = 0x1.0p-53;
    double *m = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double *h = (double *)malloc(sizeof(double) * (size_t)k);
    double *hsum = (double *)malloc(sizeof(double) * (size_t)k);
    if (!m || !w || !h || !hsum) {
        free(m);
        free(w);
        free(h);
        free(hsum);
        return OR_ENOMEM;
    }
    for (int64_t q = 0; q < (int64_t)(k + 1) * d; ++q) H[q] = 0.0;

    /* g = S r; b_1 = r / |r| */
    oracle_sketch_apply(n, r, seed, cycle, s, zeta, g);
    const double beta = sqrt(dot(n, r, r));
    #pragma omp parallel for num_threads(g_threads) schedule(static)
    for (int64_t i = 0; i < n; ++i) B[i] = r[i] / beta;

    int dc = d;
    for (int j = 0; j < d; ++j) { /* 0-based: column j holds b_{j+1} */
        double *bj = B + (size_t)j * n;
        oracle_csr_spmv(n, row_ptr, col_idx, val, bj, m);
        oracle_sketch_apply(n, bj, seed, cycle, s, zeta, SB + (size_t)j * s);
        oracle_sketch_apply(n, m, seed, cycle, s, zeta, SAB + (size_t)j * s);
        if (j == d - 1) break;

        /* window W = [b_j, b_{j-1}, ..., b_{j-kw+1}] (R-window), newest first */
        const int kw = (j + 1 < k) ? j + 1 : k;
        memcpy(w, m, sizeof(double) * (size_t)n);
        for (int a = 0; a < kw; ++a) hsum[a] = 0.0;
        for (int pass = 0; pass < passes; ++pass) { /* R-cgs2: classical GS, twice */
            for (int a = 0; a < kw; ++a) h[a] = dot(n, B + (size_t)(j - a) * n, w);
            for (int a = 0; a < kw; ++a) {
                const double *wa = B + (size_t)(j - a) * n;
                #pragma omp parallel for num_threads(g_threads) schedule(static)
                for (int64_t i = 0; i < n; ++i) w[i] -= h[a] * wa[i];
                hsum[a] += h[a];
            }
        }
        const double nu = sqrt(dot(n, w, w));
        const double mnorm = sqrt(dot(n, m, m));
        for (int a = 0; a < kw; ++a) H[(size_t)j * (k + 1) + a] = hsum[a];
        H[(size_t)j * (k + 1) + k] = nu;
        if (!(nu > 4.0 * u * mnorm)) { /* R-break: Krylov space is invariant */
            dc = j + 1;
            *flags |= OR_FLAG_BREAKDOWN;
            break;
        }
        double *bn = B + (size_t)(j + 1) * n;
        #pragma omp parallel for num_threads(g_threads) schedule(static)
        for (int64_t i = 0; i < n; ++i) bn[i] = w[i] / nu;
    }
    free(m);
    free(w);
    free(h);
    free(hsum);
    return dc;
}

/* ------------------------------------------------------------------------ */
/* One cycle of the shifted-and-scaled Chebyshev basis (Section 4.4) with      */
/* sketching (R-cheb).  The spectrum of A lies in the box [c - dx, c + dx] x   */
/* [-dy, dy]; rho = max(dx, dy).  The recurrence, in the paper's scaling:      */
/*   b_1 = r / |r|,   b_2 = (A - c I) b_1 / (2 rho),                           */
/*   b_j = [ (A - c I) b_{j-1} - (dx^2 - dy^2) / (4 rho) b_{j-2} ] / rho.      */
/* Outputs (column-major, caller-allocated):                                  */
/*   B   n x d   normalised columns b_j / |b_j|                                */
/*   SB  s x d   S of the normalised columns                                   */
/*   SAB s x d   S (A times the normalised columns)                            */
/*   nrm d       |b_j| of the unnormalised recurrence vectors                  */
/*   g   s       S r                                                           */
/* The unnormalised vectors shrink like 2^(1-j) for an interval box, so d is   */
/* limited to where they stay normal numbers (d of a few hundred).             */
/* ------------------------------------------------------------------------ */
int oracle_chebyshev_cycle(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                           const double *val, const double *r, int d, int s, int zeta,
                           uint64_t seed, uint32_t cycle, double c, double dx, double dy,
                           double *B, double *SB, double *SAB, double *nrm, double *g) {
    if (n < 1 || d < 1 || s < 1 || zeta < 1 || zeta > s || !(dx >= 0.0) || !(dy >= 0.0)) return OR_EINVAL;
    const double rho = dx > dy ? dx : dy;
    if (!(rho > 0.0)) return OR_EINVAL;
    double *prev = (double *)calloc((size_t)n, sizeof(double)); /* b_{j-2} */
    double *cur = (double *)malloc(sizeof(double) * (size_t)n);  /* b_{j-1} */
    double *nxt = (double *)malloc(sizeof(double) * (size_t)n);  /* b_j */
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    if (!prev || !cur || !nxt || !t) {
        free(prev);
        free(cur);
        free(nxt);
        free(t);
        return OR_ENOMEM;
    }
    oracle_sketch_apply(n, r, seed, cycle, s, zeta, g);
    const double beta = sqrt(dot(n, r, r));
    const double qcoef = (dx * dx - dy * dy) / (4.0 * rho);
    for (int j = 0; j < d; ++j) { /* 0-based: this iteration forms b_{j+1} */
        if (j == 0) {
            #pragma omp parallel for num_threads(g_threads) schedule(static)
            for (int64_t i = 0; i < n; ++i) nxt[i] = r[i] / beta;
        } else {
            oracle_csr_spmv(n, row_ptr, col_idx, val, cur, t); /* t = A b_{j} (1-based j) */
            #pragma omp parallel for num_threads(g_threads) schedule(static)
            for (int64_t i = 0; i < n; ++i) t[i] -= c * cur[i];
            if (j == 1) {
                #pragma omp parallel for num_threads(g_threads) schedule(static)
                for (int64_t i = 0; i < n; ++i) nxt[i] = t[i] / (2.0 * rho);
            } else {
                #pragma omp parallel for num_threads(g_threads) schedule(static)
                for (int64_t i = 0; i < n; ++i) nxt[i] = (t[i] - qcoef * prev[i]) / rho;
            }
        }
        /* normalised copy into B (the recurrence keeps the raw vector) */
        const double nj = sqrt(dot(n, nxt, nxt));
        nrm[j] = nj;
        double *bj = B + (size_t)j * n;
        #pragma omp parallel for num_threads(g_threads) schedule(static)
        for (int64_t i = 0; i < n; ++i) bj[i] = nj > 0.0 ? nxt[i] / nj : 0.0;
        oracle_csr_spmv(n, row_ptr, col_idx, val, bj, t);
        oracle_sketch_apply(n, bj, seed, cycle, s, zeta, SB + (size_t)j * s);
        oracle_sketch_apply(n, t, seed, cycle, s, zeta, SAB + (size_t)j * s);
        double *tmp = prev;
        prev = cur;
        cur = nxt;
        nxt = tmp;
    }
    free(prev);
    free(cur);
    free(nxt);
    free(t);
    return d;
}

/* ------------------------------------------------------------------------ */
/* Sketched least squares, Algorithm 1 lines 9-13 and Section 3.3.             */
/*                                                                            */
/* C (s x dc, column-major, leading dim s) is overwritten by its Householder   */
/* factorisation: T in the upper triangle, reflector tails below it.  g (s) is */
/* overwritten by Q^T g.  On return y[0..d_eff) solves T[:d_eff,:d_eff] y =    */
/* (Q^T g)[:d_eff]; *rest = |(Q^T g)[d_eff:s]| (= r_est of eq. sgmres-rhat for */
/* the prefix); *kappa = kappa_est(d_eff).                                     */
/* ------------------------------------------------------------------------ */
int oracle_sketched_lsq(int s, int dc, double *C, double *g, double kappa_max, double *y,
                        double *tau, int *d_eff_out, double *rest, double *kappa, int *flags) {
    if (s < 1 || dc < 0 || dc > s) return OR_EINVAL;
    for (int p = 0; p < dc; ++p) {
        double *cp = C + (size_t)p * s;
        const double alpha = cp[p];
        double xn2 = 0.0;
        for (int i = p + 1; i < s; ++i) xn2 += cp[i] * cp[i];
        double beta, t;
        if (xn2 == 0.0) { /* H = I (LAPACK dlarfg convention) */
            t = 0.0;
            beta = alpha;
        } else {
            const double nrm = sqrt(alpha * alpha + xn2);
            beta = (alpha >= 0.0) ? -nrm : nrm; /* beta = -sign(alpha)|x|, sign(0) = + */
            t = (beta - alpha) / beta;
            const double sc = 1.0 / (alpha - beta);
            for (int i = p + 1; i < s; ++i) cp[i] *= sc;
        }
        cp[p] = beta;
        tau[p] = t;
        if (t != 0.0) {
            /* apply I - t v v^T (v = [1; cp[p+1:s]]) to trailing columns and g */
            for (int c = p + 1; c < dc; ++c) {
                double *cc = C + (size_t)c * s;
                double sdot = cc[p];
                for (int i = p + 1; i < s; ++i) sdot += cp[i] * cc[i];
                sdot *= t;
                cc[p] -= sdot;
                for (int i = p + 1; i < s; ++i) cc[i] -= sdot * cp[i];
            }
            double sdot = g[p];
            for (int i = p + 1; i < s; ++i) sdot += cp[i] * g[i];
            sdot *= t;
            g[p] -= sdot;
            for (int i = p + 1; i < s; ++i) g[i] -= sdot * cp[i];
        }
    }
    /* R-kappa: longest prefix whose diagonal ratio stays within kappa_max */
    int d_eff = 0;
    double tmax = 0.0, tmin = INFINITY, kap = 0.0;
    for (int j = 0; j < dc; ++j) {
        const double a = fabs(C[(size_t)j * s + j]);
        const double nmax = a > tmax ? a : tmax;
        const double nmin = a < tmin ? a : tmin;
        if (!(nmin > 0.0) || nmax / nmin > kappa_max) break;
        tmax = nmax;
        tmin = nmin;
        kap = tmax / tmin;
        d_eff = j + 1;
    }
    if (d_eff < dc) *flags |= OR_FLAG_KAPPA_TRUNC;
    /* back substitution T y = z */
    for (int i = d_eff - 1; i >= 0; --i) {
        double acc = g[i];
        for (int c = i + 1; c < d_eff; ++c) acc -= C[(size_t)c * s + i] * y[c];
        y[i] = acc / C[(size_t)i * s + i];
    }
    double rr = 0.0;
    for (int i = d_eff; i < s; ++i) rr += g[i] * g[i];
    *rest = sqrt(rr);
    *kappa = kap;
    *d_eff_out = d_eff;
    return OR_OK;
}

/* x <- x + B[:, :d_eff] y   (R-soln) */
void oracle_basis_combine(int64_t n, int d_eff, const double *B, const double *y, double *x) {
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int c = 0; c < d_eff; ++c) acc += B[(size_t)c * n + i] * y[c];
        x[i] += acc;
    }
}

/* ------------------------------------------------------------------------ */
/* Restarted sGMRES (Algorithm 1 per cycle; restarts of Section 3.5).          */
/*                                                                            */
/* x is in/out (initial guess on entry).  Stops when |b - A x|/|b| <= tol      */
/* (R-tol) or after restarts+1 cycles.  info (nullable, 8 doubles):            */
/*   [0] cycles run  [1] total basis columns  [2] d_eff of the last cycle      */
/*   [3] flags (OR of all cycles)  [4] final relative residual                 */
/*   [5] last r_est / |b|  [6] last kappa_est  [7] unused                      */
/* ------------------------------------------------------------------------ */
/* basis: 0 = k-truncated Arnoldi; 1 = Chebyshev for the box (c, dx, dy), k unused. */
int oracle_sgmres_solve_basis(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                              const double *val, const double *b, double *x, int d, int k, int s,
                              int zeta, uint64_t seed, double tol, int restarts, double kappa_max,
                              int basis, double c, double dx, double dy, double *info) {
    if (n < 1 || d < 1 || d > n || k < 1 || s < d + 1 || zeta < 1 || zeta > s || !(tol >= 0.0) ||
        restarts < 0 || (basis != 0 && basis != 1))
        return OR_EINVAL;
    double stat[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int flags = 0;
    if (!all_finite(n, b) || !all_finite(n, x) || !all_finite(row_ptr[n], val)) return OR_ENONFINITE;
    const double nf = sqrt(dot(n, b, b));
    if (nf == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        if (info) memcpy(info, stat, sizeof stat);
        return OR_OK;
    }
    const int kk = k > d - 1 ? (d - 1 > 0 ? d - 1 : 1) : k;
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *B = (double *)malloc(sizeof(double) * (size_t)n * d);
    double *SB = (double *)malloc(sizeof(double) * (size_t)s * d);
    double *SAB = (double *)malloc(sizeof(double) * (size_t)s * d);
    double *H = (double *)malloc(sizeof(double) * (size_t)(kk + 1) * d);
    double *nrm = (double *)malloc(sizeof(double) * (size_t)d);
    double *g = (double *)malloc(sizeof(double) * (size_t)s);
    double *y = (double *)malloc(sizeof(double) * (size_t)d);
    double *tau = (double *)malloc(sizeof(double) * (size_t)d);
    int rc = OR_OK;
    if (!r || !B || !SB || !SAB || !H || !nrm || !g || !y || !tau) {
        rc = OR_ENOMEM;
        goto done;
    }
    double rho = 0.0;
    int cycles = 0;
    for (;;) {
        const double beta = oracle_residual(n, row_ptr, col_idx, val, b, x, r);
        if (!isfinite(beta)) {
            rc = OR_ENONFINITE;
            break;
        }
        rho = beta / nf;
        if (rho <= tol) {
            rc = OR_OK;
            break;
        }
        if (cycles > restarts) {
            rc = OR_NOT_CONVERGED;
            break;
        }
        const int dc = basis == 0 ? oracle_arnoldi_cycle(n, row_ptr, col_idx, val, r, d, kk, s, zeta, seed,
                                                         (uint32_t)cycles, 2, B, SB, SAB, H, g, &flags)
                                  : oracle_chebyshev_cycle(n, row_ptr, col_idx, val, r, d, s, zeta, seed,
                                                           (uint32_t)cycles, c, dx, dy, B, SB, SAB, nrm, g);
        if (dc < 0) {
            rc = dc;
            break;
        }
        int d_eff = 0;
        double rest = 0.0, kap = 0.0;
        oracle_sketched_lsq(s, dc, SAB, g, kappa_max, y, tau, &d_eff, &rest, &kap, &flags);
        oracle_basis_combine(n, d_eff, B, y, x);
        ++cycles;
        stat[1] += dc;
        stat[2] = d_eff;
        stat[5] = rest / nf;
        stat[6] = kap;
    }
    stat[0] = cycles;
    stat[3] = flags;
    stat[4] = rho;
    if (info) memcpy(info, stat, sizeof stat);
done:
    free(r);
    free(B);
    free(SB);
    free(SAB);
    free(H);
    free(nrm);
    free(g);
    free(y);
    free(tau);
    return rc;
}

int oracle_sgmres_solve(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                        const double *val, const double *b, double *x, int d, int k, int s,
                        int zeta, uint64_t seed, double tol, int restarts, double kappa_max,
                        double *info) {
    return oracle_sgmres_solve_basis(n, row_ptr, col_idx, val, b, x, d, k, s, zeta, seed, tol, restarts,
                                     kappa_max, 0, 0.0, 0.0, 0.0, info);
}

/* Solve A^T x = b: transpose once, then the same restarted method. */
int oracle_sgmres_solve_transposed(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                                   const double *val, const double *b, double *x, int d, int k,
                                   int s, int zeta, uint64_t seed, double tol, int restarts,
                                   double kappa_max, double *info) {
    if (n < 1) return OR_EINVAL;
    const int64_t nnz = row_ptr[n];
    int32_t *trp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *tci = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    double *tv = (double *)malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    int rc = OR_ENOMEM;
    if (trp && tci && tv) {
        rc = oracle_csr_transpose(n, row_ptr, col_idx, val, trp, tci, tv);
        if (rc == OR_OK)
            rc = oracle_sgmres_solve(n, trp, tci, tv, b, x, d, k, s, zeta, seed, tol, restarts,
                                     kappa_max, info);
    }
    free(trp);
    free(tci);
    free(tv);
    return rc;
}

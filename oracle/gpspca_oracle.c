/*
 * FP64 reference ("oracle") of the generalized power method for sparse PCA
 * (GP-SPCA), all four formulations of Table 1 of the paper: single-unit L1
 * (SL1), single-unit L0 (SL0), block L1 (BL1) and block L0 (BL0), plus the
 * other reading of the block-L1 row (BL1X, below).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into its own shared
 * library and is used by the tests, the smoke check and the CPU-baseline leg
 * of the benchmark.  It shares no source, header, table or helper with the
 * GPU library, and the GPU library never calls it.
 *
 * Everything is plain double-precision loops in the order of the method:
 *   pass:    y_ij = a_i^T x_j                        (Table 1, a_i^T x terms)
 *            threshold  (soft for l1, hard for l0)   (Table 1; t_+ = max(0,t))
 *            g_j = mu_j * sum_i s_ij a_i             (gradient of the Table 1
 *                                                     reformulation, up to a
 *                                                     uniform factor 2)
 *   retract: x = g/||g|| on the sphere (m = 1), polar factor on the Stiefel
 *            manifold (block forms)                  (Section 2, feasible sets)
 *
 * The iteration itself is not printed in the paper; it is the power method
 * for a convex function over the sphere or the Stiefel manifold (Section 2):
 * the next iterate maximizes the linearization <grad F(X_k), Y> over the
 * feasible set, which is the normalized gradient on the sphere and the polar
 * factor of the gradient on the Stiefel manifold.
 *
 * Readings where the paper is silent or garbled (all listed in the design
 * notes):
 *  - the block-L1 reformulation is read with the bracket squared, so that
 *    m = 1, mu = 1 reduces to the single-unit L1 row of Table 1;
 *  - BL1X is the block-L1 row read from its original form instead: for fixed
 *    X the maximum over unit-norm z_j of mu_j x_j^T A z_j - gamma ||z_j||_1 is
 *    ||s_j|| (s_ij the soft-thresholded correlation), so the objective is
 *    F = sum_j ||s_j|| and its gradient in x_j is mu_j A s_j / ||s_j||: the
 *    pass of BL1 with column j of G divided by ||s_j||, and F summed from the
 *    square roots of the per-component terms;
 *  - the block-L0 row is read with x_j for x;
 *  - the Stiefel manifold is read in R^{p x m};
 *  - gamma_j = gamma for every component;
 *  - thresholds are strict (t > 0, q > 0) and sign(0) = 0;
 *  - components whose thresholded column is empty ("dead") are completed by
 *    the polar factor of the previous iterate's columns projected off the
 *    live part, and the run is flagged degenerate;
 *  - stopping: F_k = 0, or k >= 1 and |F_k - F_{k-1}| < tol*|F_{k-1}|, or
 *    k + 1 = max_iter; the returned triple (X_k, Z(X_k), F_k) is consistent.
 *
 * Reductions over columns run in fixed chunks of ORC_CHUNK columns that are
 * added in chunk order, so results do not depend on the OpenMP thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_SL1 0
#define ORC_SL0 1
#define ORC_BL1 2
#define ORC_BL0 3
#define ORC_BL1X 4

#define ORC_OK 0
#define ORC_MAXITER 1
#define ORC_DEGENERATE 2
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-3)
#define ORC_ENONFINITE (-5)

#define ORC_CHUNK 1024

static int is_l0(int form) { return form == ORC_SL0 || form == ORC_BL0; }
static int is_block(int form) { return form == ORC_BL1 || form == ORC_BL0 || form == ORC_BL1X; }

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* Euclidean norm of every column a_i (used by the default initialization). */
int orc_column_norms(const double* A, int64_t p, int64_t n, int64_t lda, double* c) {
    if (!A || !c || p < 1 || n < 1 || lda < p) return ORC_EINVAL;
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t r = 0; r < p; ++r) s += A[i * lda + r] * A[i * lda + r];
        c[i] = sqrt(s);
    }
    return ORC_OK;
}

/* Indices of the m largest entries of c, ordered by (-c_i, i): ties go to the
 * lower index.  Plain selection: m rounds of a linear scan. */
int orc_top_m(const double* c, int64_t n, int m, int64_t* idx) {
    if (!c || !idx || m < 1 || m > n) return ORC_EINVAL;
    unsigned char* taken = (unsigned char*)calloc((size_t)n, 1);
    if (!taken) return ORC_ENOMEM;
    for (int k = 0; k < m; ++k) {
        int64_t best = -1;
        for (int64_t i = 0; i < n; ++i) {
            if (taken[i]) continue;
            if (best < 0 || c[i] > c[best]) best = i;
        }
        taken[best] = 1;
        idx[k] = best;
    }
    free(taken);
    return ORC_OK;
}

/*
 * Polar factor X = U V^T of a p x m matrix G (column-major, leading dim p) by
 * the one-sided Jacobi SVD (Hestenes): plane rotations applied to pairs of
 * columns until every pair is orthogonal, accumulating V.  Then the columns
 * are W = U Sigma, and X = U V^T.
 *
 * sv (optional, m entries) receives the singular values.  *rank_def is set
 * when sigma_min <= m * eps * sigma_max (the polar factor is then not unique).
 */
int orc_polar(const double* G, int64_t p, int m, double* X, double* sv, int* rank_def) {
    if (!G || !X || p < 1 || m < 1 || m > p) return ORC_EINVAL;
    double* W = (double*)malloc(sizeof(double) * (size_t)(p * m));
    double* V = (double*)calloc((size_t)(m * m), sizeof(double));
    double* s = (double*)malloc(sizeof(double) * (size_t)m);
    if (!W || !V || !s) { free(W); free(V); free(s); return ORC_ENOMEM; }
    memcpy(W, G, sizeof(double) * (size_t)(p * m));
    for (int j = 0; j < m; ++j) V[j * m + j] = 1.0;

    const double eps = 2.220446049250313e-16;
    for (int sweep = 0; sweep < 80; ++sweep) {
        int rotated = 0;
        for (int j = 0; j < m - 1; ++j) {
            for (int k = j + 1; k < m; ++k) {
                double* wj = W + (int64_t)j * p;
                double* wk = W + (int64_t)k * p;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int64_t r = 0; r < p; ++r) {
                    al += wj[r] * wj[r];
                    be += wk[r] * wk[r];
                    ga += wj[r] * wk[r];
                }
                if (ga == 0.0 || fabs(ga) <= eps * sqrt(al * be)) continue;
                rotated = 1;
                double zeta = (be - al) / (2.0 * ga);
                double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double cs = 1.0 / sqrt(1.0 + t * t);
                double sn = cs * t;
                for (int64_t r = 0; r < p; ++r) {
                    double a = wj[r], b = wk[r];
                    wj[r] = cs * a - sn * b;
                    wk[r] = sn * a + cs * b;
                }
                for (int r = 0; r < m; ++r) {
                    double a = V[j * m + r], b = V[k * m + r];
                    V[j * m + r] = cs * a - sn * b;
                    V[k * m + r] = sn * a + cs * b;
                }
            }
        }
        if (!rotated) break;
    }
    double smax = 0.0, smin = INFINITY;
    for (int j = 0; j < m; ++j) {
        double q = 0.0;
        for (int64_t r = 0; r < p; ++r) q += W[(int64_t)j * p + r] * W[(int64_t)j * p + r];
        s[j] = sqrt(q);
        if (s[j] > smax) smax = s[j];
        if (s[j] < smin) smin = s[j];
    }
    if (rank_def) *rank_def = (smin <= (double)m * eps * smax) ? 1 : 0;
    /* X = U V^T with U_j = W_j / s_j. */
    for (int64_t r = 0; r < p; ++r) {
        for (int c = 0; c < m; ++c) {
            double acc = 0.0;
            for (int j = 0; j < m; ++j) {
                double u = s[j] > 0.0 ? W[(int64_t)j * p + r] / s[j] : 0.0;
                acc += u * V[j * m + c];
            }
            X[(int64_t)c * p + r] = acc;
        }
    }
    if (sv) memcpy(sv, s, sizeof(double) * (size_t)m);
    free(W); free(V); free(s);
    return ORC_OK;
}

/* Threshold of one correlation y for component weight mu (Table 1).
 * l1: t = mu|y| - gamma; active iff t > 0; s = sign(y) t; objective += t^2.
 * l0: q = (mu y)^2 - gamma; active iff q > 0; s = mu y;  objective += q.   */
static int threshold(int l0, double mu, double gamma, double y, double* s, double* f) {
    if (l0) {
        double q = (mu * y) * (mu * y) - gamma;
        if (q > 0.0) { *s = mu * y; *f = q; return 1; }
    } else {
        double t = mu * fabs(y) - gamma;
        if (t > 0.0) { *s = (y > 0.0) ? t : (y < 0.0 ? -t : 0.0); *f = t * t; return 1; }
    }
    *s = 0.0; *f = 0.0;
    return 0;
}

/*
 * One pass of the power iteration at X (p x m, column-major, leading dim p).
 * Outputs (any may be NULL except G and f):
 *   Y   n x m correlations a_i^T x_j          (column-major, leading dim n)
 *   S   n x m thresholded correlations         (column-major, leading dim n)
 *   G   p x m gradient direction, G = A S N    (column-major, leading dim p)
 *   f   m per-component objective terms; F = sum_j f_j
 *   nnz m per-component support sizes
 * mask (n x m, may be NULL) restricts the pass to a frozen support: where
 * mask[j*n + i] == 0 the thresholded value is forced to 0 (refinement on a
 * support found by a reduced-precision run).
 */
int orc_pass(const double* A, int64_t p, int64_t n, int64_t lda, int form, int m,
             double gamma, const double* mu, const double* X, const unsigned char* mask,
             double* Y, double* S, double* G, double* f, int64_t* nnz) {
    if (!A || !X || !G || !f || p < 1 || n < 1 || lda < p || m < 1) return ORC_EINVAL;
    const int l0 = is_l0(form);
    const int64_t nch = (n + ORC_CHUNK - 1) / ORC_CHUNK;
    double* Gc = (double*)calloc((size_t)(nch * p * m), sizeof(double));
    double* fc = (double*)calloc((size_t)(nch * m), sizeof(double));
    int64_t* nc = (int64_t*)calloc((size_t)(nch * m), sizeof(int64_t));
    if (!Gc || !fc || !nc) { free(Gc); free(fc); free(nc); return ORC_ENOMEM; }

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t c = 0; c < nch; ++c) {
        double* yv = (double*)malloc(sizeof(double) * (size_t)m);
        double* gc = Gc + c * p * m;
        const int64_t i0 = c * ORC_CHUNK, i1 = (i0 + ORC_CHUNK < n) ? i0 + ORC_CHUNK : n;
        for (int64_t i = i0; i < i1; ++i) {
            const double* a = A + i * lda;
            for (int j = 0; j < m; ++j) yv[j] = 0.0;
            for (int64_t r = 0; r < p; ++r)
                for (int j = 0; j < m; ++j) yv[j] += a[r] * X[(int64_t)j * p + r];
            for (int j = 0; j < m; ++j) {
                const double muj = mu ? mu[j] : 1.0;
                double s, fj;
                int act = threshold(l0, muj, gamma, yv[j], &s, &fj);
                if (mask && !mask[(int64_t)j * n + i]) { act = 0; s = 0.0; }
                if (Y) Y[(int64_t)j * n + i] = yv[j];
                if (S) S[(int64_t)j * n + i] = s;
                if (act) {
                    fc[c * m + j] += fj;
                    nc[c * m + j] += 1;
                    const double w = muj * s;
                    for (int64_t r = 0; r < p; ++r) gc[(int64_t)j * p + r] += w * a[r];
                }
            }
        }
        free(yv);
    }
    memset(G, 0, sizeof(double) * (size_t)(p * m));
    for (int j = 0; j < m; ++j) { f[j] = 0.0; if (nnz) nnz[j] = 0; }
    for (int64_t c = 0; c < nch; ++c) {
        for (int64_t e = 0; e < p * m; ++e) G[e] += Gc[c * p * m + e];
        for (int j = 0; j < m; ++j) {
            f[j] += fc[c * m + j];
            if (nnz) nnz[j] += nc[c * m + j];
        }
    }
    free(Gc); free(fc); free(nc);
    return ORC_OK;
}

/*
 * BL1X (original form of the block-L1 row): objective and ascent direction
 * from the pass's per-component terms f_j = ||s_j||^2.  Returns
 * F = sum_j sqrt(f_j) and divides column j of G (p x m) by sqrt(f_j) where
 * f_j > 0 (an empty column stays 0: a dead component).
 */
double orc_bl1x_direction(int64_t p, int m, const double* f, double* G) {
    double F = 0.0;
    for (int j = 0; j < m; ++j) {
        if (!(f[j] > 0.0)) continue;
        const double nr = sqrt(f[j]);
        F += nr;
        for (int64_t r = 0; r < p; ++r) G[(int64_t)j * p + r] /= nr;
    }
    return F;
}

/*
 * Retraction of the gradient direction G onto the feasible set.
 *  m = 1 (single-unit): x = g / ||g||.
 *  block: X = polar(G) when every component is live.  With dead components
 *  (nnz_j = 0, so g_j = 0), X_L = polar(G_L) on the live set and
 *  X_D = polar(H) with H = X_k[:,D] - X_L (X_L^T X_k[:,D]); this is still a
 *  maximizer of <G, Y> over the Stiefel manifold.
 * *degenerate is set when dead components were completed or G is rank
 * deficient.  Requires at least one live component.
 */
int orc_retract(int64_t p, int m, const double* G, const int64_t* nnz, const double* Xk,
                double* Xn, int* degenerate) {
    if (!G || !Xn || p < 1 || m < 1) return ORC_EINVAL;
    *degenerate = 0;
    if (m == 1) {
        double s = 0.0;
        for (int64_t r = 0; r < p; ++r) s += G[r] * G[r];
        double nr = sqrt(s);
        if (!(nr > 0.0)) return ORC_EINVAL;
        for (int64_t r = 0; r < p; ++r) Xn[r] = G[r] / nr;
        return ORC_OK;
    }
    int nl = 0;
    for (int j = 0; j < m; ++j) nl += (nnz[j] > 0);
    if (nl == 0) return ORC_EINVAL;
    int rank_def = 0;
    if (nl == m) {
        int rc = orc_polar(G, p, m, Xn, NULL, &rank_def);
        *degenerate = rank_def;
        return rc;
    }
    const int nd = m - nl;
    double* GL = (double*)malloc(sizeof(double) * (size_t)(p * nl));
    double* XL = (double*)malloc(sizeof(double) * (size_t)(p * nl));
    double* H = (double*)malloc(sizeof(double) * (size_t)(p * nd));
    double* XD = (double*)malloc(sizeof(double) * (size_t)(p * nd));
    if (!GL || !XL || !H || !XD) { free(GL); free(XL); free(H); free(XD); return ORC_ENOMEM; }
    int a = 0, b = 0;
    for (int j = 0; j < m; ++j) {
        if (nnz[j] > 0) memcpy(GL + (int64_t)(a++) * p, G + (int64_t)j * p, sizeof(double) * (size_t)p);
        else memcpy(H + (int64_t)(b++) * p, Xk + (int64_t)j * p, sizeof(double) * (size_t)p);
    }
    int rc = orc_polar(GL, p, nl, XL, NULL, &rank_def);
    if (rc == ORC_OK) {
        /* H = X_D - X_L (X_L^T X_D), column by column from the previous iterate. */
        b = 0;
        for (int j = 0; j < m; ++j) {
            if (nnz[j] > 0) continue;
            const double* xd = Xk + (int64_t)j * p;
            double* h = H + (int64_t)(b++) * p;
            for (int64_t r = 0; r < p; ++r) h[r] = xd[r];
            for (int l = 0; l < nl; ++l) {
                const double* xl = XL + (int64_t)l * p;
                double c = 0.0;
                for (int64_t r = 0; r < p; ++r) c += xl[r] * xd[r];
                for (int64_t r = 0; r < p; ++r) h[r] -= c * xl[r];
            }
        }
        int rd2 = 0;
        rc = orc_polar(H, p, nd, XD, NULL, &rd2);
        a = 0; b = 0;
        for (int j = 0; j < m; ++j) {
            const double* src = (nnz[j] > 0) ? XL + (int64_t)(a++) * p : XD + (int64_t)(b++) * p;
            memcpy(Xn + (int64_t)j * p, src, sizeof(double) * (size_t)p);
        }
        *degenerate = 1;
    }
    free(GL); free(XL); free(H); free(XD);
    return rc;
}

/* Project a starting point onto the feasible set: x0/||x0|| (m = 1) or the
 * polar factor (block).  Rank-deficient starting points are rejected. */
int orc_project(int64_t p, int m, const double* X0, double* X) {
    if (!X0 || !X || p < 1 || m < 1 || m > p) return ORC_EINVAL;
    if (m == 1) {
        double s = 0.0;
        for (int64_t r = 0; r < p; ++r) s += X0[r] * X0[r];
        if (!(s > 0.0) || !isfinite(s)) return ORC_EINVAL;
        double nr = sqrt(s);
        for (int64_t r = 0; r < p; ++r) X[r] = X0[r] / nr;
        return ORC_OK;
    }
    int rd = 0;
    int rc = orc_polar(X0, p, m, X, NULL, &rd);
    if (rc != ORC_OK) return rc;
    return rd ? ORC_EINVAL : ORC_OK;
}

/* Default starting point: the m columns of largest norm (ties to the lower
 * index), projected onto the feasible set. */
int orc_init(const double* A, int64_t p, int64_t n, int64_t lda, int m, double* X, int64_t* idx_out) {
    if (!A || !X || m < 1 || m > n || m > p) return ORC_EINVAL;
    double* c = (double*)malloc(sizeof(double) * (size_t)n);
    int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
    double* X0 = (double*)malloc(sizeof(double) * (size_t)(p * m));
    if (!c || !idx || !X0) { free(c); free(idx); free(X0); return ORC_ENOMEM; }
    int rc = orc_column_norms(A, p, n, lda, c);
    if (rc == ORC_OK) rc = orc_top_m(c, n, m, idx);
    if (rc == ORC_OK) {
        for (int j = 0; j < m; ++j)
            memcpy(X0 + (int64_t)j * p, A + idx[j] * lda, sizeof(double) * (size_t)p);
        rc = orc_project(p, m, X0, X);
        if (idx_out) memcpy(idx_out, idx, sizeof(int64_t) * (size_t)m);
    }
    free(c); free(idx); free(X0);
    return rc;
}

/*
 * Full solve.  Inputs: A (p x n, column-major, leading dim lda), form, m,
 * gamma (absolute), mu (m weights, NULL = all 1; ignored by single-unit
 * forms), X0 (p x m or NULL for the default start), tol, max_iter.
 * Outputs: X (p x m) = X_k at the stopping pass; Z (n x m, unit-norm columns
 * or 0); support (n x m bytes, 1 where s_ij != 0); trace (max_iter entries,
 * F_0..F_k); *n_iter = k + 1.  Returns the status.
 */
int orc_solve(const double* A, int64_t p, int64_t n, int64_t lda, int form, int m,
              double gamma, const double* mu, const double* X0, const unsigned char* mask,
              double tol, int max_iter,
              double* X, double* Z, unsigned char* support, double* trace, int* n_iter) {
    if (!A || !X || !trace || !n_iter) return ORC_EINVAL;
    if (p < 1 || n < 1 || lda < p) return ORC_EINVAL;
    if (form < 0 || form > 4) return ORC_EINVAL;
    if (!is_block(form) && m != 1) return ORC_EINVAL;
    if (m < 1 || m > p) return ORC_EINVAL;
    if (!(gamma >= 0.0) || !isfinite(gamma)) return ORC_EINVAL;
    if (!(tol >= 0.0) || !isfinite(tol) || max_iter < 1) return ORC_EINVAL;
    double* muv = (double*)malloc(sizeof(double) * (size_t)m);
    if (!muv) return ORC_ENOMEM;
    for (int j = 0; j < m; ++j) {
        muv[j] = (is_block(form) && mu) ? mu[j] : 1.0;
        if (!(muv[j] > 0.0) || !isfinite(muv[j])) { free(muv); return ORC_EINVAL; }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t r = 0; r < p; ++r)
            if (!isfinite(A[i * lda + r])) { free(muv); return ORC_ENONFINITE; }

    double* Xk = (double*)malloc(sizeof(double) * (size_t)(p * m));
    double* Xn = (double*)malloc(sizeof(double) * (size_t)(p * m));
    double* G = (double*)malloc(sizeof(double) * (size_t)(p * m));
    double* S = (double*)malloc(sizeof(double) * (size_t)(n * m));
    double* f = (double*)malloc(sizeof(double) * (size_t)m);
    int64_t* nnz = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
    int rc = ORC_OK;
    if (!Xk || !Xn || !G || !S || !f || !nnz) { rc = ORC_ENOMEM; goto done; }

    if (X0) rc = orc_project(p, m, X0, Xk);
    else rc = orc_init(A, p, n, lda, m, Xk, NULL);
    if (rc != ORC_OK) goto done;

    int degenerate_seen = 0, converged = 0, k = 0;
    for (k = 0; k < max_iter; ++k) {
        rc = orc_pass(A, p, n, lda, form, m, gamma, muv, Xk, mask, NULL, S, G, f, nnz);
        if (rc != ORC_OK) goto done;
        double F = 0.0;
        if (form == ORC_BL1X) F = orc_bl1x_direction(p, m, f, G);
        else for (int j = 0; j < m; ++j) F += f[j];
        trace[k] = F;
        if (F == 0.0) { degenerate_seen = 1; break; }
        if (k >= 1 && fabs(F - trace[k - 1]) < tol * fabs(trace[k - 1])) { converged = 1; break; }
        if (k + 1 == max_iter) break;
        int deg = 0;
        rc = orc_retract(p, m, G, nnz, Xk, Xn, &deg);
        if (rc != ORC_OK) goto done;
        degenerate_seen |= deg;
        double* t = Xk; Xk = Xn; Xn = t;
    }
    if (k == max_iter) k = max_iter - 1;
    *n_iter = k + 1;
    memcpy(X, Xk, sizeof(double) * (size_t)(p * m));
    for (int j = 0; j < m; ++j) {
        double q = 0.0;
        for (int64_t i = 0; i < n; ++i) q += S[(int64_t)j * n + i] * S[(int64_t)j * n + i];
        double nr = sqrt(q);
        for (int64_t i = 0; i < n; ++i) {
            double s = S[(int64_t)j * n + i];
            if (Z) Z[(int64_t)j * n + i] = nr > 0.0 ? s / nr : 0.0;
            if (support) support[(int64_t)j * n + i] = (s != 0.0);
        }
    }
    if (degenerate_seen) rc = ORC_DEGENERATE;
    else if (!converged) rc = ORC_MAXITER;
    else rc = ORC_OK;
done:
    free(muv); free(Xk); free(Xn); free(G); free(S); free(f); free(nnz);
    return rc;
}

/* ------------------------------------------------------------------------
 * Reduced-precision storage of A (test reference for the quantized path).
 *
 * The paper computes in full precision; storing A in 16 or 8 bits is an
 * extension whose readings are:
 *  - bfloat16: the FP32 value rounded to 8 significant bits, ties to the even
 *    significand (subnormal FP32 values round to multiples of 2^-133, the
 *    bfloat16 subnormal spacing); column scale 1.
 *  - OCP float8 e4m3fn (4 exponent bits, bias 7, 3 mantissa bits, no
 *    infinities, largest finite 448, smallest normal 2^-6, subnormal spacing
 *    2^-9): column i is scaled by scale_i = max_r |a_ri| / 448 computed in
 *    FP32 (1 for a zero column), each a_ri / scale_i (FP32 division) is rounded
 *    to the nearest e4m3 value, ties to even, and saturated at +-448.
 * The dequantized matrix holds code_value * scale_i, exact in FP64.
 * ------------------------------------------------------------------------ */

/* Nearest multiple of 2^q to v (|v| small enough to be exact), ties to even. */
static double round_to_quantum(double v, int q) {
    return ldexp(nearbyint(ldexp(v, -q)), q);
}

uint16_t orc_bf16_code(float v) {
    const double a = fabs((double)v);
    double r;
    if (a == 0.0) {
        r = 0.0;
    } else if (a < ldexp(1.0, -126)) {
        r = round_to_quantum(a, -133);
    } else {
        int e;
        frexp(a, &e);                      /* a = f 2^e, 0.5 <= f < 1 */
        r = round_to_quantum(a, e - 8);    /* 8 significant bits */
    }
    float rf = (float)r;                   /* exact (or +inf past the top binade) */
    if (v < 0 || (v == 0 && signbit(v))) rf = -rf;
    uint32_t u;
    memcpy(&u, &rf, 4);
    return (uint16_t)(u >> 16);
}

double orc_bf16_value(uint16_t c) {
    uint32_t u = (uint32_t)c << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

uint8_t orc_e4m3_code(float v) {
    const uint8_t sign = (v < 0 || (v == 0 && signbit(v))) ? 0x80 : 0x00;
    const double a = fabs((double)v);
    if (a >= 448.0) return sign | 0x7E;
    if (a < ldexp(1.0, -6)) {
        /* subnormal range: multiples of 2^-9 (a result of 8 * 2^-9 is the
         * smallest normal, whose code is also 8) */
        const double k = nearbyint(ldexp(a, 9));
        return sign | (uint8_t)k;
    }
    int e;
    frexp(a, &e);
    int E = e - 1;                         /* 2^E <= a < 2^(E+1) */
    double k = nearbyint(ldexp(a, 3 - E)); /* significand in eighths: 8..16 */
    if (k == 16.0) { k = 8.0; E += 1; }
    return sign | (uint8_t)(((E + 7) << 3) | ((int)k - 8));
}

double orc_e4m3_value(uint8_t c) {
    const int e = (c >> 3) & 15, mt = c & 7;
    double v = (e == 0) ? ldexp((double)mt, -9) : ldexp((double)(8 + mt), e - 10);
    return (c & 0x80) ? -v : v;
}

/*
 * Quantize the FP32 matrix A (p x n, leading dim lda) to `to` (1 = bfloat16,
 * 2 = e4m3fn) into codes (leading dim ldq >= p, uint16 or uint8 elements) and
 * scale (n floats; all 1 for bfloat16).
 */
int orc_quantize(const float* A, int64_t p, int64_t n, int64_t lda, int to, void* codes,
                 int64_t ldq, float* scale) {
    if (!A || !codes || !scale || p < 1 || n < 1 || lda < p || ldq < p) return ORC_EINVAL;
    if (to != 1 && to != 2) return ORC_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const float* a = A + i * lda;
        if (to == 1) {
            uint16_t* q = (uint16_t*)codes + i * ldq;
            for (int64_t r = 0; r < p; ++r) q[r] = orc_bf16_code(a[r]);
            scale[i] = 1.0f;
        } else {
            uint8_t* q = (uint8_t*)codes + i * ldq;
            float mx = 0.0f;
            for (int64_t r = 0; r < p; ++r) {
                const float t = fabsf(a[r]);
                if (t > mx) mx = t;
            }
            const float sc = (mx > 0.0f) ? mx / 448.0f : 1.0f;
            for (int64_t r = 0; r < p; ++r) q[r] = orc_e4m3_code(a[r] / sc);
            scale[i] = sc;
        }
    }
    return ORC_OK;
}

/* FP64 matrix of the dequantized values code_value * scale_i (leading dim p). */
int orc_dequantize(const void* codes, int64_t p, int64_t n, int64_t ldq, int to,
                   const float* scale, double* out) {
    if (!codes || !out || p < 1 || n < 1 || ldq < p) return ORC_EINVAL;
    if (to != 1 && to != 2) return ORC_EINVAL;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double sc = scale ? (double)scale[i] : 1.0;
        for (int64_t r = 0; r < p; ++r) {
            const double v = (to == 1) ? orc_bf16_value(((const uint16_t*)codes)[i * ldq + r])
                                       : orc_e4m3_value(((const uint8_t*)codes)[i * ldq + r]);
            out[i * p + r] = v * sc;
        }
    }
    return ORC_OK;
}

/* Element-wise codes and values (no column scaling), for checks. */
int orc_encode(const float* v, int64_t cnt, int to, void* out) {
    if (!v || !out || cnt < 0 || (to != 1 && to != 2)) return ORC_EINVAL;
    for (int64_t k = 0; k < cnt; ++k) {
        if (to == 1) ((uint16_t*)out)[k] = orc_bf16_code(v[k]);
        else ((uint8_t*)out)[k] = orc_e4m3_code(v[k]);
    }
    return ORC_OK;
}

int orc_decode(const void* c, int64_t cnt, int to, double* out) {
    if (!c || !out || cnt < 0 || (to != 1 && to != 2)) return ORC_EINVAL;
    for (int64_t k = 0; k < cnt; ++k)
        out[k] = (to == 1) ? orc_bf16_value(((const uint16_t*)c)[k])
                           : orc_e4m3_value(((const uint8_t*)c)[k]);
    return ORC_OK;
}

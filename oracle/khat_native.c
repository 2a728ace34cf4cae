/* Matrix-free products with K_hat for the CPU oracle, in plain C.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by oracle/gp_oracle.py for the full-size
 * reference runs (n = 100,000 and beyond), where the NumPy row blocks are too
 * slow.  Shares no code with the HIP library.
 *
 * K_hat = K(X, X) + sigma^2 I with k(x, x') = s * kappa(r) and
 * r^2 = sum_j ((x_j - x'_j) / ls_j)^2 computed by direct differences, exactly
 * as the NumPy oracle does (Section 2.1; kernels in the forms of Rasmussen &
 * Williams 2006, Sec. 4.2).  Every entry and every sum is FP64; rows are
 * processed independently, so the result does not depend on the thread count.
 *
 *   gcc -O3 -fopenmp -shared -fPIC oracle/khat_native.c -o oracle/liboracle_khat.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { K_RBF = 0, K_MATERN32 = 1, K_MATERN52 = 2, K_RATQUAD = 3 };

#define ROWS 16   /* rows of one task */
#define COLS 256  /* columns of X (and rows of V) per inner block */

static double kappa(int kind, double alpha, double r2)
{
    double r;
    switch (kind) {
    case K_RBF:
        return exp(-0.5 * r2);
    case K_MATERN32:
        r = sqrt(r2);
        return (1.0 + sqrt(3.0) * r) * exp(-sqrt(3.0) * r);
    case K_MATERN52:
        r = sqrt(r2);
        return (1.0 + sqrt(5.0) * r + (5.0 / 3.0) * r2) * exp(-sqrt(5.0) * r);
    default:
        return pow(1.0 + r2 / (2.0 * alpha), -alpha);
    }
}

/* g(r) with d kappa / d ls_j = g(r) * dtilde_j^2 / ls_j, dtilde = scaled difference */
static double gfun(int kind, double alpha, double r2)
{
    double r;
    switch (kind) {
    case K_RBF:
        return exp(-0.5 * r2);
    case K_MATERN32:
        r = sqrt(r2);
        return 3.0 * exp(-sqrt(3.0) * r);
    case K_MATERN52:
        r = sqrt(r2);
        return (5.0 / 3.0) * (1.0 + sqrt(5.0) * r) * exp(-sqrt(5.0) * r);
    default:
        return pow(1.0 + r2 / (2.0 * alpha), -alpha - 1.0);
    }
}

static double sqdist(const double* xa, const double* xb, const double* ls, int d)
{
    double r2 = 0.0;
    for (int k = 0; k < d; ++k) {
        double u = (xa[k] - xb[k]) / ls[k];
        r2 += u * u;
    }
    return r2;
}

/* out[a, :] = K_hat[rows[a], :] @ V for a < m (rows == NULL: rows[a] = a).
 * X: n x d row-major; V: n x t row-major; out: m x t row-major. */
int oracle_khat_matvec(int64_t n, int32_t d, const double* X, const double* ls, double s, double s2,
                       int32_t kind, double alpha, int32_t t, const double* V, int64_t m,
                       const int64_t* rows, double* out)
{
    if (n < 1 || d < 1 || t < 1 || m < 0) return -1;
    const int64_t ntask = (m + ROWS - 1) / ROWS;
#pragma omp parallel
    {
        double* kv = (double*)malloc(sizeof(double) * ROWS * COLS);
#pragma omp for schedule(dynamic, 1)
        for (int64_t task = 0; task < ntask; ++task) {
            const int64_t a0 = task * ROWS;
            const int nr = (int)((m - a0) < ROWS ? (m - a0) : ROWS);
            double* o = out + a0 * t;
            memset(o, 0, sizeof(double) * (size_t)nr * (size_t)t);
            for (int64_t j0 = 0; j0 < n; j0 += COLS) {
                const int nc = (int)((n - j0) < COLS ? (n - j0) : COLS);
                for (int r = 0; r < nr; ++r) {
                    const int64_t i = rows ? rows[a0 + r] : a0 + r;
                    for (int c = 0; c < nc; ++c)
                        kv[r * COLS + c] = s * kappa(kind, alpha, sqdist(X + i * d, X + (j0 + c) * d, ls, d));
                }
                for (int r = 0; r < nr; ++r) {
                    double* orow = o + (int64_t)r * t;
                    for (int c = 0; c < nc; ++c) {
                        const double k = kv[r * COLS + c];
                        const double* v = V + (j0 + c) * t;
                        for (int q = 0; q < t; ++q) orow[q] += k * v[q];
                    }
                }
            }
            for (int r = 0; r < nr; ++r) {
                const int64_t i = rows ? rows[a0 + r] : a0 + r;
                for (int q = 0; q < t; ++q) o[(int64_t)r * t + q] += s2 * V[i * t + q];
            }
        }
        free(kv);
    }
    return 0;
}

/* sum_pq M_pq dK_hat_pq / dtheta for M = A C^T (A, C: n x t row-major), over the
 * rows p0 <= p < p1 of M (0, n: all of it).
 * out[0..d): per-dimension terms sum_pq W_pq dtilde_pqj^2 / ls_j with
 * W = s g(r) M (the lengthscale derivatives of an ARD kernel; an isotropic
 * kernel sums them); out[d]: sum_pq M_pq kappa(r_pq) (outputscale);
 * out[d + 1]: sum_p M_pp (noise).  Partial sums per task are added in task
 * order, so the result does not depend on the thread count. */
int oracle_dkhat_lowrank(int64_t n, int32_t d, const double* X, const double* ls, double s, int32_t kind,
                         double alpha, int32_t t, const double* A, const double* C, int64_t p0, int64_t p1,
                         double* out)
{
    if (n < 1 || d < 1 || t < 1 || p0 < 0 || p1 > n || p0 > p1) return -1;
    const int64_t ntask = (p1 - p0 + ROWS - 1) / ROWS;
    const int np = d + 2;
    double* part = (double*)calloc((size_t)ntask * (size_t)np, sizeof(double));
    if (!part) return -2;
#pragma omp parallel
    {
        double* dt = (double*)malloc(sizeof(double) * (size_t)d);
#pragma omp for schedule(dynamic, 1)
        for (int64_t task = 0; task < ntask; ++task) {
            double* acc = part + task * np;
            const int64_t r0 = p0 + task * ROWS;
            const int64_t r1 = (r0 + ROWS) < p1 ? (r0 + ROWS) : p1;
            for (int64_t q0 = 0; q0 < n; q0 += COLS)
            for (int64_t p = r0; p < r1; ++p) {
                const double* ap = A + p * t;
                const int64_t q1 = (q0 + COLS) < n ? (q0 + COLS) : n;
                for (int64_t q = q0; q < q1; ++q) {
                    const double* cq = C + q * t;
                    double mpq = 0.0;
                    for (int c = 0; c < t; ++c) mpq += ap[c] * cq[c];
                    double r2 = 0.0;
                    for (int k = 0; k < d; ++k) {
                        dt[k] = (X[p * d + k] - X[q * d + k]) / ls[k];
                        r2 += dt[k] * dt[k];
                    }
                    const double w = s * gfun(kind, alpha, r2) * mpq;
                    for (int k = 0; k < d; ++k) acc[k] += w * dt[k] * dt[k];
                    acc[d] += kappa(kind, alpha, r2) * mpq;
                    if (q == p) acc[d + 1] += mpq;
                }
            }
        }
        free(dt);
    }
    for (int k = 0; k < np; ++k) out[k] = 0.0;
    for (int64_t task = 0; task < ntask; ++task)
        for (int k = 0; k < np; ++k) out[k] += part[task * np + k];
    for (int k = 0; k < d; ++k) out[k] /= ls[k];
    free(part);
    return 0;
}

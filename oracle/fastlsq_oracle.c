/*
 * Plain, slow FP64 CPU oracle for the FastLSQ hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or table with the HIP path.
 *
 * Each function writes out the definition it follows with explicit loops:
 *
 *   orc_assemble   -- Eq. (2) (cyclic derivative of a sinusoidal feature) summed
 *                     over the terms of a linear operator, times the row weight
 *                     of Eq. (3) and the 1/sqrt(N) factor of Eq. (1).
 *   orc_evaluate   -- D^alpha of the expansion of Eq. (1), via Eq. (2).
 *   orc_tikhonov   -- the unique minimiser of ||A beta - rhs||^2 + mu ||beta||^2
 *                     (the Tikhonov least-squares problem of Section 2.4, the
 *                     least-squares solve of Algorithm 1 / Section 2.3 "via QR"),
 *                     computed by unpivoted Householder QR of [A; sqrt(mu) I].
 *   orc_qr_factor  -- the same Householder QR of [A; sqrt(mu) I], keeping the
 *   orc_qr_solve      reflectors, and the same minimiser for right-hand sides
 *                     supplied later (a system whose matrix stays fixed while
 *                     its data change, as in the inverse application of
 *                     Section 2.5): the reflectors reach each right-hand side in
 *                     the order and arithmetic of orc_tikhonov, so both give the
 *                     same bits.
 *   orc_trisolve   -- forward / backward substitution with an upper-triangular R
 *                     (used for R^T R = A^T A + mu I in the adjoint).
 *
 * Conventions: matrices passed in and out are row-major float64; phases are
 * z = sum_k W_jk x_ik (ascending k) + b_j, evaluated in double precision with
 * the C library sin/cos.  Multi-indices are int32, one row of d per term.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Phi_{n mod 4}(z) of Eq. (2): sin, cos, -sin, -cos. */
static double cyclic_phi(int order, double s, double c)
{
    switch (order & 3) {
    case 0: return s;
    case 1: return c;
    case 2: return -s;
    default: return -c;
    }
}

/* prod_k W_jk^alpha_k by repeated multiplication. */
static double monomial(const double* Wj, const int32_t* alpha, int d)
{
    double m = 1.0;
    for (int k = 0; k < d; ++k)
        for (int p = 0; p < alpha[k]; ++p)
            m *= Wj[k];
    return m;
}

static int order_of(const int32_t* alpha, int d)
{
    int o = 0;
    for (int k = 0; k < d; ++k) o += alpha[k];
    return o;
}

static double phase(const double* Wj, const double* xi, double bj, int d)
{
    double z = 0.0;
    for (int k = 0; k < d; ++k) z += Wj[k] * xi[k];
    return z + bj;
}

/* A[i][j] = weight / sqrt(N)^normalize * sum_t coef_t * W_j^alpha_t * Phi_{|alpha_t|}(z_ij). */
void orc_assemble(int d, int n_feat, const double* W, const double* b, int normalize,
                  int64_t n_rows, const double* X, int n_terms, const double* coef,
                  const int32_t* alpha, double weight, double* A)
{
    const double scale = weight / (normalize ? sqrt((double)n_feat) : 1.0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_rows; ++i) {
        const double* xi = X + i * d;
        for (int j = 0; j < n_feat; ++j) {
            const double* Wj = W + (int64_t)j * d;
            const double z = phase(Wj, xi, b[j], d);
            const double s = sin(z), c = cos(z);
            double v = 0.0;
            for (int t = 0; t < n_terms; ++t) {
                const int32_t* at = alpha + (int64_t)t * d;
                v += coef[t] * monomial(Wj, at, d) * cyclic_phi(order_of(at, d), s, c);
            }
            A[i * n_feat + j] = scale * v;
        }
    }
}

/* out[q][a] = (1/sqrt(N))^normalize * sum_j beta_j * W_j^alpha_a * Phi_{|alpha_a|}(z_qj), j ascending. */
void orc_evaluate(int d, int n_feat, const double* W, const double* b, int normalize,
                  const double* beta, int64_t n_q, const double* Xq, int n_alpha,
                  const int32_t* alphas, double* out)
{
    const double scale = 1.0 / (normalize ? sqrt((double)n_feat) : 1.0);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n_q; ++q) {
        const double* xq = Xq + q * d;
        for (int a = 0; a < n_alpha; ++a) out[q * n_alpha + a] = 0.0;
        for (int j = 0; j < n_feat; ++j) {
            const double* Wj = W + (int64_t)j * d;
            const double z = phase(Wj, xq, b[j], d);
            const double s = sin(z), c = cos(z);
            for (int a = 0; a < n_alpha; ++a) {
                const int32_t* al = alphas + (int64_t)a * d;
                out[q * n_alpha + a] += beta[j] * monomial(Wj, al, d) * cyclic_phi(order_of(al, d), s, c);
            }
        }
        for (int a = 0; a < n_alpha; ++a) out[q * n_alpha + a] *= scale;
    }
}

/*
 * Tikhonov least squares by Householder QR of the augmented matrix.
 *
 *   minimise ||A beta - rhs||^2 + mu ||beta||^2  <=>  minimise || [A; sqrt(mu) I] beta - [rhs; 0] ||^2
 *
 * A is m x n row-major, rhs m x k row-major, beta_out n x k row-major.
 * If R_out is not NULL it receives the n x n upper-triangular factor (row-major,
 * zeros below the diagonal), so that R^T R = A^T A + mu I.
 * Returns 0 on success, 1 on a zero pivot of R, 2 on allocation failure.
 *
 * Reflector for column j: x = M[j:, j], alpha = ||x||, v = x + sign(x_0) alpha e_1
 * (sign(0) = +1), H = I - 2 v v^T / (v^T v); H x = -sign(x_0) alpha e_1.
 */
int orc_tikhonov(int64_t m, int n, const double* A, int k, const double* rhs, double mu,
                 double* beta_out, double* R_out)
{
    const int64_t rows = m + n;
    double* M = (double*)malloc(sizeof(double) * (size_t)rows * (size_t)n);  /* column-major */
    double* Y = (double*)malloc(sizeof(double) * (size_t)rows * (size_t)k);  /* column-major */
    double* v = (double*)malloc(sizeof(double) * (size_t)rows);
    if (!M || !Y || !v) { free(M); free(Y); free(v); return 2; }

    const double smu = sqrt(mu);
    for (int c = 0; c < n; ++c) {
        double* col = M + (int64_t)c * rows;
        for (int64_t i = 0; i < m; ++i) col[i] = A[i * n + c];
        for (int i = 0; i < n; ++i) col[m + i] = (i == c) ? smu : 0.0;
    }
    for (int c = 0; c < k; ++c) {
        double* col = Y + (int64_t)c * rows;
        for (int64_t i = 0; i < m; ++i) col[i] = rhs[i * k + c];
        for (int i = 0; i < n; ++i) col[m + i] = 0.0;
    }

    for (int j = 0; j < n; ++j) {
        double* x = M + (int64_t)j * rows;
        const int64_t len = rows - j;
        double nrm2 = 0.0;
        for (int64_t i = 0; i < len; ++i) nrm2 += x[j + i] * x[j + i];
        const double alpha = sqrt(nrm2);
        if (alpha == 0.0) continue;                 /* nothing to annihilate */
        const double sgn = (x[j] >= 0.0) ? 1.0 : -1.0;
        for (int64_t i = 0; i < len; ++i) v[i] = x[j + i];
        v[0] += sgn * alpha;
        double vtv = 0.0;
        for (int64_t i = 0; i < len; ++i) vtv += v[i] * v[i];
        const double tau = 2.0 / vtv;

        /* apply H to the trailing columns and to every right-hand side */
#pragma omp parallel for schedule(dynamic, 8)
        for (int c = j + 1; c < n + k; ++c) {
            double* col = (c < n) ? M + (int64_t)c * rows : Y + (int64_t)(c - n) * rows;
            double s = 0.0;
            for (int64_t i = 0; i < len; ++i) s += v[i] * col[j + i];
            s *= tau;
            for (int64_t i = 0; i < len; ++i) col[j + i] -= s * v[i];
        }
        x[j] = -sgn * alpha;
        for (int64_t i = 1; i < len; ++i) x[j + i] = 0.0;
    }

    int status = 0;
    for (int j = 0; j < n; ++j)
        if (M[(int64_t)j * rows + j] == 0.0) status = 1;

    if (status == 0) {
        /* back substitution R beta = (Q^T rhs)[0:n] for each right-hand side */
        for (int c = 0; c < k; ++c) {
            const double* y = Y + (int64_t)c * rows;
            for (int i = n - 1; i >= 0; --i) {
                double s = y[i];
                for (int jj = i + 1; jj < n; ++jj) s -= M[(int64_t)jj * rows + i] * beta_out[(int64_t)jj * k + c];
                beta_out[(int64_t)i * k + c] = s / M[(int64_t)i * rows + i];
            }
        }
    }
    if (R_out) {
        for (int i = 0; i < n; ++i)
            for (int jj = 0; jj < n; ++jj)
                R_out[(int64_t)i * n + jj] = (jj >= i) ? M[(int64_t)jj * rows + i] : 0.0;
    }
    free(M); free(Y); free(v);
    return status;
}

/*
 * Householder QR of [A; sqrt(mu) I] with the reflectors kept (the loop of
 * orc_tikhonov without right-hand sides).  V (rows x n, column-major, rows =
 * m + n) receives v_j in V[j * rows + j .. j * rows + rows - 1]; tau[j] = 2 / v_j^T v_j
 * (0 where column j had nothing to annihilate); R_out the n x n factor
 * (row-major, zeros below the diagonal).  Returns 0, 1 on a zero pivot, 2 on
 * allocation failure.
 */
int orc_qr_factor(int64_t m, int n, const double* A, double mu, double* V, double* tau, double* R_out)
{
    const int64_t rows = m + n;
    double* M = (double*)malloc(sizeof(double) * (size_t)rows * (size_t)n);  /* column-major */
    if (!M) return 2;
    const double smu = sqrt(mu);
    for (int c = 0; c < n; ++c) {
        double* col = M + (int64_t)c * rows;
        for (int64_t i = 0; i < m; ++i) col[i] = A[i * n + c];
        for (int i = 0; i < n; ++i) col[m + i] = (i == c) ? smu : 0.0;
    }
    for (int j = 0; j < n; ++j) {
        double* x = M + (int64_t)j * rows;
        double* v = V + (int64_t)j * rows + j;
        const int64_t len = rows - j;
        double nrm2 = 0.0;
        for (int64_t i = 0; i < len; ++i) nrm2 += x[j + i] * x[j + i];
        const double alpha = sqrt(nrm2);
        tau[j] = 0.0;
        if (alpha == 0.0) continue;
        const double sgn = (x[j] >= 0.0) ? 1.0 : -1.0;
        for (int64_t i = 0; i < len; ++i) v[i] = x[j + i];
        v[0] += sgn * alpha;
        double vtv = 0.0;
        for (int64_t i = 0; i < len; ++i) vtv += v[i] * v[i];
        const double t = 2.0 / vtv;
        tau[j] = t;
#pragma omp parallel for schedule(dynamic, 8)
        for (int c = j + 1; c < n; ++c) {
            double* col = M + (int64_t)c * rows;
            double s = 0.0;
            for (int64_t i = 0; i < len; ++i) s += v[i] * col[j + i];
            s *= t;
            for (int64_t i = 0; i < len; ++i) col[j + i] -= s * v[i];
        }
        x[j] = -sgn * alpha;
        for (int64_t i = 1; i < len; ++i) x[j + i] = 0.0;
    }
    int status = 0;
    for (int j = 0; j < n; ++j)
        if (M[(int64_t)j * rows + j] == 0.0) status = 1;
    for (int i = 0; i < n; ++i)
        for (int jj = 0; jj < n; ++jj)
            R_out[(int64_t)i * n + jj] = (jj >= i) ? M[(int64_t)jj * rows + i] : 0.0;
    free(M);
    return status;
}

/*
 * beta_out (n x k, row-major) = argmin ||A beta - rhs||^2 + mu ||beta||^2 for rhs (m x k,
 * row-major) with the reflectors and R of orc_qr_factor: Q^T [rhs; 0] reflector by
 * reflector, then R beta = (Q^T [rhs; 0])[0:n].  Returns 0, or 2 on allocation failure.
 */
int orc_qr_solve(int64_t m, int n, const double* V, const double* tau, const double* R, int k,
                 const double* rhs, double* beta_out)
{
    const int64_t rows = m + n;
    double* Y = (double*)malloc(sizeof(double) * (size_t)rows * (size_t)k);  /* column-major */
    if (!Y) return 2;
    for (int c = 0; c < k; ++c) {
        double* col = Y + (int64_t)c * rows;
        for (int64_t i = 0; i < m; ++i) col[i] = rhs[i * k + c];
        for (int i = 0; i < n; ++i) col[m + i] = 0.0;
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < k; ++c) {
        double* col = Y + (int64_t)c * rows;
        for (int j = 0; j < n; ++j) {
            const double t = tau[j];
            if (t == 0.0) continue;
            const double* v = V + (int64_t)j * rows + j;
            const int64_t len = rows - j;
            double s = 0.0;
            for (int64_t i = 0; i < len; ++i) s += v[i] * col[j + i];
            s *= t;
            for (int64_t i = 0; i < len; ++i) col[j + i] -= s * v[i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = col[i];
            for (int jj = i + 1; jj < n; ++jj) s -= R[(int64_t)i * n + jj] * beta_out[(int64_t)jj * k + c];
            beta_out[(int64_t)i * k + c] = s / R[(int64_t)i * n + i];
        }
    }
    free(Y);
    return 0;
}

/*
 * Triangular solves with an upper-triangular R (n x n row-major), k right-hand
 * sides (n x k row-major), in place:
 *   transpose = 0:  R   x = y   (backward substitution)
 *   transpose = 1:  R^T x = y   (forward substitution)
 */
void orc_trisolve(int n, const double* R, int k, double* Y, int transpose)
{
    for (int c = 0; c < k; ++c) {
        if (transpose) {
            for (int i = 0; i < n; ++i) {
                double s = Y[(int64_t)i * k + c];
                for (int jj = 0; jj < i; ++jj) s -= R[(int64_t)jj * n + i] * Y[(int64_t)jj * k + c];
                Y[(int64_t)i * k + c] = s / R[(int64_t)i * n + i];
            }
        } else {
            for (int i = n - 1; i >= 0; --i) {
                double s = Y[(int64_t)i * k + c];
                for (int jj = i + 1; jj < n; ++jj) s -= R[(int64_t)i * n + jj] * Y[(int64_t)jj * k + c];
                Y[(int64_t)i * k + c] = s / R[(int64_t)i * n + i];
            }
        }
    }
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

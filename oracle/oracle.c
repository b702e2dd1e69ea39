/*
 * Plain FP64 CPU oracle for the sparse-GP (GAP) fit.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this code; the GPU library
 * never does, and this file shares no code with it.
 *
 * It computes, slowly and in the order the paper states, what the GPU path
 * computes: the kernel matrices, the Cholesky factor of K_MM, the stacked
 * least-squares problem, an unblocked Householder QR with Q^T b carried along,
 * back-substitution for the weights, the loss and its gradient, the
 * prediction of total energies, and the row leverages behind CUR sparse-point
 * selection.  Every floating-point sum runs in a fixed
 * sequential order, so the result does not depend on the thread count.
 *
 * Matrices are dense, row-major: element (i, j) of an r x c matrix is at
 * [i * c + j].
 *
 * Readings of the paper taken here (each also listed in the design notes):
 *   - k(x, x') = sigma_w^2 (x . x')^zeta with integer zeta >= 1, the power
 *     formed by repeated multiplication (the paper names the dot-product
 *     covariance with its exponent but does not print the formula).
 *   - Sigma = diag(sigma_A^2) and b = [Sigma^-1/2 y ; 0]: only this right-hand
 *     side makes the least-squares objective equal to the loss (Eq. loss);
 *     the padded vector printed in Sec. Theory omits the Sigma^-1/2.
 *   - The jitter is added to the diagonal of K_MM before the Cholesky
 *     factorisation, and the same jittered K_MM is the regulariser.
 *   - Householder reflectors follow the LAPACK convention: H = I - tau v v^T,
 *     v(0) = 1, beta = -sign(alpha) * ||(alpha, x)||, sign(0) = +1, tau = 0
 *     when the part below the diagonal is exactly zero.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Return codes shared by the functions below. */
#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_ENOTPD 2
#define ORACLE_ENOMEM 3

/*
 * Dot-product covariance between two descriptors (Eq. 2 kernel, with the
 * exponent zeta and the prefactor sigma_w^2).
 */
static double covariance(const double *a, const double *b, int64_t d, int zeta, double sigma_w)
{
    double g = 0.0;
    for (int64_t p = 0; p < d; ++p)
        g += a[p] * b[p];
    double pw = g;
    for (int z = 1; z < zeta; ++z)
        pw *= g;
#ifdef ORACLE_PLANT_POWER
    pw = g; /* planted mistake: exponent dropped */
#endif
    return (sigma_w * sigma_w) * pw;
}

/*
 * K_NM (Sec. Theory, definition of K_MN: a target's row is the sum over the
 * descriptors that contribute to it).  K[A*M + j] = sum_{i in A} k(x_i, x_j),
 * atoms summed in their stored order.  X is [n_atoms x d], XM is [M x d],
 * offsets[A]..offsets[A+1] are configuration A's atoms.
 */
int oracle_knm(const double *X, const int64_t *offsets, int64_t N, const double *XM, int64_t M,
               int64_t d, int zeta, double sigma_w, double *K)
{
    if (N < 0 || M < 0 || d < 1 || zeta < 1)
        return ORACLE_EINVAL;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t A = 0; A < N; ++A) {
        for (int64_t j = 0; j < M; ++j) {
            double s = 0.0;
            int64_t end = offsets[A + 1];
#ifdef ORACLE_PLANT_SEGMENT_END
            if (end > offsets[A])
                end -= 1; /* planted mistake: a configuration's last atom dropped */
#endif
            for (int64_t i = offsets[A]; i < end; ++i)
                s += covariance(X + i * d, XM + j * d, d, zeta, sigma_w);
            K[A * M + j] = s;
        }
    }
    return ORACLE_OK;
}

/* K_MM between the sparse points, plus the jitter on its diagonal. */
int oracle_kmm(const double *XM, int64_t M, int64_t d, int zeta, double sigma_w, double jitter,
               double *K)
{
    if (M < 0 || d < 1 || zeta < 1)
        return ORACLE_EINVAL;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < M; ++i) {
        for (int64_t j = 0; j < M; ++j)
            K[i * M + j] = covariance(XM + i * d, XM + j * d, d, zeta, sigma_w);
#ifndef ORACLE_PLANT_NO_JITTER
        K[i * M + i] += jitter;
#endif
    }
    return ORACLE_OK;
}

/*
 * Cholesky-Banachiewicz factorisation K = L L^T, L lower triangular (Sec.
 * Theory, the lower block of A).  Returns ORACLE_ENOTPD and *fail_col = the
 * 0-based column whose pivot is not positive (or not finite).
 */
int oracle_cholesky(const double *K, int64_t M, double *L, int64_t *fail_col)
{
    memset(L, 0, sizeof(double) * (size_t)(M * M));
    if (fail_col)
        *fail_col = -1;
    for (int64_t i = 0; i < M; ++i) {
        for (int64_t j = 0; j <= i; ++j) {
            double s = 0.0;
            for (int64_t k = 0; k < j; ++k)
                s += L[i * M + k] * L[j * M + k];
            if (i == j) {
                double piv = K[i * M + i] - s;
                if (!(piv > 0.0) || !isfinite(piv)) {
                    if (fail_col)
                        *fail_col = i;
                    return ORACLE_ENOTPD;
                }
                L[i * M + i] = sqrt(piv);
            } else {
                L[i * M + j] = (K[i * M + j] - s) / L[j * M + j];
            }
        }
    }
    return ORACLE_OK;
}

/*
 * The stacked least-squares problem (Sec. Theory): A = [Sigma^-1/2 K_NM ; L^T]
 * of (N+M) x M and b = [Sigma^-1/2 y ; 0].  sigma[A] is the standard
 * deviation of target A, so Sigma^-1/2 divides row A by sigma[A].
 */
int oracle_stack(const double *Knm, const double *sigma, const double *y, const double *L,
                 int64_t N, int64_t M, double *A, double *b)
{
    for (int64_t r = 0; r < N; ++r) {
        for (int64_t j = 0; j < M; ++j) {
#ifdef ORACLE_PLANT_NO_ROW_SCALE
            A[r * M + j] = Knm[r * M + j];
#else
            A[r * M + j] = Knm[r * M + j] / sigma[r];
#endif
        }
#ifdef ORACLE_PLANT_B_UNSCALED
        b[r] = y[r]; /* planted mistake: targets not scaled by 1/sigma */
#else
        b[r] = y[r] / sigma[r];
#endif
    }
    for (int64_t i = 0; i < M; ++i) {
        for (int64_t j = 0; j < M; ++j) {
#ifdef ORACLE_PLANT_TRANSPOSE_L
            A[(N + i) * M + j] = L[i * M + j];
#else
            A[(N + i) * M + j] = L[j * M + i]; /* (L^T)[i][j] */
#endif
        }
        b[N + i] = 0.0;
    }
    return ORACLE_OK;
}

/*
 * Unblocked Householder QR of the m x n matrix A (m >= n), with the
 * right-hand side b carried along so that b ends as Q^T b (the effect of the
 * factorisation and the Q^T b step described in Sec. Implementation).  On
 * return R is in the upper triangle of A, the reflector tails below it (the
 * leading 1 implicit) and tau[k] holds each reflector's weight.
 */
int oracle_householder_qr(double *A, double *b, int64_t m, int64_t n, double *tau)
{
    if (m < n || n < 0)
        return ORACLE_EINVAL;
    double *v = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
    double *w = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!v || !w) {
        free(v);
        free(w);
        return ORACLE_ENOMEM;
    }
    for (int64_t k = 0; k < n; ++k) {
        double alpha = A[k * n + k];
        double xnorm2 = 0.0;
        for (int64_t i = k + 1; i < m; ++i)
            xnorm2 += A[i * n + k] * A[i * n + k];
        double t;
        if (xnorm2 == 0.0) {
            t = 0.0; /* H = I: nothing below the diagonal to annihilate */
            v[k] = 1.0;
            for (int64_t i = k + 1; i < m; ++i)
                v[i] = 0.0;
        } else {
            double norm = sqrt(alpha * alpha + xnorm2);
            double beta = (alpha >= 0.0) ? -norm : norm;
            t = (beta - alpha) / beta;
#ifdef ORACLE_PLANT_TAU
            t = (beta - alpha) / alpha; /* planted mistake: wrong denominator */
#endif
            double scale = 1.0 / (alpha - beta);
            v[k] = 1.0;
            for (int64_t i = k + 1; i < m; ++i)
                v[i] = A[i * n + k] * scale;
            A[k * n + k] = beta;
            for (int64_t i = k + 1; i < m; ++i)
                A[i * n + k] = v[i];
        }
        tau[k] = t;
        if (t == 0.0)
            continue;
        /*
         * Apply H = I - t v v^T to the remaining columns, then to b:
         * w[j] = t * sum_{i >= k} v[i] A[i][j] (each sum in ascending i), then
         * A[i][j] -= w[j] v[i].  Both loops walk A row by row (it is stored by
         * rows); every element sees the same operations in the same order as
         * the column-at-a-time form.
         */
        const int64_t nt = n - (k + 1);
#pragma omp parallel
        {
#ifdef _OPENMP
            const int64_t nth = omp_get_num_threads(), th = omp_get_thread_num();
#else
            const int64_t nth = 1, th = 0;
#endif
            const int64_t j0 = k + 1 + (nt * th) / nth, j1 = k + 1 + (nt * (th + 1)) / nth;
            for (int64_t j = j0; j < j1; ++j)
                w[j] = 0.0;
            for (int64_t i = k; i < m; ++i) {
                const double vi = v[i];
                const double *row = A + i * n;
                for (int64_t j = j0; j < j1; ++j)
                    w[j] += vi * row[j];
            }
            for (int64_t j = j0; j < j1; ++j)
                w[j] *= t;
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = k; i < m; ++i) {
            const double vi = v[i];
            double *row = A + i * n;
            for (int64_t j = k + 1; j < n; ++j)
                row[j] -= w[j] * vi;
        }
        double wb = 0.0;
        for (int64_t i = k; i < m; ++i)
            wb += v[i] * b[i];
        wb *= t;
        for (int64_t i = k; i < m; ++i)
            b[i] -= wb * v[i];
    }
    free(v);
    free(w);
    return ORACLE_OK;
}

/*
 * Back-substitution R c = rhs for the n x n upper triangle of R stored with
 * leading dimension ldr (Sec. Theory, c = R^-1 Q^T b).
 */
int oracle_back_substitution(const double *R, int64_t ldr, const double *rhs, int64_t n, double *c)
{
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = rhs[i];
        for (int64_t j = i + 1; j < n; ++j)
#ifdef ORACLE_PLANT_BACKSUB
            s -= R[j * ldr + i] * c[j]; /* planted mistake: transposed operand */
#else
            s -= R[i * ldr + j] * c[j];
#endif
        c[i] = s / R[i * ldr + i];
    }
    return ORACLE_OK;
}

/*
 * Extreme singular values of the stacked matrix A through the n x n upper
 * triangle of its QR factor R (row-major, leading dimension ldr): A = QR with
 * orthonormal columns in Q, so A and R have the same singular values and
 * kappa_2(A) = smax / smin, the factor that turns a backward-stable solver's
 * rounding into its error in c (Sec. Practical Examples compares predictions
 * because reordered fits share only a few digits of c).
 *   smax: power iteration on R^T R (x <- R^T R x, normalised).
 *   smin: inverse iteration on R^T R (x <- R^-1 R^-T x, normalised).
 * Each estimate is the Rayleigh quotient of the unit iterate (||R x||^2, and
 * ||R^-T x||^2 for the inverse), so it approaches the extreme value from
 * inside; iteration stops when the quotient changes by at most tol
 * (relative) between steps, or after max_iter steps.  iters[0], iters[1] =
 * steps taken.  Starting vector: all ones.  ORACLE_EINVAL on a zero pivot.
 */
int oracle_singular_extremes(const double *R, int64_t ldr, int64_t n, int max_iter, double tol,
                             double *smax, double *smin, int *iters)
{
    if (n < 1 || ldr < n || max_iter < 1)
        return ORACLE_EINVAL;
    for (int64_t i = 0; i < n; ++i)
        if (R[i * ldr + i] == 0.0)
            return ORACLE_EINVAL;
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *z = (double *)malloc(sizeof(double) * (size_t)n);
    if (!x || !y || !z) {
        free(x);
        free(y);
        free(z);
        return ORACLE_ENOMEM;
    }
    for (int pass = 0; pass < 2; ++pass) {
        const int inverse = (pass == 1);
        for (int64_t i = 0; i < n; ++i)
            x[i] = 1.0 / sqrt((double)n);
        double q = 0.0, q_prev = 0.0;
        int it = 0;
        while (it < max_iter) {
            ++it;
            if (!inverse) {
                /* y = R x (rows independent) */
#pragma omp parallel for schedule(static)
                for (int64_t i = 0; i < n; ++i) {
                    double s = 0.0;
                    for (int64_t j = i; j < n; ++j)
                        s += R[i * ldr + j] * x[j];
                    y[i] = s;
                }
                /* z = R^T y: z[j] = sum_{i <= j} R[i][j] y[i], ascending i */
                for (int64_t j = 0; j < n; ++j)
                    z[j] = 0.0;
                for (int64_t i = 0; i < n; ++i) {
                    const double yi = y[i];
                    for (int64_t j = i; j < n; ++j)
                        z[j] += R[i * ldr + j] * yi;
                }
            } else {
                /* y = R^-T x: forward substitution with the lower triangle R^T */
                for (int64_t i = 0; i < n; ++i)
                    z[i] = x[i];
                for (int64_t k = 0; k < n; ++k) {
                    y[k] = z[k] / R[k * ldr + k];
                    const double yk = y[k];
                    for (int64_t j = k + 1; j < n; ++j)
                        z[j] -= R[k * ldr + j] * yk;
                }
                /* z = R^-1 y: back-substitution */
                for (int64_t i = n - 1; i >= 0; --i) {
                    double s = y[i];
                    for (int64_t j = i + 1; j < n; ++j)
                        s -= R[i * ldr + j] * z[j];
                    z[i] = s / R[i * ldr + i];
                }
            }
            q = 0.0;
            for (int64_t i = 0; i < n; ++i)
                q += y[i] * y[i];
            double zn = 0.0;
            for (int64_t i = 0; i < n; ++i)
                zn += z[i] * z[i];
            zn = sqrt(zn);
            for (int64_t i = 0; i < n; ++i)
                x[i] = z[i] / zn;
            if (it > 1 && fabs(q - q_prev) <= tol * q)
                break;
            q_prev = q;
        }
        if (!inverse)
            *smax = sqrt(q);
        else
            *smin = 1.0 / sqrt(q);
        if (iters)
            iters[pass] = it;
    }
    free(x);
    free(y);
    free(z);
    return ORACLE_OK;
}

/*
 * Prediction of total energies (Eqs. 1-2): y_A = sum_{i in A} eps(x_i),
 * eps(x) = sum_j c_j k(x, x_j).
 */
int oracle_predict(const double *X, const int64_t *offsets, int64_t N, const double *XM, int64_t M,
                   int64_t d, int zeta, double sigma_w, const double *c, double *y)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t A = 0; A < N; ++A) {
        double e = 0.0;
        int64_t start = offsets[A];
#ifdef ORACLE_PLANT_PREDICT_SEGMENT
        if (start < offsets[A + 1])
            start += 1; /* planted mistake: a configuration's first atom skipped */
#endif
        for (int64_t i = start; i < offsets[A + 1]; ++i) {
            double eps = 0.0;
            for (int64_t j = 0; j < M; ++j)
                eps += c[j] * covariance(X + i * d, XM + j * d, d, zeta, sigma_w);
            e += eps;
        }
        y[A] = e;
    }
    return ORACLE_OK;
}

/*
 * The loss (Eq. loss) with Sigma = diag(sigma^2) and the jittered K_MM:
 * L = sum_A (y_A - (K_NM c)_A)^2 / sigma_A^2 + c^T Kmm c.
 */
double oracle_loss(const double *Knm, const double *sigma, const double *y, const double *Kmm,
                   const double *c, int64_t N, int64_t M)
{
    double fit = 0.0;
    for (int64_t A = 0; A < N; ++A) {
        double pred = 0.0;
        for (int64_t j = 0; j < M; ++j)
            pred += Knm[A * M + j] * c[j];
        double r = (y[A] - pred) / sigma[A];
        fit += r * r;
    }
    double reg = 0.0;
    for (int64_t i = 0; i < M; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < M; ++j)
            s += Kmm[i * M + j] * c[j];
        reg += c[i] * s;
    }
    return fit + reg;
}

/*
 * Gradient of the loss with respect to c:
 * g = 2 [ Kmm c - K_MN Sigma^-1 (y - K_NM c) ].
 */
int oracle_gradient(const double *Knm, const double *sigma, const double *y, const double *Kmm,
                    const double *c, int64_t N, int64_t M, double *g)
{
    double *r = (double *)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    if (!r)
        return ORACLE_ENOMEM;
    for (int64_t A = 0; A < N; ++A) {
        double pred = 0.0;
        for (int64_t j = 0; j < M; ++j)
            pred += Knm[A * M + j] * c[j];
        r[A] = (y[A] - pred) / (sigma[A] * sigma[A]);
    }
    for (int64_t i = 0; i < M; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < M; ++j)
            s += Kmm[i * M + j] * c[j];
        double t = 0.0;
        for (int64_t A = 0; A < N; ++A)
            t += Knm[A * M + i] * r[A];
        g[i] = 2.0 * (s - t);
    }
    free(r);
    return ORACLE_OK;
}

/*
 * The whole fit, in the paper's order: K_NM, K_MM + jitter, Cholesky, the
 * stacked problem, Householder QR with Q^T b, back-substitution.
 *
 * Outputs (all caller-allocated): c [M]; loss_tail = ||(Q^T b)[M:]||^2 (the
 * minimum of the least-squares objective); diagR [M] = diagonal of R;
 * optional (nullable) Knm_out [N x M], L_out [M x M], A_out [(N+M) x M] after
 * the QR (R and reflectors), qtb_out [N+M], tau_out [M].
 */
int oracle_fit(const double *X, const int64_t *offsets, int64_t N, const double *XM, int64_t M,
               int64_t d, int zeta, double sigma_w, double jitter, const double *sigma,
               const double *y, double *c, double *loss_tail, double *diagR, double *Knm_out,
               double *L_out, double *A_out, double *qtb_out, double *tau_out)
{
    if (N < 0 || M < 1 || d < 1 || zeta < 1)
        return ORACLE_EINVAL;
    int64_t m = N + M;
    int rc = ORACLE_ENOMEM;
    double *Knm = (double *)malloc(sizeof(double) * (size_t)(N * M + 1));
    double *Kmm = (double *)malloc(sizeof(double) * (size_t)(M * M));
    double *L = (double *)malloc(sizeof(double) * (size_t)(M * M));
    double *A = (double *)malloc(sizeof(double) * (size_t)(m * M));
    double *b = (double *)malloc(sizeof(double) * (size_t)m);
    double *tau = (double *)malloc(sizeof(double) * (size_t)M);
    if (!Knm || !Kmm || !L || !A || !b || !tau)
        goto done;
    oracle_knm(X, offsets, N, XM, M, d, zeta, sigma_w, Knm);
    oracle_kmm(XM, M, d, zeta, sigma_w, jitter, Kmm);
    rc = oracle_cholesky(Kmm, M, L, NULL);
    if (rc != ORACLE_OK)
        goto done;
    oracle_stack(Knm, sigma, y, L, N, M, A, b);
    rc = oracle_householder_qr(A, b, m, M, tau);
    if (rc != ORACLE_OK)
        goto done;
    oracle_back_substitution(A, M, b, M, c);
    {
        double t = 0.0;
        for (int64_t i = M; i < m; ++i)
            t += b[i] * b[i];
        *loss_tail = t;
    }
    for (int64_t i = 0; i < M; ++i)
        diagR[i] = A[i * M + i];
    if (Knm_out)
        memcpy(Knm_out, Knm, sizeof(double) * (size_t)(N * M));
    if (L_out)
        memcpy(L_out, L, sizeof(double) * (size_t)(M * M));
    if (A_out)
        memcpy(A_out, A, sizeof(double) * (size_t)(m * M));
    if (qtb_out)
        memcpy(qtb_out, b, sizeof(double) * (size_t)m);
    if (tau_out)
        memcpy(tau_out, tau, sizeof(double) * (size_t)M);
    rc = ORACLE_OK;
done:
    free(Knm);
    free(Kmm);
    free(L);
    free(A);
    free(b);
    free(tau);
    return rc;
}

/*
 * Statistical leverage of every descriptor row for CUR sparse-point selection
 * (Sec. Implementation: sparse points chosen by CUR-based methods, after
 * Mahoney & Drineas 2009).  With X the n x d matrix of descriptor rows, the
 * leverage of row i over the row space of X is the i-th diagonal element of
 * the hat matrix X (X^T X)^-1 X^T:
 *   lev[i] = x_i^T (X^T X)^-1 x_i = ||z_i||^2,  L z_i = x_i,  X^T X = L L^T.
 * The Gram matrix is summed over the rows in order, factored by the Cholesky
 * above, and z_i found by forward substitution.  Returns ORACLE_ENOTPD when
 * X^T X is not positive definite (X of rank below d).
 */
int oracle_cur_leverage(const double *X, int64_t n, int64_t d, double *lev)
{
    if (n < 1 || d < 1)
        return ORACLE_EINVAL;
    double *G = (double *)calloc((size_t)(d * d), sizeof(double));
    double *L = (double *)malloc(sizeof(double) * (size_t)(d * d));
    if (!G || !L) {
        free(G);
        free(L);
        return ORACLE_ENOMEM;
    }
    /* G[p][q] (q <= p) = sum over the rows r in order of X[r][p] X[r][q]; each
     * thread owns 16 rows of G and streams the rows of X once */
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p0 = 0; p0 < d; p0 += 16) {
        const int64_t p1 = p0 + 16 < d ? p0 + 16 : d;
        for (int64_t r = 0; r < n; ++r) {
            const double *x = X + r * d;
            for (int64_t p = p0; p < p1; ++p) {
                const double xp = x[p];
                double *g = G + p * d;
                for (int64_t q = 0; q <= p; ++q)
                    g[q] += xp * x[q];
            }
        }
    }
    for (int64_t p = 0; p < d; ++p)
        for (int64_t q = 0; q < p; ++q)
            G[q * d + p] = G[p * d + q];
    int rc = oracle_cholesky(G, d, L, NULL);
    if (rc == ORACLE_OK) {
#pragma omp parallel
        {
            double *z = (double *)malloc(sizeof(double) * (size_t)d);
#pragma omp for schedule(static)
            for (int64_t i = 0; i < n; ++i) {
                double s2 = 0.0;
                for (int64_t p = 0; p < d; ++p) {
                    double t = X[i * d + p];
                    for (int64_t k = 0; k < p; ++k)
                        t -= L[p * d + k] * z[k];
                    z[p] = t / L[p * d + p];
                    s2 += z[p] * z[p];
                }
                lev[i] = s2;
            }
            free(z);
        }
    }
    free(G);
    free(L);
    return rc;
}

/*
 * Derivative observation rows of K (Sec. Theory: force and virial targets are
 * obtained by differentiating the energy expression).  x_grad holds descriptor
 * gradients, row g = d x_{i(g)} / d r for one position coordinate, i(g) =
 * grad_atom[g].  Observation o is the weighted sum over its positions p =
 * obs_offsets[o] .. obs_offsets[o+1] (in order) of
 *   w_p d k(x_i, x_j) / dr = w_p zeta sigma_w^2 (x_i . x_j)^(zeta - 1) (x'_g . x_j),
 * g = pos_grad[p], w_p = pos_weight[p] (a force component takes w = -1 over the
 * gradients of its coordinate; a virial component w = -r over those of its
 * configuration).  K[o * M + j]; X is [n_atoms x d], XM [M x d], x_grad [n_grad x d].
 */
int oracle_kdm(const double *X, const double *x_grad, const int64_t *grad_atom, const int64_t *obs_offsets,
               int64_t n_obs, const int64_t *pos_grad, const double *pos_weight, const double *XM, int64_t M,
               int64_t d, int zeta, double sigma_w, double *K)
{
    if (n_obs < 0 || M < 1 || d < 1 || zeta < 1)
        return ORACLE_EINVAL;
    const double s2 = sigma_w * sigma_w;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t o = 0; o < n_obs; ++o) {
        for (int64_t j = 0; j < M; ++j) {
            const double *xj = XM + j * d;
            double s = 0.0;
            for (int64_t p = obs_offsets[o]; p < obs_offsets[o + 1]; ++p) {
                const int64_t g = pos_grad[p];
                const double *xi = X + grad_atom[g] * d, *xg = x_grad + g * d;
                double gi = 0.0, gp = 0.0;
                for (int64_t k = 0; k < d; ++k) {
                    gi += xi[k] * xj[k];
                    gp += xg[k] * xj[k];
                }
                double pw = 1.0;
                for (int z = 1; z < zeta; ++z)
                    pw *= gi;
                s += pos_weight[p] * (zeta * s2 * pw * gp);
            }
            K[o * M + j] = s;
        }
    }
    return ORACLE_OK;
}

/*
 * CPU oracle for the RBF-FD Laplacian stencil-weight path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header or table with the HIP
 * library: both implement the same definitions independently.
 *
 * Plain, slow, obviously correct FP64 C, one stencil at a time, one thread.
 * Build with -ffp-contract=off: the only fused multiply-adds are the explicit
 * fma() calls of the elimination and the substitutions.
 *
 * What each function computes, and where the definition comes from:
 *
 *   oracle_knn        N(x), the support of eq. (1): the k nodes nearest to x
 *                     (paper section II; support sizes of section V).  Keys are
 *                     (d2, j) in lexicographic order with
 *                     d2 = fl(fl(dx*dx) + fl(dy*dy)); NaN keys are never taken.
 *   oracle_assemble   the RBF-FD system for L = Laplacian with the polyharmonic
 *                     spline phi(r) = r^3 and all 2-D monomials of degree <= m
 *                     (sections I, II and V): M = [A P; P^T 0],
 *                     rhs = [lap phi(|x - x_k|) at x ; lap p_j at x], evaluated
 *                     on the shifted, scaled stencil (x_k - x) / s.
 *   oracle_lu         dense LU with partial pivoting, right-looking, unblocked;
 *                     multipliers formed with the reciprocal of the pivot.
 *   oracle_lu_solve   P b, forward substitution with unit L, back substitution
 *                     with U using the pivot reciprocals.
 *   oracle_weights    w of eq. (1): w_k = z_k / s^2 for the n support nodes.
 *   oracle_adjoint    dL/dx, dL/dy for all nodes from dL/dw (reverse mode of the
 *                     map above, with the scale s held fixed).
 *   oracle_lu32       oracle_lu in FP32 (fabsf, 1.0f / pivot, fmaf updates).
 *   oracle_weights_mixed  the same weights from an FP32 factorisation of the
 *                     FP64-assembled system, refined in FP64: residual
 *                     rhs - M z in FP64 (fused, columns ascending), FP32
 *                     correction solve, z += dz; converged when
 *                     |dz|_inf <= 1e-12 |z|_inf; an FP32 zero or non-finite
 *                     pivot, a correction above half the previous one (the
 *                     first is compared with the initial solve), a non-finite
 *                     value or 10 corrections without convergence send the
 *                     stencil to the FP64 path (status OR_FELL_BACK).  The
 *                     corrections applied, or tried before a fallback, are
 *                     reported per stencil.
 *   oracle_gj32       in-place Gauss-Jordan inversion in FP32 with the same
 *                     pivot rule (the pivot row scaled by 1.0f / pivot, fmaf
 *                     eliminations of every other row).
 *   oracle_weights_mixed_form  the mixed form with the FP32 factorisation
 *                     given as LU factors (form 0, as oracle_weights_mixed) or
 *                     as that Gauss-Jordan inverse, applied to each
 *                     right-hand side as a product (form 1).
 *   oracle_weights_mixed_op  the same for the operator of oracle_assemble_op
 *                     (the right-hand side and the scale's power change; the
 *                     refinement and the fallback rule do not).
 *   oracle_csr        the discrete operator of eq. (1) as a CSR matrix, with the
 *                     Dirichlet rows of section IV replaced by identity rows.
 *   oracle_spmv       y = W u - f, a sequential row sum in CSR order.
 *   oracle_time_steps the explicit pseudo-time loop of section IV, eq. (3).
 */

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Per-stencil status codes (values fixed by the library's specification). */
enum {
    OR_OK = 0,
    OR_SINGULAR = 1,      /* a pivot is exactly zero */
    OR_FELL_BACK = 2,     /* mixed precision only: FP64 fallback taken */
    OR_NONFINITE = 3,     /* non-finite coordinate, pivot or solution */
    OR_BAD_INDEX = 4,     /* a neighbour index is outside [0, n_nodes) */
    OR_DUPLICATE = 5      /* two support nodes coincide */
};

/* Argument errors returned by the entry points. */
#define OR_EARG (-1)
#define OR_ENOMEM (-2)

static int n_monomials(int m) { return (m + 1) * (m + 2) / 2; }

/* ---------------------------------------------------------------------- */
/* kNN by brute force                                                      */
/* ---------------------------------------------------------------------- */

static int key_before(double da, int64_t ja, double db, int64_t jb)
{
    return da < db || (da == db && ja < jb);
}

/* For every query node i (queries[t], or t itself when queries is NULL) the
 * k nearest nodes, ascending by (d2, j).  Unfilled slots (only possible when
 * fewer than k keys are not NaN) are -1.  nbr is [nq][k]. */
int oracle_knn(int64_t n_nodes, const double *x, const double *y, int32_t k,
               const int64_t *queries, int64_t nq, int32_t *nbr)
{
    if (n_nodes < 1 || k < 1 || k > n_nodes || nq < 0)
        return OR_EARG;
    double *bd = (double *)malloc(sizeof(double) * (size_t)k);
    int64_t *bj = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    if (!bd || !bj) {
        free(bd);
        free(bj);
        return OR_ENOMEM;
    }
    for (int64_t t = 0; t < nq; ++t) {
        int64_t i = queries ? queries[t] : t;
        if (i < 0 || i >= n_nodes) {
            free(bd);
            free(bj);
            return OR_EARG;
        }
        int cnt = 0;
        for (int64_t j = 0; j < n_nodes; ++j) {
            double dx = x[j] - x[i];
            double dy = y[j] - y[i];
            double ax = dx * dx;
            double ay = dy * dy;
            double d2 = ax + ay;
            if (isnan(d2))
                continue;
            if (cnt == k && !key_before(d2, j, bd[k - 1], bj[k - 1]))
                continue;
            /* insertion into the sorted list, dropping the last if full */
            int p = (cnt < k) ? cnt : k - 1;
            while (p > 0 && key_before(d2, j, bd[p - 1], bj[p - 1])) {
                bd[p] = bd[p - 1];
                bj[p] = bj[p - 1];
                --p;
            }
            bd[p] = d2;
            bj[p] = j;
            if (cnt < k)
                ++cnt;
        }
        for (int s = 0; s < k; ++s)
            nbr[t * k + s] = (s < cnt) ? (int32_t)bj[s] : -1;
    }
    free(bd);
    free(bj);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Assembly of the augmented system                                        */
/* ---------------------------------------------------------------------- */

/* Graded monomial order: degree 0..m, inside a degree b = 0..deg, exponent
 * pair (deg - b, b): 1, x, y, x^2, xy, y^2, x^3, x^2 y, ... */
static void monomial_exponents(int m, int *ea, int *eb)
{
    int j = 0;
    for (int deg = 0; deg <= m; ++deg)
        for (int b = 0; b <= deg; ++b) {
            ea[j] = deg - b;
            eb[j] = b;
            ++j;
        }
}

/* Values of all monomials of degree <= m at (u, v); powers by repeated
 * multiplication u^a = (...((1*u)*u)...)*u. */
static void monomials_at(int m, double u, double v, double *out)
{
    double pu[16], pv[16];
    pu[0] = 1.0;
    pv[0] = 1.0;
    for (int a = 1; a <= m; ++a) {
        pu[a] = pu[a - 1] * u;
        pv[a] = pv[a - 1] * v;
    }
    int ea[136], eb[136];
    monomial_exponents(m, ea, eb);
    for (int j = 0; j < n_monomials(m); ++j)
        out[j] = pu[ea[j]] * pv[eb[j]];
}

/*
 * Assemble M (K x K, row-major, K = n + M(m)) and rhs (K) for the stencil of
 * node i with support idx[0..n).  Returns a status code; on OR_OK also the
 * scale s.  Status precedence: BAD_INDEX, NONFINITE, DUPLICATE.
 *
 *   d_k  = (x[idx_k] - x_i, y[idx_k] - y_i)
 *   s    = sqrt(max_k fl(fl(dx_k^2) + fl(dy_k^2)))       (farthest support node)
 *   u_k  = d_k / s                                        (IEEE division)
 *   A_kl = rr_kl * sqrt(rr_kl),  rr_kl = fl(fl(ex^2) + fl(ey^2)), e = u_k - u_l
 *   P_kj = p_j(u_k)
 *   rhs_k     = 9 * sqrt(fl(fl(u_kx^2) + fl(u_ky^2)))     (lap r^3 = 9 r in 2-D)
 *   rhs_{n+j} = lap p_j(0) = 2 for x^2 and y^2, else 0
 */
/*
 * The same for other operators L (the extension to further operators of the
 * conclusions; eq. (1) changes only in its right-hand side [L phi_k; L p_j]):
 *   op 0: Laplacian, as above
 *   op 1: d/dx.  The r^3 of node k, differentiated at the centre (where the
 *         offset variable is 0) in unit-scale coordinates: 3 |0 - u_k|
 *         (0 - u_kx), computed as -3 * sqrt(fl(fl(u_kx^2) + fl(u_ky^2))) * u_kx
 *         (left to right); rhs_{n+j} = d/dx p_j(0) = 1 for p = x, else 0
 *   op 2: d/dy, likewise with u_ky and p = y
 * The weights are then z_k / s^2 for op 0 and z_k / s for ops 1 and 2
 * (a first derivative scales with 1/s).
 */
int oracle_assemble_op(int64_t n_nodes, const double *x, const double *y,
                       int64_t i, const int32_t *idx, int n, int m, int op,
                       double *M, double *rhs, double *s_out);

int oracle_assemble(int64_t n_nodes, const double *x, const double *y,
                    int64_t i, const int32_t *idx, int n, int m,
                    double *M, double *rhs, double *s_out)
{
    return oracle_assemble_op(n_nodes, x, y, i, idx, n, m, 0, M, rhs, s_out);
}

int oracle_assemble_op(int64_t n_nodes, const double *x, const double *y,
                       int64_t i, const int32_t *idx, int n, int m, int op,
                       double *M, double *rhs, double *s_out)
{
    const int NM = n_monomials(m);
    const int K = n + NM;
    if (m < 0 || m > 12 || n < 1 || n > 1024 || op < 0 || op > 2)
        return OR_EARG;
    for (int k = 0; k < n; ++k)
        if (idx[k] < 0 || (int64_t)idx[k] >= n_nodes || i < 0 || i >= n_nodes)
            return OR_BAD_INDEX;

    double *ux = (double *)malloc(sizeof(double) * (size_t)n * 2);
    double *uy = ux + n;
    double d2max = 0.0;
    int finite = 1;
    for (int k = 0; k < n; ++k) {
        double dx = x[idx[k]] - x[i];
        double dy = y[idx[k]] - y[i];
        if (!isfinite(dx) || !isfinite(dy))
            finite = 0;
        double d2 = dx * dx + dy * dy;
        if (d2 > d2max)
            d2max = d2;
        ux[k] = dx;
        uy[k] = dy;
    }
    if (!finite) {
        free(ux);
        return OR_NONFINITE;
    }
    double s = sqrt(d2max);
    if (!isfinite(s)) {
        free(ux);
        return OR_NONFINITE;
    }
    if (s == 0.0) {
        free(ux);
        return OR_DUPLICATE;
    }
    for (int k = 0; k < n; ++k) {
        ux[k] = ux[k] / s;
        uy[k] = uy[k] / s;
    }

    int dup = 0;
    memset(M, 0, sizeof(double) * (size_t)K * (size_t)K);
    double pk[136];
    for (int k = 0; k < n; ++k) {
        for (int l = 0; l < n; ++l) {
            double ex = ux[k] - ux[l];
            double ey = uy[k] - uy[l];
            double rr = ex * ex + ey * ey;
            if (l != k && rr == 0.0)
                dup = 1;
            M[k * K + l] = rr * sqrt(rr);
        }
        monomials_at(m, ux[k], uy[k], pk);
        for (int j = 0; j < NM; ++j) {
            M[k * K + n + j] = pk[j];     /* P   */
            M[(n + j) * K + k] = pk[j];   /* P^T */
        }
        double r0 = ux[k] * ux[k] + uy[k] * uy[k];
        if (op == 0)
            rhs[k] = 9.0 * sqrt(r0);
        else
            rhs[k] = -3.0 * sqrt(r0) * (op == 1 ? ux[k] : uy[k]);
    }
    int ea[136], eb[136];
    monomial_exponents(m, ea, eb);
    for (int j = 0; j < NM; ++j) {
        if (op == 0)
            rhs[n + j] = ((ea[j] == 2 && eb[j] == 0) || (ea[j] == 0 && eb[j] == 2)) ? 2.0 : 0.0;
        else if (op == 1)
            rhs[n + j] = (ea[j] == 1 && eb[j] == 0) ? 1.0 : 0.0;
        else
            rhs[n + j] = (ea[j] == 0 && eb[j] == 1) ? 1.0 : 0.0;
    }
    free(ux);
    if (dup)
        return OR_DUPLICATE;
    *s_out = s;
    return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Dense LU with partial pivoting and the two triangular solves            */
/* ---------------------------------------------------------------------- */

/*
 * In place: on return M holds L (unit diagonal, strictly below) and U (on and
 * above), perm[c] is the row swapped with row c at step c, and dinv[c] = 1/U_cc.
 * At step c the pivot is the first row r >= c with the largest |M_rc| (ties go
 * to the lowest row).  Returns OR_SINGULAR on a zero pivot, OR_NONFINITE on a
 * non-finite one.
 */
int oracle_lu(int K, double *M, int32_t *perm, double *dinv)
{
    for (int c = 0; c < K; ++c) {
        int p = c;
        double best = fabs(M[c * K + c]);
        for (int r = c + 1; r < K; ++r) {
            double v = fabs(M[r * K + c]);
            if (v > best) {
                best = v;
                p = r;
            }
        }
        if (!isfinite(best))
            return OR_NONFINITE;
        if (best == 0.0)
            return OR_SINGULAR;
        perm[c] = p;
        if (p != c)
            for (int q = 0; q < K; ++q) {
                double t = M[c * K + q];
                M[c * K + q] = M[p * K + q];
                M[p * K + q] = t;
            }
        double inv = 1.0 / M[c * K + c];
        dinv[c] = inv;
        for (int r = c + 1; r < K; ++r)
            M[r * K + c] = M[r * K + c] * inv;
        for (int r = c + 1; r < K; ++r) {
            double l = M[r * K + c];
            for (int q = c + 1; q < K; ++q)
                M[r * K + q] = fma(-l, M[c * K + q], M[r * K + q]);
        }
    }
    return OR_OK;
}

/* Solve (P^T L U) z = b in place: b <- P b, then L y = b column by column,
 * then U z = y from the last column back, z_c = y_c * dinv[c]. */
void oracle_lu_solve(int K, const double *LU, const int32_t *perm,
                     const double *dinv, double *b)
{
    for (int c = 0; c < K; ++c) {
        int p = perm[c];
        double t = b[c];
        b[c] = b[p];
        b[p] = t;
    }
    for (int c = 0; c < K; ++c)
        for (int r = c + 1; r < K; ++r)
            b[r] = fma(-LU[r * K + c], b[c], b[r]);
    for (int c = K - 1; c >= 0; --c) {
        b[c] = b[c] * dinv[c];
        for (int r = 0; r < c; ++r)
            b[r] = fma(-LU[r * K + c], b[c], b[r]);
    }
}

/* ---------------------------------------------------------------------- */
/* Weights                                                                 */
/* ---------------------------------------------------------------------- */

static int support_of(const int8_t *order, int32_t m_uniform, int32_t n_uniform,
                      const int32_t *n_for_m, int64_t i, int *m, int *n)
{
    if (!order) {
        *m = m_uniform;
        *n = n_uniform;
        return 0;
    }
    int mi = order[i];
    if (mi != 2 && mi != 4 && mi != 6)
        return OR_EARG;
    *m = mi;
    *n = n_for_m[mi / 2 - 1];
    return 0;
}

/* One stencil: z (K) and s.  Returns the status. */
static int stencil_solve(int64_t n_nodes, const double *x, const double *y,
                         int64_t i, const int32_t *idx, int n, int m, int op,
                         double *M, double *z, int32_t *perm, double *dinv,
                         double *s)
{
    const int K = n + n_monomials(m);
    int st = oracle_assemble_op(n_nodes, x, y, i, idx, n, m, op, M, z, s);
    if (st != OR_OK)
        return st;
    st = oracle_lu(K, M, perm, dinv);
    if (st != OR_OK)
        return st;
    oracle_lu_solve(K, M, perm, dinv, z);
    for (int q = 0; q < K; ++q)
        if (!isfinite(z[q]))
            return OR_NONFINITE;
    return OR_OK;
}

/*
 * Weights of eq. (1) for L = Laplacian at every listed node.
 * Node i = rows[t] (or t when rows is NULL) uses support nbr[i*k_stride ..][0..n)
 * and writes w[t*k_stride + k] = z_k / (s*s) for k < n and 0 for n <= k < k_stride;
 * a failed stencil gets NaN for k < n and its status code in status[t].
 * The order comes from order[i] (m in {2,4,6}, n = n_for_m[m/2-1]) or, when
 * order is NULL, from (m_uniform, n_uniform).
 */
static int weights_any(int64_t n_nodes, const double *x, const double *y,
                       const int32_t *nbr, int32_t k_stride,
                       const int8_t *order, int32_t m_uniform, int32_t n_uniform,
                       const int32_t *n_for_m, const int64_t *rows, int64_t n_rows,
                       int op, double *w, int32_t *status);

int oracle_weights(int64_t n_nodes, const double *x, const double *y,
                   const int32_t *nbr, int32_t k_stride,
                   const int8_t *order, int32_t m_uniform, int32_t n_uniform,
                   const int32_t *n_for_m, const int64_t *rows, int64_t n_rows,
                   double *w, int32_t *status)
{
    return weights_any(n_nodes, x, y, nbr, k_stride, order, m_uniform, n_uniform, n_for_m,
                       rows, n_rows, 0, w, status);
}

/* The weights of eq. (1) for the operator op of oracle_assemble_op (0, 1, 2);
 * otherwise as oracle_weights. */
int oracle_weights_op(int64_t n_nodes, const double *x, const double *y,
                      const int32_t *nbr, int32_t k_stride,
                      const int8_t *order, int32_t m_uniform, int32_t n_uniform,
                      const int32_t *n_for_m, const int64_t *rows, int64_t n_rows,
                      int32_t op, double *w, int32_t *status)
{
    if (op < 0 || op > 2)
        return OR_EARG;
    return weights_any(n_nodes, x, y, nbr, k_stride, order, m_uniform, n_uniform, n_for_m,
                       rows, n_rows, op, w, status);
}

static int weights_any(int64_t n_nodes, const double *x, const double *y,
                       const int32_t *nbr, int32_t k_stride,
                       const int8_t *order, int32_t m_uniform, int32_t n_uniform,
                       const int32_t *n_for_m, const int64_t *rows, int64_t n_rows,
                       int op, double *w, int32_t *status)
{
    int kmax = 0;
    if (order) {
        for (int q = 0; q < 3; ++q) {
            int K = n_for_m[q] + n_monomials(2 * q + 2);
            if (n_for_m[q] < n_monomials(2 * q + 2) || n_for_m[q] > k_stride)
                return OR_EARG;
            if (K > kmax)
                kmax = K;
        }
    } else {
        if (m_uniform < 0 || m_uniform > 12 || n_uniform < n_monomials(m_uniform) ||
            n_uniform > k_stride)
            return OR_EARG;
        kmax = n_uniform + n_monomials(m_uniform);
    }
    double *M = (double *)malloc(sizeof(double) * (size_t)kmax * (size_t)kmax);
    double *z = (double *)malloc(sizeof(double) * (size_t)kmax);
    double *dinv = (double *)malloc(sizeof(double) * (size_t)kmax);
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)kmax);
    if (!M || !z || !dinv || !perm) {
        free(M); free(z); free(dinv); free(perm);
        return OR_ENOMEM;
    }
    int rc = 0;
    for (int64_t t = 0; t < n_rows; ++t) {
        int64_t i = rows ? rows[t] : t;
        int m, n;
        if (i < 0 || i >= n_nodes ||
            support_of(order, m_uniform, n_uniform, n_for_m, i, &m, &n) != 0) {
            rc = OR_EARG;
            break;
        }
        double s = 0.0;
        int st = stencil_solve(n_nodes, x, y, i, nbr + i * (int64_t)k_stride,
                               n, m, op, M, z, perm, dinv, &s);
        double *wr = w + t * (int64_t)k_stride;
        if (st == OR_OK) {
            double sl = op == 0 ? s * s : s;
            for (int k = 0; k < n; ++k)
                wr[k] = z[k] / sl;
        } else {
            for (int k = 0; k < n; ++k)
                wr[k] = NAN;
        }
        for (int k = n; k < k_stride; ++k)
            wr[k] = 0.0;
        if (status)
            status[t] = st;
    }
    free(M); free(z); free(dinv); free(perm);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Mixed precision: FP32 factorisation, FP64 iterative refinement          */
/* ---------------------------------------------------------------------- */

/* oracle_lu in single precision (fabsf, 1.0f / pivot, fmaf updates). */
int oracle_lu32(int K, float *M, int32_t *perm, float *dinv)
{
    for (int c = 0; c < K; ++c) {
        int p = c;
        float best = fabsf(M[c * K + c]);
        for (int r = c + 1; r < K; ++r) {
            float v = fabsf(M[r * K + c]);
            if (v > best) {
                best = v;
                p = r;
            }
        }
        if (!isfinite(best))
            return OR_NONFINITE;
        if (best == 0.0f)
            return OR_SINGULAR;
        perm[c] = p;
        if (p != c)
            for (int q = 0; q < K; ++q) {
                float t = M[c * K + q];
                M[c * K + q] = M[p * K + q];
                M[p * K + q] = t;
            }
        float inv = 1.0f / M[c * K + c];
        dinv[c] = inv;
        for (int r = c + 1; r < K; ++r)
            M[r * K + c] = M[r * K + c] * inv;
        for (int r = c + 1; r < K; ++r) {
            float l = M[r * K + c];
            for (int q = c + 1; q < K; ++q)
                M[r * K + q] = fmaf(-l, M[c * K + q], M[r * K + q]);
        }
    }
    return OR_OK;
}

static void lu32_solve(int K, const float *LU, const int32_t *perm, const float *dinv, float *b)
{
    for (int c = 0; c < K; ++c) {
        int p = perm[c];
        float t = b[c];
        b[c] = b[p];
        b[p] = t;
    }
    for (int c = 0; c < K; ++c)
        for (int r = c + 1; r < K; ++r)
            b[r] = fmaf(-LU[r * K + c], b[c], b[r]);
    for (int c = K - 1; c >= 0; --c) {
        b[c] = b[c] * dinv[c];
        for (int r = 0; r < c; ++r)
            b[r] = fmaf(-LU[r * K + c], b[c], b[r]);
    }
}

/* In-place Gauss-Jordan inversion in single precision: for each column c,
 * the first largest |entry| among rows c..K-1 (rows swapped physically, as
 * oracle_lu32 does) is the pivot; the pivot row is scaled by the pivot's
 * reciprocal (1.0f / pivot) and its multiple f = M[r][c] is removed from
 * every other row r (fmaf(-f, pivot row, row)); column c of row r then holds
 * -f / pivot (as -f * reciprocal) and the pivot's place its reciprocal.  On
 * success M holds the inverse of the row-swapped matrix, (P M)^-1, and
 * perm[c] is the row swapped with row c at column c. */
int oracle_gj32(int K, float *M, int32_t *perm)
{
    for (int c = 0; c < K; ++c) {
        int p = c;
        float best = fabsf(M[c * K + c]);
        for (int r = c + 1; r < K; ++r) {
            float v = fabsf(M[r * K + c]);
            if (v > best) {
                best = v;
                p = r;
            }
        }
        if (!isfinite(best))
            return OR_NONFINITE;
        if (best == 0.0f)
            return OR_SINGULAR;
        perm[c] = p;
        if (p != c)
            for (int q = 0; q < K; ++q) {
                float t = M[c * K + q];
                M[c * K + q] = M[p * K + q];
                M[p * K + q] = t;
            }
        float inv = 1.0f / M[c * K + c];
        for (int q = 0; q < K; ++q)
            if (q != c)
                M[c * K + q] = M[c * K + q] * inv;
        M[c * K + c] = inv;
        for (int r = 0; r < K; ++r) {
            if (r == c)
                continue;
            float f = M[r * K + c];
            for (int q = 0; q < K; ++q)
                if (q != c)
                    M[r * K + q] = fmaf(-f, M[c * K + q], M[r * K + q]);
            M[r * K + c] = -f * inv;
        }
    }
    return OR_OK;
}

/* b <- (P M)^-1 P b: the row swaps applied to b, then the stored inverse
 * times it (each row a fused sum over the columns in order). */
static void gj32_apply(int K, const float *S, const int32_t *perm, float *b, float *tmp)
{
    for (int c = 0; c < K; ++c) {
        int p = perm[c];
        float t = b[c];
        b[c] = b[p];
        b[p] = t;
    }
    for (int r = 0; r < K; ++r) {
        float acc = 0.0f;
        for (int q = 0; q < K; ++q)
            acc = fmaf(S[r * K + q], b[q], acc);
        tmp[r] = acc;
    }
    for (int r = 0; r < K; ++r)
        b[r] = tmp[r];
}

#define MIXED_MAX_CORRECTIONS 10
#define MIXED_TOL 1e-12

/* One stencil, mixed precision, for the operator op of oracle_assemble_op
 * (the system is the same for every operator; only the right-hand side
 * differs).  Returns the status; *iters = number of corrections applied,
 * or tried before the stencil fell back (0 when the assembly or the FP32
 * factorisation failed). */
static int stencil_solve_mixed(int64_t n_nodes, const double *x, const double *y,
                               int64_t i, const int32_t *idx, int n, int m, int op,
                               double *M, double *z, float *M32, float *d32,
                               int32_t *perm, float *dinv32, double *dinv, double *rhs,
                               double *s, int *iters, int form)
{
    const int K = n + n_monomials(m);
    *iters = 0;
    int st = oracle_assemble_op(n_nodes, x, y, i, idx, n, m, op, M, rhs, s);
    if (st != OR_OK)
        return st;
    for (int e = 0; e < K * K; ++e)
        M32[e] = (float)M[e];
    /* form 0: LU factors and triangular solves; form 1: the Gauss-Jordan
     * inverse applied to each right-hand side (dinv32 is its scratch row) */
    int ok = (form == 0 ? oracle_lu32(K, M32, perm, dinv32) : oracle_gj32(K, M32, perm)) == OR_OK;
    if (ok) {
        for (int q = 0; q < K; ++q)
            d32[q] = (float)rhs[q];
        if (form == 0)
            lu32_solve(K, M32, perm, dinv32, d32);
        else
            gj32_apply(K, M32, perm, d32, dinv32);
        double prev = 0.0;
        for (int q = 0; q < K; ++q) {
            z[q] = (double)d32[q];
            if (fabs(z[q]) > prev)
                prev = fabs(z[q]);
        }
        int converged = 0;
        for (int it = 1; it <= MIXED_MAX_CORRECTIONS && ok; ++it) {
            for (int r = 0; r < K; ++r) {
                double acc = rhs[r];
                for (int c = 0; c < K; ++c)
                    acc = fma(-M[r * K + c], z[c], acc);
                d32[r] = (float)acc;
            }
            if (form == 0)
                lu32_solve(K, M32, perm, dinv32, d32);
            else
                gj32_apply(K, M32, perm, d32, dinv32);
            double dn = 0.0, zn = 0.0;
            int bad = 0;
            for (int q = 0; q < K; ++q) {
                z[q] = z[q] + (double)d32[q];
                double a = fabs((double)d32[q]);
                if (!isfinite(a) || !isfinite(z[q]))
                    bad = 1;
                if (a > dn)
                    dn = a;
                if (fabs(z[q]) > zn)
                    zn = fabs(z[q]);
            }
            *iters = it;
            if (bad)
                ok = 0;
            else if (dn <= MIXED_TOL * zn)
                converged = 1;
            else if (dn > 0.5 * prev)
                ok = 0;
            prev = dn;
            if (converged)
                break;
        }
        if (!converged)
            ok = 0;
    }
    if (ok)
        return OR_OK;
    /* FP64 path from scratch; *iters keeps the corrections tried */
    st = stencil_solve(n_nodes, x, y, i, idx, n, m, op, M, z, perm, dinv, s);
    return st == OR_OK ? OR_FELL_BACK : st;
}

/* As oracle_weights_op, mixed precision.  iters (may be NULL) receives the
 * number of FP64 refinement corrections per listed node.  form: 0 solves
 * with FP32 LU factors, 1 applies the FP32 Gauss-Jordan inverse. */
int oracle_weights_mixed_op(int64_t n_nodes, const double *x, const double *y,
                            const int32_t *nbr, int32_t k_stride,
                            const int8_t *order, int32_t m_uniform, int32_t n_uniform,
                            const int32_t *n_for_m, const int64_t *rows, int64_t n_rows,
                            double *w, int32_t *status, int32_t *iters, int32_t form,
                            int32_t op)
{
    if ((form != 0 && form != 1) || op < 0 || op > 2)
        return OR_EARG;
    int kmax = 0;
    if (order) {
        for (int q = 0; q < 3; ++q) {
            int K = n_for_m[q] + n_monomials(2 * q + 2);
            if (n_for_m[q] < n_monomials(2 * q + 2) || n_for_m[q] > k_stride)
                return OR_EARG;
            if (K > kmax)
                kmax = K;
        }
    } else {
        if (m_uniform < 0 || m_uniform > 12 || n_uniform < n_monomials(m_uniform) ||
            n_uniform > k_stride)
            return OR_EARG;
        kmax = n_uniform + n_monomials(m_uniform);
    }
    size_t kk = (size_t)kmax * (size_t)kmax;
    double *M = (double *)malloc(sizeof(double) * kk);
    float *M32 = (float *)malloc(sizeof(float) * kk);
    double *z = (double *)malloc(sizeof(double) * (size_t)kmax * 3);
    double *dinv = z + kmax, *rhs = z + 2 * kmax;
    float *d32 = (float *)malloc(sizeof(float) * (size_t)kmax * 2);
    float *dinv32 = d32 + kmax;
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)kmax);
    if (!M || !M32 || !z || !d32 || !perm) {
        free(M); free(M32); free(z); free(d32); free(perm);
        return OR_ENOMEM;
    }
    int rc = 0;
    for (int64_t t = 0; t < n_rows; ++t) {
        int64_t i = rows ? rows[t] : t;
        int m, n, it = 0;
        if (i < 0 || i >= n_nodes ||
            support_of(order, m_uniform, n_uniform, n_for_m, i, &m, &n) != 0) {
            rc = OR_EARG;
            break;
        }
        double s = 0.0;
        int st = stencil_solve_mixed(n_nodes, x, y, i, nbr + i * (int64_t)k_stride, n, m, op,
                                     M, z, M32, d32, perm, dinv32, dinv, rhs, &s, &it, form);
        double *wr = w + t * (int64_t)k_stride;
        if (st == OR_OK || st == OR_FELL_BACK) {
            double s2 = op == 0 ? s * s : s;
            for (int k = 0; k < n; ++k)
                wr[k] = z[k] / s2;
        } else {
            for (int k = 0; k < n; ++k)
                wr[k] = NAN;
        }
        for (int k = n; k < k_stride; ++k)
            wr[k] = 0.0;
        if (status)
            status[t] = st;
        if (iters)
            iters[t] = it;
    }
    free(M); free(M32); free(z); free(d32); free(perm);
    return rc;
}

/* The Laplacian (op 0). */
int oracle_weights_mixed_form(int64_t n_nodes, const double *x, const double *y,
                              const int32_t *nbr, int32_t k_stride,
                              const int8_t *order, int32_t m_uniform, int32_t n_uniform,
                              const int32_t *n_for_m, const int64_t *rows, int64_t n_rows,
                              double *w, int32_t *status, int32_t *iters, int32_t form)
{
    return oracle_weights_mixed_op(n_nodes, x, y, nbr, k_stride, order, m_uniform, n_uniform,
                                   n_for_m, rows, n_rows, w, status, iters, form, 0);
}

int oracle_weights_mixed(int64_t n_nodes, const double *x, const double *y,
                         const int32_t *nbr, int32_t k_stride,
                         const int8_t *order, int32_t m_uniform, int32_t n_uniform,
                         const int32_t *n_for_m, const int64_t *rows, int64_t n_rows,
                         double *w, int32_t *status, int32_t *iters)
{
    return oracle_weights_mixed_form(n_nodes, x, y, nbr, k_stride, order, m_uniform, n_uniform,
                                     n_for_m, rows, n_rows, w, status, iters, 0);
}

/* ---------------------------------------------------------------------- */
/* Adjoint                                                                 */
/* ---------------------------------------------------------------------- */

/*
 * Reverse mode of the weights map, for every node's stencil, accumulated in
 * node order.  Given G = dL/dw ([n_nodes][k_stride]), with u_k the scaled
 * offsets, (w_hat, lambda) = z and mu = M^{-1} [G/s^2 ; 0] (M is symmetric, so
 * the factors of M serve the transposed solve):
 *
 *   dL/du_k = 9 mu_k u_k / |u_k|
 *           - sum_l 3 r_kl (u_k - u_l) (mu_k w_l + mu_l w_k)
 *           - sum_j grad p_j(u_k) (mu_k lambda_j + w_k mu_{n+j})
 *
 * and, with s held fixed (w does not depend on s, so this is exact),
 * dL/dx_{idx_k} += dL/du_k / s and dL/dx_i -= dL/du_k / s.  Support nodes that
 * are the stencil's own node have u_k identically 0 and contribute nothing.
 * grad_x, grad_y are overwritten.  Returns the number of failed stencils
 * (their terms are skipped), or a negative argument error.
 */
int oracle_adjoint_rows(int64_t n_nodes, const double *x, const double *y,
                        const int32_t *nbr, int32_t k_stride,
                        const int8_t *order, int32_t m_uniform, int32_t n_uniform,
                        const int32_t *n_for_m, const double *G,
                        const int64_t *rows, int64_t n_rows,
                        double *grad_x, double *grad_y);

int oracle_adjoint(int64_t n_nodes, const double *x, const double *y,
                   const int32_t *nbr, int32_t k_stride,
                   const int8_t *order, int32_t m_uniform, int32_t n_uniform,
                   const int32_t *n_for_m, const double *G,
                   double *grad_x, double *grad_y)
{
    return oracle_adjoint_rows(n_nodes, x, y, nbr, k_stride, order, m_uniform, n_uniform,
                               n_for_m, G, NULL, n_nodes, grad_x, grad_y);
}

/* As oracle_adjoint, with only the stencils of the listed nodes (in list
 * order; rows == NULL: every node) contributing to the gradients. */
int oracle_adjoint_rows(int64_t n_nodes, const double *x, const double *y,
                        const int32_t *nbr, int32_t k_stride,
                        const int8_t *order, int32_t m_uniform, int32_t n_uniform,
                        const int32_t *n_for_m, const double *G,
                        const int64_t *rows, int64_t n_rows,
                        double *grad_x, double *grad_y)
{
    int kmax = 0;
    if (order) {
        for (int q = 0; q < 3; ++q) {
            int K = n_for_m[q] + n_monomials(2 * q + 2);
            if (K > kmax)
                kmax = K;
        }
    } else {
        kmax = n_uniform + n_monomials(m_uniform);
    }
    double *M = (double *)malloc(sizeof(double) * (size_t)kmax * (size_t)kmax);
    double *z = (double *)malloc(sizeof(double) * (size_t)kmax);
    double *mu = (double *)malloc(sizeof(double) * (size_t)kmax);
    double *dinv = (double *)malloc(sizeof(double) * (size_t)kmax);
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)kmax);
    double *ux = (double *)malloc(sizeof(double) * (size_t)kmax * 2);
    double *uy = ux + kmax;
    if (!M || !z || !mu || !dinv || !perm || !ux) {
        free(M); free(z); free(mu); free(dinv); free(perm); free(ux);
        return OR_ENOMEM;
    }
    memset(grad_x, 0, sizeof(double) * (size_t)n_nodes);
    memset(grad_y, 0, sizeof(double) * (size_t)n_nodes);
    int failed = 0;
    for (int64_t t = 0; t < n_rows; ++t) {
        const int64_t i = rows ? rows[t] : t;
        int m, n;
        if (i < 0 || i >= n_nodes ||
            support_of(order, m_uniform, n_uniform, n_for_m, i, &m, &n) != 0) {
            failed = OR_EARG;
            break;
        }
        const int NM = n_monomials(m);
        const int K = n + NM;
        const int32_t *idx = nbr + i * (int64_t)k_stride;
        double s = 0.0;
        int st = stencil_solve(n_nodes, x, y, i, idx, n, m, 0, M, z, perm, dinv, &s);
        if (st != OR_OK) {
            ++failed;
            continue;
        }
        double s2 = s * s;
        for (int k = 0; k < n; ++k)
            mu[k] = G[i * (int64_t)k_stride + k] / s2;
        for (int j = 0; j < NM; ++j)
            mu[n + j] = 0.0;
        oracle_lu_solve(K, M, perm, dinv, mu);
        for (int k = 0; k < n; ++k) {
            ux[k] = (x[idx[k]] - x[i]) / s;
            uy[k] = (y[idx[k]] - y[i]) / s;
        }
        int ea[136], eb[136];
        monomial_exponents(m, ea, eb);
        for (int k = 0; k < n; ++k) {
            if (idx[k] == i)
                continue;
            double gx = 0.0, gy = 0.0;
            double rk = sqrt(ux[k] * ux[k] + uy[k] * uy[k]);
            if (rk > 0.0) {
                gx += 9.0 * mu[k] * ux[k] / rk;
                gy += 9.0 * mu[k] * uy[k] / rk;
            }
            for (int l = 0; l < n; ++l) {
                double ex = ux[k] - ux[l];
                double ey = uy[k] - uy[l];
                double r = sqrt(ex * ex + ey * ey);
                double c = 3.0 * r * (mu[k] * z[l] + mu[l] * z[k]);
                gx -= c * ex;
                gy -= c * ey;
            }
            for (int j = 0; j < NM; ++j) {
                /* grad of u^a v^b = (a u^(a-1) v^b, b u^a v^(b-1)) */
                int a = ea[j], b = eb[j];
                double dpx = 0.0, dpy = 0.0;
                if (a > 0)
                    dpx = (double)a * pow(ux[k], a - 1) * pow(uy[k], b);
                if (b > 0)
                    dpy = (double)b * pow(ux[k], a) * pow(uy[k], b - 1);
                double c = mu[k] * z[n + j] + z[k] * mu[n + j];
                gx -= dpx * c;
                gy -= dpy * c;
            }
            gx /= s;
            gy /= s;
            grad_x[idx[k]] += gx;
            grad_y[idx[k]] += gy;
            grad_x[i] -= gx;
            grad_y[i] -= gy;
        }
    }
    free(M); free(z); free(mu); free(dinv); free(perm); free(ux);
    return failed;
}

/* ---------------------------------------------------------------------- */
/* CSR operator and SpMV                                                   */
/* ---------------------------------------------------------------------- */

/*
 * Row i: boundary -> the single entry (i, 1.0); interior -> the pairs
 * (nbr[i][k], w[i][k]), k < n_i, sorted by (column, k).  row_ptr has
 * n_nodes + 1 entries; col/val are sized by the caller to at least the nnz.
 */
int oracle_csr(int64_t n_nodes, const int32_t *nbr, int32_t k_stride,
               const int8_t *order, int32_t n_uniform, const int32_t *n_for_m,
               const double *w, const uint8_t *is_boundary,
               int64_t *row_ptr, int32_t *col, double *val)
{
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n_nodes; ++i) {
        int n = order ? n_for_m[order[i] / 2 - 1] : n_uniform;
        int64_t at = row_ptr[i];
        if (is_boundary && is_boundary[i]) {
            col[at] = (int32_t)i;
            val[at] = 1.0;
            row_ptr[i + 1] = at + 1;
            continue;
        }
        const int32_t *c = nbr + i * (int64_t)k_stride;
        const double *v = w + i * (int64_t)k_stride;
        /* selection of the entries in (column, slot) order */
        for (int k = 0; k < n; ++k) {
            int rank = 0;
            for (int l = 0; l < n; ++l)
                if (c[l] < c[k] || (c[l] == c[k] && l < k))
                    ++rank;
            col[at + rank] = c[k];
            val[at + rank] = v[k];
        }
        row_ptr[i + 1] = at + n;
    }
    return 0;
}

/* y_i = sum over the row in CSR order of fma(val, u[col], acc), minus f_i. */
int oracle_spmv(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                const double *val, const double *u, const double *f, double *y)
{
    for (int64_t i = 0; i < n_rows; ++i) {
        double acc = 0.0;
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            acc = fma(val[e], u[col[e]], acc);
        y[i] = f ? acc - f[i] : acc;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Explicit pseudo-time loop (section IV, eq. (3))                         */
/* ---------------------------------------------------------------------- */

/* n_steps steps of u_2 = u_1 + dt (f + lap u_1) at the interior nodes, the
 * Laplacian being the stencil sum over the first n supports of each row
 * (fma over k ascending from 0); t = f + sum, then u_1 + dt * t.  Boundary
 * nodes (is_boundary[i] != 0, or none when NULL) keep their values.  A
 * support index outside [0, n_nodes) makes the node's value NaN.  u holds
 * the initial values and receives the final ones. */
int oracle_time_steps(int64_t n_nodes, const int32_t *nbr, int32_t k_stride, int32_t n,
                      const double *w, const uint8_t *is_boundary, const double *f, double dt,
                      int64_t n_steps, double *u)
{
    if (n_nodes < 1 || n < 1 || k_stride < n || n_steps < 0)
        return OR_EARG;
    double *next = (double *)malloc(sizeof(double) * (size_t)n_nodes);
    if (!next)
        return OR_ENOMEM;
    for (int64_t t = 0; t < n_steps; ++t) {
        for (int64_t i = 0; i < n_nodes; ++i) {
            if (is_boundary && is_boundary[i]) {
                next[i] = u[i];
                continue;
            }
            double lap = 0.0;
            int bad = 0;
            for (int k = 0; k < n; ++k) {
                int32_t j = nbr[i * k_stride + k];
                if (j < 0 || j >= n_nodes) {
                    bad = 1;
                    continue;
                }
                lap = fma(w[i * k_stride + k], u[j], lap);
            }
            double tt = f[i] + lap;
            next[i] = bad ? NAN : u[i] + dt * tt;
        }
        memcpy(u, next, sizeof(double) * (size_t)n_nodes);
    }
    free(next);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Three dimensions (eq. (1) and eq. (2) are written for any d)            */
/* ---------------------------------------------------------------------- */

/*
 *   oracle_knn3       N(x) for nodes in R^3, keys (d2, j) with
 *                     d2 = fl(fl(fl(dx*dx) + fl(dy*dy)) + fl(dz*dz)).
 *   oracle_weights3   w of eq. (1) for L = Laplacian in d = 3: phi(r) = r^3
 *                     (lap r^3 = (3d + 3) r = 12 r), all 3-D monomials of
 *                     degree <= m in graded order (inside a degree the x
 *                     exponent descending, then the y exponent descending:
 *                     1, x, y, z, x^2, xy, xz, y^2, yz, z^2, ...), evaluated
 *                     as (u^a * v^b) * t^c with powers by repeated
 *                     multiplication; rhs_{n+j} = lap p_j(0) = 2 for x^2,
 *                     y^2, z^2, else 0.  Scale, LU, solves, w = z / s^2 and
 *                     the status rules as in two dimensions.
 */

static int n_monomials3(int m) { return (m + 1) * (m + 2) * (m + 3) / 6; }

int oracle_knn3(int64_t n_nodes, const double *x, const double *y, const double *z,
                int32_t k, const int64_t *queries, int64_t nq, int32_t *nbr)
{
    if (n_nodes < 1 || k < 1 || k > n_nodes || nq < 0)
        return OR_EARG;
    double *bd = (double *)malloc(sizeof(double) * (size_t)k);
    int64_t *bj = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    if (!bd || !bj) {
        free(bd);
        free(bj);
        return OR_ENOMEM;
    }
    for (int64_t t = 0; t < nq; ++t) {
        int64_t i = queries ? queries[t] : t;
        if (i < 0 || i >= n_nodes) {
            free(bd);
            free(bj);
            return OR_EARG;
        }
        int cnt = 0;
        for (int64_t j = 0; j < n_nodes; ++j) {
            double dx = x[j] - x[i];
            double dy = y[j] - y[i];
            double dz = z[j] - z[i];
            double ax = dx * dx;
            double ay = dy * dy;
            double az = dz * dz;
            double d2 = (ax + ay) + az;
            if (isnan(d2))
                continue;
            if (cnt == k && !key_before(d2, j, bd[k - 1], bj[k - 1]))
                continue;
            int p = (cnt < k) ? cnt : k - 1;
            while (p > 0 && key_before(d2, j, bd[p - 1], bj[p - 1])) {
                bd[p] = bd[p - 1];
                bj[p] = bj[p - 1];
                --p;
            }
            bd[p] = d2;
            bj[p] = j;
            if (cnt < k)
                ++cnt;
        }
        for (int s = 0; s < k; ++s)
            nbr[t * k + s] = (s < cnt) ? (int32_t)bj[s] : -1;
    }
    free(bd);
    free(bj);
    return 0;
}

static void monomial_exponents3(int m, int *ea, int *eb, int *ec)
{
    int j = 0;
    for (int deg = 0; deg <= m; ++deg)
        for (int a = deg; a >= 0; --a)
            for (int b = deg - a; b >= 0; --b) {
                ea[j] = a;
                eb[j] = b;
                ec[j] = deg - a - b;
                ++j;
            }
}

/* M (K x K, K = n + M3(m)) and rhs for node i of a 3-D node set; returns the
 * status and, on OR_OK, the scale s.  Same definitions as oracle_assemble
 * with a third coordinate.  op 0 is the Laplacian; ops 1, 2, 3 are d/dx,
 * d/dy, d/dz: rhs_k = -3 * sqrt(r0) * (u_k, v_k or t_k), left to right (the
 * derivative of r^3 of node k at the centre), rhs_{n+j} = 1 for the monomial
 * x, y or z, else 0. */
int oracle_assemble3_op(int64_t n_nodes, const double *x, const double *y, const double *z,
                        int64_t i, const int32_t *idx, int n, int m, int op,
                        double *M, double *rhs, double *s_out);

int oracle_assemble3(int64_t n_nodes, const double *x, const double *y, const double *z,
                     int64_t i, const int32_t *idx, int n, int m,
                     double *M, double *rhs, double *s_out)
{
    return oracle_assemble3_op(n_nodes, x, y, z, i, idx, n, m, 0, M, rhs, s_out);
}

int oracle_assemble3_op(int64_t n_nodes, const double *x, const double *y, const double *z,
                        int64_t i, const int32_t *idx, int n, int m, int op,
                        double *M, double *rhs, double *s_out)
{
    const int NM = n_monomials3(m);
    const int K = n + NM;
    if (m < 0 || m > 6 || n < 1 || n > 1024 || op < 0 || op > 3)
        return OR_EARG;
    for (int k = 0; k < n; ++k)
        if (idx[k] < 0 || (int64_t)idx[k] >= n_nodes || i < 0 || i >= n_nodes)
            return OR_BAD_INDEX;
    double *u = (double *)malloc(sizeof(double) * (size_t)n * 3);
    double *v = u + n, *t = u + 2 * n;
    double d2max = 0.0;
    int finite = 1;
    for (int k = 0; k < n; ++k) {
        double dx = x[idx[k]] - x[i];
        double dy = y[idx[k]] - y[i];
        double dz = z[idx[k]] - z[i];
        if (!isfinite(dx) || !isfinite(dy) || !isfinite(dz))
            finite = 0;
        double d2 = (dx * dx + dy * dy) + dz * dz;
        if (d2 > d2max)
            d2max = d2;
        u[k] = dx;
        v[k] = dy;
        t[k] = dz;
    }
    if (!finite) {
        free(u);
        return OR_NONFINITE;
    }
    double s = sqrt(d2max);
    if (!isfinite(s)) {
        free(u);
        return OR_NONFINITE;
    }
    if (s == 0.0) {
        free(u);
        return OR_DUPLICATE;
    }
    for (int k = 0; k < n; ++k) {
        u[k] = u[k] / s;
        v[k] = v[k] / s;
        t[k] = t[k] / s;
    }
    int ea[84], eb[84], ec[84];
    monomial_exponents3(m, ea, eb, ec);
    int dup = 0;
    memset(M, 0, sizeof(double) * (size_t)K * (size_t)K);
    for (int k = 0; k < n; ++k) {
        for (int l = 0; l < n; ++l) {
            double ex = u[k] - u[l];
            double ey = v[k] - v[l];
            double ez = t[k] - t[l];
            double rr = (ex * ex + ey * ey) + ez * ez;
            if (l != k && rr == 0.0)
                dup = 1;
            M[k * K + l] = rr * sqrt(rr);
        }
        double pu[8], pv[8], pt[8];
        pu[0] = pv[0] = pt[0] = 1.0;
        for (int a = 1; a <= m; ++a) {
            pu[a] = pu[a - 1] * u[k];
            pv[a] = pv[a - 1] * v[k];
            pt[a] = pt[a - 1] * t[k];
        }
        for (int j = 0; j < NM; ++j) {
            double p = (pu[ea[j]] * pv[eb[j]]) * pt[ec[j]];
            M[k * K + n + j] = p;
            M[(n + j) * K + k] = p;
        }
        double r0 = (u[k] * u[k] + v[k] * v[k]) + t[k] * t[k];
        if (op == 0)
            rhs[k] = 12.0 * sqrt(r0);
        else
            rhs[k] = -3.0 * sqrt(r0) * (op == 1 ? u[k] : (op == 2 ? v[k] : t[k]));
    }
    for (int j = 0; j < NM; ++j) {
        int sq = (ea[j] == 2 && eb[j] == 0 && ec[j] == 0) ||
                 (ea[j] == 0 && eb[j] == 2 && ec[j] == 0) ||
                 (ea[j] == 0 && eb[j] == 0 && ec[j] == 2);
        int lin = ea[j] + eb[j] + ec[j] == 1 &&
                  ((op == 1 && ea[j] == 1) || (op == 2 && eb[j] == 1) || (op == 3 && ec[j] == 1));
        rhs[n + j] = op == 0 ? (sq ? 2.0 : 0.0) : (lin ? 1.0 : 0.0);
    }
    free(u);
    if (dup)
        return OR_DUPLICATE;
    *s_out = s;
    return OR_OK;
}

/* Weights of eq. (1) (Laplacian, d = 3) for every listed node: node
 * i = rows[t] (or t) uses nbr[i*k_stride ..][0..n) and writes
 * w[t*k_stride + k] = z_k / (s*s) for k < n, 0 up to k_stride, NaN and the
 * status code for a failed stencil. */
int oracle_weights3_op(int64_t n_nodes, const double *x, const double *y, const double *z,
                       const int32_t *nbr, int32_t k_stride, int32_t m, int32_t n,
                       const int64_t *rows, int64_t n_rows, int32_t op, double *w,
                       int32_t *status);

int oracle_weights3(int64_t n_nodes, const double *x, const double *y, const double *z,
                    const int32_t *nbr, int32_t k_stride, int32_t m, int32_t n,
                    const int64_t *rows, int64_t n_rows, double *w, int32_t *status)
{
    return oracle_weights3_op(n_nodes, x, y, z, nbr, k_stride, m, n, rows, n_rows, 0, w,
                              status);
}

/* The weights of the operator op of oracle_assemble3_op: z_k / s^2 for the
 * Laplacian, z_k / s for the first derivatives. */
int oracle_weights3_op(int64_t n_nodes, const double *x, const double *y, const double *z,
                       const int32_t *nbr, int32_t k_stride, int32_t m, int32_t n,
                       const int64_t *rows, int64_t n_rows, int32_t op, double *w,
                       int32_t *status)
{
    if (m < 0 || m > 6 || n < n_monomials3(m) || n > k_stride || n > 1024 || op < 0 || op > 3)
        return OR_EARG;
    const int K = n + n_monomials3(m);
    double *M = (double *)malloc(sizeof(double) * (size_t)K * (size_t)K);
    double *b = (double *)malloc(sizeof(double) * (size_t)K);
    double *dinv = (double *)malloc(sizeof(double) * (size_t)K);
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)K);
    if (!M || !b || !dinv || !perm) {
        free(M); free(b); free(dinv); free(perm);
        return OR_ENOMEM;
    }
    int rc = 0;
    for (int64_t t = 0; t < n_rows; ++t) {
        int64_t i = rows ? rows[t] : t;
        if (i < 0 || i >= n_nodes) {
            rc = OR_EARG;
            break;
        }
        double s = 0.0;
        int st = oracle_assemble3_op(n_nodes, x, y, z, i, nbr + i * (int64_t)k_stride, n, m,
                                     op, M, b, &s);
        if (st == OR_OK)
            st = oracle_lu(K, M, perm, dinv);
        if (st == OR_OK) {
            oracle_lu_solve(K, M, perm, dinv, b);
            for (int q = 0; q < K; ++q)
                if (!isfinite(b[q]))
                    st = OR_NONFINITE;
        }
        double *wr = w + t * (int64_t)k_stride;
        for (int k = 0; k < n; ++k)
            wr[k] = st == OR_OK ? b[k] / (op == 0 ? s * s : s) : NAN;
        for (int k = n; k < k_stride; ++k)
            wr[k] = 0.0;
        if (status)
            status[t] = st;
    }
    free(M); free(b); free(dinv); free(perm);
    return rc;
}

/*
 * FP64 CPU oracle for the convex-regression constraint operators.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the package smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the HIP library.
 *
 * The least-squares convex-regression QP (paper, eq. "original") has one
 * constraint per ordered pair (i, j), i != j:
 *
 *     y_i >= y_j + xi_j^T (x_i - x_j)            (i = l1, j = l2)
 *
 * Written compactly (eq. "original_compact") as A1 y + A2 xi >= 0, row (i,j)
 * of A1 holds +1 in column i and -1 in column j, and row (i,j) of A2 holds
 * -(x_i - x_j)^T in block j.  The paper (Sec. II-E, ALCC) notes that the
 * costly step of every first-order iteration is multiplying by A1, A2 and
 * their transposes, and that only the points x_l need to be stored.  This file
 * is exactly those four products, written from the row definition above:
 *
 *   cro_forward : R = A1 y + A2 xi, stored as an N x N array R[i*N + j]
 *   cro_adjoint : u = A1^T z and v = A2^T z for a pair array z[i*N + j]
 *
 * Diagonal entries (i == j) are not constraints; cro_forward writes 0 there
 * and cro_adjoint ignores them.  All arithmetic is IEEE double.  Loops are
 * parallel only over the index that owns the output, and every sum runs in
 * increasing index order, so the result does not depend on the thread count.
 */
#include <stdint.h>
#include <string.h>

/* r_ij = y_i - y_j - xi_j^T (x_i - x_j): the (i,j) row of A1 y + A2 xi. */
static double pair_residual(int n, const double* X, const double* y,
                            const double* xi, int64_t i, int64_t j)
{
    const double* xi_j = xi + j * n;
    const double* x_i = X + i * n;
    const double* x_j = X + j * n;
    double hyper = 0.0;
    for (int k = 0; k < n; ++k) hyper += xi_j[k] * (x_i[k] - x_j[k]);
    return y[i] - y[j] - hyper;
}

void cro_forward(int64_t N, int n, const double* X, const double* y,
                 const double* xi, double* R)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t j = 0; j < N; ++j) {
            R[i * N + j] = (i == j) ? 0.0 : pair_residual(n, X, y, xi, i, j);
        }
    }
}

/*
 * u = A1^T z:  u_m = sum_{j != m} z_{m j} - sum_{i != m} z_{i m}
 * v = A2^T z:  v_m = - sum_{i != m} z_{i m} (x_i - x_m)       (block m, n entries)
 */
void cro_adjoint(int64_t N, int n, const double* X, const double* Z,
                 double* u, double* v)
{
#pragma omp parallel for schedule(static)
    for (int64_t m = 0; m < N; ++m) {
        double out_rows = 0.0;          /* pairs (m, j): A1 entry +1 at m */
        for (int64_t j = 0; j < N; ++j)
            if (j != m) out_rows += Z[m * N + j];
        double in_cols = 0.0;           /* pairs (i, m): A1 entry -1 at m */
        for (int64_t i = 0; i < N; ++i)
            if (i != m) in_cols += Z[i * N + m];
        u[m] = out_rows - in_cols;

        const double* x_m = X + m * n;
        for (int k = 0; k < n; ++k) {
            double acc = 0.0;           /* pairs (i, m): A2 block m is -(x_i - x_m) */
            for (int64_t i = 0; i < N; ++i)
                if (i != m) acc += Z[i * N + m] * (X[i * n + k] - x_m[k]);
            v[m * n + k] = -acc;
        }
    }
}

/* Single-pair residual, exposed so that tests can sample entries at sizes
 * where the full N x N array is not wanted. */
double cro_pair_residual(int n, const double* X, const double* y,
                         const double* xi, int64_t i, int64_t j)
{
    return pair_residual(n, X, y, xi, i, j);
}

/*
 * Column m of A1^T z and A2^T z restricted to one output index m, for a pair
 * array given only through a callback-free dense row/column: zrow[j] = z_{m j}
 * and zcol[i] = z_{i m}.  Used to check single outputs at full problem sizes.
 */
void cro_adjoint_one(int64_t N, int n, const double* X, int64_t m,
                     const double* zrow, const double* zcol,
                     double* u_m, double* v_m)
{
    double out_rows = 0.0, in_cols = 0.0;
    for (int64_t j = 0; j < N; ++j) if (j != m) out_rows += zrow[j];
    for (int64_t i = 0; i < N; ++i) if (i != m) in_cols += zcol[i];
    *u_m = out_rows - in_cols;
    const double* x_m = X + m * n;
    for (int k = 0; k < n; ++k) {
        double acc = 0.0;
        for (int64_t i = 0; i < N; ++i)
            if (i != m) acc += zcol[i] * (X[i * n + k] - x_m[k]);
        v_m[k] = -acc;
    }
}

/* Row m (pairs (m, j)) and column m (pairs (i, m)) of A1 y + A2 xi, with the
 * diagonal entry set to 0; for sampled checks at full problem sizes. */
void cro_residual_row_col(int64_t N, int n, const double* X, const double* y,
                          const double* xi, int64_t m, double* row, double* col)
{
    for (int64_t j = 0; j < N; ++j)
        row[j] = (j == m) ? 0.0 : pair_residual(n, X, y, xi, m, j);
    for (int64_t i = 0; i < N; ++i)
        col[i] = (i == m) ? 0.0 : pair_residual(n, X, y, xi, i, m);
}

/*
 * Oracle (test infrastructure only; never linked into the GPU library).
 *
 * Cyclic-by-row Jacobi eigendecomposition of a dense symmetric matrix in
 * float64 -- the textbook method (Golub & Van Loan, "symmetric Jacobi"), with
 * Rutishauser's stable choice of rotation.  The density-matrix oracle builds
 * D = sum_i f(lambda_i) q_i q_i^T from these eigenpairs (paper Sec. II.A).
 *
 * oracle_jacobi_eigh(n, A, w, V, rel_tol, max_sweeps)
 *   A   : n*n row-major symmetric input, overwritten (ends near-diagonal)
 *   w   : n eigenvalues, unsorted (diagonal of the rotated A)
 *   V   : n*n row-major, column k is the eigenvector of w[k]
 *   stop: when off(A) <= rel_tol * ||A||_F  (off = Frobenius norm of the
 *         off-diagonal part), or after max_sweeps sweeps.
 * Returns the number of sweeps run, or -1 if it did not converge.
 */
#include <math.h>
#include <stddef.h>

static double frob2(int n, const double *A) {
    double s = 0.0;
    for (size_t k = 0; k < (size_t)n * n; ++k) s += A[k] * A[k];
    return s;
}

static double off2(int n, const double *A) {
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (i != j) s += A[(size_t)i * n + j] * A[(size_t)i * n + j];
    return s;
}

int oracle_jacobi_eigh(int n, double *A, double *w, double *V, double rel_tol, int max_sweeps) {
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    const double target = rel_tol * sqrt(frob2(n, A));
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        if (sqrt(off2(n, A)) <= target) break;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                const double app = A[(size_t)p * n + p];
                const double aqq = A[(size_t)q * n + q];
                /* rotation angle: theta = (a_qq - a_pp) / (2 a_pq);
                   t = sgn(theta) / (|theta| + sqrt(1 + theta^2)) is the
                   smaller root of t^2 + 2 theta t - 1 = 0. */
                const double theta = (aqq - app) / (2.0 * apq);
                double t = 1.0 / (fabs(theta) + sqrt(1.0 + theta * theta));
                if (theta < 0.0) t = -t;
                const double c = 1.0 / sqrt(1.0 + t * t);
                const double s = t * c;
                /* A <- J^T A J with J the rotation in the (p, q) plane */
                for (int k = 0; k < n; ++k) {
                    const double akp = A[(size_t)k * n + p];
                    const double akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = c * akp - s * akq;
                    A[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = A[(size_t)p * n + k];
                    const double aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk - s * aqk;
                    A[(size_t)q * n + k] = s * apk + c * aqk;
                }
                /* the rotation zeroes the (p, q) pair exactly in exact arithmetic */
                A[(size_t)p * n + q] = 0.0;
                A[(size_t)q * n + p] = 0.0;
                /* V <- V J */
                for (int k = 0; k < n; ++k) {
                    const double vkp = V[(size_t)k * n + p];
                    const double vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = c * vkp - s * vkq;
                    V[(size_t)k * n + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
    return (sqrt(off2(n, A)) <= target) ? sweep : -1;
}

/* Reference inter-body sum, FP64, OpenMP.  TEST INFRASTRUCTURE ONLY.
 *
 * (B q)_i = sum_{j : body(j) != body(i)} G(x_i, x_j) q_j  with q_j = w_j sigma_j,
 * G(x, y) = d phi/d n(y) + gamma phi,  phi = exp(i kappa R) / (4 pi R),  R = |x - y|,
 * gamma = i eta for kappa > 0, eta at kappa = 0 (the Laplace equation of Sec. 6.1)
 * (the combined-field kernel of Sec. 2 and the naive Nystrom entries of the
 * off-diagonal blocks, Sec. 3.3).  Written straight from the definition:
 * one complex exponential per pair, no blocking, no reordering.
 *
 * x, n : [N][3] row-major; q : [r][N] complex interleaved; out : [r][nrows]
 * complex interleaved.  Returns 0.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int oracle_direct_rows(int64_t N, const double *x, const double *n, const double *q,
                       const int64_t *body, double kappa, double gam_re, double gam_im, int64_t r,
                       const int64_t *rows, int64_t nrows, double *out) {
    const double complex *qc = (const double complex *)q;
    double complex *oc = (double complex *)out;
    const double complex gam = gam_re + I * gam_im;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t a = 0; a < nrows; ++a) {
        int64_t i = rows[a];
        for (int64_t c = 0; c < r; ++c) oc[c * nrows + a] = 0.0;
        for (int64_t j = 0; j < N; ++j) {
            if (body[j] == body[i]) continue;
            double dx = x[3 * i] - x[3 * j], dy = x[3 * i + 1] - x[3 * j + 1],
                   dz = x[3 * i + 2] - x[3 * j + 2];
            double R = sqrt(dx * dx + dy * dy + dz * dz);
            double nd = n[3 * j] * dx + n[3 * j + 1] * dy + n[3 * j + 2] * dz;
            double complex phi = cexp(I * kappa * R) / (4.0 * M_PI * R);
            double complex G = phi * (nd * (1.0 - I * kappa * R) / (R * R) + gam);
            for (int64_t c = 0; c < r; ++c) oc[c * nrows + a] += G * qc[c * N + j];
        }
    }
    return 0;
}

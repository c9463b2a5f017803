/* Oracle helper: Galerkin product-rule sums for piecewise-constant bases.
 *
 * TEST INFRASTRUCTURE ONLY (part of the oracle; never linked into the
 * product library).  Plain C99, FP64, OpenMP over rows.
 *
 * out[r][c] = sum_{p,q} w_i[p] w_j[q] g(x_i[p], x_j[q])         for i != j
 *           = sum_{p,q} w_i[p] w_i[q] rho(|x_i[p] - x_i[q]|)     for i == j
 * with g(x,y) = exp(i kappa r) / (4 pi r), r = |x - y| (eq. (helmholtz)),
 * rho(r) = (exp(i kappa r) - 1) / r written as (-2 sin^2(kappa r/2) + i sin(kappa r)) / r,
 * rho(0) = i kappa.  The diagonal case returns only the bounded remainder; the
 * caller adds the closed-form Laplace part and the 1/(4 pi) factor.
 * i = rows[r], j = cols[c]; points xq[idx][nq][3], weights wq[idx][nq];
 * out is interleaved complex (re, im), row-major [nr][nc].
 */
#include <math.h>
#include <stdint.h>

void oracle_pair_sums(int64_t nr, const int64_t *rows, int64_t nc, const int64_t *cols,
                      int64_t nq, const double *xq, const double *wq, double kappa,
                      double *out)
{
    const double inv4pi = 1.0 / (4.0 * 3.14159265358979323846);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nr; ++r) {
        const int64_t i = rows[r];
        const double *xi = xq + 3 * nq * i;
        const double *wi = wq + nq * i;
        for (int64_t c = 0; c < nc; ++c) {
            const int64_t j = cols[c];
            const double *xj = xq + 3 * nq * j;
            const double *wj = wq + nq * j;
            double sre = 0.0, sim = 0.0;
            for (int64_t p = 0; p < nq; ++p) {
                for (int64_t q = 0; q < nq; ++q) {
                    double dx = xi[3 * p + 0] - xj[3 * q + 0];
                    double dy = xi[3 * p + 1] - xj[3 * q + 1];
                    double dz = xi[3 * p + 2] - xj[3 * q + 2];
                    double rr = sqrt(dx * dx + dy * dy + dz * dz);
                    double w = wi[p] * wj[q];
                    if (i != j) {
                        double f = w * inv4pi / rr;
                        sre += f * cos(kappa * rr);
                        sim += f * sin(kappa * rr);
                    } else if (rr == 0.0) {
                        sim += w * kappa;
                    } else {
                        double h = sin(0.5 * kappa * rr);
                        sre += w * (-2.0 * h * h) / rr;
                        sim += w * sin(kappa * rr) / rr;
                    }
                }
            }
            out[2 * (r * nc + c) + 0] = sre;
            out[2 * (r * nc + c) + 1] = sim;
        }
    }
}

/* FP64 direct summation oracle (CPU, OpenMP).  TEST INFRASTRUCTURE ONLY:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
 *
 * Computes the particle sum the fast multipole method approximates (the
 * N-body sum of the FMM-accelerated evaluation paragraph, Methods) with the
 * free-space Green's functions of the boundary integral formulation:
 *   Laplace  g(r) = 1 / (4 pi r)
 *   Yukawa   g(r) = exp(-kappa r) / (4 pi r)
 *   pot_i  = sum_{j : r_ij > 0} g(r_ij) q_j
 *   grad_i = sum_{j : r_ij > 0} g'(r_ij) (x_i - x_j) / r_ij q_j      (+grad_x)
 * with g'(r)/r = -(1 + kappa r) exp(-kappa r) / (4 pi r^3).
 * Pairs at zero distance (bitwise-equal coordinates) contribute nothing.
 * Every quantity is double precision; the source loop accumulates in order.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

static const double FOUR_PI = 12.566370614359172953850573533118;

void oracle_direct(int64_t nt, const double *tx, int64_t ns, const double *sx,
                   const double *q, int yukawa, double kappa,
                   double *pot, double *grad)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nt; ++i) {
        const double xi = tx[3 * i], yi = tx[3 * i + 1], zi = tx[3 * i + 2];
        double p = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
        for (int64_t j = 0; j < ns; ++j) {
            const double dx = xi - sx[3 * j], dy = yi - sx[3 * j + 1], dz = zi - sx[3 * j + 2];
            const double r2 = dx * dx + dy * dy + dz * dz;
            if (r2 == 0.0) continue;
            const double r = sqrt(r2);
            double g, dg; /* g(r) and g'(r)/r, without the 1/(4 pi) */
            if (yukawa) {
                const double e = exp(-kappa * r);
                g = e / r;
                dg = -(1.0 + kappa * r) * e / (r2 * r);
            } else {
                g = 1.0 / r;
                dg = -1.0 / (r2 * r);
            }
            p += g * q[j];
            gx += dg * dx * q[j];
            gy += dg * dy * q[j];
            gz += dg * dz * q[j];
        }
        pot[i] = p / FOUR_PI;
        if (grad) {
            grad[3 * i] = gx / FOUR_PI;
            grad[3 * i + 1] = gy / FOUR_PI;
            grad[3 * i + 2] = gz / FOUR_PI;
        }
    }
}

/* Same sum, several density columns q[c*ns + j]; outputs pot[c*nt + i],
 * grad[(c*nt + i)*3 + d]. */
void oracle_direct_multi(int64_t nt, const double *tx, int64_t ns, const double *sx,
                         const double *q, int nrhs, int yukawa, double kappa,
                         double *pot, double *grad)
{
    for (int c = 0; c < nrhs; ++c)
        oracle_direct(nt, tx, ns, sx, q + (int64_t)c * ns, yukawa, kappa,
                      pot + (int64_t)c * nt, grad ? grad + (int64_t)c * nt * 3 : NULL);
}

int oracle_num_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}

/*
 * ORACLE -- test infrastructure only.  Nothing in the product library links,
 * calls or includes this file; only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load the shared object built from it.
 *
 * Plain, slow, obviously correct CPU double-precision sums:
 *
 *   oracle_stokeslet_direct   free-space point sum with the self term
 *                             excluded (Introduction, eq. stokes_stress_sum
 *                             with the 3D Stokeslet of eq.
 *                             stokeslet_def_deriv):
 *                               u_j(x_b) = sum_{a != b} S_jl(x_b - x_a) f_{a,l},
 *                               S_jl(y) = (1/8pi) (delta_jl/r + y_j y_l / r^3).
 *
 *   oracle_stokeslet_ewald_real
 *                             the real-space half of the classical Hasimoto
 *                             (Gaussian) Ewald split of the periodic sum
 *                             (eq. periodic_sum, split eq. hasimoto-split),
 *                             written through the general residual formula
 *                             (eq. res_stokeslet / Soffdiag) with the Gaussian
 *                             window phi_G(r) = (xi/sqrt(pi)) exp(-xi^2 r^2),
 *                             whose erfc-like function is Phi_G(r) = erfc(xi r):
 *                               S_R = (1/8pi)[(erfc(xi r) - 2 xi r e^{-xi^2 r^2}/sqrt(pi)) delta/r
 *                                           + (erfc(xi r) + 2 xi r e^{-xi^2 r^2}/sqrt(pi)) y y^T / r^3].
 *                             The Fourier half and the self term live in
 *                             ewald.py.
 *
 *   oracle_stresslet_direct   free-space stresslet sum (eq. stokes_stress_sum
 *                             with the 3D stresslet of eq. stresslet_def_deriv):
 *                               u_j(x_b) = sum_{a != b} T_jlm(x_b - x_a) f_{a,l} n_{a,m},
 *                               T_jlm(y) = -(3/4pi) y_j y_l y_m / r^5.
 *
 *   oracle_stresslet_ewald_real
 *                             the real-space half of the Hasimoto (Gaussian)
 *                             Ewald split of the periodic stresslet sum, from
 *                             the general residual stresslet (eq. res_stresslet
 *                             with R_Tdiag, R_Toffd of eq. T-offd) with the
 *                             Gaussian window phi_G(r) = (xi/sqrt(pi)) e^{-xi^2 r^2},
 *                             phi_G'(r) = -2 xi^2 r phi_G(r), Phi_G = erfc(xi r):
 *                               R_Tdiag = 4 xi^2 r^3 phi_G,
 *                               R_Toffd = erfc(xi r) + 2 r phi_G + (4/3) xi^2 r^3 phi_G,
 *                               T_R : (f n^T) = R_Tdiag [(y.n) f + (y.f) n + (f.n) y] / (8 pi r^3)
 *                                             - (3/4pi) R_Toffd (y.f)(y.n) y / r^5.
 *                             The Fourier half and the k = 0 term live in ewald.py.
 *
 * Conventions: points and forces are row-major (n,3) arrays; targets are a
 * list of source indices (the target is also a source, and the pair a == b is
 * skipped).  A pair of distinct but coincident points (r == 0) contributes
 * nothing -- the paper does not define it.  Sums are Neumaier-compensated.
 */
#include <math.h>
#include <stdint.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

static inline void neumaier_add(double *s, double *c, double v)
{
    double t = *s + v;
    if (fabs(*s) >= fabs(v))
        *c += (*s - t) + v;
    else
        *c += (v - t) + *s;
    *s = t;
}

void oracle_stokeslet_direct(const double *x, const double *f, int64_t n,
                             const int64_t *tgt, int64_t m, double *u)
{
    const double c8 = 1.0 / (8.0 * M_PI);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < m; ++t) {
        const int64_t b = tgt[t];
        const double xb0 = x[3 * b], xb1 = x[3 * b + 1], xb2 = x[3 * b + 2];
        double s0 = 0, s1 = 0, s2 = 0, c0 = 0, c1 = 0, c2 = 0;
        for (int64_t a = 0; a < n; ++a) {
            if (a == b)
                continue;
            const double y0 = xb0 - x[3 * a], y1 = xb1 - x[3 * a + 1], y2 = xb2 - x[3 * a + 2];
            const double r2 = y0 * y0 + y1 * y1 + y2 * y2;
            if (r2 == 0.0)
                continue;
            const double r = sqrt(r2);
            const double ir = 1.0 / r;
            const double ir3 = ir * ir * ir;
            const double f0 = f[3 * a], f1 = f[3 * a + 1], f2 = f[3 * a + 2];
            const double yf = y0 * f0 + y1 * f1 + y2 * f2;
            neumaier_add(&s0, &c0, c8 * (f0 * ir + yf * y0 * ir3));
            neumaier_add(&s1, &c1, c8 * (f1 * ir + yf * y1 * ir3));
            neumaier_add(&s2, &c2, c8 * (f2 * ir + yf * y2 * ir3));
        }
        u[3 * t] = s0 + c0;
        u[3 * t + 1] = s1 + c1;
        u[3 * t + 2] = s2 + c2;
    }
}

/*
 * Real-space Ewald part on the unit cell [0,1)^3.  Requires rc <= 1/2, so the
 * minimum image of a difference vector is the only image that can lie within
 * rc (every other image is at least 1/2 away in some coordinate).  The pair
 * (a == b, image 0) is skipped.
 */
void oracle_stresslet_direct(const double *x, const double *f, const double *nv, int64_t n,
                             const int64_t *tgt, int64_t m, double *u)
{
    const double c = -3.0 / (4.0 * M_PI);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < m; ++t) {
        const int64_t b = tgt[t];
        const double xb0 = x[3 * b], xb1 = x[3 * b + 1], xb2 = x[3 * b + 2];
        double s0 = 0, s1 = 0, s2 = 0, c0 = 0, c1 = 0, c2 = 0;
        for (int64_t a = 0; a < n; ++a) {
            if (a == b)
                continue;
            const double y0 = xb0 - x[3 * a], y1 = xb1 - x[3 * a + 1], y2 = xb2 - x[3 * a + 2];
            const double r2 = y0 * y0 + y1 * y1 + y2 * y2;
            if (r2 == 0.0)
                continue;
            const double r = sqrt(r2);
            const double yf = y0 * f[3 * a] + y1 * f[3 * a + 1] + y2 * f[3 * a + 2];
            const double yn = y0 * nv[3 * a] + y1 * nv[3 * a + 1] + y2 * nv[3 * a + 2];
            const double w = c * yf * yn / (r2 * r2 * r);
            neumaier_add(&s0, &c0, w * y0);
            neumaier_add(&s1, &c1, w * y1);
            neumaier_add(&s2, &c2, w * y2);
        }
        u[3 * t] = s0 + c0;
        u[3 * t + 1] = s1 + c1;
        u[3 * t + 2] = s2 + c2;
    }
}

int oracle_stokeslet_ewald_real(const double *x, const double *f, int64_t n,
                                const int64_t *tgt, int64_t m, double xi, double rc,
                                double *u)
{
    if (!(rc > 0.0 && rc <= 0.5) || !(xi > 0.0))
        return -1;
    const double c8 = 1.0 / (8.0 * M_PI);
    const double two_over_sqrtpi = 2.0 / sqrt(M_PI);
    const double rc2 = rc * rc;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < m; ++t) {
        const int64_t b = tgt[t];
        const double xb0 = x[3 * b], xb1 = x[3 * b + 1], xb2 = x[3 * b + 2];
        double s0 = 0, s1 = 0, s2 = 0, c0 = 0, c1 = 0, c2 = 0;
        for (int64_t a = 0; a < n; ++a) {
            if (a == b)
                continue;
            double y0 = xb0 - x[3 * a], y1 = xb1 - x[3 * a + 1], y2 = xb2 - x[3 * a + 2];
            y0 -= nearbyint(y0);
            y1 -= nearbyint(y1);
            y2 -= nearbyint(y2);
            const double r2 = y0 * y0 + y1 * y1 + y2 * y2;
            if (r2 >= rc2 || r2 == 0.0)
                continue;
            const double r = sqrt(r2);
            const double e = erfc(xi * r);
            const double g = two_over_sqrtpi * xi * r * exp(-xi * xi * r2);
            const double sdiag = e - g, soffd = e + g;
            const double f0 = f[3 * a], f1 = f[3 * a + 1], f2 = f[3 * a + 2];
            const double yf = y0 * f0 + y1 * f1 + y2 * f2;
            const double a1 = c8 * sdiag / r, a2 = c8 * soffd * yf / (r2 * r);
            neumaier_add(&s0, &c0, a1 * f0 + a2 * y0);
            neumaier_add(&s1, &c1, a1 * f1 + a2 * y1);
            neumaier_add(&s2, &c2, a1 * f2 + a2 * y2);
        }
        u[3 * t] = s0 + c0;
        u[3 * t + 1] = s1 + c1;
        u[3 * t + 2] = s2 + c2;
    }
    return 0;
}

int oracle_stresslet_ewald_real(const double *x, const double *f, const double *nv, int64_t n,
                                const int64_t *tgt, int64_t m, double xi, double rc, double *u)
{
    if (!(rc > 0.0 && rc <= 0.5) || !(xi > 0.0))
        return -1;
    const double c8 = 1.0 / (8.0 * M_PI), c34 = 3.0 / (4.0 * M_PI);
    const double rc2 = rc * rc;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t t = 0; t < m; ++t) {
        const int64_t b = tgt[t];
        const double xb0 = x[3 * b], xb1 = x[3 * b + 1], xb2 = x[3 * b + 2];
        double s0 = 0, s1 = 0, s2 = 0, c0 = 0, c1 = 0, c2 = 0;
        for (int64_t a = 0; a < n; ++a) {
            if (a == b)
                continue;
            double y0 = xb0 - x[3 * a], y1 = xb1 - x[3 * a + 1], y2 = xb2 - x[3 * a + 2];
            y0 -= nearbyint(y0);
            y1 -= nearbyint(y1);
            y2 -= nearbyint(y2);
            const double r2 = y0 * y0 + y1 * y1 + y2 * y2;
            if (r2 >= rc2 || r2 == 0.0)
                continue;
            const double r = sqrt(r2);
            const double phi = xi / sqrt(M_PI) * exp(-xi * xi * r2);
            const double tdiag = 4.0 * xi * xi * r2 * r * phi;
            const double toffd = erfc(xi * r) + 2.0 * r * phi + (4.0 / 3.0) * xi * xi * r2 * r * phi;
            const double f0 = f[3 * a], f1 = f[3 * a + 1], f2 = f[3 * a + 2];
            const double n0 = nv[3 * a], n1 = nv[3 * a + 1], n2 = nv[3 * a + 2];
            const double yf = y0 * f0 + y1 * f1 + y2 * f2;
            const double yn = y0 * n0 + y1 * n1 + y2 * n2;
            const double fn = f0 * n0 + f1 * n1 + f2 * n2;
            const double d = c8 * tdiag / (r2 * r);
            const double o = c34 * toffd * yf * yn / (r2 * r2 * r);
            neumaier_add(&s0, &c0, d * (yn * f0 + yf * n0 + fn * y0) - o * y0);
            neumaier_add(&s1, &c1, d * (yn * f1 + yf * n1 + fn * y1) - o * y1);
            neumaier_add(&s2, &c2, d * (yn * f2 + yf * n2 + fn * y2) - o * y2);
        }
        u[3 * t] = s0 + c0;
        u[3 * t + 1] = s1 + c1;
        u[3 * t + 2] = s2 + c2;
    }
    return 0;
}

int oracle_num_threads(void)
{
    int nt = 1;
#pragma omp parallel
    {
#pragma omp master
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            nt = omp_get_num_threads();
#endif
        }
    }
    return nt;
}

/* Sets the number of OpenMP threads later oracle calls use (timing only; the
 * per-target sums do not depend on it). */
void oracle_set_num_threads(int nt)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(nt > 0 ? nt : 1);
#else
    (void)nt;
#endif
}

// Host-side kernel-splitting mathematics (double precision, once per tolerance).
#include "kernel_math.hpp"

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>

namespace dmk {

namespace {
constexpr double kPi = 3.14159265358979323846;

struct Row {
    double tol;
    int q, p, n1, nper, ns;
    int p_used;      // Chebyshev order the plan uses
    int q_used = 0;  // window parameter the plan uses (0: the printed q)
};
// Table "tab:params" (Stokeslet, PSWF split) and the 3D leaf sizes of
// Sec. "Numerical results".  The table was tuned on uniform free-space
// points; on periodic and clustered inputs p = 33 at 1e-9 leaves errors at or
// just above the tolerance (the Chebyshev interpolation term dominates: a
// larger q makes it worse, a larger p removes it), so that row is stepped up
// to p = 36 in the spirit of the parameter-selection discussion of Sec.
// "Error control and parameter selection".
const Row kRows[4] = {
    {1e-3, 10, 12, 19, 3, 600, 12},
    {1e-6, 17, 23, 33, 5, 1200, 23},
    {1e-9, 25, 33, 49, 9, 2000, 36},
    {1e-12, 31, 44, 61, 11, 3000, 44},
};
// The Gaussian columns of the same table: q = (6/pi) sigma^-2, p^G, N_1^G,
// N_per^G.  Only the rows down to 1e-6 are offered: from 1e-9 on the
// Gaussian's radial fits need more than the 24 coefficients the near-field
// kernel holds in scalar registers (and the 1e-12 row, p^G = 58, also exceeds
// the compiled proxy kernels).  Measured on periodic, 9-level clustered and
// shallow 500-point inputs, the printed rows leave up to 1.05 tol (1e-3) and
// 0.88 tol (1e-6); they run as (q, p) = (14, 16) and (27, 33), at most 0.36
// tol on the same inputs.
// Stresslet columns (prolate) of the same table.  Measured against direct
// sums, the printed rows leave errors of 1.0 to 1.9 times the tolerance on
// some inputs: shallow trees of a few hundred points with random orientation
// vectors are the hardest (up to 1.9 tol at 1e-3, 1.6 at 1e-6), clustered
// inputs of 9 levels next.  Both the Fourier truncation (q) and the
// interpolation (p) contribute; stepping both up, in the spirit of the
// parameter-selection discussion of Sec. "Error control and parameter
// selection", gives at most 0.37, 0.26, 0.39 and 0.79 tol on the same
// inputs: (q, p) = (11, 14), (19, 26), (26, 36), (32, 48).  (At 1e-12 a
// larger q makes the residual's radial functions need more than the 24
// coefficients the near-field kernel holds.)
const Row kRowsT[4] = {
    {1e-3, 9, 11, 17, 3, 600, 14, 11},
    {1e-6, 17, 22, 33, 5, 1200, 26, 19},
    {1e-9, 25, 33, 49, 9, 2000, 36, 26},
    {1e-12, 32, 44, 63, 11, 3000, 48, 32},
};
const Row kRowsG[2] = {
    {1e-3, 14, 14, 27, 5, 600, 16, 14},
    {1e-6, 25, 28, 49, 9, 1200, 33, 27},
};
}  // namespace

bool select_params(double tol, Params* out, int window, int kernel)
{
    if (kernel == 1 && window != 0)
        return false;
    const Row* rows = kernel == 1 ? kRowsT : (window == 1 ? kRowsG : kRows);
    const int nrow = window == 1 ? 2 : 4;
    const double tmin = window == 1 ? 1e-6 : 1e-12;
    if (!(tol >= tmin * (1 - 1e-9) && tol <= 1e-3 * (1 + 1e-9)))
        return false;
    const double lt = std::log10(tol);
    int hit = -1;
    for (int i = 0; i < nrow; ++i)
        if (std::fabs(lt - std::log10(rows[i].tol)) < 1e-9)
            hit = i;
    if (hit < 0) {
        // between rows: the row with the largest tolerance below tol
        hit = 0;
        while (hit < nrow - 1 && rows[hit].tol > tol)
            ++hit;
    }
    const int q = rows[hit].q_used > 0 ? rows[hit].q_used : rows[hit].q;
    out->tol = tol;
    out->kernel = kernel;
    out->window = window;
    out->q = q;
    out->c = q * kPi / 3.0;
    out->sigma = window == 1 ? std::sqrt(6.0 / (kPi * q)) : 0.0;
    out->p = rows[hit].p_used;
    // strict truncation |k_i| < K_max / r_{l+1} with h_l = 2 pi/(3 r_l)
    // (Sec. "Error control and parameter selection") gives |m_i| <= q-1
    out->n1 = 2 * q - 1;
    // periodic root k = 2 pi kappa, |k_i| < K_max
    out->nper = 2 * ((q + 5) / 6) - 1;
    out->ns = rows[hit].ns;
    return true;
}

void override_params(Params* prm, int q, int p)
{
    if (q > 0) {
        prm->q = q;
        prm->c = q * kPi / 3.0;
        prm->sigma = prm->window == 1 ? std::sqrt(6.0 / (kPi * q)) : 0.0;
        prm->n1 = 2 * q - 1;
        prm->nper = 2 * ((q + 5) / 6) - 1;
    }
    if (p > 0)
        prm->p = p;
}

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double pp = 0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
            }
            pp = n * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / pp;
            z -= dz;
            if (std::fabs(dz) < 1e-16)
                break;
        }
        {
            double p0 = 1.0, p1 = 0.0;
            for (int j = 1; j <= n; ++j) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
            }
            pp = n * (z * p0 - p1) / (z * z - 1.0);
        }
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

// ---------------------------------------------------------------------------
// Prolate: the prolate operator L = -d/dx (1-x^2) d/dx + c^2 x^2 is symmetric
// tridiagonal on the even normalised Legendre functions sqrt(k+1/2) P_k.
// psi_0 is its eigenvector of smallest eigenvalue (published Legendre-Galerkin
// approach for prolates; the operator commutes with the band-limited Fourier
// operator that defines psi_0 in Sec. "Prolate spheroidal wave functions").
Prolate::Prolate(double c) : c_(c)
{
    const int M = (int)(0.6 * c) + 32;
    std::vector<double> d(M), e(M, 0.0);
    for (int i = 0; i < M; ++i) {
        const double k = 2.0 * i;
        d[i] = k * (k + 1) + c * c * (2 * k * k + 2 * k - 1) / ((2 * k - 1) * (2 * k + 3));
        if (i + 1 < M)
            e[i] = c * c * (k + 1) * (k + 2) / ((2 * k + 3) * std::sqrt((2 * k + 1) * (2 * k + 5)));
    }
    // smallest eigenvalue by Sturm-sequence bisection
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < M; ++i) {
        const double rad = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + std::fabs(e[i]);
        lo = std::min(lo, d[i] - rad);
        hi = std::max(hi, d[i] + rad);
    }
    auto count_below = [&](double x) {
        int cnt = 0;
        double q = d[0] - x;
        if (q < 0)
            ++cnt;
        for (int i = 1; i < M; ++i) {
            if (q == 0.0)
                q = 1e-300;
            q = (d[i] - x) - e[i - 1] * e[i - 1] / q;
            if (q < 0)
                ++cnt;
        }
        return cnt;
    };
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (count_below(mid) >= 1)
            hi = mid;
        else
            lo = mid;
        if (hi - lo <= 1e-15 * std::max(1.0, std::fabs(hi)))
            break;
    }
    chi_ = 0.5 * (lo + hi);
    // inverse iteration (tridiagonal solve without pivoting, slightly shifted)
    const double shift = chi_ - 1e-10 * std::max(1.0, std::fabs(chi_));
    std::vector<double> v(M, 1.0), cp(M), dp(M);
    for (int it = 0; it < 4; ++it) {
        double b0 = d[0] - shift;
        cp[0] = e[0] / b0;
        dp[0] = v[0] / b0;
        for (int i = 1; i < M; ++i) {
            const double den = (d[i] - shift) - e[i - 1] * cp[i - 1];
            cp[i] = (i + 1 < M ? e[i] / den : 0.0);
            dp[i] = (v[i] - e[i - 1] * dp[i - 1]) / den;
        }
        v[M - 1] = dp[M - 1];
        for (int i = M - 2; i >= 0; --i)
            v[i] = dp[i] - cp[i] * v[i + 1];
        double nrm = 0;
        for (double a : v)
            nrm += a * a;
        nrm = std::sqrt(nrm);
        for (double& a : v)
            a /= nrm;
    }
    beta_.resize(M);
    // psi(0) > 0: P_{2i}(0) = (-1)^i (2i-1)!!/(2i)!!
    double psi0 = 0, p0 = 1.0;
    for (int i = 0; i < M; ++i) {
        if (i > 0)
            p0 *= -(2.0 * i - 1) / (2.0 * i);
        psi0 += v[i] * std::sqrt(2.0 * i + 0.5) * p0;
    }
    const double sgn = psi0 > 0 ? 1.0 : -1.0;
    for (int i = 0; i < M; ++i)
        beta_[i] = sgn * v[i] * std::sqrt(2.0 * i + 0.5);  // coefficient of plain P_{2i}
    // int_{-1}^{1} psi = 2 * beta_0 (only P_0 has a nonzero integral)
    norm_ = 2.0 * beta_[0];
    std::vector<double> x, w;
    gauss_legendre(320, x, w);
    gl_t_.resize(320);
    gl_w_.resize(320);
    for (int i = 0; i < 320; ++i) {
        gl_t_[i] = 0.5 * (x[i] + 1.0);
        gl_w_[i] = 0.5 * w[i];
    }
    gl_phi_.resize(320);
    for (int i = 0; i < 320; ++i)
        gl_phi_[i] = gl_w_[i] * phi(gl_t_[i]);
}

void Prolate::legendre_all(double x, std::vector<double>& P) const
{
    const int n = 2 * (int)beta_.size() + 1;
    P.resize(n + 1);
    P[0] = 1.0;
    P[1] = x;
    for (int j = 1; j < n; ++j)
        P[j + 1] = ((2.0 * j + 1) * x * P[j] - j * P[j - 1]) / (j + 1);
}

double Prolate::phi(double r) const
{
    r = std::fabs(r);
    if (r > 1.0)
        return 0.0;
    std::vector<double> P;
    legendre_all(r, P);
    double s = 0;
    for (size_t i = 0; i < beta_.size(); ++i)
        s += beta_[i] * P[2 * i];
    return s / norm_;
}

double Prolate::dphi(double r) const
{
    const double sg = r < 0 ? -1.0 : 1.0;
    r = std::fabs(r);
    if (r > 1.0)
        return 0.0;
    std::vector<double> P;
    legendre_all(r, P);
    // P'_{n+1} = P'_{n-1} + (2n+1) P_n
    const int n = (int)P.size();
    std::vector<double> dP(n, 0.0);
    dP[0] = 0.0;
    if (n > 1)
        dP[1] = 1.0;
    for (int j = 1; j + 1 < n; ++j)
        dP[j + 1] = dP[j - 1] + (2.0 * j + 1) * P[j];
    double s = 0;
    for (size_t i = 0; i < beta_.size(); ++i)
        s += beta_[i] * dP[2 * i];
    return sg * s / norm_;
}

double Prolate::int_phi(double r) const
{
    r = std::min(std::fabs(r), 1.0);
    std::vector<double> P;
    legendre_all(r, P);
    // int_0^r P_0 = r;  int_0^r P_n = (P_{n+1}(r) - P_{n-1}(r))/(2n+1) for even n >= 2
    double s = beta_[0] * r;
    for (size_t i = 1; i < beta_.size(); ++i) {
        const int n = 2 * (int)i;
        s += beta_[i] * (P[n + 1] - P[n - 1]) / (2.0 * n + 1);
    }
    return s / norm_;
}

double Prolate::Phi(double r) const
{
    r = std::fabs(r);
    if (r >= 1.0)
        return 0.0;
    return 1.0 - 2.0 * int_phi(r);
}

double Prolate::phihat(double k) const
{
    double s = 0;
    for (size_t i = 0; i < gl_t_.size(); ++i)
        s += gl_phi_[i] * std::cos(k * gl_t_[i]);
    return 2.0 * s;
}

double Prolate::dphihat(double k) const
{
    double s = 0;
    for (size_t i = 0; i < gl_t_.size(); ++i)
        s += gl_phi_[i] * gl_t_[i] * std::sin(k * gl_t_[i]);
    return -2.0 * s;
}

double Prolate::gammahat(double k) const
{
    return phihat(k) - 0.5 * k * dphihat(k);
}

double ChebFit::eval(double s) const
{
    const double t = 2.0 * s - 1.0;
    double b1 = 0, b2 = 0;
    for (int k = (int)a.size() - 1; k >= 1; --k) {
        const double b0 = 2.0 * t * b1 - b2 + a[k];
        b2 = b1;
        b1 = b0;
    }
    return t * b1 - b2 + a[0];
}

double GaussWindow::phi(double r) const
{
    r = std::fabs(r);
    return r <= 1.0 ? std::exp(-r * r / (s_ * s_)) / (s_ * std::sqrt(kPi)) : 0.0;
}
double GaussWindow::dphi(double r) const
{
    return std::fabs(r) <= 1.0 ? -2.0 * r / (s_ * s_) * std::exp(-r * r / (s_ * s_)) / (s_ * std::sqrt(kPi)) : 0.0;
}
double GaussWindow::Phi(double r) const { return std::erfc(std::fabs(r) / s_); }
double GaussWindow::phihat(double k) const { return std::exp(-k * k * s_ * s_ / 4.0); }
double GaussWindow::dphihat(double k) const { return -0.5 * k * s_ * s_ * phihat(k); }
double GaussWindow::gammahat(double k) const { return phihat(k) - 0.5 * k * dphihat(k); }

RadialFits fit_radial(const Window& w, double fit_tol)
{
    // E(s) = int_0^1 phi(rho v) dv,  E - G = -rho int_0^1 v phi'(rho v) dv
    // (integration by parts, no cancellation), Q = (E - G)/s.
    std::vector<double> gx, gw;
    gauss_legendre(120, gx, gw);
    for (size_t i = 0; i < gx.size(); ++i) {
        gx[i] = 0.5 * (gx[i] + 1.0);
        gw[i] *= 0.5;
    }
    auto PQ = [&](double s, double* P, double* Q) {
        const double rho = std::sqrt(s);
        double E = 0, H = 0;
        for (size_t i = 0; i < gx.size(); ++i) {
            E += gw[i] * w.phi(rho * gx[i]);
            H += gw[i] * gx[i] * w.dphi(rho * gx[i]);
        }
        const double G = w.phi(rho);
        *P = E + G;
        *Q = -H / rho;  // (E-G)/s = -rho H / rho^2
    };
    const int N = 96;
    std::vector<double> fp(N), fq(N);
    for (int j = 0; j < N; ++j) {
        const double s = 0.5 * (1.0 + std::cos((2.0 * j + 1) * kPi / (2.0 * N)));
        PQ(s, &fp[j], &fq[j]);
    }
    auto coeffs = [&](const std::vector<double>& f) {
        std::vector<double> a(N);
        for (int k = 0; k < N; ++k) {
            double s = 0;
            for (int j = 0; j < N; ++j)
                s += f[j] * std::cos(k * (2.0 * j + 1) * kPi / (2.0 * N));
            a[k] = (k == 0 ? 1.0 : 2.0) * s / N;
        }
        return a;
    };
    // keep coefficients up to the point where the series first stays below
    // the threshold for 8 consecutive terms (beyond it is rounding noise)
    auto trunc = [&](std::vector<double> a, double scale) {
        const double thr = std::max(fit_tol, 2e-14) * scale;
        int d = (int)a.size() - 1;
        for (int k = 1; k + 8 < (int)a.size(); ++k) {
            bool small = true;
            for (int j = k; j < k + 8; ++j)
                small = small && std::fabs(a[j]) < thr;
            if (small) {
                d = k - 1;
                break;
            }
        }
        a.resize(d + 1);
        return a;
    };
    RadialFits out;
    double scale = std::fabs(fp[N - 1]);  // ~P(0) = 2 phi(0)
    for (double v : fp)
        scale = std::max(scale, std::fabs(v));
    out.P.a = trunc(coeffs(fp), scale);
    out.Q.a = trunc(coeffs(fq), scale);
    out.max_err_P = out.max_err_Q = 0;
    for (int j = 0; j <= 200; ++j) {
        const double s = j / 200.0 * (1 - 1e-12) + 1e-12;
        double P, Q;
        PQ(s, &P, &Q);
        out.max_err_P = std::max(out.max_err_P, std::fabs(out.P.eval(s) - P));
        out.max_err_Q = std::max(out.max_err_Q, std::fabs(out.Q.eval(s) - Q));
    }
    return out;
}

RadialFits fit_radial_stresslet(const Window& w, double fit_tol)
{
    // psi(sigma) = phi'(r)/r, r = sqrt(sigma), smooth in sigma (phi is even);
    // A(s) = (1/s) int_0^1 u^2 [psi(s) - psi(s u^2)] du (from E - G =
    // -rho^2 int_0^1 u^2 psi(s u^2) du and rho phi'(rho)/3 = rho^2 psi(s)/3,
    // no cancellation at small s), D(s) = -psi(s).
    std::vector<double> gx, gw;
    gauss_legendre(120, gx, gw);
    for (size_t i = 0; i < gx.size(); ++i) {
        gx[i] = 0.5 * (gx[i] + 1.0);
        gw[i] *= 0.5;
    }
    auto psi = [&](double sig) {
        const double r = std::sqrt(sig);
        return w.dphi(r) / r;
    };
    auto AD = [&](double s, double* A, double* D) {
        const double ps = psi(s);
        double acc = 0;
        for (size_t i = 0; i < gx.size(); ++i)
            acc += gw[i] * gx[i] * gx[i] * (ps - psi(s * gx[i] * gx[i]));
        *A = acc / s;
        *D = -ps;
    };
    const int N = 96;
    std::vector<double> fa(N), fd(N);
    for (int j = 0; j < N; ++j) {
        const double s = 0.5 * (1.0 + std::cos((2.0 * j + 1) * kPi / (2.0 * N)));
        AD(s, &fa[j], &fd[j]);
    }
    auto coeffs = [&](const std::vector<double>& f) {
        std::vector<double> a(N);
        for (int k = 0; k < N; ++k) {
            double acc = 0;
            for (int j = 0; j < N; ++j)
                acc += f[j] * std::cos(k * (2.0 * j + 1) * kPi / (2.0 * N));
            a[k] = (k == 0 ? 1.0 : 2.0) * acc / N;
        }
        return a;
    };
    auto trunc = [&](std::vector<double> a, double scale) {
        const double thr = std::max(fit_tol, 2e-14) * scale;
        int d = (int)a.size() - 1;
        for (int k = 1; k + 8 < (int)a.size(); ++k) {
            bool small = true;
            for (int j = k; j < k + 8; ++j)
                small = small && std::fabs(a[j]) < thr;
            if (small) {
                d = k - 1;
                break;
            }
        }
        a.resize(d + 1);
        return a;
    };
    double scale = 1.0;
    for (int j = 0; j < N; ++j)
        scale = std::max({scale, std::fabs(fa[j]), std::fabs(fd[j])});
    RadialFits out;
    out.P.a = trunc(coeffs(fa), scale);
    out.Q.a = trunc(coeffs(fd), scale);
    out.max_err_P = out.max_err_Q = 0;
    for (int j = 0; j <= 200; ++j) {
        const double s = j / 200.0 * (1 - 1e-12) + 1e-12;
        double A, D;
        AD(s, &A, &D);
        out.max_err_P = std::max(out.max_err_P, std::fabs(out.P.eval(s) - A));
        out.max_err_Q = std::max(out.max_err_Q, std::fabs(out.Q.eval(s) - D));
    }
    return out;
}

void cheb_nodes(int p, std::vector<double>& t, std::vector<double>& bw)
{
    t.resize(p);
    bw.resize(p);
    for (int a = 0; a < p; ++a) {
        const double th = (2.0 * a + 1) * kPi / (2.0 * p);
        t[a] = std::cos(th);
        bw[a] = ((a & 1) ? -1.0 : 1.0) * std::sin(th);
    }
}

void lagrange_basis(const std::vector<double>& t, const std::vector<double>& bw, double x, double* out)
{
    const int p = (int)t.size();
    for (int a = 0; a < p; ++a)
        if (x == t[a]) {
            for (int b = 0; b < p; ++b)
                out[b] = (a == b) ? 1.0 : 0.0;
            return;
        }
    double den = 0;
    for (int a = 0; a < p; ++a) {
        out[a] = bw[a] / (x - t[a]);
        den += out[a];
    }
    for (int a = 0; a < p; ++a)
        out[a] /= den;
}

double btrunc_hat(double k, double R)
{
    const double x = k * R;
    if (x >= 0.2)
        return (1.0 + 0.5 * std::cos(x) - 1.5 * std::sin(x) / x) / (k * k * k * k);
    // 1 + cos(x)/2 - 3 sin(x)/(2x) = sum_{n>=2} (-1)^n x^{2n} [1/(2 (2n)!) - 3/(2 (2n+1)!)]
    double acc = 0, f2n = 24.0;  // (2n)! at n = 2
    double x2 = x * x, xp = 1.0;  // x^{2n-4}
    for (int n = 2; n < 12; ++n) {
        if (n > 2)
            f2n *= (2.0 * n - 1) * (2.0 * n);
        const double f2n1 = f2n * (2.0 * n + 1);
        acc += ((n & 1) ? -1.0 : 1.0) * (0.5 / f2n - 1.5 / f2n1) * xp;
        xp *= x2;
    }
    return acc * R * R * R * R;
}

namespace {

void plane_wave_mats(int p, int mmax, double alpha, const std::vector<double>& t,
                     std::vector<std::complex<double>>& e_half, std::vector<std::complex<double>>& e_full,
                     std::vector<std::complex<double>>& g_half, std::vector<std::complex<double>>& g_full)
{
    // outgoing: exp(-i alpha m t_a); incoming: exp(+i alpha m t_a) (weight 2 for m1 > 0)
    const int nh = mmax + 1, nf = 2 * mmax + 1;
    e_half.resize((size_t)nh * p);
    e_full.resize((size_t)nf * p);
    g_half.resize((size_t)p * nh);
    g_full.resize((size_t)p * nf);
    for (int m = 0; m < nh; ++m)
        for (int a = 0; a < p; ++a) {
            const double ph = alpha * m * t[a];
            e_half[(size_t)m * p + a] = std::complex<double>(std::cos(ph), -std::sin(ph));
            g_half[(size_t)a * nh + m] = (m == 0 ? 1.0 : 2.0) * std::complex<double>(std::cos(ph), std::sin(ph));
        }
    for (int mi = 0; mi < nf; ++mi)
        for (int a = 0; a < p; ++a) {
            const double ph = alpha * (mi - mmax) * t[a];
            e_full[(size_t)mi * p + a] = std::complex<double>(std::cos(ph), -std::sin(ph));
            g_full[(size_t)a * nf + mi] = std::complex<double>(std::cos(ph), std::sin(ph));
        }
}

Tables::PW fold_pw(int p, int M, double theta, const std::vector<double>& t)
{
    const int h = (p + 1) / 2;
    Tables::PW w;
    w.M = M;
    w.out.resize((size_t)2 * (M + 1) * h);
    w.in_full.resize((size_t)2 * h * (M + 1));
    w.in_half.resize((size_t)2 * h * (M + 1));
    for (int m = 0; m <= M; ++m)
        for (int j = 0; j < h; ++j) {
            const double ph = theta * m * t[j];
            const double c = std::cos(ph), s = std::sin(ph);
            w.out[2 * ((size_t)m * h + j)] = c;
            w.out[2 * ((size_t)m * h + j) + 1] = s;
            w.in_full[2 * ((size_t)j * (M + 1) + m)] = c;
            w.in_full[2 * ((size_t)j * (M + 1) + m) + 1] = s;
            const double wm = m == 0 ? 1.0 : 2.0;
            w.in_half[2 * ((size_t)j * (M + 1) + m)] = wm * c;
            w.in_half[2 * ((size_t)j * (M + 1) + m) + 1] = wm * s;
        }
    return w;
}

Tables* build_tables(const Params& prm)
{
    const double tol = prm.tol;
    Tables* T = new Tables();
    T->prm = prm;
    Prolate wp(prm.window == 1 ? 1.0 : prm.c);
    GaussWindow wg(prm.sigma > 0 ? prm.sigma : 1.0);
    const Window& w = prm.window == 1 ? (const Window&)wg : (const Window&)wp;
    T->phi0 = w.phi(0.0);
    T->fits = prm.kernel == 1 ? fit_radial_stresslet(w, 1e-3 * tol) : fit_radial(w, 1e-3 * tol);
    const int p = prm.p, q = prm.q;
    std::vector<double> t, bw;
    cheb_nodes(p, t, bw);
    T->cheb_t = t;
    T->up.assign((size_t)p * 2 * p, 0.0);
    T->down.assign((size_t)2 * p * p, 0.0);
    std::vector<double> L(p);
    for (int A = 0; A < 2 * p; ++A) {
        const double x = A < p ? 0.5 * (t[A] - 1.0) : 0.5 * (t[A - p] + 1.0);
        lagrange_basis(t, bw, x, L.data());
        for (int a = 0; a < p; ++a) {
            T->up[(size_t)a * 2 * p + A] = L[a];
            T->down[(size_t)A * p + a] = L[a];
        }
    }
    plane_wave_mats(p, q - 1, kPi / 3.0, t, T->e_half, T->e_full, T->g_half, T->g_full);
    const int m2max = 3 * (q - 1) * (q - 1);
    T->wdiff.assign(m2max + 1, 0.0);
    for (int m2 = 1; m2 <= m2max; ++m2) {
        const double m = std::sqrt((double)m2);
        T->wdiff[m2] = (w.gammahat(kPi * m / 3.0) - w.gammahat(2.0 * kPi * m / 3.0)) / (12.0 * kPi * kPi * m2);
    }
    // stresslet difference symbol i [(m_m d_jl + m_j d_lm + m_l d_mj) m^2 - 2 m_j m_l m_m] W_t(|m|),
    // from eq. moll_stresslet at k = h_l m with weight (h_l / 2 pi)^3: W_t = dgammahat / (18 pi |m|^4) / r_l^2
    T->wdiff_t.assign(m2max + 1, 0.0);
    for (int m2 = 1; m2 <= m2max; ++m2) {
        const double m = std::sqrt((double)m2);
        T->wdiff_t[m2] = (w.gammahat(kPi * m / 3.0) - w.gammahat(2.0 * kPi * m / 3.0)) / (18.0 * kPi * m2 * m2);
    }
    // free-space root: truncated kernel B^R with R = 1 + sqrt(3) on the unit
    // box; M_0^R is supported in |x| <= R + 1, differences of root proxy
    // nodes have |x_i| <= 1, so a trapezoid period P > 3 + sqrt(3) avoids
    // aliasing.  Modes up to |k_i| <= 1.25 c.
    T->root_R = 1.0 + std::sqrt(3.0);
    T->root_period = 5.0;
    T->root_m = (int)std::ceil(1.25 * prm.c * T->root_period / (2.0 * kPi));
    plane_wave_mats(p, T->root_m, kPi / T->root_period, t, T->r_e_half, T->r_e_full, T->r_g_half, T->r_g_full);
    const int r2max = 3 * T->root_m * T->root_m;
    T->wroot.assign(r2max + 1, 0.0);
    for (int m2 = 1; m2 <= r2max; ++m2) {
        const double k = 2.0 * kPi * std::sqrt((double)m2) / T->root_period;
        const double P3 = T->root_period * T->root_period * T->root_period;
        T->wroot[m2] = k * k * btrunc_hat(k, T->root_R) * w.gammahat(k) / P3;
    }
    T->wroot_t.assign(r2max + 1, 0.0);
    for (int m2 = 1; m2 <= r2max; ++m2) {
        const double k = 2.0 * kPi * std::sqrt((double)m2) / T->root_period;
        const double P3 = T->root_period * T->root_period * T->root_period;
        T->wroot_t[m2] = btrunc_hat(k, T->root_R) * w.gammahat(k) / P3;
    }
    // periodic root: Poisson summation over k = 2 pi kappa, k = 0 dropped
    T->per_m = (prm.nper - 1) / 2;
    plane_wave_mats(p, T->per_m, kPi, t, T->p_e_half, T->p_e_full, T->p_g_half, T->p_g_full);
    const int p2max = 3 * T->per_m * T->per_m;
    T->wper.assign(p2max + 1, 0.0);
    for (int m2 = 1; m2 <= p2max; ++m2) {
        const double k = 2.0 * kPi * std::sqrt((double)m2);
        T->wper[m2] = w.gammahat(k) / (k * k);
    }
    T->wper_t.assign(p2max + 1, 0.0);
    for (int m2 = 1; m2 <= p2max; ++m2) {
        const double k = 2.0 * kPi * std::sqrt((double)m2);
        T->wper_t[m2] = w.gammahat(k) / (k * k * k * k);
    }
    // folded stage matrices
    const int h = (p + 1) / 2;
    T->pw = fold_pw(p, q - 1, kPi / 3.0, t);
    T->pw_root = fold_pw(p, T->root_m, kPi / T->root_period, t);
    T->pw_per = fold_pw(p, T->per_m, kPi, t);
    T->merge_mat.resize((size_t)2 * h * p);
    for (int i = 0; i < h; ++i)
        for (int j = 0; j < p; ++j) {
            const double a = T->up[(size_t)i * 2 * p + j], b = T->up[(size_t)i * 2 * p + (2 * p - 1 - j)];
            T->merge_mat[2 * ((size_t)i * p + j)] = 0.5 * (a + b);
            T->merge_mat[2 * ((size_t)i * p + j) + 1] = 0.5 * (a - b);
        }
    T->interp_mat.resize((size_t)2 * p * h);
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < h; ++j) {
            const double a = T->down[(size_t)i * p + j], b = T->down[(size_t)i * p + (p - 1 - j)];
            T->interp_mat[2 * ((size_t)i * h + j)] = 0.5 * (a + b);
            T->interp_mat[2 * ((size_t)i * h + j) + 1] = 0.5 * (a - b);
        }
    return T;
}

}  // namespace

const Tables* get_tables(const Params& prm)
{
    static std::mutex mu;
    static std::map<std::tuple<double, int, int, int>, Tables*> cache;
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_tuple(prm.tol, prm.window * 2 + prm.kernel, prm.q, prm.p);
    auto it = cache.find(key);
    if (it != cache.end())
        return it->second;
    Tables* T = build_tables(prm);
    if (T)
        cache[key] = T;
    return T;
}

const Tables* get_tables(double tol)
{
    Params prm;
    if (!select_params(tol, &prm))
        return nullptr;
    return get_tables(prm);
}

}  // namespace dmk

namespace dmk {

static bool ewald_grid_build(const Params& prm, int L, EwaldGrid* out);

bool ewald_grid(const Params& prm, int L, EwaldGrid* out)
{
    // the symbol table costs about 10^4 mollifier evaluations: computed once
    // per (tolerance, q, split level) and process
    static std::mutex mu;
    static std::map<std::tuple<double, int, int>, EwaldGrid> cache;
    const auto key = std::make_tuple(prm.tol, prm.q, L);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            *out = it->second;
            return true;
        }
    }
    if (!ewald_grid_build(prm, L, out))
        return false;
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = *out;
    return true;
}

static bool ewald_grid_build(const Params& prm, int L, EwaldGrid* out)
{
    if (L < 1 || L > 8 || prm.window != 0 || prm.kernel != 0)
        return false;
    EwaldGrid& E = *out;
    E.L = L;
    const double rc = 1.0 / (double)(1 << L);
    // strict |k_i| < c / r_c with k = 2 pi kappa: |kappa_i| < q 2^L / 6
    const double lim = prm.q * (double)(1 << L) / 6.0;
    E.K = (int)std::ceil(lim) - 1;
    // gridding kernel width: the aliasing error of a prolate kernel of width w
    // at oversampling sigma falls like exp(-pi w (1 - 1/(2 sigma)))
    E.w = prm.tol >= 1e-3 * (1 - 1e-9) ? 6 : prm.tol >= 1e-6 * (1 - 1e-9) ? 8 : prm.tol >= 1e-9 * (1 - 1e-9) ? 11 : 0;
    if (E.w == 0)
        return false;
    // grid M = B 2^Lt, B in {6, 8}, the smallest with oversampling >= 1.9
    const int need = (int)std::ceil(1.9 * (2 * E.K + 1));
    int best = 0, bB = 0, bL = 0;
    for (int B : {6, 8})
        for (int Lt = 0; Lt <= 9; ++Lt) {
            const int M = B << Lt;
            // the interpolation block holds one component's (B + w)^3 region and
            // the stencil weights of 64 points in LDS: at most 80 KB, two blocks per CU
            const bool fits =
                (size_t)(B + E.w) * (B + E.w) * (B + E.w) * 8 + 64 * 3 * 12 * 8 + 64 * 3 * 4 <= 80 * 1024;
            if (M >= need && (best == 0 || M < best) && 2 * B >= E.w && fits) {
                best = M;
                bB = B;
                bL = Lt;
            }
        }
    if (best == 0)
        return false;
    E.M = best;
    E.B = bB;
    E.Lt = bL;
    E.sigma = (double)E.M / (2 * E.K + 1);
    E.beta = kPi * E.w * (1.0 - 1.0 / (2.0 * E.sigma));
    const Prolate g(E.beta);
    const double g0 = g.phi(0.0);
    // Chebyshev coefficients in v = 2 t^2 - 1 on [-1, 1]
    const int N = 64;
    std::vector<double> fv(N);
    for (int j = 0; j < N; ++j) {
        const double v = std::cos((2.0 * j + 1) * kPi / (2.0 * N));
        fv[j] = g.phi(std::sqrt(0.5 * (v + 1.0))) / g0;
    }
    std::vector<double> a(N);
    for (int k = 0; k < N; ++k) {
        double acc = 0;
        for (int j = 0; j < N; ++j)
            acc += fv[j] * std::cos(k * (2.0 * j + 1) * kPi / (2.0 * N));
        a[k] = (k == 0 ? 1.0 : 2.0) * acc / N;
    }
    // keep the terms up to where the series first stays below 1e-15 for 6
    // consecutive terms (beyond it is rounding noise)
    int d = N - 1;
    for (int k = 1; k + 6 < N; ++k) {
        bool small = true;
        for (int j = k; j < k + 6; ++j)
            small = small && std::fabs(a[j]) < 1e-15;
        if (small) {
            d = k - 1;
            break;
        }
    }
    a.resize(d + 1);
    E.g_cheb = a;
    // ghat: g as a function of x in cell units has half-width alpha = w / (2M):
    // ghat(k) = alpha phihat(k alpha) / phi(0)
    const double alpha = E.w / (2.0 * E.M);
    E.ghat.assign(E.M / 2 + 1, 0.0);
    for (int kap = 0; kap <= E.M / 2; ++kap)
        E.ghat[kap] = alpha * g.phihat(2.0 * kPi * kap * alpha) / g0;
    // symbol with the grid factors h^6 folded in
    const double h = 1.0 / E.M, h6 = h * h * h * h * h * h;
    const Prolate win(prm.c);
    const int m2max = 3 * E.K * E.K;
    E.wsym.assign(m2max + 1, 0.0);
    for (int m2 = 1; m2 <= m2max; ++m2) {
        const double k = 2.0 * kPi * std::sqrt((double)m2);
        E.wsym[m2] = h6 * win.gammahat(k * rc) / (k * k);
    }
    return true;
}

}  // namespace dmk

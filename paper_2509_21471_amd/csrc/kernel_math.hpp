// Host-side kernel-splitting mathematics for the DMK Stokeslet: parameter
// selection, the prolate window, the biharmonic mollifier, the radial fits
// used by the near-field kernel and the level-independent Fourier tables.
// Everything here runs once per tolerance in double precision.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace dmk {

// Parameters for one tolerance (Table "tab:params", Stokeslet, PSWF columns;
// leaf size from Sec. "Numerical results").
struct Params {
    double tol;
    int kernel;   // 0: Stokeslet, 1: stresslet
    int window;   // 0: prolate (PSWF), 1: Gaussian
    int q;        // 3c/pi (prolate) or (6/pi) sigma^-2 (Gaussian)
    double c;     // Fourier truncation K_max = q pi / 3 (the PSWF band limit; 2/sigma^2 for the Gaussian)
    double sigma; // Gaussian shape parameter (0 for the prolate)
    int p;        // Chebyshev points per dimension on every proxy grid
    int n1;       // plane-wave modes per dimension, 2q - 1
    int nper;     // periodic root modes per dimension, 2 ceil(q/6) - 1
    int ns;       // maximum points per leaf
};

// Returns false if tol is outside [1e-12, 1e-3] (Gaussian window: [1e-6, 1e-3]).
bool select_params(double tol, Params* out, int window = 0, int kernel = 0);
// Replaces q (and with it c, n1, nper) and/or p when the value is > 0.
void override_params(Params* prm, int q, int p);

// Zeroth-order prolate spheroidal wave function psi_0^c as an even Legendre
// series (Legendre-Galerkin form of the prolate differential operator,
// smallest eigenvalue; sign psi(0) > 0) and the window phi = psi / int psi.
// The window function of the split and the quantities the tables need
// (eqs. wfunchat_prol_G / wfunc_prol_G, def_erfc_like_fcn, gammaB_in_phi).
class Window {
  public:
    virtual ~Window() = default;
    virtual double phi(double r) const = 0;       // |r| <= 1, else 0
    virtual double dphi(double r) const = 0;
    virtual double Phi(double r) const = 0;       // 1 - 2 int_0^r phi
    virtual double phihat(double k) const = 0;
    virtual double dphihat(double k) const = 0;
    virtual double gammahat(double k) const = 0;  // phihat - k phihat'/2
};

// Gaussian window phi(r) = exp(-r^2/sigma^2) / (sigma sqrt(pi)), truncated at
// r = 1; phihat(k) = exp(-k^2 sigma^2/4), Phi = erfc(r/sigma) (the Hasimoto
// split, eq. hasimoto-split).
class GaussWindow : public Window {
  public:
    explicit GaussWindow(double sigma) : s_(sigma) {}
    double phi(double r) const override;
    double dphi(double r) const override;
    double Phi(double r) const override;
    double phihat(double k) const override;
    double dphihat(double k) const override;
    double gammahat(double k) const override;

  private:
    double s_;
};

class Prolate : public Window {
  public:
    explicit Prolate(double c);
    double c() const { return c_; }
    double phi(double r) const override;       // |r| <= 1, else 0
    double dphi(double r) const override;
    double int_phi(double r) const;            // int_0^r phi, r in [0,1]
    double Phi(double r) const override;       // 2 int_r^inf phi = 1 - 2 int_0^r phi
    double phihat(double k) const override;    // int phi(t) e^{-ikt} dt
    double dphihat(double k) const override;
    double gammahat(double k) const override;  // phihat - k phihat'/2
    double chi() const { return chi_; }

  private:
    void legendre_all(double x, std::vector<double>& P) const;
    double c_, chi_, norm_;
    std::vector<double> beta_;  // coefficient of normalised P_{2i}
    std::vector<double> gl_t_, gl_w_, gl_phi_;  // Gauss-Legendre on [0,1] for transforms
};

// Chebyshev series on s in [0,1] (t = 2s-1), evaluated by Clenshaw.
struct ChebFit {
    std::vector<double> a;
    double eval(double s) const;
};

// Radial functions of the residual Stokeslet at unit scale, written as
//   S_R(y) = S(y) - [P(s) I + Q(s) y y^T] / (4 pi),  s = |y|^2,  |y| < 1,
// with E(s) = rho^{-1} int_0^rho phi, G(s) = phi(rho), rho = sqrt(s),
// P = E + G and Q = (E - G)/s  (rearrangement of eq. res_stokeslet/Soffdiag).
struct RadialFits {
    ChebFit P, Q;
    double max_err_P, max_err_Q;
};
RadialFits fit_radial(const Window& w, double fit_tol);
// Radial functions of the residual stresslet at unit scale (eq. res_stresslet
// with R_Tdiag, R_Toffd of eq. T-offd, rearranged):
//   T_R(y) = T(y) + (3/(2 pi)) A(s) y y y + (1/(4 pi)) D(s) (delta y + ...),
// A(s) = [E - G + rho phi'(rho)/3] / s^2,  D(s) = -phi'(rho)/rho,  s = |y|^2.
// Returned in the P (= A) and Q (= D) slots.
RadialFits fit_radial_stresslet(const Window& w, double fit_tol);

// Single-level spectral Ewald on the periodic unit cell with the prolate
// split at r_c = 2^-L (the uniform-data variant of the method, Sec.
// "Ewald summation"): near field = the residual between cells of side r_c;
// far field = sum over 0 < |kappa_i| <= K of (I - k k^T/k^2) gammahat(k r_c)/k^2
// F(k) e^{ik.x}, k = 2 pi kappa, by spreading to an M^3 grid with a prolate
// gridding kernel of w points, FFT, scaling, inverse FFT and interpolation.
struct EwaldGrid {
    int L;            // split level
    int K;            // |kappa_i| <= K (strict |k_i| < c / r_c)
    int M;            // grid points per dimension, M = B 2^Lt
    int B, Lt;        // tile side in grid points, tile level
    int w;            // gridding kernel width in grid points
    double beta;      // prolate parameter of the gridding kernel
    double sigma;     // oversampling M / (2K + 1)
    // gridding kernel g(t) = psi_0^beta(t)/psi_0^beta(0), |t| <= 1, t = (X - n)/(w/2)
    // in grid units, as sum_k a_k T_k(2 t^2 - 1)
    std::vector<double> g_cheb;
    std::vector<double> ghat;   // kappa = 0..M/2: 1D transform of g(x) at k = 2 pi kappa (x in cell units)
    std::vector<double> wsym;   // by |kappa|^2 <= 3 K^2: h^6 gammahat(k r_c)/k^2 (0 at kappa = 0)
};
// Fills the grid parameters for tol's row (q) and split level L (1..8);
// false when the kernel width the tolerance needs does not fit the LDS tiles.
bool ewald_grid(const Params& prm, int L, EwaldGrid* out);

// Gauss-Legendre nodes and weights on [-1,1].
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);

// Chebyshev nodes of the first kind t_a = cos((2a+1) pi / (2p)), a = 0..p-1,
// and barycentric Lagrange basis evaluation.
void cheb_nodes(int p, std::vector<double>& t, std::vector<double>& bw);
void lagrange_basis(const std::vector<double>& t, const std::vector<double>& bw,
                    double x, double* out);

// Truncated biharmonic symbol in 3D (eq. Btrunc_hat).
double btrunc_hat(double k, double R);

// All per-tolerance tables, in the layouts the device kernels use.
struct Tables {
    Params prm;
    RadialFits fits;
    double phi0;                 // phi(0)
    std::vector<double> cheb_t;  // p nodes
    // child interpolation: up[a][A] = L_a(child node A), A in [0,2p):
    // A < p -> lower child (x = (t_A - 1)/2), else upper child (x = (t_{A-p}+1)/2)
    std::vector<double> up;      // p x 2p
    std::vector<double> down;    // 2p x p  (down[A][a] = up[a][A])
    // plane waves at level l: k = h_l m, h_l = 2 pi /(3 r_l), phases (pi/3) m t_a
    std::vector<std::complex<double>> e_half;   // q  x p : exp(-i pi/3 m t_a), m = 0..q-1
    std::vector<std::complex<double>> e_full;   // n1 x p : exp(-i pi/3 m t_a), m = -(q-1)..q-1
    std::vector<std::complex<double>> g_half;   // p x q  : w(m) exp(+i pi/3 m t_a), w = 1 (m=0) or 2
    std::vector<std::complex<double>> g_full;   // p x n1 : exp(+i pi/3 m t_a)
    std::vector<double> wdiff;   // by |m|^2: [gammahat(pi|m|/3) - gammahat(2 pi |m|/3)]/(12 pi^2 |m|^2)
    // stresslet: by |m|^2: [gammahat(pi|m|/3) - gammahat(2 pi |m|/3)]/(18 pi |m|^4)
    std::vector<double> wdiff_t;
    // free-space root: truncated mollified kernel (eq. Bmollhat_trunc) on a
    // trapezoid grid of period root_period, modes |m_i| <= root_m
    double root_period, root_R;
    int root_m;
    std::vector<std::complex<double>> r_e_half, r_e_full, r_g_half, r_g_full;
    std::vector<double> wroot;   // by |m|^2: (1/P^3) k^2 Bhat^R(k) gammahat(k), k = 2 pi |m| / P
    std::vector<double> wroot_t; // stresslet: by |m|^2: (1/P^3) Bhat^R(k) gammahat(k)
    // periodic root: k = 2 pi kappa, |kappa_i| <= per_m
    int per_m;
    std::vector<std::complex<double>> p_e_half, p_e_full, p_g_half, p_g_full;
    std::vector<double> wper;    // by |kappa|^2: gammahat(2 pi |kappa|) / (4 pi^2 |kappa|^2)
    std::vector<double> wper_t;  // stresslet: by |kappa|^2: gammahat(k) / k^4, k = 2 pi |kappa|
    // folded stage matrices, (Me, Mo) pairs, row-major Nh x Kh (see the
    // separable-stage kernel): h = ceil(p/2)
    struct PW {
        int M;                    // modes -M..M (half axis 0..M)
        std::vector<double> out;  // (M+1) x h : cos(th m t_j), sin(th m t_j)
        std::vector<double> in_full;  // h x (M+1): cos(th m t_i), sin(th m t_i)
        std::vector<double> in_half;  // h x (M+1): w_m cos, w_m sin, w_0 = 1, w_m = 2
    };
    PW pw, pw_root, pw_per;
    std::vector<double> merge_mat;   // h x p  : (up[i][j] +- up[i][2p-1-j]) / 2
    std::vector<double> interp_mat;  // p x h  : (down[i][j] +- down[i][p-1-j]) / 2
};

// Builds (and caches per tolerance) the tables.  Returns nullptr on bad tol.
const Tables* get_tables(double tol);
// Tables for explicit parameters (cached per (tol, window, q, p)).
const Tables* get_tables(const Params& prm);

}  // namespace dmk

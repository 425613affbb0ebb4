"""Pins for the oracle's kernel-splitting functions.

Each check is fixed by the paper's mathematics rather than by re-typing a
formula:
* the prolate function satisfies the integral eigen-relation of Sec.
  "Prolate spheroidal wave functions" and is positive and even;
* phihat(k) = psi(k/c)/psi(0) for |k| <= c (eq. PSWFhat / wfunchat_prol_G),
  computed here by quadrature of the window;
* the mollifier conditions gammahat(0) = 1, gammahat''(0) = 0
  (Definition wfunhat) and the 1D inverse transform of eq.
  biharmonic_screen_R;
* with a Gaussian window the generic formulas reproduce the Hasimoto split
  (eq. hasimoto-split) and its derivatives (eq. BR_ders);
* the residual Stokeslet equals D_S applied to the residual biharmonic of
  Theorem Bres (eq. BR_gen with eq. dsf);
* residual + mollified = full Stokeslet, the mollified part by the appendix's
  independent Fourier route (eqs. STterms, dFterms, msdiag);
* compact support (Corollary, eq. reskernelproperty) and the self term
  (eq. S_self) obtained three ways."""
import numpy as np
import pytest
import scipy.special as sp
from numpy.polynomial.legendre import leggauss

from oracle import splitting as S

QS = [10, 17, 25, 31]


@pytest.fixture(scope="module", params=QS)
def win(request):
    return S.ProlateWindow(S.prolate_c(request.param))


def test_prolate_eigen_relation(win):
    t, w = leggauss(300)
    psi_t = win.psi(t)
    xs = np.linspace(-1.0, 1.0, 23)
    lhs = np.array([(psi_t * np.cos(win.c * t * x) * w).sum() for x in xs])
    lam = (psi_t * w).sum() / win.psi(0.0)  # lambda psi(0) = int psi
    assert np.max(np.abs(lhs - lam * win.psi(xs))) < 1e-12 * win.psi(0.0)
    assert np.all(win.psi(np.linspace(-1, 1, 101)) > 0)
    assert np.max(np.abs(win.psi(xs) - win.psi(-xs))) < 1e-13 * win.psi(0.0)


def test_window_normalisation_and_transform(win):
    assert abs(win.Phi(0.0)[0] - 1.0) < 5e-14
    assert abs(win.Phi(1.0)[0]) < 1e-13
    k = np.linspace(0.0, win.c, 9)
    ph = win.phihat(k)
    assert abs(ph[0] - 1.0) < 1e-13
    assert np.allclose(ph, win.psi(k / win.c) / win.psi(0.0), rtol=0, atol=1e-12)


def test_mollifier_conditions(win):
    assert abs(win.gammahat(0.0)[0] - 1.0) < 1e-13
    h = 1e-2
    g = win.gammahat(np.array([-2 * h, -h, 0.0, h, 2 * h]))
    d2 = (-g[0] + 16 * g[1] - 30 * g[2] + 16 * g[3] - g[4]) / (12 * h * h)
    phd2 = win.phihat(np.array([-h, 0.0, h]))
    assert abs(d2) < 1e-6 * abs((phd2[0] - 2 * phd2[1] + phd2[2]) / h ** 2)


def test_gamma_1d_inverse_transform(win):
    # gamma(x) = (1/pi) int_0^inf cos(kx) gammahat(k) dk = (3/2) phi + (1/2) x phi'
    t, w = leggauss(40)
    edges = np.linspace(0.0, 300.0, 301)
    ks = (0.5 * (t[None, :] + 1) + edges[:-1, None]).ravel()
    ws = np.tile(0.5 * w, 300)
    gh = win.gammahat(ks)
    for x in (0.0, 0.2, 0.45, 0.7):
        num = (np.cos(ks * x) * gh * ws).sum() / np.pi
        ref = 1.5 * win.phi(x) + 0.5 * x * win.dphi(x)
        # the truncated window's transform has a tail ~phi(1) cos(k); allow that
        assert abs(num - ref) < 1e-8 + 50 * win.phi(1.0)


def test_gaussian_window_is_hasimoto():
    xi = 7.0
    g = S.GaussianWindow(xi)
    r = np.linspace(0.01, 0.6, 25)
    assert np.allclose(g.Phi(r), sp.erfc(xi * r), rtol=0, atol=1e-14)
    ex = 2 * xi * r * np.exp(-(xi * r) ** 2) / np.sqrt(np.pi)
    assert np.allclose(g.Sdiag(r), sp.erfc(xi * r) - ex, atol=1e-14)
    assert np.allclose(g.Soffd(r), sp.erfc(xi * r) + ex, atol=1e-14)
    # Hasimoto residual biharmonic and its derivatives (eq. BR_ders)
    sig = 1 / xi
    BR = lambda rr: -rr / (8 * np.pi) * sp.erfc(rr / sig) + sig / (8 * np.pi ** 1.5) * np.exp(-rr ** 2 / sig ** 2)
    h = 1e-4
    d1 = (BR(r + h) - BR(r - h)) / (2 * h)
    d2 = (BR(r + h) - 2 * BR(r) + BR(r - h)) / h ** 2
    assert np.allclose(d1, -g.Phi(r) / (8 * np.pi), atol=1e-9)
    assert np.allclose(d2, g.phi(r) / (4 * np.pi), atol=1e-6)
    # gammahat of the Gaussian window is the Hasimoto mollifier
    k = np.linspace(0, 40, 9)
    assert np.allclose(g.gammahat(k), np.exp(-k ** 2 / (4 * xi ** 2)) * (1 + k ** 2 / (4 * xi ** 2)), atol=1e-12)


def test_residual_from_residual_biharmonic(win):
    """Sdiag = -8 pi (B_R' + r B_R''), Soffd = 8 pi (-B_R' + r B_R'') (appendix,
    d = 3) with B_R from Theorem Bres evaluated by quadrature."""
    t, w = leggauss(80)

    def BR(r):
        a = np.array([(win.phi(rr * 0.5 * (t + 1)) * 0.5 * w).sum() * rr for rr in np.atleast_1d(r)])
        b = np.array([(rr * 0.5 * (t + 1) * win.phi(rr * 0.5 * (t + 1)) * 0.5 * w).sum() * rr for rr in np.atleast_1d(r)])
        inf = (0.5 * (t + 1) * win.phi(0.5 * (t + 1)) * 0.5 * w).sum()
        return -(r - 2 * r * a + 2 * b - 2 * inf) / (8 * np.pi)

    r = np.linspace(0.05, 0.95, 10)
    h = 1e-3
    d1 = (BR(r - 2 * h) - 8 * BR(r - h) + 8 * BR(r + h) - BR(r + 2 * h)) / (12 * h)
    d2 = (-BR(r + 2 * h) + 16 * BR(r + h) - 30 * BR(r) + 16 * BR(r - h) - BR(r - 2 * h)) / (12 * h * h)
    assert np.allclose(-8 * np.pi * (d1 + r * d2), win.Sdiag(r), atol=2e-8)
    assert np.allclose(8 * np.pi * (-d1 + r * d2), win.Soffd(r), atol=2e-8)


@pytest.mark.parametrize("q", [17, 25])
def test_residual_plus_mollified_is_full(q):
    win = S.ProlateWindow(S.prolate_c(q))
    r = np.array([0.03, 0.1, 0.25, 0.5, 0.8, 0.97, 1.2, 1.6])
    md, mo = S.mollified_S_fourier(win, r, kmax=400.0)
    tol = 2e-8 + 20 * win.phi(1.0)
    assert np.allclose(win.Sdiag(r) + md, 1.0, atol=tol)
    assert np.allclose(win.Soffd(r) + mo, 1.0, atol=tol)


def test_compact_support(win):
    r = np.array([1.0, 1.0 + 1e-9, 1.3, 2.0])
    assert np.all(win.Sdiag(r[1:]) == 0.0) and np.all(win.Soffd(r[1:]) == 0.0)
    assert abs(win.Sdiag(np.array([1 - 1e-12]))[0]) < 3 * win.phi(1.0)
    y = np.array([[0.0, 0.0, 0.5], [0.3, 0.0, 0.0]])
    Sr = S.residual_stokeslet(win, y, nu=0.25)
    assert np.all(Sr == 0.0)


def test_self_term_three_ways(win):
    # (1) eq. S_self: lim S_M = phi(0)/(2 pi) I
    ref = win.phi(0.0) / (2 * np.pi)
    # (2) closed form: S_M = S - S_R at tiny r
    y = np.array([[1e-5, 2e-5, -1.5e-5]])
    SM = S.stokeslet(y) - S.residual_stokeslet(win, y)
    assert np.allclose(SM[0], ref * np.eye(3), rtol=0, atol=1e-8 * ref)
    # (3) appendix: S_M(0) = (1/8pi) (8/(3 pi)) int_0^inf gammahat dk
    t, w = leggauss(40)
    K = 200.0 * np.pi + np.pi / 2  # end on a zero of the cos tail
    edges = np.linspace(0.0, K, 401)
    ks = (0.5 * (edges[1:] - edges[:-1])[:, None] * (t[None, :] + 1) + edges[:-1, None]).ravel()
    ws = (0.5 * (edges[1:] - edges[:-1])[:, None] * w[None, :]).ravel()
    val = (8 / (3 * np.pi)) * (win.gammahat(ks) * ws).sum() / (8 * np.pi)
    assert abs(val - ref) < 1e-8 + 10 * win.phi(1.0)

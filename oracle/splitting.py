"""ORACLE -- test infrastructure only.  Kernel-splitting functions in float64.

An independent evaluation of the pieces of the biharmonic/Stokeslet split,
used to pin the method's host tables and its residual-kernel pair sums.  It
shares no code with the product library: the prolate function comes from a
Chebyshev collocation of the prolate differential operator (the product uses a
Legendre-Galerkin form), every integral is a Gauss-Legendre quadrature
written out here.

Definitions followed (section / equation of the paper):

* window (Sec. "Prolate spheroidal wave functions", eq. wfunc_prol_G):
    phi(r) = psi_0^c(r) / int_{-1}^{1} psi_0^c,  |r| <= 1, and 0 for |r| > 1;
* erfc-like function (eq. def_erfc_like_fcn): Phi(r) = 2 int_r^inf phi
  = 1 - 2 int_0^r phi;
* 1D transform phihat(k) = int phi(t) e^{-ikt} dt = 2 int_0^1 phi(t) cos(kt) dt;
* biharmonic mollifier (eq. gammaB_in_phi): gammahat = phihat - k phihat'/2;
* residual Stokeslet (eq. res_stokeslet, Soffdiag) at length scale nu
  (the remark on scaling: real-space functions at r/nu):
    S_R(y) = Sdiag(r/nu) I/(8 pi r) + Soffd(r/nu) y y^T/(8 pi r^3),
    Sdiag = Phi - 2 rho phi,  Soffd = Phi + 2 rho phi;
* mollified Stokeslet by the numerical Fourier route of the appendix
  (eqs. STterms, dFterms, msdiag): radial Gauss-Legendre integrals of the
  differentiated sinc kernel against the truncated biharmonic symbol
  (eq. Btrunc_hat) times gammahat, plus the constant correction 2r/R.
"""
from __future__ import annotations

import numpy as np
import scipy.special as sp
from numpy.polynomial.legendre import leggauss


def _gl01(n):
    t, w = leggauss(n)
    return 0.5 * (t + 1.0), 0.5 * w


class Window:
    """Generic even window with int phi = 1; Phi and transforms by quadrature."""

    def phi(self, r):
        raise NotImplementedError

    def dphi(self, r):
        raise NotImplementedError

    support = np.inf

    def Phi(self, r, n=64):
        """Phi(r) = 2 int_r^inf phi: integrated over [r, support] for a compactly
        supported window (exactly 0 beyond it), else as 1 - 2 int_0^r phi."""
        r = np.atleast_1d(np.abs(np.asarray(r, dtype=np.float64)))
        t, w = _gl01(n)
        if np.isfinite(self.support):
            a = np.minimum(r, self.support)
            L = self.support - a
            pts = a[:, None] + L[:, None] * t[None, :]
            return 2.0 * (self.phi(pts) * w[None, :]).sum(axis=1) * L
        pts = r[:, None] * t[None, :]
        return 1.0 - 2.0 * (self.phi(pts) * w[None, :]).sum(axis=1) * r

    def phihat(self, k, n=400):
        k = np.atleast_1d(np.asarray(k, dtype=np.float64))
        L = self.support if np.isfinite(self.support) else 12.0 / getattr(self, "xi", 1.0)
        t, w = _gl01(n)
        t = t * L
        w = w * L
        return 2.0 * (np.cos(np.outer(k, t)) * (self.phi(t) * w)[None, :]).sum(axis=1)

    def dphihat(self, k, n=400):
        k = np.atleast_1d(np.asarray(k, dtype=np.float64))
        L = self.support if np.isfinite(self.support) else 12.0 / getattr(self, "xi", 1.0)
        t, w = _gl01(n)
        t = t * L
        w = w * L
        return -2.0 * (np.sin(np.outer(k, t)) * (t * self.phi(t) * w)[None, :]).sum(axis=1)

    def gammahat(self, k):
        k = np.atleast_1d(np.asarray(k, dtype=np.float64))
        return self.phihat(k) - 0.5 * k * self.dphihat(k)

    def Sdiag(self, rho):
        rho = np.asarray(rho, dtype=np.float64)
        return self.Phi(rho) - 2.0 * rho * self.phi(rho)

    def Soffd(self, rho):
        rho = np.asarray(rho, dtype=np.float64)
        return self.Phi(rho) + 2.0 * rho * self.phi(rho)

    def Tdiag(self, rho):
        """R_Tdiag of eq. T-offd."""
        rho = np.asarray(rho, dtype=np.float64)
        return -2.0 * rho ** 2 * self.dphi(rho)

    def Toffd(self, rho):
        """R_Toffd of eq. T-offd."""
        rho = np.asarray(rho, dtype=np.float64)
        return self.Phi(rho) + 2.0 * rho * self.phi(rho) - (2.0 / 3.0) * rho ** 2 * self.dphi(rho)


def _cheb_lobatto(N):
    """Chebyshev-Lobatto points x_j = cos(j pi/N) and the spectral
    differentiation matrix (standard textbook construction)."""
    x = np.cos(np.pi * np.arange(N + 1) / N)
    c = np.ones(N + 1)
    c[0] = c[-1] = 2.0
    c = c * (-1.0) ** np.arange(N + 1)
    X = np.tile(x, (N + 1, 1)).T
    dX = X - X.T
    D = np.outer(c, 1.0 / c) / (dX + np.eye(N + 1))
    D = D - np.diag(D.sum(axis=1))
    return D, x


def _bary_lobatto(xn, fn, x):
    """Barycentric interpolation from Chebyshev-Lobatto data."""
    N = len(xn) - 1
    w = (-1.0) ** np.arange(N + 1)
    w[0] *= 0.5
    w[-1] *= 0.5
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    d = x[:, None] - xn[None, :]
    exact = d == 0.0
    d = np.where(exact, 1.0, d)
    t = w[None, :] / d
    out = (t * fn[None, :]).sum(axis=1) / t.sum(axis=1)
    hit = exact.any(axis=1)
    if np.any(hit):
        out[hit] = fn[np.argmax(exact[hit], axis=1)]
    return out


class ProlateWindow(Window):
    """phi = psi_0^c / int psi_0^c on [-1,1], zero outside.

    psi_0^c is the eigenfunction of the prolate differential operator
    L psi = -((1 - x^2) psi')' + c^2 x^2 psi with the smallest eigenvalue; that
    operator commutes with the band-limited Fourier operator whose top
    eigenfunction the paper uses (Sec. "Prolate spheroidal wave functions"),
    so both define the same function.  Here L is discretised by Chebyshev
    collocation (a dense non-symmetric eigenproblem solved by numpy) and psi
    is interpolated barycentrically; the tests pin the result against the
    paper's integral eigen-relation.  Sign: psi(0) > 0."""

    support = 1.0

    def __init__(self, c: float, N: int = 80):
        self.c = float(c)
        D, x = _cheb_lobatto(N)
        L = -D @ np.diag(1.0 - x * x) @ D + np.diag(self.c ** 2 * x * x)
        ev, V = np.linalg.eig(L)
        i = int(np.argmin(ev.real))
        v = V[:, i].real
        v = v * np.sign(_bary_lobatto(x, v, 0.0)[0])
        self.chi = float(ev[i].real)
        self._x, self._v, self._dv = x, v, D @ v
        t, w = leggauss(200)
        self.norm = float((self.psi(t) * w).sum())

    def psi(self, x):
        x = np.asarray(x, dtype=np.float64)
        return _bary_lobatto(self._x, self._v, np.clip(x, -1.0, 1.0).ravel()).reshape(x.shape)

    def dpsi(self, x):
        x = np.asarray(x, dtype=np.float64)
        return _bary_lobatto(self._x, self._dv, np.clip(x, -1.0, 1.0).ravel()).reshape(x.shape)

    def phi(self, r):
        r = np.asarray(r, dtype=np.float64)
        inside = np.abs(r) <= 1.0
        return np.where(inside, self.psi(np.where(inside, r, 0.0)) / self.norm, 0.0)

    def dphi(self, r):
        r = np.asarray(r, dtype=np.float64)
        inside = np.abs(r) <= 1.0
        return np.where(inside, self.dpsi(np.where(inside, r, 0.0)) / self.norm, 0.0)


class GaussianWindow(Window):
    """phi_G(r) = (xi/sqrt(pi)) exp(-xi^2 r^2), xi = 1/sigma (eq. wfunc_prol_G)."""

    def __init__(self, xi: float):
        self.xi = float(xi)

    def phi(self, r):
        r = np.asarray(r, dtype=np.float64)
        return self.xi / np.sqrt(np.pi) * np.exp(-(self.xi * r) ** 2)

    def dphi(self, r):
        r = np.asarray(r, dtype=np.float64)
        return -2.0 * self.xi ** 2 * r * self.phi(r)


def prolate_c(q: int) -> float:
    """Bandlimit from the integer 3c/pi that Table 1 lists."""
    return q * np.pi / 3.0


def stokeslet(y):
    """Free-space Stokeslet tensors S(y), y of shape (m,3) -> (m,3,3)."""
    y = np.asarray(y, dtype=np.float64)
    r = np.linalg.norm(y, axis=-1)
    I = np.eye(3)
    return (I[None] / r[:, None, None] + y[:, :, None] * y[:, None, :] / r[:, None, None] ** 3) / (8 * np.pi)


def residual_stokeslet(win: Window, y, nu: float = 1.0):
    """S_R at length scale nu (eq. res_stokeslet with the scaling remark)."""
    y = np.asarray(y, dtype=np.float64)
    r = np.linalg.norm(y, axis=-1)
    rho = r / nu
    sd = win.Sdiag(rho)
    so = win.Soffd(rho)
    I = np.eye(3)
    return (sd[:, None, None] * I[None] / r[:, None, None]
            + so[:, None, None] * y[:, :, None] * y[:, None, :] / r[:, None, None] ** 3) / (8 * np.pi)


def stresslet(y):
    """Free-space stresslet tensors T(y) (eq. stresslet_def_deriv), (m,3) -> (m,3,3,3)."""
    y = np.asarray(y, dtype=np.float64)
    r = np.linalg.norm(y, axis=-1)
    return -3.0 / (4 * np.pi) * np.einsum("ai,aj,ak->aijk", y, y, y) / r[:, None, None, None] ** 5


def residual_stresslet(win: Window, y, nu: float = 1.0):
    """T_R at length scale nu (eq. res_stresslet with R_Tdiag, R_Toffd of eq.
    T-offd evaluated at r/nu), (m,3) -> (m,3,3,3)."""
    y = np.asarray(y, dtype=np.float64)
    r = np.linalg.norm(y, axis=-1)
    rho = r / nu
    td = win.Tdiag(rho)
    to = win.Toffd(rho)
    I = np.eye(3)
    sym = (np.einsum("jl,am->ajlm", I, y) + np.einsum("lm,aj->ajlm", I, y) + np.einsum("mj,al->ajlm", I, y))
    return (td[:, None, None, None] * sym / (8 * np.pi * r[:, None, None, None] ** 3)
            - 3.0 / (4 * np.pi) * to[:, None, None, None] * np.einsum("ai,aj,ak->aijk", y, y, y)
            / r[:, None, None, None] ** 5)


def residual_stresslet_pair_sum(win: Window, xt, xs, fs, ns, nu):
    """Brute-force sum_a T_R^nu(x_t - x_a) : (f_a n_a) over all sources
    (pairs with r = 0 or r >= nu contribute nothing)."""
    xt = np.asarray(xt, dtype=np.float64)
    out = np.zeros((xt.shape[0], 3))
    for t in range(xt.shape[0]):
        y = xt[t][None, :] - xs
        r = np.linalg.norm(y, axis=1)
        keep = (r > 0) & (r < nu)
        if not np.any(keep):
            continue
        T = residual_stresslet(win, y[keep], nu)
        out[t] = np.einsum("ajlm,al,am->j", T, fs[keep], ns[keep])
    return out


def Btrunc_hat(k, R):
    """Truncated biharmonic symbol in 3D (eq. Btrunc_hat); series near k = 0."""
    k = np.atleast_1d(np.asarray(k, dtype=np.float64))
    x = k * R
    out = np.empty_like(k)
    small = x < 0.2
    xs = x[~small]
    ks = k[~small]
    out[~small] = (1.0 + 0.5 * np.cos(xs) - 1.5 * np.sin(xs) / xs) / ks ** 4
    # 1 + cos(x)/2 - 3 sin(x)/(2x) = sum_{n>=2} (-1)^n x^{2n} [1/(2 (2n)!) - 3/(2 (2n+1)!)]
    xm = x[small]
    acc = np.zeros_like(xm)
    for nn in range(2, 12):
        coef = (-1) ** nn * (0.5 / sp.factorial(2 * nn) - 1.5 / sp.factorial(2 * nn + 1))
        acc += coef * xm ** (2 * nn - 4)
    out[small] = acc * R ** 4
    return out


def mollified_S_fourier(win: Window, r, R=1.0 + np.sqrt(3.0), kmax=None, panels=None, order=32):
    """Mollified Stokeslet radial functions (M_Sdiag, M_Soffd) at unit scale by
    the appendix's Fourier route: with z = k r,
      F_Sdiag(k,r) = -8 pi (F_k' + r F_k'') = 8 pi k (z j0(z) - j1(z)),
      F_Soffd(k,r) =  8 pi (-F_k' + r F_k'') = 8 pi k (3 j1(z) - z j0(z)),
      M^R = (1/(2 pi^2)) int_0^inf F(k,r) Bhat^R(k) gammahat(k) k^2 dk,
    and M_Sdiag = M^R_Sdiag + 2 r / R, M_Soffd = M^R_Soffd (eq. msdiag)."""
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    if kmax is None:
        kmax = 400.0
    if panels is None:
        panels = int(kmax / 1.0)
    t, w = leggauss(order)
    edges = np.linspace(0.0, kmax, panels + 1)
    ks = (0.5 * (edges[1:] - edges[:-1])[:, None] * (t[None, :] + 1.0) + edges[:-1, None]).ravel()
    ws = (0.5 * (edges[1:] - edges[:-1])[:, None] * w[None, :]).ravel()
    g = win.gammahat(ks) * Btrunc_hat(ks, R) * ks ** 2 * ws
    z = np.outer(r, ks)
    j0 = sp.spherical_jn(0, z)
    j1 = sp.spherical_jn(1, z)
    fd = 8 * np.pi * ks[None, :] * (z * j0 - j1)
    fo = 8 * np.pi * ks[None, :] * (3 * j1 - z * j0)
    md = (fd * g[None, :]).sum(axis=1) / (2 * np.pi ** 2) + 2.0 * r / R
    mo = (fo * g[None, :]).sum(axis=1) / (2 * np.pi ** 2)
    return md, mo


def residual_pair_sum(win: Window, xt, xs, fs, nu, self_index=None, shifts=None):
    """Brute-force sum_a S_R^nu(x_t - x_a + shift) f_a over all given sources
    (pairs with r >= support*nu or r == 0 contribute nothing).

    ``self_index[t]`` (optional) is the index into xs of the target itself,
    whose zero-shift pair is skipped.  ``shifts`` (optional, (s,3)) are image
    shifts added to the difference vectors (periodic images)."""
    xt = np.asarray(xt, dtype=np.float64)
    xs = np.asarray(xs, dtype=np.float64)
    fs = np.asarray(fs, dtype=np.float64)
    if shifts is None:
        shifts = np.zeros((1, 3))
    out = np.zeros((xt.shape[0], 3))
    for t in range(xt.shape[0]):
        acc = np.zeros(3)
        for sh in shifts:
            y = xt[t][None, :] - xs + sh[None, :]
            r = np.linalg.norm(y, axis=1)
            ok = (r > 0) & (r < win.support * nu)
            if self_index is not None and not np.any(sh):
                ok[self_index[t]] = False
            if not np.any(ok):
                continue
            S = residual_stokeslet(win, y[ok], nu)
            acc += np.einsum("mij,mj->i", S, fs[ok])
        out[t] = acc
    return out

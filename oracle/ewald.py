"""ORACLE -- test infrastructure only.  Periodic Stokeslet and stresslet sums
on the unit cell.

The periodic sum (eq. periodic_sum) is evaluated with the classical
Hasimoto/Gaussian Ewald split (eq. hasimoto-split), which shares nothing with
the method under test (the method uses a prolate window):

  u(x_b) = u_real(x_b) + u_fourier(x_b) + u_self(x_b)

  u_real     sum over source images within rc of the Gaussian residual
             Stokeslet (direct.c, oracle_stokeslet_ewald_real);
  u_fourier  Poisson-summed mollified part over k = 2 pi kappa, kappa in Z^3,
             0 < |k| < kc (eq. ewald_far, mollified Stokeslet eq.
             moll_stokeslet with the Hasimoto biharmonic symbol):
               S_M(k) = (I - k k^T / k^2) k^-2 (1 + k^2/(4 xi^2)) exp(-k^2/(4 xi^2)),
             the k = 0 term dropped (zero mean flow);
  u_self     -lim_{x->0} S_M(x) f_b = -(phi_G(0)/(2 pi)) f_b = -xi/(2 pi^{3/2}) f_b
             (eq. S_self with phi_G(0) = xi/sqrt(pi)).

Truncation: erfc(xi rc) and exp(-kc^2/(4 xi^2)) are both e^{-E}; the default
E = 30 gives about 1e-13 relative accuracy.

The periodic stresslet sum (stresslet_ewald) splits the same way:

  u_real     Gaussian residual stresslet (direct.c, oracle_stresslet_ewald_real);
  u_fourier  the mollified stresslet over 0 < |k| < kc (eq. moll_stresslet with
             the Hasimoto symbol): for the symmetric density rho = sym(f n^T),
               u_j(k) = i [k^2 (2 (rho k)_j + k_j tr rho) - 2 k_j k.rho.k]
                        (1 + k^2/(4 xi^2)) exp(-k^2/(4 xi^2)) / k^4;
  u^(0)      the k = 0 term the paper fixes for the stresslet (after eq.
             ewald_far): u^(0)(x_t) = -sum_s (x_t - x_s)(f_s . n_s), positions
             in the unit cell;
  no self term (the stresslet's vanishes).
"""
from __future__ import annotations

import numpy as np

from . import ewald_real, stresslet_ewald_real


def ewald_params(rc: float = 0.5, E: float = 30.0):
    xi = np.sqrt(E) / rc
    kc = 2.0 * xi * np.sqrt(E)
    return float(xi), float(rc), float(kc)


def _fourier(x, f, xt, xi, kc, chunk=8192):
    K = int(np.floor(kc / (2 * np.pi)))
    kx = np.arange(0, K + 1)                 # half space kappa_x >= 0
    ky = np.arange(-K, K + 1)
    n = x.shape[0]
    nK = ky.size
    # structure factor F(kappa) = sum_a f_a exp(-i k.x_a), kappa_x >= 0
    F = np.zeros((kx.size, nK, nK, 3), dtype=np.complex128)
    for s in range(0, n, chunk):
        xs = x[s:s + chunk]
        fs = f[s:s + chunk]
        ex = np.exp(-2j * np.pi * np.outer(xs[:, 0], kx))
        ey = np.exp(-2j * np.pi * np.outer(xs[:, 1], ky))
        ez = np.exp(-2j * np.pi * np.outer(xs[:, 2], ky))
        B = (ez[:, :, None] * fs[:, None, :]).reshape(xs.shape[0], nK * 3)
        for i in range(kx.size):
            A = ex[:, i:i + 1] * ey
            F[i] += (A.T @ B).reshape(nK, nK, 3)
    KX, KY, KZ = np.meshgrid(2 * np.pi * kx, 2 * np.pi * ky, 2 * np.pi * ky, indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    mask = (k2 > 0) & (k2 < kc * kc)
    k2s = np.where(mask, k2, 1.0)
    s = np.where(mask, (1.0 + k2s / (4 * xi * xi)) * np.exp(-k2s / (4 * xi * xi)) / k2s, 0.0)
    # Hermitian pairs: kappa_x > 0 stands for itself and its mirror
    s = s * np.where(kx[:, None, None] > 0, 2.0, 1.0)
    kdotF = (KX * F[..., 0] + KY * F[..., 1] + KZ * F[..., 2]) / k2s
    G = np.empty_like(F)
    G[..., 0] = s * (F[..., 0] - KX * kdotF)
    G[..., 1] = s * (F[..., 1] - KY * kdotF)
    G[..., 2] = s * (F[..., 2] - KZ * kdotF)
    # evaluate Re sum_k G(k) exp(i k.x_t)
    u = np.zeros((xt.shape[0], 3))
    for s0 in range(0, xt.shape[0], 256):
        xb = xt[s0:s0 + 256]
        ex = np.exp(2j * np.pi * np.outer(xb[:, 0], kx))
        ey = np.exp(2j * np.pi * np.outer(xb[:, 1], ky))
        ez = np.exp(2j * np.pi * np.outer(xb[:, 2], ky))
        # sum over kz first: H[t, i, j, c] = sum_kz G[i, j, kz, c] ez[t, kz]
        H = np.einsum("ijkc,tk->tijc", G, ez, optimize=True)
        H = np.einsum("tijc,tj->tic", H, ey, optimize=True)
        u[s0:s0 + 256] = np.einsum("tic,ti->tc", H, ex, optimize=True).real
    return u


def ewald(x, f, targets, xi=None, rc=0.5, kc=None, E=30.0):
    """Periodic Stokeslet sum on the unit cell at the listed target indices."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    if xi is None or kc is None:
        xi0, rc, kc0 = ewald_params(rc, E)
        xi = xi0 if xi is None else xi
        kc = kc0 if kc is None else kc
    xm = x - np.floor(x)
    u_real = ewald_real(xm, f, targets, xi, rc)
    u_four = _fourier(xm, f, xm[targets], xi, kc)
    u_self = -xi / (2.0 * np.pi ** 1.5) * f[targets]
    return u_real + u_four + u_self


def _fourier_stresslet(x, f, nv, xt, xi, kc, chunk=8192):
    K = int(np.floor(kc / (2 * np.pi)))
    kx = np.arange(0, K + 1)                 # half space kappa_x >= 0
    ky = np.arange(-K, K + 1)
    n = x.shape[0]
    nK = ky.size
    # symmetric density per source: (11, 22, 33, 12, 13, 23) of sym(f n^T)
    rho = np.stack([f[:, 0] * nv[:, 0], f[:, 1] * nv[:, 1], f[:, 2] * nv[:, 2],
                    0.5 * (f[:, 0] * nv[:, 1] + f[:, 1] * nv[:, 0]),
                    0.5 * (f[:, 0] * nv[:, 2] + f[:, 2] * nv[:, 0]),
                    0.5 * (f[:, 1] * nv[:, 2] + f[:, 2] * nv[:, 1])], axis=1)
    F = np.zeros((kx.size, nK, nK, 6), dtype=np.complex128)
    for s in range(0, n, chunk):
        xs = x[s:s + chunk]
        rs = rho[s:s + chunk]
        ex = np.exp(-2j * np.pi * np.outer(xs[:, 0], kx))
        ey = np.exp(-2j * np.pi * np.outer(xs[:, 1], ky))
        ez = np.exp(-2j * np.pi * np.outer(xs[:, 2], ky))
        B = (ez[:, :, None] * rs[:, None, :]).reshape(xs.shape[0], nK * 6)
        for i in range(kx.size):
            A = ex[:, i:i + 1] * ey
            F[i] += (A.T @ B).reshape(nK, nK, 6)
    KX, KY, KZ = np.meshgrid(2 * np.pi * kx, 2 * np.pi * ky, 2 * np.pi * ky, indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    mask = (k2 > 0) & (k2 < kc * kc)
    k2s = np.where(mask, k2, 1.0)
    w = np.where(mask, (1.0 + k2s / (4 * xi * xi)) * np.exp(-k2s / (4 * xi * xi)) / (k2s * k2s), 0.0)
    w = w * np.where(kx[:, None, None] > 0, 2.0, 1.0)
    r11, r22, r33, r12, r13, r23 = (F[..., c] for c in range(6))
    rk = [r11 * KX + r12 * KY + r13 * KZ, r12 * KX + r22 * KY + r23 * KZ, r13 * KX + r23 * KY + r33 * KZ]
    tr = r11 + r22 + r33
    krk = KX * rk[0] + KY * rk[1] + KZ * rk[2]
    G = np.empty((kx.size, nK, nK, 3), dtype=np.complex128)
    for j, Kj in enumerate((KX, KY, KZ)):
        G[..., j] = 1j * w * (k2 * (2.0 * rk[j] + Kj * tr) - 2.0 * Kj * krk)
    u = np.zeros((xt.shape[0], 3))
    for s0 in range(0, xt.shape[0], 256):
        xb = xt[s0:s0 + 256]
        ex = np.exp(2j * np.pi * np.outer(xb[:, 0], kx))
        ey = np.exp(2j * np.pi * np.outer(xb[:, 1], ky))
        ez = np.exp(2j * np.pi * np.outer(xb[:, 2], ky))
        H = np.einsum("ijkc,tk->tijc", G, ez, optimize=True)
        H = np.einsum("tijc,tj->tic", H, ey, optimize=True)
        u[s0:s0 + 256] = np.einsum("tic,ti->tc", H, ex, optimize=True).real
    return u


def stresslet_u0(x, f, nv, xt):
    """k = 0 term of the periodic stresslet sum: -sum_s (x_t - x_s)(f_s . n_s)."""
    fn = np.einsum("ij,ij->i", f, nv)
    return -(xt * fn.sum() - (x * fn[:, None]).sum(axis=0))


def stresslet_ewald(x, f, nv, targets, xi=None, rc=0.5, kc=None, E=30.0):
    """Periodic stresslet sum on the unit cell at the listed target indices
    (points are taken modulo the cell)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    nv = np.ascontiguousarray(nv, dtype=np.float64)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    if xi is None or kc is None:
        xi0, rc, kc0 = ewald_params(rc, E)
        xi = xi0 if xi is None else xi
        kc = kc0 if kc is None else kc
    xm = x - np.floor(x)
    u_real = stresslet_ewald_real(xm, f, nv, targets, xi, rc)
    u_four = _fourier_stresslet(xm, f, nv, xm[targets], xi, kc)
    return u_real + u_four + stresslet_u0(xm, f, nv, xm[targets])

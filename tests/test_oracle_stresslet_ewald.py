"""Pins of the oracle's periodic stresslet sum (Gaussian Ewald split plus the
k = 0 term of the paper, after eq. ewald_far) and of its free-space direct sum,
against facts that do not come from the oracle's own formulas:

* the double-layer identity of a closed surface with constant density f:
  sum_s T(x - x_s) : (f n_s^T) w_s over a quadrature of the surface equals f
  inside and 0 outside (the Gauss-type jump of the stresslet; each image is
  compactly supported, so the periodic sum is f times the periodic
  indicator, and the k = 0 term is what restores the mean f V);
* independence of the Ewald result from the split parameter xi."""
import numpy as np
import pytest

import oracle
from oracle.ewald import stresslet_ewald


def _sphere_quadrature(c, R, nt=40, nph=80):
    ct, wt = np.polynomial.legendre.leggauss(nt)
    ph = np.arange(nph) * 2 * np.pi / nph
    CT, PH = np.meshgrid(ct, ph, indexing="ij")
    W = np.outer(wt, np.full(nph, 2 * np.pi / nph)) * R * R
    st = np.sqrt(1 - CT ** 2)
    nv = np.stack([st * np.cos(PH), st * np.sin(PH), CT], -1).reshape(-1, 3)
    return np.asarray(c) + R * nv, nv, W.ravel()


def _with_targets(xs, fs, ns, tg):
    x = np.concatenate([xs, tg])
    f = np.concatenate([fs, np.zeros_like(tg)])
    n = np.concatenate([ns, np.zeros_like(tg)])
    return x, f, n, np.arange(xs.shape[0], x.shape[0])


TARGETS = np.array([[0.55, 0.47, 0.52], [0.5, 0.5, 0.5], [0.42, 0.6, 0.45],   # inside
                    [0.85, 0.5, 0.5], [0.1, 0.2, 0.9], [0.02, 0.98, 0.5]])  # outside
INSIDE = np.array([1, 1, 1, 0, 0, 0], dtype=float)


def test_free_space_double_layer_identity():
    xs, nv, w = _sphere_quadrature([0.5, 0.5, 0.5], 0.2)
    f0 = np.array([0.3, -0.7, 0.5])
    x, f, n, t = _with_targets(xs, f0 * w[:, None], nv, TARGETS)
    u = oracle.stresslet_direct(x, f, n, t)
    # quadrature error of the nearest target (0.06 from the surface): ~3e-12
    assert np.abs(u - INSIDE[:, None] * f0).max() < 1e-10


def test_periodic_double_layer_identity():
    xs, nv, w = _sphere_quadrature([0.5, 0.5, 0.5], 0.2)
    f0 = np.array([0.3, -0.7, 0.5])
    x, f, n, t = _with_targets(xs, f0 * w[:, None], nv, TARGETS)
    u = stresslet_ewald(x, f, n, t)
    assert np.abs(u - INSIDE[:, None] * f0).max() < 1e-10


def test_periodic_double_layer_identity_off_centre():
    # a sphere that crosses the cell faces: its images enter through the
    # minimum-image real part and the Fourier part; the indicator is periodic
    xs, nv, w = _sphere_quadrature([0.9, 0.15, 0.5], 0.2, nt=60, nph=120)
    f0 = np.array([-0.2, 0.4, 0.9])
    # inside: near the centre, and through the x face (image centre at x = -0.1);
    # outside: the cell centre and two far points
    tg = np.array([[0.95, 0.12, 0.45], [0.02, 0.15, 0.5], [0.9, 0.15, 0.5], [0.5, 0.5, 0.5], [0.3, 0.7, 0.1],
                   [0.5, 0.97, 0.2]])
    inside = np.array([1, 1, 1, 0, 0, 0], dtype=float)
    # the quadrature nodes wrapped into the cell; the k = 0 term then takes
    # their wrapped positions, so the identity holds only for the sum of all
    # images -- compare with the unwrapped sphere's moment explicitly
    x, f, n, t = _with_targets(xs - np.floor(xs), f0 * w[:, None], nv, tg)
    u = stresslet_ewald(x, f, n, t)
    # wrapping source s by a lattice vector p_s changes -sum (x_t - x_s)(f.n) by -sum p_s (f.n_s)
    p = np.floor(xs)
    shift = -(p * (n[:xs.shape[0]] * f[:xs.shape[0]]).sum(axis=1)[:, None]).sum(axis=0)
    assert np.abs(u - shift - inside[:, None] * f0).max() < 1e-10


def test_ewald_independent_of_xi():
    rng = np.random.default_rng(5)
    x = rng.random((300, 3))
    f = rng.normal(size=(300, 3))
    nv = rng.normal(size=(300, 3))
    t = np.arange(0, 300, 7)
    a = stresslet_ewald(x, f, nv, t, rc=0.5, E=30.0)
    b = stresslet_ewald(x, f, nv, t, rc=0.3, E=32.0)
    assert np.abs(a - b).max() < 1e-10 * np.abs(a).max()

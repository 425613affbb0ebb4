"""Pins for the free-space direct-sum oracle (Introduction, eq. stokeslet_def_deriv
and eq. stokes_stress_sum).  None of these re-types the oracle's formula: they
use hand-computed values, finite-difference derivatives of the biharmonic
Green's function, symmetry, homogeneity and the divergence-free property."""
import numpy as np
import pytest

import oracle

INV8PI = 1.0 / (8.0 * np.pi)


def kernel_matrix(y):
    """S(y) read back from the oracle with unit forces at a second point."""
    x = np.array([[0.0, 0.0, 0.0], -np.asarray(y, dtype=float)])
    S = np.zeros((3, 3))
    for l in range(3):
        f = np.zeros((2, 3))
        f[1, l] = 1.0
        S[:, l] = oracle.direct(x, f, [0])[0]
    return S


def test_two_points_by_hand_axis():
    # y = x_1 - x_2 = (-1,0,0), r = 1: S = (1/8pi) diag(2,1,1)
    x = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    f = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 3.0]])
    u = oracle.direct(x, f)
    assert np.allclose(u[0], np.array([2.0, 2.0, 3.0]) * INV8PI, rtol=0, atol=1e-15)
    assert np.allclose(u[1], 0.0, atol=0)


def test_two_points_by_hand_oblique():
    # y = (1/3, 2/3, 2/3), r = 1, f = (3,0,0): S f = (1/8pi)(f + (y.f) y) = (1/8pi)(10/3, 2/3, 2/3)
    x = np.array([[1 / 3, 2 / 3, 2 / 3], [0.0, 0.0, 0.0]])
    f = np.array([[0.0, 0.0, 0.0], [3.0, 0.0, 0.0]])
    u = oracle.direct(x, f, [0])[0]
    assert np.allclose(u, np.array([10 / 3, 2 / 3, 2 / 3]) * INV8PI, rtol=1e-14, atol=0)


def test_three_points_superposition_by_hand():
    # x0 at origin, sources at (2,0,0) with f=(0,1,0) and (0,0,-1) with f=(0,0,1)
    # first: y=(-2,0,0), r=2, y.f=0 -> (1/8pi)(0,1/2,0)
    # second: y=(0,0,1), r=1, y.f=1 -> (1/8pi)((0,0,1) + (0,0,1)) = (1/8pi)(0,0,2)
    x = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [0.0, 0.0, -1.0]])
    f = np.array([[5.0, 5.0, 5.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    u = oracle.direct(x, f, [0])[0]
    assert np.allclose(u, np.array([0.0, 0.5, 2.0]) * INV8PI, rtol=1e-14, atol=1e-17)


def test_matches_biharmonic_second_derivatives():
    """S = (-I lap + grad grad) B with B = -r/(8 pi) (eq. stokeslet_def_deriv,
    eq. biharmonic_green_def), Hessian of B by 4th-order central differences."""
    rng = np.random.default_rng(0)
    B = lambda p: -np.linalg.norm(p) / (8 * np.pi)
    def hessian(y, h):
        H = np.zeros((3, 3))
        for i in range(3):
            for j in range(3):
                ei = np.eye(3)[i] * h
                ej = np.eye(3)[j] * h
                if i == j:
                    H[i, i] = (-B(y + 2 * ei) + 16 * B(y + ei) - 30 * B(y) + 16 * B(y - ei) - B(y - 2 * ei)) / (12 * h * h)
                else:
                    H[i, j] = (B(y + ei + ej) - B(y + ei - ej) - B(y - ei + ej) + B(y - ei - ej)) / (4 * h * h)
        return H

    for _ in range(5):
        y = rng.normal(size=3)
        y *= 0.7 / np.linalg.norm(y)
        H = (4 * hessian(y, 1e-3) - hessian(y, 2e-3)) / 3  # Richardson step on the O(h^2) terms
        DS = -np.trace(H) * np.eye(3) + H
        assert np.allclose(kernel_matrix(y), DS, rtol=0, atol=2e-9)


def test_symmetry_homogeneity_reciprocity():
    rng = np.random.default_rng(1)
    for _ in range(4):
        y = rng.normal(size=3)
        S = kernel_matrix(y)
        assert np.allclose(S, S.T, atol=1e-16, rtol=1e-14)
        assert np.allclose(kernel_matrix(3.0 * y), S / 3.0, rtol=1e-13)
    x = rng.random((50, 3))
    f1 = rng.normal(size=(50, 3))
    f2 = rng.normal(size=(50, 3))
    a = np.sum(f2 * oracle.direct(x, f1))
    b = np.sum(f1 * oracle.direct(x, f2))
    assert abs(a - b) <= 1e-13 * abs(a)


def test_divergence_free():
    rng = np.random.default_rng(2)
    h = 1e-4
    for _ in range(4):
        xs = rng.normal(size=3)
        fs = rng.normal(size=3)
        xp = xs + 0.5 * rng.normal(size=3)
        div = 0.0
        for i in range(3):
            e = np.eye(3)[i] * h
            up = oracle.direct(np.array([xp + e, xs]), np.array([np.zeros(3), fs]), [0])[0]
            um = oracle.direct(np.array([xp - e, xs]), np.array([np.zeros(3), fs]), [0])[0]
            div += (up[i] - um[i]) / (2 * h)
        mag = np.linalg.norm(oracle.direct(np.array([xp, xs]), np.array([np.zeros(3), fs]), [0])[0])
        assert abs(div) < 1e-7 * mag / np.linalg.norm(xp - xs)


def test_self_and_coincident_points_excluded():
    x = np.array([[0.1, 0.2, 0.3], [0.1, 0.2, 0.3], [0.5, 0.5, 0.5]])
    f = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 0]])
    u = oracle.direct(x, f, [2])
    ref = oracle.direct(np.array([x[2], x[0]]), np.array([f[2], f[0] + f[1]]), [0])
    assert np.allclose(u, ref, rtol=1e-15)
    u0 = oracle.direct(x, f, [0])
    assert np.allclose(u0, 0.0)


def test_subset_targets_match_full():
    rng = np.random.default_rng(3)
    x = rng.random((300, 3))
    f = rng.normal(size=(300, 3))
    full = oracle.direct(x, f)
    idx = np.array([0, 17, 299])
    assert np.array_equal(oracle.direct(x, f, idx), full[idx])

"""Pins for the periodic (Gaussian-Ewald) oracle (eq. periodic_sum, split
eq. hasimoto-split, zero-mean-flow convention of eq. ewald_far).

* the split parameter xi is arbitrary: three (rc, xi, kc) triples must agree;
* a single force in the unit cell feels its images through the classical
  simple-cubic lattice constant: u = -2.837297 f / (6 pi)  (Hasimoto 1959; the
  same constant appears in finite-size corrections of periodic Stokes flows);
* invariance under translation of all points (mod 1), under moving one
  point by a lattice vector, and reciprocity;
* a tiny zero-net-force cluster sees almost no images: the periodic sum
  tends to the free-space direct sum (difference O(a^3) relative)."""
import numpy as np

import oracle
from oracle.ewald import ewald


def test_xi_independence():
    rng = np.random.default_rng(10)
    x = rng.random((40, 3))
    f = rng.normal(size=(40, 3))
    f -= f.mean(axis=0)
    t = np.arange(40)
    u1 = ewald(x, f, t, rc=0.5, E=30)
    u2 = ewald(x, f, t, rc=0.35, E=30)
    u3 = ewald(x, f, t, rc=0.25, E=32)
    assert oracle.rel_l2(u2, u1) < 1e-12
    assert oracle.rel_l2(u3, u1) < 1e-12


def test_simple_cubic_lattice_constant():
    x = np.array([[0.3, 0.6, 0.2]])
    for d in range(3):
        f = np.zeros((1, 3))
        f[0, d] = 1.0
        u = ewald(x, f, [0])
        expect = np.zeros(3)
        expect[d] = -2.837297 / (6 * np.pi)
        assert np.allclose(u[0], expect, rtol=0, atol=1e-6 / (6 * np.pi))  # the constant is quoted to 6 decimals


def test_translation_and_lattice_invariance_and_reciprocity():
    rng = np.random.default_rng(11)
    x = rng.random((30, 3))
    f = rng.normal(size=(30, 3))
    f -= f.mean(axis=0)
    t = np.arange(30)
    u = ewald(x, f, t)
    xs = (x + np.array([0.37, -0.81, 0.55])) % 1.0
    assert oracle.rel_l2(ewald(xs, f, t), u) < 1e-12
    x2 = x.copy()
    x2[3] += np.array([1.0, -2.0, 0.0])
    assert oracle.rel_l2(ewald(x2, f, t), u) < 1e-12
    g = rng.normal(size=(30, 3))
    g -= g.mean(axis=0)
    a = np.sum(g * u)
    b = np.sum(f * ewald(x, g, t))
    assert abs(a - b) < 1e-12 * abs(a)


def test_small_cluster_tends_to_free_space():
    rng = np.random.default_rng(12)
    a = 0.01
    x = 0.5 + a * (rng.random((20, 3)) - 0.5)
    f = rng.normal(size=(20, 3))
    f -= f.mean(axis=0)
    t = np.arange(20)
    up = ewald(x, f, t)
    ud = oracle.direct(x, f)
    assert oracle.rel_l2(up, ud) < 1e-4

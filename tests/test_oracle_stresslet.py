"""Pins of the stresslet oracle against the paper's definitions and plain
mathematics (CPU only).

* T = [-(delta_jl d_m + delta_lm d_j + delta_mj d_l) lap + 2 d_j d_l d_m] B
  (eq. stresslet_def_deriv) with B = -r/(8 pi), by Cartesian finite
  differences (Richardson-extrapolated third differences);
* the residual stresslet of eq. res_stresslet / T-offd equals the same
  operator applied to the residual biharmonic kernel of Theorem Bres
  (evaluated by quadrature);
* zero divergence, symmetry in (f, n), hand values for two points, compact
  support.
"""
import numpy as np
import pytest
from numpy.polynomial.legendre import leggauss

import oracle
from oracle import splitting as S


def _d3(F, x, a, b, c, h):
    """d_a d_b d_c F at x by the product of three central differences."""
    e = np.eye(3)
    acc = 0.0
    for s1 in (-1, 1):
        for s2 in (-1, 1):
            for s3 in (-1, 1):
                acc += s1 * s2 * s3 * F(x + h * (s1 * e[a] + s2 * e[b] + s3 * e[c]))
    return acc / (8 * h ** 3)


def _DT(F, x, h):
    """The stresslet operator of eq. stresslet_def_deriv applied to F at x,
    Richardson-extrapolated in h."""
    def once(hh):
        d = np.zeros((3, 3, 3))
        for j in range(3):
            for l in range(3):
                for m in range(3):
                    d[j, l, m] = _d3(F, x, j, l, m, hh)
        lapgrad = np.array([sum(d[a, a, m] for a in range(3)) for m in range(3)])
        I = np.eye(3)
        T = (-(np.einsum("jl,m->jlm", I, lapgrad) + np.einsum("lm,j->jlm", I, lapgrad)
               + np.einsum("mj,l->jlm", I, lapgrad)) + 2 * d)
        return T
    return (4 * once(h / 2) - once(h)) / 3


PTS = np.array([[0.3, -0.2, 0.5], [0.05, 0.4, -0.1], [-0.6, 0.1, 0.2], [0.2, 0.2, 0.2]])


def test_stresslet_is_DT_of_biharmonic():
    B = lambda x: -np.linalg.norm(x) / (8 * np.pi)
    for x in PTS:
        got = _DT(B, x, 0.01 * np.linalg.norm(x))
        ref = S.stresslet(x[None])[0]
        assert np.abs(got - ref).max() < 1e-6 * np.abs(ref).max(), x


def test_c_oracle_matches_tensor_and_symmetry():
    rng = np.random.default_rng(5)
    x = rng.random((60, 3))
    f = rng.normal(size=(60, 3))
    nv = rng.normal(size=(60, 3))
    u = oracle.stresslet_direct(x, f, nv)
    ref = np.zeros((60, 3))
    for b in range(60):
        y = x[b] - np.delete(x, b, axis=0)
        ref[b] = np.einsum("ajlm,al,am->j", S.stresslet(y), np.delete(f, b, axis=0), np.delete(nv, b, axis=0))
    assert np.abs(u - ref).max() < 1e-12 * np.abs(ref).max()
    assert np.abs(oracle.stresslet_direct(x, nv, f) - u).max() < 1e-12 * np.abs(u).max()


def test_two_points_by_hand():
    x = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 2.0]])
    f = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    nv = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    u = oracle.stresslet_direct(x, f, nv)
    # target 1: y = (1,2,2), r = 3, y.f_0 = 1, y.n_0 = 2: u = -(3/4pi) y * 2 / 243
    assert np.allclose(u[1], -3 / (4 * np.pi) * np.array([1.0, 2.0, 2.0]) * 2 / 243, rtol=1e-14)
    # target 0: y = -(1,2,2), y.f_1 = -2, y.n_1 = -1
    assert np.allclose(u[0], -3 / (4 * np.pi) * -np.array([1.0, 2.0, 2.0]) * 2 / 243, rtol=1e-14)


def test_stresslet_divergence_free():
    h = 1e-4
    for x in PTS:
        div = sum((S.stresslet((x + h * np.eye(3)[j])[None])[0][j] - S.stresslet((x - h * np.eye(3)[j])[None])[0][j])
                  / (2 * h) for j in range(3))
        assert np.abs(div).max() < 1e-6 * np.abs(S.stresslet(x[None])[0]).max() / np.linalg.norm(x)


@pytest.mark.parametrize("q", [17, 25])
def test_residual_stresslet_is_DT_of_residual_biharmonic(q):
    win = S.ProlateWindow(S.prolate_c(q))
    t, w = leggauss(80)
    inf = (0.5 * (t + 1) * win.phi(0.5 * (t + 1)) * 0.5 * w).sum()

    def BR(x):
        rr = np.linalg.norm(x)
        a = (win.phi(rr * 0.5 * (t + 1)) * 0.5 * w).sum() * rr
        b = (rr * 0.5 * (t + 1) * win.phi(rr * 0.5 * (t + 1)) * 0.5 * w).sum() * rr
        return -(rr - 2 * rr * a + 2 * b - 2 * inf) / (8 * np.pi)

    for x in np.array([[0.3, -0.2, 0.4], [0.05, 0.2, -0.1], [-0.5, 0.1, 0.3], [0.1, 0.1, 0.1]]):
        got = _DT(BR, x, 0.01 * np.linalg.norm(x))
        ref = S.residual_stresslet(win, x[None])[0]
        scale = np.abs(S.stresslet(x[None])[0]).max()
        assert np.abs(got - ref).max() < 1e-6 * scale, x


def test_residual_stresslet_compact_support():
    win = S.ProlateWindow(S.prolate_c(17))
    r = np.array([1.0 + 1e-9, 1.3, 2.0])
    assert np.all(win.Tdiag(r) == 0.0) and np.all(win.Toffd(r) == 0.0)
    # the residual tends to the full kernel at r -> 0
    assert abs(win.Toffd(1e-4) - 1.0) < 1e-6 and abs(win.Tdiag(1e-4)) < 1e-6

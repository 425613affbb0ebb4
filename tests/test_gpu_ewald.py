"""GPU parity of the single-level spectral Ewald method (DMK_METHOD_EWALD)
against the oracle's Gaussian Ewald sum (a different split and no FFT), and
against the multilevel DMK on the same points, through the C ABI."""
import os

import numpy as np
import pytest

import oracle
import workloads
from oracle.ewald import ewald

pytestmark = pytest.mark.gpu


def _dmk():
    import paper_2509_21471_amd as dmk
    return dmk


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9])
@pytest.mark.parametrize("n,leaf", [(3000, 0), (20000, 300)])
def test_matches_ewald_oracle(dev, tol, n, leaf):
    dmk = _dmk()
    x, f = workloads.make("periodic", n, seed=200 + n)
    plan = dmk.Plan(_t(x), periodic=True, tol=tol, leaf_size=leaf, method=dmk.METHOD_EWALD)
    info = plan.info()
    u = plan.eval(_t(f)).cpu().numpy()
    t = np.arange(0, n, max(1, n // 500))
    err = oracle.rel_l2(u[t], ewald(x, f, t))
    print(f"spectral Ewald n={n} tol={tol}: L={info['levels'] - 1} M={info['ewald_grid']} "
          f"K={info['ewald_modes']} w={info['ewald_width']} err/tol={err / tol:.3f}")
    assert info["method"] == dmk.METHOD_EWALD
    assert err < tol


def test_agrees_with_dmk(dev):
    dmk = _dmk()
    x, f = workloads.make("periodic", 30000, seed=211)
    a = dmk.Plan(_t(x), periodic=True, tol=1e-9, leaf_size=200, method=dmk.METHOD_EWALD).eval(_t(f)).cpu().numpy()
    b = dmk.Plan(_t(x), periodic=True, tol=1e-9, leaf_size=200).eval(_t(f)).cpu().numpy()
    assert oracle.rel_l2(a, b) < 2e-9


def test_multi_rhs_equals_single(dev):
    dmk = _dmk()
    x, f = workloads.make("periodic", 4000, seed=212, n_rhs=2)
    plan = dmk.Plan(_t(x), periodic=True, tol=1e-6, method=dmk.METHOD_EWALD)
    both = plan.eval(_t(f)).cpu().numpy()
    for r in range(2):
        assert np.array_equal(both[r], plan.eval(_t(f[r])).cpu().numpy())


def test_periodic_2e6_stored_ewald(dev):
    """The 2e6-point periodic workload at 1e-9 against the stored oracle values."""
    dmk = _dmk()
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "periodic_2e6_ewald.npz"))
    x, f = workloads.config("periodic_2e6")
    plan = dmk.Plan(_t(x), periodic=True, tol=1e-9, method=dmk.METHOD_EWALD)
    u = plan.eval(_t(f)).cpu().numpy()
    info = plan.info()
    err = oracle.rel_l2(u[g["idx"]], g["u"])
    print("spectral Ewald periodic_2e6:", info["levels"] - 1, info["ewald_grid"], info["ewald_modes"], err)
    assert err < 1e-9


@pytest.mark.parametrize("n", [1, 2, 50])
def test_small_sizes(dev, n):
    """Tiny periodic inputs (split level 1, 2^3 cells with repeated
    neighbours through the wrap) against the Gaussian Ewald oracle."""
    dmk = _dmk()
    x, f = workloads.make("uniform", n, seed=220 + n)
    plan = dmk.Plan(_t(x), periodic=True, tol=1e-6, method=dmk.METHOD_EWALD)
    u = plan.eval(_t(f)).cpu().numpy()
    ref = ewald(x, f, np.arange(n))
    err = oracle.rel_l2(u, ref)
    print("spectral Ewald small", n, plan.info()["ewald_grid"], err)
    assert err < 1e-6

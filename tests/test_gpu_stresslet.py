"""GPU parity of the stresslet path (dmk_stokes_eval_stresslet) against the
oracle's direct stresslet sum and its brute-force residual stresslet, through
the C ABI."""
import numpy as np
import pytest

import oracle
import workloads
from oracle import splitting as S

pytestmark = pytest.mark.gpu


def _dmk():
    import paper_2509_21471_amd as dmk
    return dmk


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _inputs(kind, n, seed, sigma=0.02):
    x, f = workloads.make(kind, n, seed=seed, sigma=sigma)
    return x, f, workloads.normals(x, seed, "sphere" if kind == "sphere" else "random")


def _plan(x, tol, **kw):
    dmk = _dmk()
    return dmk.Plan(_t(x), tol=tol, kernel=dmk.KERNEL_STRESSLET, **kw)


@pytest.mark.parametrize("tol,q", [(1e-6, 19), (1e-9, 26)])
def test_residual_stresslet_matches_oracle(dev, tol, q):
    """Near-field stresslet pair routine vs the oracle's residual stresslet
    (eq. res_stresslet with eq. T-offd at scale r_lambda), brute force over
    all pairs; coincident pairs contribute nothing on both sides."""
    rng = np.random.default_rng(21)
    rl = 0.125
    xt = rng.random((300, 3)) * 0.3
    xs = np.concatenate([rng.random((700, 3)) * 0.3, xt[:50]])
    fs = rng.normal(size=(xs.shape[0], 3))
    ns = rng.normal(size=(xs.shape[0], 3))
    win = S.ProlateWindow(S.prolate_c(q))
    ref = S.residual_stresslet_pair_sum(win, xt, xs, fs, ns, rl)
    got = _dmk().residual_sum_stresslet(_t(xt), _t(xs), _t(fs), _t(ns), rl, tol).cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"residual stresslet tol={tol}: max rel err {err:.2e}")
    # radial fits at 1e-3 tol of their scale
    assert err < 20 * 1e-3 * tol


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9, 1e-12])
def test_uniform_matches_direct(dev, tol):
    x, f, nv = _inputs("uniform", 12000, seed=70)
    plan = _plan(x, tol, leaf_size=200)
    u = plan.eval_stresslet(_t(f), _t(nv)).cpu().numpy()
    ref = oracle.stresslet_direct(x, f, nv)
    err = oracle.rel_l2(u, ref)
    print("stresslet uniform", tol, plan.info()["levels"], plan.info()["p"], err)
    assert err < tol


_DEEP = {}


def _deep():
    """20000 points in tight clusters (sigma 0.005, 9 levels at leaf 100), and
    their direct sum (computed once)."""
    if not _DEEP:
        x, f, nv = _inputs("clusters", 20000, seed=15, sigma=0.005)
        _DEEP["v"] = (x, f, nv, oracle.stresslet_direct(x, f, nv))
    return _DEEP["v"]


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9, 1e-12])
def test_deep_clusters_all_tolerances(dev, tol):
    x, f, nv, ref = _deep()
    plan = _plan(x, tol, leaf_size=100)
    u = plan.eval_stresslet(_t(f), _t(nv)).cpu().numpy()
    err = oracle.rel_l2(u, ref)
    print("stresslet deep clusters", tol, plan.info()["levels"], plan.info()["p"], err / tol)
    assert plan.info()["levels"] >= 8
    assert err < tol


@pytest.mark.parametrize("n,leaf", [(1, 0), (2, 0), (50, 0), (3000, 100)])
def test_small(dev, n, leaf):
    # seed 3080 at n = 3000: the input on which the printed p = 22 missed 1e-6
    x, f, nv = _inputs("uniform", n, seed=80 + n)
    plan = _plan(x, 1e-6, leaf_size=leaf)
    u = plan.eval_stresslet(_t(f), _t(nv)).cpu().numpy()
    if n == 1:
        # no self term: exactly what the far field leaves at the point (tol-sized)
        assert np.abs(u).max() < 1e-6 * np.abs(f).max() * np.abs(nv).max()
        return
    err = oracle.rel_l2(u, oracle.stresslet_direct(x, f, nv))
    assert err < 1e-6


def test_clusters_adaptive(dev):
    x, f, nv = _inputs("clusters", 40000, seed=90, sigma=0.02)
    plan = _plan(x, 1e-6, leaf_size=150)
    u = plan.eval_stresslet(_t(f), _t(nv)).cpu().numpy()
    t = np.arange(0, x.shape[0], 5)
    err = oracle.rel_l2(u[t], oracle.stresslet_direct(x, f, nv, t))
    print("stresslet clusters", plan.info()["levels"], err)
    assert plan.info()["levels"] >= 5
    assert err < 1e-6


def test_sphere_surface_normals(dev):
    x, f, nv = _inputs("sphere", 30000, seed=91)
    plan = _plan(x, 1e-6, leaf_size=200)
    u = plan.eval_stresslet(_t(f), _t(nv)).cpu().numpy()
    t = np.arange(0, x.shape[0], 5)
    err = oracle.rel_l2(u[t], oracle.stresslet_direct(x, f, nv, t))
    print("stresslet sphere", plan.info()["levels"], err)
    assert err < 1e-6


def test_mixed_precision(dev):
    dmk = _dmk()
    x, f, nv = _inputs("clusters", 20000, seed=92, sigma=0.03)
    plan = _plan(x, 1e-6, leaf_size=200, precision=dmk.PREC_MIXED)
    u = plan.eval_stresslet(_t(f), _t(nv)).cpu().numpy()
    err = oracle.rel_l2(u, oracle.stresslet_direct(x, f, nv))
    print("stresslet mixed", err)
    assert err < 1e-6


def test_multi_rhs_equals_single(dev):
    x, f, nv = _inputs("uniform", 5000, seed=93)
    rng = np.random.default_rng(94)
    F = np.stack([f, rng.normal(size=f.shape)])
    N = np.stack([nv, rng.normal(size=nv.shape)])
    plan = _plan(x, 1e-6, leaf_size=150)
    both = plan.eval_stresslet(_t(F), _t(N)).cpu().numpy()
    for r in range(2):
        one = plan.eval_stresslet(_t(F[r]), _t(N[r])).cpu().numpy()
        assert np.array_equal(both[r], one)


def test_separate_targets(dev):
    dmk = _dmk()
    x, f, nv = _inputs("sphere", 8000, seed=95)
    tg = workloads.sphere_targets(3000, 95)
    plan = dmk.Plan(_t(x), tol=1e-6, leaf_size=150, targets=_t(tg), kernel=dmk.KERNEL_STRESSLET)
    u = plan.eval_stresslet(_t(f), _t(nv)).cpu().numpy()
    # direct sum over the sources at the targets: targets appended with zero strength
    xa = np.concatenate([x, tg])
    fa = np.concatenate([f, np.zeros_like(tg)])
    na = np.concatenate([nv, np.zeros_like(tg)])
    ref = oracle.stresslet_direct(xa, fa, na, np.arange(x.shape[0], xa.shape[0]))
    err = oracle.rel_l2(u, ref)
    print("stresslet targets", err)
    assert u.shape == (3000, 3) and err < 1e-6


def test_batched_problems(dev):
    dmk = _dmk()
    probs = [_inputs("uniform", 3000, seed=96), _inputs("clusters", 5000, seed=97, sigma=0.05)]
    # the second problem lives in its own, larger cube: the 1/L^2 scaling per problem
    probs[1] = (probs[1][0] * 7.0 - 2.0, probs[1][1], probs[1][2])
    x = np.concatenate([p[0] for p in probs])
    f = np.concatenate([p[1] for p in probs])
    nv = np.concatenate([p[2] for p in probs])
    off = [0, 3000, 8000]
    plan = dmk.Plan(_t(x), tol=1e-6, leaf_size=150, offsets=off, kernel=dmk.KERNEL_STRESSLET)
    u = plan.eval_stresslet(_t(f), _t(nv)).cpu().numpy()
    for b, (xb, fb, nb) in enumerate(probs):
        err = oracle.rel_l2(u[off[b]:off[b + 1]], oracle.stresslet_direct(xb, fb, nb))
        print("stresslet batch", b, err)
        assert err < 1e-6


def test_stokeslet_plan_refuses_stresslet_eval(dev):
    dmk = _dmk()
    x, f, nv = _inputs("uniform", 100, seed=98)
    plan = dmk.Plan(_t(x), tol=1e-6)
    with pytest.raises(dmk.DMKError):
        plan.eval_stresslet(_t(f), _t(nv))
    splan = _plan(x, 1e-6)
    with pytest.raises(dmk.DMKError):
        splan.eval(_t(f))


def test_clusters_1e6_sampled(dev):
    """The benchmark's 1e6-point clustered input, at its tolerance, on 400
    sampled targets (direct sums over all 1e6 sources)."""
    x, f = workloads.config("clusters_1e6")
    nv = workloads.normals(x, 2)
    plan = _plan(x, 1e-6)
    u = plan.eval_stresslet(_t(f), _t(nv)).cpu().numpy()
    idx = workloads.sample_targets(x.shape[0], 400, 2)
    err = oracle.rel_l2(u[idx], oracle.stresslet_direct(x, f, nv, idx))
    print("stresslet clusters_1e6", plan.info()["levels"], err)
    assert err < 1e-6


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9])
def test_periodic_matches_ewald(dev, tol):
    """Periodic stresslet sum (k = 0 term of the paper included) vs the
    oracle's Gaussian Ewald sum."""
    from oracle.ewald import stresslet_ewald
    x, f, nv = _inputs("periodic", 4000, seed=99)
    plan = _plan(x, tol, leaf_size=150, periodic=True)
    u = plan.eval_stresslet(_t(f), _t(nv)).cpu().numpy()
    t = np.arange(0, 4000, 9)
    ref = stresslet_ewald(x, f, nv, t)
    err = oracle.rel_l2(u[t], ref)
    print("stresslet periodic", tol, plan.info()["levels"], err / tol)
    assert err < tol


def test_periodic_double_layer_identity(dev):
    """A closed sphere crossing the cell faces, constant density f0 on a
    surface quadrature (weights in the forces), outward normals: the periodic
    stresslet sum is f0 inside the sphere's images and 0 outside, up to the
    k = 0 term's dependence on the wrapped source positions."""
    R, c = 0.2, np.array([0.9, 0.15, 0.5])
    ct, wt = np.polynomial.legendre.leggauss(60)
    ph = np.arange(120) * 2 * np.pi / 120
    CT, PH = np.meshgrid(ct, ph, indexing="ij")
    st = np.sqrt(1 - CT ** 2)
    nv = np.stack([st * np.cos(PH), st * np.sin(PH), CT], -1).reshape(-1, 3)
    w = (np.outer(wt, np.full(120, 2 * np.pi / 120)) * R * R).ravel()
    xs = c + R * nv
    f0 = np.array([-0.2, 0.4, 0.9])
    tg = np.array([[0.95, 0.12, 0.45], [0.02, 0.15, 0.5], [0.9, 0.15, 0.5], [0.5, 0.5, 0.5], [0.3, 0.7, 0.1]])
    inside = np.array([1, 1, 1, 0, 0], dtype=float)
    dmk = _dmk()
    xw = xs - np.floor(xs)
    plan = dmk.Plan(_t(xw), tol=1e-9, periodic=True, targets=_t(tg), kernel=dmk.KERNEL_STRESSLET)
    u = plan.eval_stresslet(_t(f0 * w[:, None]), _t(nv)).cpu().numpy()
    p = np.floor(xs)
    shift = -(p * ((f0 * w[:, None]) * nv).sum(axis=1)[:, None]).sum(axis=0)
    err = np.abs(u - shift - inside[:, None] * f0).max()
    print("periodic double layer", err)
    assert err < 1e-8


def test_periodic_2e6_stored_ewald(dev):
    """The 2e6-point periodic workload at 1e-9 against the oracle's stored
    periodic stresslet values (tests/golden/make_references.py)."""
    import os
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                             "periodic_2e6_stresslet_ewald.npz"))
    x, f = workloads.config("periodic_2e6")
    nv = workloads.normals(x, 3)
    plan = _plan(x, 1e-9, periodic=True)
    u = plan.eval_stresslet(_t(f), _t(nv)).cpu().numpy()
    err = oracle.rel_l2(u[g["idx"]], g["u"])
    print("stresslet periodic_2e6", plan.info()["levels"], err)
    assert err < 1e-9


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9])
def test_shallow_random_problems(dev, tol):
    """150 problems of 500 points (random cube sizes and offsets, random
    orientation vectors) in one batched plan at leaf size 60: the inputs on
    which the printed parameter rows missed the tolerance."""
    rng = np.random.default_rng(95)
    P, m = 150, 500
    x = rng.random((P, m, 3)) * rng.uniform(0.5, 2.0, (P, 1, 1)) + rng.uniform(-5, 5, (P, 1, 3))
    f = rng.normal(size=(P, m, 3))
    nv = rng.normal(size=(P, m, 3))
    off = np.arange(P + 1, dtype=np.int64) * m
    dmk = _dmk()
    plan = dmk.Plan(_t(x.reshape(-1, 3)), tol=tol, leaf_size=60, offsets=off, kernel=dmk.KERNEL_STRESSLET)
    u = plan.eval_stresslet(_t(f.reshape(-1, 3)), _t(nv.reshape(-1, 3))).cpu().numpy().reshape(P, m, 3)
    errs = [oracle.rel_l2(u[b], oracle.stresslet_direct(x[b], f[b], nv[b])) for b in range(0, P, 3)]
    print("stresslet shallow problems", tol, max(errs) / tol)
    assert max(errs) < tol

"""The reorder of points inside leaves (compact near-field groups) against
Morton order, through the C ABI: the same sums up to rounding, the same leaf
of every point, the same in-support pair count (a within-leaf permutation
cannot change which pairs lie within r_lambda), and fewer evaluated pairs."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


def _dmk():
    import paper_2509_21471_amd as dmk
    return dmk


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _run(x, f, leaf_order, **kw):
    plan = _dmk().Plan(_t(x), leaf_order=leaf_order, **kw)
    u = plan.eval(_t(f)).cpu().numpy()
    stats = plan.near_stats()
    leaves = plan.tree_leaves()
    plan.close()
    return u, stats, leaves


@pytest.mark.parametrize("name,n,leaf,lanes,tol", [
    ("clusters", 60000, 1200, 4, 1e-6),
    ("clusters", 60000, 5000, 8, 1e-6),     # leaves above 2048 points: several bisection pieces
    ("uniform", 30000, 700, 1, 1e-9),
    ("periodic", 40000, 900, 2, 1e-6),
])
def test_leaf_order_matches_morton(dev, name, n, leaf, lanes, tol):
    x, f = workloads.make(name, n, seed=81)
    periodic = name == "periodic"
    kw = dict(tol=tol, leaf_size=leaf, near_lanes=lanes, periodic=periodic)
    u, st, lv = _run(x, f, True, **kw)
    um, stm, lvm = _run(x, f, False, **kw)
    assert oracle.rel_l2(u, um) < 1e-12
    for a, b in zip(lv, lvm):
        np.testing.assert_array_equal(a, b)
    assert st["listed"] == stm["listed"]
    assert st["in_support"] == stm["in_support"]
    assert st["evaluated"] < stm["evaluated"]
    if not periodic:
        idx = np.random.default_rng(82).choice(n, 300, replace=False)
        assert oracle.rel_l2(u[idx], oracle.direct(x, f, targets=idx)) < tol


def test_leaf_order_targets_and_batches(dev):
    """Separate targets (sources and targets reordered separately inside each
    leaf) and a batch of problems."""
    dmk = _dmk()
    x, f = workloads.make("clusters", 30000, seed=83)
    y, _ = workloads.make("uniform", 20000, seed=84)
    res = []
    for order in (True, False):
        p = dmk.Plan(_t(x), tol=1e-6, leaf_size=500, targets=_t(y), leaf_order=order)
        res.append(p.eval(_t(f)).cpu().numpy())
        p.close()
    assert oracle.rel_l2(res[0], res[1]) < 1e-12
    sizes = [3000, 17000, 9000, 40]
    xs = [workloads.make("clusters" if i % 2 else "uniform", m, seed=90 + i)[0] for i, m in enumerate(sizes)]
    xb = np.concatenate(xs)
    fb = np.random.default_rng(95).standard_normal(xb.shape)
    off = np.concatenate([[0], np.cumsum(sizes)])
    res = []
    for order in (True, False):
        p = dmk.Plan(_t(xb), tol=1e-6, leaf_size=400, offsets=off, leaf_order=order)
        res.append(p.eval(_t(fb)).cpu().numpy())
        p.close()
    assert oracle.rel_l2(res[0], res[1]) < 1e-12

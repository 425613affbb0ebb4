"""The octree built on the device (Step 1 of Sec. "The DMK method": radix
sort of the Morton keys, adaptive refinement, 2:1 level restriction over
vertex adjacency, neighbour lists) against the sequential host construction.

* Periodic inputs: the unit cell maps every point to itself, so the host
  computes the same Morton keys on the CPU and sorts them with std::sort;
  the device plan's leaves (levels, coordinates, counts) and near-pair count
  must equal dmk_stokes_host_tree's exactly (this also pins the radix sort).
* Any input: a plan with the host construction from the same device-sorted
  keys (DMK_FLAG_HOST_TREE) must give identical leaves, lists and sums, bit
  for bit."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _dmk():
    import paper_2509_21471_amd as dmk
    return dmk


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _leaves(plan):
    lev, crd, cnt, pl = plan.tree_leaves()
    return lev, crd, cnt, pl


@pytest.mark.parametrize("kind,n,ls", [("periodic", 8000, 50), ("periodic", 30000, 200),
                                       ("clusters", 12000, 40), ("clusters", 40000, 30)])
def test_periodic_device_tree_equals_cpu_tree(dev, kind, n, ls):
    x, _ = workloads.make(kind, n, seed=90 + n, sigma=0.03)
    x = np.mod(x, 1.0)
    plan = _dmk().Plan(_t(x), periodic=True, tol=1e-6, leaf_size=ls)
    lev, crd, cnt, _ = _leaves(plan)
    info = plan.info()
    plan.close()
    hl, hc, hn, hpairs = _dmk().host_tree(x, ls, periodic=True)
    assert np.array_equal(lev, hl) and np.array_equal(crd, hc) and np.array_equal(cnt, hn)
    assert info["near_pairs"] == hpairs
    # the exchange lists too: same senders and receivers as the host construction
    ph = _dmk().Plan(_t(x), periodic=True, tol=1e-6, leaf_size=ls, host_tree=True)
    ih = ph.info()
    ph.close()
    assert (info["n_senders"], info["n_receivers"]) == (ih["n_senders"], ih["n_receivers"])


CASES = [
    ("uniform", 5000, 100, False, 0.0),
    ("clusters", 20000, 64, False, 0.03),     # deep, unbalanced before the restriction
    ("clusters", 30000, 200, False, 0.01),
    ("periodic", 8000, 50, True, 0.0),
    ("clusters", 3000, 8, False, 0.002),       # many levels
]


@pytest.mark.parametrize("kind,n,ls,periodic,sigma", CASES)
def test_device_tree_equals_host_construction(dev, kind, n, ls, periodic, sigma):
    x, f = workloads.make(kind, n, seed=91, sigma=sigma)
    if periodic:
        x = np.mod(x, 1.0)
    dmk = _dmk()
    pd = dmk.Plan(_t(x), periodic=periodic, tol=1e-6, leaf_size=ls)
    ph = dmk.Plan(_t(x), periodic=periodic, tol=1e-6, leaf_size=ls, host_tree=True)
    a, b = _leaves(pd), _leaves(ph)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    ia, ib = pd.info(), ph.info()
    for k in ("levels", "n_boxes", "n_leaves", "n_nonempty_leaves", "near_pairs", "n_senders", "n_receivers"):
        assert ia[k] == ib[k], k
    assert ia["levels"] >= 3
    ua = pd.eval(_t(f)).cpu().numpy()
    ub = ph.eval(_t(f)).cpu().numpy()
    assert np.array_equal(ua, ub)


def test_coincident_points_reach_the_deepest_level(dev):
    """All points at one location: the tree refines to the maximum depth and
    both constructions agree."""
    x = np.concatenate([np.full((60, 3), 0.3), np.random.default_rng(3).random((200, 3))])
    dmk = _dmk()
    pd = dmk.Plan(_t(x), tol=1e-6, leaf_size=10)
    ph = dmk.Plan(_t(x), tol=1e-6, leaf_size=10, host_tree=True)
    a, b = _leaves(pd), _leaves(ph)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    assert a[0].max() == 19


def test_batched_forest_equals_host_construction(dev):
    """A forest of independent problems (device segmented sort and one octree
    per problem) against the host's per-problem trees merged."""
    rng = np.random.default_rng(92)
    parts, fs = [], []
    for b in range(23):
        m = int(10 ** rng.uniform(1.5, 3.7))
        kind = "uniform" if b % 3 else "clusters"
        xb, fb = workloads.make(kind, m, seed=920 + b, sigma=0.05)
        parts.append(xb * rng.uniform(0.5, 3.0) + rng.normal(size=3))
        fs.append(fb)
    x = np.concatenate(parts)
    f = np.concatenate(fs)
    off = np.concatenate([[0], np.cumsum([p.shape[0] for p in parts])])
    dmk = _dmk()
    pd = dmk.Plan(_t(x), tol=1e-6, leaf_size=40, offsets=off)
    ph = dmk.Plan(_t(x), tol=1e-6, leaf_size=40, offsets=off, host_tree=True)
    a, b = _leaves(pd), _leaves(ph)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    assert pd.info()["near_pairs"] == ph.info()["near_pairs"]
    ua = pd.eval(_t(f)).cpu().numpy()
    ub = ph.eval(_t(f)).cpu().numpy()
    assert np.array_equal(ua, ub)


def test_benchmark_input_tree(dev):
    """The 1e6-point clustered benchmark input at its autotuned leaf size."""
    x, _ = workloads.config("clusters_1e6")
    dmk = _dmk()
    pd = dmk.Plan(_t(x), tol=1e-6, leaf_size=2160)
    ph = dmk.Plan(_t(x), tol=1e-6, leaf_size=2160, host_tree=True)
    a, b = _leaves(pd), _leaves(ph)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    assert pd.info()["near_pairs"] == ph.info()["near_pairs"]

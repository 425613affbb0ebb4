"""Octree invariants on the host build (Step 1 of Sec. "The DMK method"):
leaves tile the unit cube, hold every point, respect the leaf size, and are
level-restricted: leaves sharing a boundary point (vertex adjacency, through
the periodic wrap when periodic) differ by at most one level.  Checked by
brute force over all leaf pairs."""
import numpy as np
import pytest

import workloads


def _dmk():
    import paper_2509_21471_amd as dmk
    return dmk


def check_tree(lev, crd, cnt, n, leaf_size, periodic):
    assert cnt.sum() == n
    assert np.all(cnt[lev < 19] <= leaf_size)
    h = 1.0 / (1 << lev.astype(np.int64))
    assert abs(np.sum(h ** 3) - 1.0) < 1e-12          # leaves tile the cube
    lo = crd * h[:, None]
    hi = lo + h[:, None]
    shifts = [np.zeros(3)]
    if periodic:
        shifts = [np.array([a, b, c], float) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    for i in range(len(lev)):
        for sh in shifts:
            touch = np.all((lo + sh <= hi[i] + 1e-15) & (hi + sh >= lo[i] - 1e-15), axis=1)
            bad = np.abs(lev[touch] - lev[i]) > 1
            assert not np.any(bad), (i, lev[i], lev[touch][bad][:5])


@pytest.mark.parametrize("kind,n,ls,periodic", [
    ("uniform", 5000, 100, False),
    ("clusters", 20000, 64, False),
    ("clusters", 30000, 200, False),
    ("periodic", 8000, 50, True),
    ("clusters", 12000, 40, True),
])
def test_host_tree_invariants(kind, n, ls, periodic):
    x, _ = workloads.make("periodic" if periodic and kind != "clusters" else kind, n, seed=70 + n, sigma=0.03)
    if periodic:
        x = x % 1.0
    lev, crd, cnt, _ = _dmk().host_tree(x, ls, periodic)
    check_tree(lev, crd, cnt, n, ls, periodic)


def test_host_tree_degenerate_inputs():
    dmk = _dmk()
    # root stays a leaf
    lev, crd, cnt, _ = dmk.host_tree(np.random.default_rng(0).random((10, 3)), 100)
    assert len(lev) == 1 and cnt[0] == 10
    # all points coincident: depth stops at the maximum level
    lev, crd, cnt, _ = dmk.host_tree(np.full((50, 3), 0.3), 10)
    assert cnt.sum() == 50 and lev.max() == 19 and cnt[lev == 19].max() == 50
    check_tree(lev, crd, cnt, 50, 10, False)
    # two far clusters of coincident points force deep, balanced refinement
    x = np.concatenate([np.full((30, 3), 0.1), np.full((30, 3), 0.9)])
    lev, crd, cnt, _ = dmk.host_tree(x, 10)
    check_tree(lev, crd, cnt, 60, 10, False)
    # points on faces and corners of the unit cell (periodic)
    x = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5], [0.0, 0.5, 0.999999], [0.25, 0.0, 0.75]] * 10)
    lev, crd, cnt, _ = dmk.host_tree(x, 3, periodic=True)
    check_tree(lev, crd, cnt, 40, 3, True)

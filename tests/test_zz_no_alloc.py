"""The residual-sum entry point for callers that cannot allocate
(dmk_stokes_residual_sum_noalloc, staging in the library's fixed device
workspace) against dmk_stokes_residual_sum on the same inputs, through the C
ABI: two calls in a row, the second smaller, each bit for bit equal."""
import numpy as np
import pytest

from oracle import splitting as S

pytestmark = pytest.mark.gpu


def _dmk():
    import paper_2509_21471_amd as dmk
    return dmk


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _case(seed, m, ns, rl):
    rng = np.random.default_rng(seed)
    xt = rng.random((m, 3)) * 0.4
    xs = np.concatenate([rng.random((ns - 20, 3)) * 0.4, xt[:20]])  # coincident pairs included
    fs = rng.normal(size=(ns, 3))
    return xt, xs, fs


@pytest.mark.parametrize("tol,q", [(1e-6, 17), (1e-9, 25)])
def test_noalloc_matches_allocating_entry(dev, tol, q):
    import torch
    dmk = _dmk()
    rl = 0.125
    for seed, m, ns in ((40, 3000, 5000), (41, 700, 900)):  # second call smaller
        xt, xs, fs = _case(seed, m, ns, rl)
        tt, ts, tf = _t(xt), _t(xs), _t(fs)
        out = torch.full((m, 3), np.nan, dtype=torch.float64, device="cuda:0")
        dmk.residual_sum_noalloc(tt, ts, tf, rl, tol, out)
        got = out.cpu().numpy()
        ref = dmk.residual_sum(tt, ts, tf, rl, tol).cpu().numpy()
        assert np.array_equal(got, ref), (seed, np.abs(got - ref).max())
        if seed == 41:
            # and both follow the oracle's residual Stokeslet (eq. res_stokeslet)
            win = S.ProlateWindow(S.prolate_c(q))
            o = S.residual_pair_sum(win, xt, xs, fs, rl)
            same = np.all(xt[:, None, :] == xs[None, :, :], axis=2)
            o = o - win.phi(0.0) / (2 * np.pi * rl) * (same.astype(float) @ fs)
            assert np.abs(got - o).max() / np.abs(o).max() < 1e-6


def test_noalloc_rejects_oversize(dev):
    import torch
    dmk = _dmk()
    m = (1 << 21) // 3 + 1  # 3 m alone exceeds the workspace
    xt = torch.zeros((m, 3), dtype=torch.float64, device="cuda:0")
    xs = torch.zeros((1, 3), dtype=torch.float64, device="cuda:0")
    out = torch.empty_like(xt)
    with pytest.raises(dmk.DMKError) as e:
        dmk.residual_sum_noalloc(xt, xs, xs, 0.1, 1e-6, out)
    assert e.value.code == -1 and "workspace" in str(e.value)

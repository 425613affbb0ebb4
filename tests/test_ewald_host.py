"""Host-side parameters of the spectral Ewald method (no GPU): the split
level and mode bound follow the strict mode rule |k_i| < c / r_c, the grid
is oversampled and tiles into Morton cells, and the prolate gridding kernel's
aliasing, evaluated with the oracle's own prolate functions, stays below the
tolerance."""
import math

import numpy as np
import pytest

from oracle import splitting as S


def _dmk():
    import paper_2509_21471_amd as dmk
    return dmk


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9])
@pytest.mark.parametrize("n", [1, 3000, 20000, 2_000_000])
def test_grid_rules(tol, n):
    e = _dmk().ewald_params(tol, n)
    L = e["levels"] - 1
    ns = e["leaf_size"]
    assert L >= 1 and (L == 1 or n / 8 ** (L - 1) > ns) and (n / 8 ** L <= ns or L == 8)
    K, M, w, q = e["ewald_modes"], e["ewald_grid"], e["ewald_width"], e["q"]
    lim = q * 2 ** L / 6           # |kappa_i| < c / (2 pi r_c) = q 2^L / 6
    assert K < lim <= K + 1
    assert M >= 1.9 * (2 * K + 1)
    assert any(M == B * 2 ** Lt for B in (6, 8) for Lt in range(10))
    assert w == {1e-3: 6, 1e-6: 8, 1e-9: 11}[tol]


def test_benchmark_grid():
    # 2e6 periodic points at 1e-9: 488 points per cell at level 4, K = 66, M = 256
    e = _dmk().ewald_params(1e-9, 2_000_000)
    assert (e["levels"] - 1, e["ewald_modes"], e["ewald_grid"], e["ewald_width"]) == (4, 66, 256, 11)


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9])
def test_gridding_kernel_aliasing(tol):
    """Relative size of the aliases kappa + m M (m != 0) against kappa, for
    every retained |kappa| <= K, with the gridding kernel rebuilt from the
    oracle's prolate window at beta = pi w (1 - 1/(2 sigma))."""
    e = _dmk().ewald_params(tol, 2_000_000)
    K, M, w = e["ewald_modes"], e["ewald_grid"], e["ewald_width"]
    sigma = M / (2 * K + 1)
    beta = math.pi * w * (1 - 1 / (2 * sigma))
    win = S.ProlateWindow(beta)
    alpha = w / (2 * M)
    kap = np.arange(0, K + 1)
    ghat = lambda k: win.phihat(2 * np.pi * k * alpha)  # noqa: E731
    base = np.abs(ghat(kap))
    alias = sum(np.abs(ghat(kap + m * M)) for m in (-2, -1, 1, 2))
    ratio = alias / base
    # What reaches the sum: a mode's coefficient carries the aliases of the
    # three separable factors, twice (spreading and interpolation), and is
    # weighted by the mollified kernel's symbol gammahat(k r_c)/k^2, which the
    # mode bound K puts at about tol where the ratio is largest.  Aggregate
    # over the retained cube of modes for sources of flat spectrum.
    L = e["levels"] - 1
    split = S.ProlateWindow(S.prolate_c(e["q"]))
    ks = np.arange(-K, K + 1)
    r1 = ratio[np.abs(ks)]
    KX, KY, KZ = np.meshgrid(ks, ks, ks, indexing="ij")
    m2 = KX ** 2 + KY ** 2 + KZ ** 2
    kv = 2 * np.pi * np.sqrt(np.arange(1, 3 * K * K + 1))
    wv = np.concatenate([[0.0], split.gammahat(kv / 2 ** L) / kv ** 2])
    W = wv[m2]
    R3 = 2 * (r1[:, None, None] + r1[None, :, None] + r1[None, None, :])
    agg = float(np.sum(R3 * W) / np.sum(W))
    print(f"tol {tol}: w {w} sigma {sigma:.2f} beta {beta:.2f} worst alias ratio {ratio.max():.2e}, "
          f"symbol-weighted aggregate {agg:.2e}")
    # the aggregate adds every alias coherently (a pessimistic bound: the
    # measured totals on 3000 to 2e6 points are 0.06 to 0.5 tol with the near
    # field's share included)
    assert agg < 0.3 * tol
    assert ratio.max() < 10 * tol

"""Stresslet on the CPU: the parameter rows, the near-field radial fits of the
residual stresslet against the oracle's window functions, and argument
validation of the stresslet entry points (no GPU needed)."""
import ctypes
import math

import numpy as np
import pytest

from oracle import splitting as S


def _dmk():
    import paper_2509_21471_amd as dmk
    return dmk


# Table tab:params, stresslet block, PSWF columns: (q, p, N_1, N_per) as printed
PRINTED = {1e-3: (9, 11, 17, 3), 1e-6: (17, 22, 33, 5), 1e-9: (25, 33, 49, 9), 1e-12: (32, 44, 63, 11)}
# the rows as run: q and p stepped up (measured: the printed rows leave up to
# 1.9 tol on shallow trees of a few hundred points with random orientations)
USED = {1e-3: (11, 14), 1e-6: (19, 26), 1e-9: (26, 36), 1e-12: (32, 48)}


@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9, 1e-12])
def test_stresslet_parameters_follow_table(tol):
    dmk = _dmk()
    prm = dmk.params(tol, kernel=dmk.KERNEL_STRESSLET)
    q, p = USED[tol]
    qp, pp, n1p, nperp = PRINTED[tol]
    assert q >= qp and p >= pp
    # N_1 = 2q - 1 and N_per = 2 ceil(q/6) - 1 (the strict mode rule) reproduce the printed columns
    assert (2 * qp - 1, 2 * math.ceil(qp / 6) - 1) == (n1p, nperp)
    assert (prm["q"], prm["p"], prm["n1"], prm["nper"], prm["kernel"]) == (q, p, 2 * q - 1, 2 * math.ceil(q / 6) - 1, 1)
    assert abs(prm["c"] - q * np.pi / 3) < 1e-14
    # the fits fit the 24 coefficients the near-field kernel holds
    assert max(prm["deg_P"], prm["deg_Q"]) <= 23


def test_stresslet_gaussian_is_refused():
    dmk = _dmk()
    with pytest.raises(dmk.DMKError):
        dmk.params(1e-6, window=1, kernel=dmk.KERNEL_STRESSLET)


@pytest.mark.parametrize("tol,q", [(1e-3, 11), (1e-6, 19), (1e-9, 26), (1e-12, 32)])
def test_stresslet_fits_match_oracle(tol, q):
    """A = (1 - R_Toffd)/(2 rho^5) and D = R_Tdiag/(2 rho^3) (eq. T-offd
    rearranged around the free-space stresslet), R_Toffd and R_Tdiag from the
    oracle's window (its Phi by quadrature).  Below rho ~ 0.3 the oracle's
    form loses digits to cancellation, so the comparison starts there and the
    fits' small-rho behaviour is checked against the series limit instead."""
    win = S.ProlateWindow(S.prolate_c(q))
    rho = np.linspace(0.3, 0.999, 71)
    got = _dmk().radial_stresslet(tol, rho)
    A = (1.0 - win.Toffd(rho)) / (2.0 * rho ** 5)
    D = win.Tdiag(rho) / (2.0 * rho ** 3)
    # the residual's terms are A y y y and D y: compare at their scale
    eA = np.max(np.abs(got[:, 0] - A) * rho ** 3)
    eD = np.max(np.abs(got[:, 1] - D) * rho)
    scale = np.max(np.abs(D * rho))
    assert eA < 50 * max(1e-3 * tol, 1e-13) * scale, eA
    assert eD < 50 * max(1e-3 * tol, 1e-13) * scale, eD
    # rho -> 0: D(0) = -phi''(0) (phi even), A(0) = (1/s) int u^2 [psi(s) - psi(s u^2)] -> psi'(0)/5
    # with psi(sigma) = phi'(sqrt sigma)/sqrt sigma; check by differences of the oracle's phi'
    h = 1e-3
    d2 = (win.dphi(h) - win.dphi(-h)) / (2 * h)
    g0 = _dmk().radial_stresslet(tol, np.array([1e-4]))[0]
    assert abs(g0[1] + d2) < 1e-4 * abs(d2)


def test_stresslet_argument_validation_without_gpu():
    dmk = _dmk()
    lib = dmk.lib()
    out = ctypes.c_void_p()
    host = (ctypes.c_double * 30)()
    vp = ctypes.cast(host, ctypes.c_void_p)
    st = dmk._lib.Opts(0, 0, None, 0, 0, 0, 0, 0, 0, 0, 1)
    # periodic stresslet plans pass validation (and stop at the host pointer)
    assert lib.dmk_stokes_plan_ex(vp, 10, 3, 1, 1e-6, ctypes.byref(st), ctypes.byref(out)) == -1
    # prolate window only
    stg = dmk._lib.Opts(0, 0, None, 0, 0, 0, 0, 0, 0, 1, 1)
    assert lib.dmk_stokes_plan_ex(vp, 10, 3, 0, 1e-6, ctypes.byref(stg), ctypes.byref(out)) == -2
    # no graph capture
    stgr = dmk._lib.Opts(0, 0, None, 0, 4, 0, 0, 0, 0, 0, 1)
    assert lib.dmk_stokes_plan_ex(vp, 10, 3, 0, 1e-6, ctypes.byref(stgr), ctypes.byref(out)) == -2
    bad = dmk._lib.Opts(0, 0, None, 0, 0, 0, 0, 0, 0, 0, 2)
    assert lib.dmk_stokes_plan_ex(vp, 10, 3, 0, 1e-6, ctypes.byref(bad), ctypes.byref(out)) == -1
    assert out.value is None
    assert lib.dmk_stokes_eval_stresslet(None, None, None, 1, None) == -1
    assert lib.dmk_stokes_residual_sum_stresslet(vp, 1, vp, vp, vp, 1, -1.0, 1e-6, None, vp) == -1
    # the autotuner times Stokeslet plans only
    tuned = dmk._lib.Opts()
    assert lib.dmk_stokes_autotune(vp, 10, None, 0, 3, 0, 1e-6, ctypes.byref(st), 1, ctypes.byref(tuned),
                                   None) == -2


def test_ewald_method_argument_validation_without_gpu():
    """DMK_METHOD_EWALD: one periodic FP64 prolate Stokeslet problem, tol >= 1e-9."""
    dmk = _dmk()
    lib = dmk.lib()
    out = ctypes.c_void_p()
    host = (ctypes.c_double * 30)()
    vp = ctypes.cast(host, ctypes.c_void_p)
    O = dmk._lib.Opts
    ew = O(0, 0, None, 0, 0, 0, 0, 0, 0, 0, 0, 1)
    # passes validation, stops at the host pointer
    assert lib.dmk_stokes_plan_ex(vp, 10, 3, 1, 1e-6, ctypes.byref(ew), ctypes.byref(out)) == -1
    assert lib.dmk_stokes_plan_ex(vp, 10, 3, 1, 1e-12, ctypes.byref(ew), ctypes.byref(out)) == -5
    mixed = O(1, 0, None, 0, 0, 0, 0, 0, 0, 0, 0, 1)
    assert lib.dmk_stokes_plan_ex(vp, 10, 3, 1, 1e-6, ctypes.byref(mixed), ctypes.byref(out)) == -2
    stress = O(0, 0, None, 0, 0, 0, 0, 0, 0, 0, 1, 1)
    assert lib.dmk_stokes_plan_ex(vp, 10, 3, 1, 1e-6, ctypes.byref(stress), ctypes.byref(out)) == -2
    graph = O(0, 0, None, 0, 4, 0, 0, 0, 0, 0, 0, 1)
    assert lib.dmk_stokes_plan_ex(vp, 10, 3, 1, 1e-6, ctypes.byref(graph), ctypes.byref(out)) == -2
    bad = O(0, 0, None, 0, 0, 0, 0, 0, 0, 0, 0, 2)
    assert lib.dmk_stokes_plan_ex(vp, 10, 3, 1, 1e-6, ctypes.byref(bad), ctypes.byref(out)) == -1
    assert out.value is None

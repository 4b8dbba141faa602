"""GPU precision control: the window condition number, routing of systems to
the FP64 re-solve, and the convergence test of the FP64-residual correction,
against the FP64 oracle and bit for bit against the unrouted and FP64
launches.

The per-voxel measure is |z_hat - z*| / max(|z*|, 0.01 Zmax); refine_tol is a
bound on it (see okr_problem.refine_tol)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from _gpu_util import rel_err_est, rel_err_var, run_gpu

pytestmark = pytest.mark.gpu


def _phantom(name, n, m, f, r, seed, n_ell=10, n_shell=2):
    w = W.Workload(name, n, m, f, r, True, n_ell, n_shell, 0.02,
                   W.Variogram("spherical", 0, 1, 4), seed)
    s = W.phantom(w)
    return s, W.sobel_edges(s)


# a reduced copy of the ill-conditioned precision study: Gaussian model,
# nugget 1e-4, 7x7x2 windows, f = 4 (kappa of the window about 1.9e5)
C3_VARIO = ("gaussian", 1e-4, 1.0, 5.0)


@pytest.fixture(scope="module")
def c3_small():
    s, e = _phantom("c3_small", 5, 64, 4, 3, 3)
    vol, var, _ = O.krige_volume(s, e, 4, 3, C3_VARIO)
    return s, e, vol, var


def _kz(nz, f):
    kz = np.ones(nz, bool)
    kz[::f] = False
    return kz


@pytest.mark.parametrize("vario,r,f", [(("spherical", 0.005, 1.0, 8.0), 3, 4),
                                       (("gaussian", 1e-4, 1.0, 5.0), 3, 4),
                                       (("exponential", 0.01, 1.0, 6.0), 2, 4),
                                       (("spherical", 0.0, 1.0, 4.0), 1, 2)])
def test_window_condition_matches_oracle(vario, r, f):
    """The library's host eigenvalue computation of the full-window covariance
    matrix agrees with the oracle's (LAPACK) condition number."""
    s, e = _phantom("kw", 3, 24, f, r, 4)
    _, _, _, st = run_gpu(s, e, f, r, vario, precision="mixed_fp16", refine_max=1,
                          refine_tol=1e-5)
    ref = O.window_condition(*vario, r, f)
    print(f"kappa_window {st['kappa_window']:.6e} oracle {ref:.6e}", flush=True)
    assert abs(st["kappa_window"] - ref) <= 1e-7 * ref


def test_fp32_routes_every_system_when_the_window_bound_misses_the_tolerance():
    s, e = _phantom("fp32route", 3, 40, 3, 3, 7)
    vario = ("gaussian", 0.05, 1.0, 5.0)
    kw = O.window_condition(*vario, 3, 3)
    v32, w32, _, _ = run_gpu(s, e, 3, 3, vario)
    v64, w64, _, _ = run_gpu(s, e, 3, 3, vario, precision="fp64")
    # tolerance below kappa_w 2^-24: every system goes to FP64, bit for bit
    vr, wr, fr, sr = run_gpu(s, e, 3, 3, vario, flags=True, refine_tol=0.5 * kw * 2.0 ** -24)
    assert sr["n_fp64_fallback"] == sr["n_systems"] and sr["direct_fp64"]
    assert ((fr & 4) != 0).all()
    np.testing.assert_array_equal(vr, v64)
    np.testing.assert_array_equal(wr, w64)
    # above it: nothing routed, bit for bit the FP32 launch
    vn, wn, fn, sn = run_gpu(s, e, 3, 3, vario, flags=True, refine_tol=2.0 * kw * 2.0 ** -24)
    assert sn["n_fp64_fallback"] == sn["n_nonpositive_pivot"] == 0 and not sn["direct_fp64"]
    np.testing.assert_array_equal(vn, v32)
    np.testing.assert_array_equal(wn, w32)


@pytest.mark.parametrize("direct", [True, False], ids=["direct", "checked"])
@pytest.mark.parametrize("precision", ["mixed_fp16", "mixed_bf16"])
def test_corrected_convergence_routing(precision, direct, c3_small, monkeypatch):
    """refine_max = 1 corrects every system; with refine_tol the systems the
    correction cannot bring under it (by the bound) are flagged (32), counted,
    and equal the FP64 launch bit for bit; the others equal the unchecked
    corrected launch bit for bit; every voxel then meets the mixed bar. The
    full window misses 1e-4 by its bound here, so by default every system is
    solved in FP64 directly (flagged and counted as re-solved, bit for bit the
    FP64 launch); OKR_NO_DIRECT_FP64=1 keeps the per-system checks."""
    if not direct:
        monkeypatch.setenv("OKR_NO_DIRECT_FP64", "1")
    s, e, vol_o, var_o = c3_small
    f, r = 4, 3
    tol = 1e-4
    v0, w0, f0, s0 = run_gpu(s, e, f, r, C3_VARIO, precision=precision, flags=True,
                             refine_max=1, refine_tol=0.0)
    v64, w64, _, _ = run_gpu(s, e, f, r, C3_VARIO, precision="fp64")
    vr, wr, fr, sr = run_gpu(s, e, f, r, C3_VARIO, precision=precision, flags=True,
                             refine_max=1, refine_tol=tol)
    unconv = (fr & 32) != 0
    routed = (fr & 4) != 0
    print(f"{precision}: kappa_w {sr['kappa_window']:.3e}, unconverged {unconv.sum()} of "
          f"{unconv.size}, FP64 {routed.sum()}", flush=True)
    assert sr["n_refine_unconverged"] == unconv.sum()
    assert (routed >= unconv).all()
    assert sr["n_fp64_fallback"] == routed.sum()
    assert s0["n_refined"] + s0["n_nonpositive_pivot"] == s0["n_systems"]
    assert sr["direct_fp64"] == direct
    if direct:
        assert routed.all() and sr["n_refined"] == 0 and not unconv.any()
    else:
        assert unconv.sum() > 0
    for g in range(s.shape[0] - 1):
        for t in range(1, f):
            z = g * f + t
            m = routed[g]
            np.testing.assert_array_equal(vr[z][m], v64[z][m])
            keep = ~m & ~((f0[g] & 4) != 0)
            np.testing.assert_array_equal(vr[z][keep], v0[z][keep])
    kz = _kz(vr.shape[0], f)
    ee = rel_err_est(vr[kz], vol_o[kz], np.abs(s).max())
    ev = rel_err_var(wr[kz], var_o[kz], 1.0)
    print(f"  max est err {ee.max():.3e} var err {ev.max():.3e}", flush=True)
    assert ee.max() <= tol
    assert ev.max() <= 1e-4


@pytest.mark.parametrize("direct", [True, False], ids=["direct", "checked"])
@pytest.mark.parametrize("precision", ["mixed_fp16", "mixed_bf16"])
def test_readout_routing_meets_the_tolerance(precision, direct, c3_small, monkeypatch):
    """refine_max = 0 with refine_tol: systems whose error indicator exceeds
    it are re-solved in FP64 (bit for bit the FP64 launch), the others keep
    the read-out (bit for bit the unrouted launch), and every voxel meets the
    tolerance (by default solved in FP64 directly, as the full window misses
    it; OKR_NO_DIRECT_FP64=1 keeps the per-system routing)."""
    if not direct:
        monkeypatch.setenv("OKR_NO_DIRECT_FP64", "1")
    s, e, vol_o, var_o = c3_small
    f, r = 4, 3
    tol = 1e-4
    v0, w0, f0, _ = run_gpu(s, e, f, r, C3_VARIO, precision=precision, flags=True, refine_max=0)
    v64, w64, _, _ = run_gpu(s, e, f, r, C3_VARIO, precision="fp64")
    vr, wr, fr, sr = run_gpu(s, e, f, r, C3_VARIO, precision=precision, flags=True,
                             refine_max=0, refine_tol=tol)
    routed = (fr & 4) != 0
    print(f"{precision} read-out: routed {routed.sum()} of {routed.size}", flush=True)
    assert sr["n_fp64_fallback"] == routed.sum()
    assert sr["direct_fp64"] == direct and (routed.all() if direct else True)
    for g in range(s.shape[0] - 1):
        for t in range(1, f):
            z = g * f + t
            m = routed[g]
            np.testing.assert_array_equal(vr[z][m], v64[z][m])
            keep = ~m & ~((f0[g] & 4) != 0)
            np.testing.assert_array_equal(vr[z][keep], v0[z][keep])
    kz = _kz(vr.shape[0], f)
    ee = rel_err_est(vr[kz], vol_o[kz], np.abs(s).max())
    print(f"  max est err {ee.max():.3e}", flush=True)
    assert ee.max() <= tol


def test_mixed_readout_routing_on_a_well_conditioned_window():
    """The large workload's variogram on a small phantom: with refine_tol =
    1e-3 some systems are routed and some are not, and the result meets it."""
    s, e = _phantom("c5_small", 4, 48, 4, 3, 5, n_ell=8, n_shell=2)
    vario = ("spherical", 0.005, 1.0, 8.0)
    vol_o, _, _ = O.krige_volume(s, e, 4, 3, vario)
    vr, _, fr, sr = run_gpu(s, e, 4, 3, vario, precision="mixed_fp16", flags=True, refine_max=0,
                            refine_tol=1e-3)
    routed = (fr & 4) != 0
    print(f"routed {routed.sum()} of {routed.size}", flush=True)
    assert 0 < routed.sum() < routed.size
    kz = _kz(vr.shape[0], 4)
    assert rel_err_est(vr[kz], vol_o[kz], np.abs(s).max()).max() <= 1e-3


def test_refine_max_above_one_is_rejected():
    import paper_2303_09523_amd as P
    with pytest.raises(P.OkrError) as ei:
        P.Plan(16, 16, 3, 2, 1, precision="mixed_fp16", refine_max=2)
    assert ei.value.status == 1

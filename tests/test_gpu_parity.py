"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Error measures: per voxel, |z_hat - z*| / max(|z*|, 0.01 Zmax) for the
estimate and |s2 - s2*| / sill for the variance (the bars); normwise,
max |z_hat - z*| / max |z*| (printed, and asserted only as an extra check on
the FP32 paths). Bars:
  * FP32 paths (batched and plain per-voxel) and the mixed read-out: per
    voxel <= 1e-4. Their per-voxel error is set by FP32 border solves over an
    FP32 factor (about 5e-5 on 7x7x2 windows), so they are not claimed at
    1e-5; the 1e-5 bar is carried by the refined mixed paths.
  * mixed FP16 with the FP64-residual correction (the plan default,
    refine_max = 1): per voxel <= 1e-5.
  * mixed BF16 with the correction: per voxel <= 1e-4.
  * FP64: per voxel <= 1.2e-7 (outputs are written as float32).
  * integer selection: bit-exact.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from _gpu_util import canonical_bits, rel_err_est, rel_err_var, run_gpu

pytestmark = pytest.mark.gpu

# per-voxel bars; FP32 paths also carry a normwise 1e-5 bar
TOL = {"fp32": 1e-4, "fp64": 1.2e-7, "mixed_fp16": 1e-5, "mixed_bf16": 1e-4}
NORMWISE_FP32 = 1e-5

# (name, nslices, ny, nx, f, r, model, nugget, sill, range, masked, seed)
CASES = [
    ("c1_full", 8, 64, 64, 2, 1, "spherical", 0.0, 1.0, 4.0, False, 1),
    ("edge_r2_f4", 5, 53, 47, 4, 2, "exponential", 0.01, 1.0, 6.0, True, 2),
    ("edge_r3_f4", 4, 45, 38, 4, 3, "spherical", 0.005, 1.0, 8.0, True, 5),
    ("edge_r3_f3_gauss", 3, 33, 40, 3, 3, "gaussian", 0.05, 1.0, 5.0, True, 7),
    ("edge_r2_f5", 3, 29, 70, 5, 2, "exponential", 0.02, 2.0, 4.0, True, 8),
    ("r0_f2", 4, 17, 19, 2, 0, "spherical", 0.0, 1.0, 4.0, False, 9),
    ("tiny_image", 3, 2, 3, 4, 3, "exponential", 0.01, 1.0, 6.0, True, 10),
    # largest systems: full 7x7x2 windows with the most targets (f = 15, sixteen
    # border rows: the last block holds no data column; unmasked, so interior
    # systems keep all 98 candidates and need NB = 8)
    ("r3_f15_max", 3, 20, 22, 15, 3, "spherical", 0.01, 1.0, 8.0, False, 12),
]


def _inputs(name, n, ny, nx, f, r, masked, seed):
    w = W.Workload(name, n, max(ny, nx), f, r, masked, 6, 2, 0.02,
                   W.Variogram("spherical", 0, 1, 4), seed)
    s = W.phantom(w)[:, :ny, :nx].copy()
    e = W.sobel_edges(s) if masked else None
    if masked:
        # add random edge pixels so every rule branch and the floor are exercised
        rng = np.random.default_rng(seed + 100)
        e = np.maximum(e, (rng.random(e.shape) < 0.15).astype(np.uint8))
    return s, e


@pytest.fixture(scope="module")
def oracle_cache():
    return {}


def _oracle(cache, case):
    name, n, ny, nx, f, r, model, nug, sill, rng_, masked, seed = case
    if name not in cache:
        s, e = _inputs(name, n, ny, nx, f, r, masked, seed)
        vol, var, npts = O.krige_volume(s, e, f, r, (model, nug, sill, rng_),
                                        min_points=min(4, 2 * (2 * r + 1) ** 2))
        cache[name] = (s, e, vol, var, npts)
    return cache[name]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", ["fp32", "fp64", "mixed_fp16", "mixed_bf16"])
def test_batched_vs_oracle(case, precision, oracle_cache):
    name, n, ny, nx, f, r, model, nug, sill, rng_, masked, seed = case
    s, e, vol_o, var_o, npts = _oracle(oracle_cache, case)
    print(f"case {name} precision {precision}", flush=True)
    vol, var, fl, st = run_gpu(s, e, f, r, (model, nug, sill, rng_), precision=precision,
                               min_points=min(4, 2 * (2 * r + 1) ** 2))
    # known slices bit-exact, variance 0 there
    np.testing.assert_array_equal(vol[::f], s)
    assert (var[::f] == 0).all()
    kz = np.ones(vol.shape[0], bool)
    kz[::f] = False
    zmax = np.abs(s).max()
    ee = rel_err_est(vol[kz], vol_o[kz], zmax)
    ev = rel_err_var(var[kz], var_o[kz], sill)
    nw = np.abs(vol[kz].astype(np.float64) - vol_o[kz]).max() / np.abs(vol_o[kz]).max()
    print(f"  max est err {ee.max():.3e} var err {ev.max():.3e} normwise {nw:.3e}", flush=True)
    assert ee.max() <= TOL[precision]
    assert ev.max() <= max(TOL[precision], 1e-5)
    if precision == "fp32":
        assert nw <= NORMWISE_FP32
    # bucket histogram equals the oracle's neighbour counts
    hist = np.bincount(npts.ravel(), minlength=128)
    assert st["bucket"] == hist.tolist()


@pytest.mark.parametrize("refine_max", [1, 0])
@pytest.mark.parametrize("case", CASES[:4], ids=[c[0] for c in CASES[:4]])
def test_plain_vs_oracle(case, refine_max, oracle_cache):
    """The per-voxel comparison kernel: with its FP64-residual refinement step
    per voxel <= 1e-5, without it the FP32 bar."""
    name, n, ny, nx, f, r, model, nug, sill, rng_, masked, seed = case
    s, e, vol_o, var_o, _ = _oracle(oracle_cache, case)
    vol, var, _, _ = run_gpu(s, e, f, r, (model, nug, sill, rng_), algo="plain",
                             min_points=min(4, 2 * (2 * r + 1) ** 2), refine_max=refine_max)
    np.testing.assert_array_equal(vol[::f], s)
    kz = np.ones(vol.shape[0], bool)
    kz[::f] = False
    zmax = np.abs(s).max()
    ee = rel_err_est(vol[kz], vol_o[kz], zmax)
    ev = rel_err_var(var[kz], var_o[kz], sill)
    nw = np.abs(vol[kz].astype(np.float64) - vol_o[kz]).max() / np.abs(vol_o[kz]).max()
    print(f"case {name} plain refine_max={refine_max}: max est err {ee.max():.3e} "
          f"var err {ev.max():.3e} normwise {nw:.3e}", flush=True)
    assert ee.max() <= (1e-5 if refine_max else TOL["fp32"])
    assert ev.max() <= 1e-5
    assert nw <= NORMWISE_FP32


@pytest.mark.parametrize("r", [0, 1, 2, 3])
@pytest.mark.parametrize("density", [0.05, 0.3, 0.9])
def test_select_bit_exact(r, density):
    import torch
    import paper_2303_09523_amd as P
    rng = np.random.default_rng(1000 + 10 * r + int(density * 10))
    n, ny, nx = 4, 37, 41
    e = (rng.random((n, ny, nx)) < density).astype(np.uint8)
    mp = min(4, 2 * (2 * r + 1) ** 2)
    plan = P.Plan(nx, ny, n, 2, r, mp)
    bits, count = plan.select(torch.from_numpy(e).cuda())
    bits = bits.cpu().numpy().view(np.uint64)
    count = count.cpu().numpy()
    plan.close()
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    for g in range(n - 1):
        S = ny * nx
        gs = np.full(S, g)
        kept, _ = O.select_neighbours((e[gs], e[gs + 1]), yy.ravel(), xx.ravel(), r, mp, (ny, nx))
        lo, hi = canonical_bits(kept)
        sl = slice(g * S, (g + 1) * S)
        np.testing.assert_array_equal(bits[sl, 0], lo)
        np.testing.assert_array_equal(bits[sl, 1], hi)
        np.testing.assert_array_equal(count[sl] & 0x7f, kept.sum(axis=1))


def test_degenerate_shapes():
    vario = ("exponential", 0.01, 1.0, 6.0)
    rng = np.random.default_rng(3)
    # f = 1: nothing to krige, the volume is the slices
    s = rng.normal(size=(3, 5, 6)).astype(np.float32)
    vol, var, _, _ = run_gpu(s, None, 1, 2, vario)
    np.testing.assert_array_equal(vol, s)
    # a single slice
    s1 = s[:1].copy()
    vol, var, _, _ = run_gpu(s1, None, 4, 2, vario)
    np.testing.assert_array_equal(vol, s1)
    # 1-pixel-wide image with a window wider than the image
    s2 = rng.normal(size=(2, 9, 1)).astype(np.float32)
    vol, var, _, _ = run_gpu(s2, None, 3, 3, vario)
    vo, va, _ = O.krige_volume(s2, None, 3, 3, vario)
    assert np.abs(vol - vo).max() <= 1e-5 * max(1.0, np.abs(vo).max())


def test_nonfinite_input_reported():
    import torch
    import paper_2303_09523_amd as P
    s = np.zeros((2, 8, 8), np.float32)
    s[1, 3, 3] = np.nan
    plan = P.Plan(8, 8, 2, 2, 1)
    plan.execute(torch.from_numpy(s).cuda(), ("spherical", 0.0, 1.0, 4.0))
    with pytest.raises(P.OkrError) as ei:
        plan.stats()
    assert ei.value.status == 3
    plan.close()


def test_bitwise_repeatable():
    case = CASES[1]
    name, n, ny, nx, f, r, model, nug, sill, rng_, masked, seed = case
    s, e = _inputs(name, n, ny, nx, f, r, masked, seed)
    a = run_gpu(s, e, f, r, (model, nug, sill, rng_))
    b = run_gpu(s, e, f, r, (model, nug, sill, rng_))
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_forced_fp64_fallback(monkeypatch):
    monkeypatch.setenv("OKR_FORCE_FALLBACK", "1")
    case = CASES[2]
    name, n, ny, nx, f, r, model, nug, sill, rng_, masked, seed = case
    s, e = _inputs(name, n, ny, nx, f, r, masked, seed)
    vol, var, fl, st = run_gpu(s, e, f, r, (model, nug, sill, rng_), flags=True)
    monkeypatch.delenv("OKR_FORCE_FALLBACK")
    v64, s64, _, _ = run_gpu(s, e, f, r, (model, nug, sill, rng_), precision="fp64")
    assert st["n_fp64_fallback"] == (n - 1) * ny * nx
    assert (fl & 4).all()
    np.testing.assert_array_equal(vol, v64)
    np.testing.assert_array_equal(var, s64)


READOUT_CASES = CASES[:4] + [CASES[7]]


@pytest.mark.parametrize("case", READOUT_CASES, ids=[c[0] for c in READOUT_CASES])
def test_mixed_factor_readout_only(case, oracle_cache):
    """refine_max = 0: the split-FP16 factorisation's own Schur read-out meets
    the FP32 bars; no system is marked refined."""
    name, n, ny, nx, f, r, model, nug, sill, rng_, masked, seed = case
    s, e, vol_o, var_o, _ = _oracle(oracle_cache, case)
    mp = min(4, 2 * (2 * r + 1) ** 2)
    vol, var, fl, st = run_gpu(s, e, f, r, (model, nug, sill, rng_), precision="mixed_fp16",
                               min_points=mp, flags=True, refine_max=0)
    kz = np.ones(vol.shape[0], bool)
    kz[::f] = False
    zmax = np.abs(s).max()
    ee = rel_err_est(vol[kz], vol_o[kz], zmax)
    nw = np.abs(vol[kz].astype(np.float64) - vol_o[kz]).max() / np.abs(vol_o[kz]).max()
    print(f"case {name} mixed read-out: max est err {ee.max():.3e} normwise {nw:.3e}", flush=True)
    assert ee.max() <= TOL["fp32"]
    assert nw <= NORMWISE_FP32
    assert st["n_refined"] == 0
    assert not (fl & 2).any()


def test_strict_mode_reports_failed_systems():
    """A near-singular Gaussian model: strict mode turns an FP64 re-solve that
    still meets a non-positive pivot into OKR_E_NOT_CONVERGED at the sync; the
    same run without strict only counts it."""
    import torch
    import paper_2303_09523_amd as P
    rng = np.random.default_rng(11)
    s = rng.normal(size=(3, 20, 21)).astype(np.float32)
    vario = ("gaussian", 0.0, 1.0, 40.0)
    st = torch.from_numpy(s).cuda()
    plan = P.Plan(21, 20, 3, 2, 3, precision="fp32", refine_tol=1e-7)
    plan.execute(st, vario)
    stats = plan.stats()
    plan.close()
    failed = stats["n_not_converged"]
    print(f"fp64 re-solves {stats['n_fp64_fallback']}, failed {failed}", flush=True)
    assert stats["n_fp64_fallback"] > 0
    plan = P.Plan(21, 20, 3, 2, 3, precision="fp32", refine_tol=1e-7, strict=True)
    plan.execute(st, vario)
    if failed:
        with pytest.raises(P.OkrError) as ei:
            plan.stats()
        assert ei.value.status == 7
    else:
        plan.stats()
    plan.close()


# f = 14 puts the cache's inverse range at n >= 66 (drop counts up to 32, the
# largest the k x k solves take); the masks leave systems across that range
PATTERN_CASES = CASES + [
    ("r3_f14_k32", 3, 30, 33, 14, 3, "exponential", 0.01, 1.0, 6.0, True, 14)]


@pytest.mark.parametrize("case", PATTERN_CASES, ids=[c[0] for c in PATTERN_CASES])
@pytest.mark.parametrize("precision", ["fp32", "mixed_fp16"])
def test_pattern_cache_vs_oracle(case, precision, oracle_cache):
    """PATTERN_CACHE: full-window systems from the cached FP64 weights, the rest
    batched; the same bars as the batched path."""
    name, n, ny, nx, f, r, model, nug, sill, rng_, masked, seed = case
    s, e, vol_o, var_o, npts = _oracle(oracle_cache, case)
    vol, var, fl, st = run_gpu(s, e, f, r, (model, nug, sill, rng_), precision=precision,
                               algo="pattern", min_points=min(4, 2 * (2 * r + 1) ** 2))
    np.testing.assert_array_equal(vol[::f], s)
    kz = np.ones(vol.shape[0], bool)
    kz[::f] = False
    zmax = np.abs(s).max()
    ee = rel_err_est(vol[kz], vol_o[kz], zmax)
    ev = rel_err_var(var[kz], var_o[kz], sill)
    nw = np.abs(vol[kz].astype(np.float64) - vol_o[kz]).max() / np.abs(vol_o[kz]).max()
    print(f"case {name} pattern {precision}: est {ee.max():.3e} var {ev.max():.3e} "
          f"normwise {nw:.3e} full-window systems {st['bucket'][2 * (2 * r + 1) ** 2]}",
          flush=True)
    assert ee.max() <= TOL[precision]
    assert ev.max() <= max(TOL[precision], 1e-5)
    if precision == "fp32":
        assert nw <= NORMWISE_FP32
    assert st["bucket"] == np.bincount(npts.ravel(), minlength=128).tolist()
    if name == "r3_f14_k32":
        assert sum(st["bucket"][66:76]) > 0   # drop counts 23..32 present


def _downdate_floor(ncand, nb, max_drop=32):
    """Smallest neighbour count the weight cache serves from the full
    window's inverse: the lowest 16-wide size class (16 (NB - 1) - nb < n <=
    16 NB - nb) that drops at most max_drop candidates; ncand when none."""
    for NB in range(1, 9):
        lo = max(1, 16 * (NB - 1) - nb + 1)
        if ncand - max_drop <= lo <= ncand - 1:
            return lo
    return ncand


@pytest.mark.parametrize("drift", [None, "linear_z"], ids=["ok", "drift"])
@pytest.mark.parametrize("case", [CASES[0], CASES[2]], ids=[CASES[0][0], CASES[2][0]])
def test_pattern_cache_splits_exactly(case, drift):
    """Systems below the cache's range are bit-identical to the batched
    launch; full-window systems, and those that drop at most 32 candidates
    (weights from the full window's inverse), match the FP64 batched solve to
    float32 rounding; with and without the slice predictor."""
    import torch
    import paper_2303_09523_amd as P
    name, n, ny, nx, f, r, model, nug, sill, rng_, masked, seed = case
    s, _ = _inputs(name, n, ny, nx, f, r, masked, seed)
    e = W.sobel_edges(s) if masked else None      # phantom edges only: full windows exist
    vario = (model, nug, sill, rng_)
    mp = min(4, 2 * (2 * r + 1) ** 2)
    kw = {"drift": drift} if drift else {}
    vb, wb, _, _ = run_gpu(s, e, f, r, vario, precision="mixed_fp16", min_points=mp,
                           refine_max=0, **kw)
    vp, wp, fp, sp = run_gpu(s, e, f, r, vario, precision="mixed_fp16", min_points=mp,
                             algo="pattern", refine_max=0, flags=True, **kw)
    v64, w64, _, _ = run_gpu(s, e, f, r, vario, precision="fp64", min_points=mp, **kw)
    plan = P.Plan(nx, ny, n, f, r, mp)
    _, count = plan.select(torch.from_numpy(e).cuda() if e is not None else None)
    plan.close()
    ncand = 2 * (2 * r + 1) ** 2
    cnt = (count.cpu().numpy() & 0x7f).reshape(n - 1, ny, nx)
    full = cnt >= _downdate_floor(ncand, f + 1 + (1 if drift else 0))
    print(f"full-window systems {(cnt == ncand).sum()}, from the inverse "
          f"{full.sum() - (cnt == ncand).sum()}, batched {(~full).sum()} of {full.size}",
          flush=True)
    assert (cnt == ncand).sum() > 0 and (full & (cnt < ncand)).sum() > 0
    zmax = np.abs(s).max()
    for g in range(n - 1):
        for t in range(1, f):
            z = g * f + t
            m = full[g]
            np.testing.assert_array_equal(vp[z][~m], vb[z][~m])
            np.testing.assert_array_equal(wp[z][~m], wb[z][~m])
            assert rel_err_est(vp[z][m], v64[z][m].astype(np.float64), zmax).max() <= 1.2e-7
            assert np.abs(wp[z][m] - w64[z][m]).max() <= 1.2e-7 * sill


DRIFT_CASES = [CASES[1], CASES[2], CASES[4], CASES[5],
               # the most targets the slice predictor allows (f = 14: sixteen border rows)
               ("r3_f14_drift", 3, 18, 21, 14, 3, "exponential", 0.01, 1.0, 6.0, False, 13)]


@pytest.mark.parametrize("case", DRIFT_CASES, ids=[c[0] for c in DRIFT_CASES])
@pytest.mark.parametrize("precision", ["fp32", "fp64", "mixed_fp16"])
def test_drift_vs_oracle(case, precision, oracle_cache):
    """Universal kriging with the slice predictor (drift = linear_z) against
    the oracle's Appendix A solve with the same predictors."""
    name, n, ny, nx, f, r, model, nug, sill, rng_, masked, seed = case
    key = name + "/drift"
    if key not in oracle_cache:
        s, e = _inputs(name, n, ny, nx, f, r, masked, seed)
        vol, var, _ = O.krige_volume(s, e, f, r, (model, nug, sill, rng_),
                                     min_points=min(4, 2 * (2 * r + 1) ** 2), drift="linear_z")
        oracle_cache[key] = (s, e, vol, var)
    s, e, vol_o, var_o = oracle_cache[key]
    vol, var, _, _ = run_gpu(s, e, f, r, (model, nug, sill, rng_), precision=precision,
                             min_points=min(4, 2 * (2 * r + 1) ** 2), drift="linear_z",
                             refine_max=0)
    np.testing.assert_array_equal(vol[::f], s)
    kz = np.ones(vol.shape[0], bool)
    kz[::f] = False
    zmax = np.abs(s).max()
    ee = rel_err_est(vol[kz], vol_o[kz], zmax)
    ev = rel_err_var(var[kz], var_o[kz], sill)
    nw = np.abs(vol[kz].astype(np.float64) - vol_o[kz]).max() / np.abs(vol_o[kz]).max()
    print(f"case {name} drift {precision}: est {ee.max():.3e} var {ev.max():.3e} normwise {nw:.3e}",
          flush=True)
    bar = TOL["fp64"] if precision == "fp64" else TOL["fp32"]
    assert ee.max() <= bar
    assert ev.max() <= max(bar, 1e-5)
    if precision != "fp64":
        assert nw <= NORMWISE_FP32


@pytest.mark.parametrize("case", DRIFT_CASES, ids=[c[0] for c in DRIFT_CASES])
def test_drift_fp64_correction_vs_oracle(case, oracle_cache):
    """The mixed FP16 factorisation with the FP64 correction in the
    slice-predictor form (two multipliers) reaches the corrected path's bar."""
    name, n, ny, nx, f, r, model, nug, sill, rng_, masked, seed = case
    key = name + "/drift"
    if key not in oracle_cache:
        s, e = _inputs(name, n, ny, nx, f, r, masked, seed)
        vol, var, _ = O.krige_volume(s, e, f, r, (model, nug, sill, rng_),
                                     min_points=min(4, 2 * (2 * r + 1) ** 2), drift="linear_z")
        oracle_cache[key] = (s, e, vol, var)
    s, e, vol_o, var_o = oracle_cache[key]
    vol, var, fl, st = run_gpu(s, e, f, r, (model, nug, sill, rng_), precision="mixed_fp16",
                               min_points=min(4, 2 * (2 * r + 1) ** 2), drift="linear_z",
                               refine_max=1, refine_tol=0.0, flags=True)
    np.testing.assert_array_equal(vol[::f], s)
    kz = np.ones(vol.shape[0], bool)
    kz[::f] = False
    ee = rel_err_est(vol[kz], vol_o[kz], np.abs(s).max())
    ev = rel_err_var(var[kz], var_o[kz], sill)
    print(f"case {name} drift corrected: est {ee.max():.3e} var {ev.max():.3e} "
          f"refined {st['n_refined']}", flush=True)
    assert st["n_refined"] + st["n_fp64_fallback"] == (n - 1) * ny * nx
    assert ee.max() <= TOL["mixed_fp16"]
    assert ev.max() <= 1e-5


# unmasked cases: full windows exist (with the random edges of the masked ones
# they may not)
@pytest.mark.parametrize("case", [CASES[0], CASES[5], DRIFT_CASES[-1]],
                         ids=[CASES[0][0], CASES[5][0], DRIFT_CASES[-1][0]])
@pytest.mark.parametrize("precision", ["fp32", "mixed_fp16"])
def test_pattern_cache_drift_vs_oracle(case, precision, oracle_cache):
    """The full-window weights of the slice-predictor form, cached in FP64,
    and the batched path for the other systems, against the oracle."""
    name, n, ny, nx, f, r, model, nug, sill, rng_, masked, seed = case
    key = name + "/drift"
    if key not in oracle_cache:
        s, e = _inputs(name, n, ny, nx, f, r, masked, seed)
        vol, var, _ = O.krige_volume(s, e, f, r, (model, nug, sill, rng_),
                                     min_points=min(4, 2 * (2 * r + 1) ** 2), drift="linear_z")
        oracle_cache[key] = (s, e, vol, var)
    s, e, vol_o, var_o = oracle_cache[key]
    vol, var, _, st = run_gpu(s, e, f, r, (model, nug, sill, rng_), precision=precision,
                              algo="pattern", min_points=min(4, 2 * (2 * r + 1) ** 2),
                              drift="linear_z", refine_max=0)
    np.testing.assert_array_equal(vol[::f], s)
    kz = np.ones(vol.shape[0], bool)
    kz[::f] = False
    ee = rel_err_est(vol[kz], vol_o[kz], np.abs(s).max())
    ev = rel_err_var(var[kz], var_o[kz], sill)
    print(f"case {name} pattern drift {precision}: est {ee.max():.3e} var {ev.max():.3e}",
          flush=True)
    assert st["bucket"][2 * (2 * r + 1) ** 2] > 0
    assert ee.max() <= TOL["fp32"]
    assert ev.max() <= 1e-5


def test_drift_reproduces_linear_trend_gpu():
    """A field linear across the gap is reproduced at every target."""
    n, ny, nx, f, r = 4, 21, 23, 4, 2
    planes = np.array([0.3 + 0.7 * k for k in range(n)], dtype=np.float32)
    s = np.broadcast_to(planes[:, None, None], (n, ny, nx)).copy()
    rng = np.random.default_rng(5)
    e = (rng.random((n, ny, nx)) < 0.2).astype(np.uint8)
    for precision, tol in (("fp64", 2e-7), ("fp32", 2e-5), ("mixed_fp16", 2e-5)):
        vol, _, _, _ = run_gpu(s, e, f, r, ("exponential", 0.01, 1.0, 6.0), precision=precision,
                               drift="linear_z", refine_max=0)
        for g in range(n - 1):
            for t in range(1, f):
                exact = float(planes[g]) + (float(planes[g + 1]) - float(planes[g])) * t / f
                assert np.abs(vol[g * f + t] - exact).max() <= tol * max(1.0, abs(exact)), \
                    (precision, g, t)

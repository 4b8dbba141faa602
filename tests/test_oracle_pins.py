"""Pins for the FP64 oracle: each test fixes part of the oracle against
something other than the oracle itself (closed forms, invariants, brute force,
a 50-digit second arithmetic, hand-derived fixtures, finite differences)."""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


# --- covariance model --------------------------------------------------------

def test_practical_range_definition():
    # practical range: exponential / gaussian reach 95% of the partial sill
    # (rho = exp(-3)) at h = a; spherical reaches it exactly and stays there.
    for model in ("exponential", "gaussian"):
        assert O.correlation(model, 7.0, 7.0) == pytest.approx(np.exp(-3.0), rel=1e-15)
    assert O.correlation("spherical", 7.0, 7.0) == 0.0
    assert O.correlation("spherical", 9.0, 7.0) == 0.0
    # continuity of the spherical model at the range, smoothness at 0
    assert O.correlation("spherical", 7.0 - 1e-9, 7.0) == pytest.approx(0.0, abs=1e-15)
    assert O.correlation("spherical", 0.0, 7.0) == 1.0
    # Cov(0) = sill, gamma jumps by the nugget at the origin
    assert O.covariance("exponential", 0.1, 2.0, 5.0, 0.0) == 2.0
    assert O.semivariogram("exponential", 0.1, 2.0, 5.0, 1e-12) == pytest.approx(0.1, abs=1e-11)


def test_covariance_derivatives_vs_complex_step():
    # complex-step derivative of the analytic exponential / gaussian models
    h = np.array([0.5, 1.0, 2.3, 4.0])
    for model in ("exponential", "gaussian"):
        nug, sill, a = 0.03, 1.3, 4.5
        d = O.covariance_derivatives(model, nug, sill, a, h)
        eps = 1e-30
        def cov(nug_, sill_, a_):
            if model == "exponential":
                rho = np.exp(-3.0 * h / a_)
            else:
                rho = np.exp(-3.0 * (h / a_) ** 2)
            return (sill_ - nug_) * rho
        cs = [cov(nug + 1j * eps, sill, a).imag / eps,
              cov(nug, sill + 1j * eps, a).imag / eps,
              cov(nug, sill, a + 1j * eps).imag / eps]
        np.testing.assert_allclose(d, np.stack(cs), rtol=1e-14, atol=1e-300)
    # spherical by central differences
    d = O.covariance_derivatives("spherical", 0.03, 1.3, 4.5, h)
    for k in range(3):
        th = np.array([0.03, 1.3, 4.5])
        tp, tm = th.copy(), th.copy()
        tp[k] += 1e-6
        tm[k] -= 1e-6
        fd = (O.covariance("spherical", *tp, h) - O.covariance("spherical", *tm, h)) / 2e-6
        np.testing.assert_allclose(d[k], fd, rtol=1e-7, atol=1e-9)


# --- P1, P2, P3: closed forms ------------------------------------------------

@pytest.mark.parametrize("model", ["spherical", "exponential", "gaussian"])
def test_P1_single_point(model):
    nug, sill, a = 0.05, 1.5, 5.0
    est, var, w, mu = O.krige_points([[0, 0, 0]], [3.25], [[1.0, 2.0, 2.0]], model, nug, sill, a)
    assert w[0, 0] == pytest.approx(1.0, abs=1e-15)
    assert est[0] == pytest.approx(3.25, abs=1e-14)
    g = O.semivariogram(model, nug, sill, a, 3.0)
    assert var[0] == pytest.approx(2.0 * g, rel=1e-13)


def test_P2_two_points_spherical_exact():
    gold = _gold("closed_forms.json")["two_points_spherical"]
    est, var, w, mu = O.krige_points([[0, 0, 0], [0, 0, 2]], [1.0, 3.0], [[0, 0, 1]],
                                     gold["model"], gold["nugget"], gold["sill"], gold["range"])
    np.testing.assert_allclose(w[:, 0], [0.5, 0.5], atol=1e-15)
    assert var[0] == pytest.approx(gold["variance"], abs=1e-15)
    assert est[0] == pytest.approx(2.0, abs=1e-15)


def test_P2_volume_geometry_r0():
    # r = 0 reduces the window to the two vertically adjacent known voxels at
    # distance t and f - t: with f = 2 this is the two-point case above for
    # every kriged voxel, which pins the z spacing of the volume path.
    gold = _gold("closed_forms.json")["two_points_spherical"]
    rng = np.random.default_rng(0)
    s = rng.normal(size=(3, 5, 4)).astype(np.float32)
    vol, var, n = O.krige_volume(s, None, 2, 0, ("spherical", 0.0, 1.0, 4.0))
    np.testing.assert_allclose(var[1::2], gold["variance"], atol=1e-14)
    np.testing.assert_allclose(vol[1::2], 0.5 * (s[:-1].astype(np.float64) + s[1:]), atol=1e-14)
    assert (n == 2).all()


@pytest.mark.parametrize("model", ["exponential", "gaussian"])
def test_P2_two_points_other_models(model):
    nug, sill, a = 0.02, 0.9, 6.0
    h, d = np.sqrt(1 + 1.5 ** 2), 3.0
    est, var, w, mu = O.krige_points([[0, 1, 0], [0, 1, 3]], [0.0, 1.0], [[0, 0, 1.5]], model,
                                     nug, sill, a)
    gh = O.semivariogram(model, nug, sill, a, h)
    gd = O.semivariogram(model, nug, sill, a, d)
    assert var[0] == pytest.approx(2 * gh - 0.5 * gd, rel=1e-13)
    np.testing.assert_allclose(w[:, 0], [0.5, 0.5], atol=1e-14)


def test_P3_pure_nugget():
    gold = _gold("closed_forms.json")["pure_nugget"]
    rng = np.random.default_rng(1)
    s = rng.normal(size=(2, 7, 7)).astype(np.float32)
    vol, var, n = O.krige_volume(s, None, 2, 1, ("spherical", 0.0, 1.0, 0.9))
    assert n[0, 3, 3] == gold["n"]
    assert var[1, 3, 3] == pytest.approx(gold["variance"], rel=1e-14)
    expect = s[:, 2:5, 2:5].astype(np.float64).mean()
    assert vol[1, 3, 3] == pytest.approx(expect, abs=1e-14)


# --- P4-P8: invariants and brute force ---------------------------------------

def _random_system(rng, n, model="exponential"):
    pts = rng.integers(-3, 4, size=(n * 3, 3)).astype(np.float64)
    pts = np.unique(pts, axis=0)[:n]
    vals = rng.normal(size=len(pts))
    tgt = np.array([[0.25, -0.5, 0.75], [1.5, 0.5, 0.5]])
    return pts, vals, tgt


@pytest.mark.parametrize("model", ["spherical", "exponential", "gaussian"])
def test_P4_P5_P7_invariants(model):
    rng = np.random.default_rng(2)
    nug = 0.0 if model != "gaussian" else 0.05
    pts, vals, tgt = _random_system(rng, 14, model)
    est, var, w, mu = O.krige_points(pts, vals, tgt, model, nug, 1.0, 4.0)
    np.testing.assert_allclose(w.sum(axis=0), 1.0, atol=1e-12)               # P4
    est_c, _, _, _ = O.krige_points(pts, np.full(len(pts), 7.5), tgt, model, nug, 1.0, 4.0)
    np.testing.assert_allclose(est_c, 7.5, rtol=1e-12)                       # P5
    assert (var >= -1e-12).all()                                             # P7


@pytest.mark.parametrize("nug", [0.0, 0.1])
def test_P6_exact_reproduction(nug):
    rng = np.random.default_rng(3)
    pts, vals, _ = _random_system(rng, 10)
    est, var, w, mu = O.krige_points(pts, vals, pts[4:5], "exponential", nug, 1.0, 3.0)
    assert est[0] == pytest.approx(vals[4], abs=1e-12)
    assert var[0] == pytest.approx(0.0, abs=1e-12)
    assert w[4, 0] == pytest.approx(1.0, abs=1e-12)


def test_P8_brute_force_optimality():
    rng = np.random.default_rng(4)
    pts, vals, tgt = _random_system(rng, 9)
    model, nug, sill, a = "spherical", 0.02, 1.0, 5.0
    est, var, w, mu = O.krige_points(pts, vals, tgt[:1], model, nug, sill, a)
    d = np.linalg.norm(pts[:, None] - pts[None], axis=2)
    d0 = np.linalg.norm(pts - tgt[0], axis=1)
    C = O.covariance(model, nug, sill, a, d)
    c0 = O.covariance(model, nug, sill, a, d0)
    def Q(v):
        return v @ C @ v - 2 * v @ c0 + sill
    ws = w[:, 0]
    assert Q(ws) == pytest.approx(var[0], abs=1e-13)
    for i in range(len(ws)):
        for j in range(len(ws)):
            if i != j:
                for eps in (1e-3, -1e-3):
                    v = ws.copy()
                    v[i] += eps
                    v[j] -= eps
                    assert Q(v) >= Q(ws) - 1e-15


# --- P9: second arithmetic ---------------------------------------------------

def test_P9_mpmath_volume():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 50
    rng = np.random.default_rng(5)
    s = rng.normal(size=(3, 6, 6)).astype(np.float32)
    e = (rng.random((3, 6, 6)) < 0.25).astype(np.uint8)
    f, r = 3, 1
    nug, sill, a = mp.mpf("0.01"), mp.mpf(1), mp.mpf(6)
    vol, var, n = O.krige_volume(s, e, f, r, ("exponential", 0.01, 1.0, 6.0))
    cands = O.candidates(r)
    for g in range(2):
        gs = np.full(36, g)
        yy, xx = np.meshgrid(np.arange(6), np.arange(6), indexing="ij")
        kept, _ = O.select_neighbours((e[gs], e[gs + 1]), yy.ravel(), xx.ravel(), r, 4, (6, 6))
        for i in range(36):
            y, x = divmod(i, 6)
            pts = [(x + cands[c][0], y + cands[c][1], (g + cands[c][2]) * f)
                   for c in np.nonzero(kept[i])[0]]
            vals = [mp.mpf(float(s[g + cands[c][2], y + cands[c][1], x + cands[c][0]]))
                    for c in np.nonzero(kept[i])[0]]
            nn = len(pts)
            def cov(p, q):
                h = mp.sqrt(sum((mp.mpf(p[k]) - mp.mpf(q[k])) ** 2 for k in range(3)))
                return sill if h == 0 else (sill - nug) * mp.e ** (-3 * h / a)
            K = mp.matrix(nn + 1, nn + 1)
            for p in range(nn):
                for q in range(nn):
                    K[p, q] = cov(pts[p], pts[q])
                K[p, nn] = 1
                K[nn, p] = 1
            for t in range(1, f):
                tgt = (x, y, g * f + t)
                rhs = mp.matrix([cov(p, tgt) for p in pts] + [1])
                sol = mp.lu_solve(K, rhs)
                est = sum(sol[p] * vals[p] for p in range(nn))
                vv = sill - sum(sol[p] * rhs[p] for p in range(nn)) - sol[nn]
                assert abs(float(est) - vol[g * f + t, y, x]) <= 1e-13 * max(1.0, abs(float(est)))
                assert abs(float(vv) - var[g * f + t, y, x]) <= 1e-13


# --- P10: translation invariance = a fixed stencil on an unmasked interior ----

def test_P10_interior_stencil():
    w = W.workload("plain_8x64")
    s, _ = W.make_inputs(w)
    vol, var, n = O.krige_volume(s[:3], None, 2, 1, w.vario)
    # weights of one interior system from an explicit point solve
    pts = [(dx, dy, 2 * sl) for sl in (0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    _, v0, wts, _ = O.krige_points(pts, np.zeros(18), [[0, 0, 1]], *O.kriging._vtuple(w.vario))
    st = wts[:, 0].reshape(2, 3, 3)                       # [slice][dy][dx]
    sd = s.astype(np.float64)
    for g in range(2):
        acc = np.zeros((62, 62))
        for sl in (0, 1):
            for dy in range(3):
                for dx in range(3):
                    acc += st[sl, dy, dx] * sd[g + sl, dy:dy + 62, dx:dx + 62]
        np.testing.assert_allclose(vol[2 * g + 1, 1:63, 1:63], acc, atol=1e-13)
        np.testing.assert_allclose(var[2 * g + 1, 1:63, 1:63], v0[0], atol=1e-14)
    # the two slices get equal weights at mid-gap, and they are not uniform
    np.testing.assert_allclose(st[0], st[1], atol=1e-14)
    assert st[0, 1, 1] > st[0, 0, 1] > 0 > st[0, 0, 0]


# --- edge rule and floor (hand-derived fixtures) ------------------------------

def test_edge_paths_fixture():
    gold = _gold("edge_rule_cases.json")["paths"]
    for key, path in gold.items():
        dx, dy = map(int, key.split(","))
        assert O.edge_path(dx, dy) == [tuple(p) for p in path], key


def test_edge_path_d4_symmetry():
    for dx in range(-3, 4):
        for dy in range(-3, 4):
            if (dx, dy) == (0, 0):
                continue
            p = O.edge_path(dx, dy)
            assert O.edge_path(dy, dx) == [(b, a) for a, b in p]
            assert O.edge_path(-dx, dy) == [(-a, b) for a, b in p]
            assert O.edge_path(dx, -dy) == [(a, -b) for a, b in p]
            assert p[-1] == (dx, dy) and len(p) == max(abs(dx), abs(dy))


def test_floor_all_edges():
    gold = _gold("edge_rule_cases.json")["floor_all_edges_r1"]
    e = np.ones((1, 5, 5), dtype=np.uint8)
    kept, _ = O.select_neighbours((e, e), [2], [2], 1, 4, (5, 5))
    assert list(np.nonzero(kept[0])[0]) == gold["kept_indices"]


def test_single_edge_pixel():
    gold = _gold("edge_rule_cases.json")["single_edge_r2"]
    lo = np.zeros((1, 9, 9), dtype=np.uint8)
    hi = np.zeros((1, 9, 9), dtype=np.uint8)
    lo[0, 4, 5] = 1                                      # (x+1, y) of column (4, 4)
    kept, inimg = O.select_neighbours((lo, hi), [4], [4], 2, 4, (9, 9))
    dropped = sorted(np.nonzero(~kept[0] & inimg[0])[0].tolist())
    assert dropped == gold["dropped_indices"]
    # the transposed pixel drops the transposed candidates: x and y are not mixed up
    lo2 = np.zeros((1, 9, 9), dtype=np.uint8)
    lo2[0, 5, 4] = 1                                     # (x, y+1)
    kept2, _ = O.select_neighbours((lo2, hi), [4], [4], 2, 4, (9, 9))
    # (dx=0,dy=1) -> (1+2)*5+2 = 17 and (0,2) -> 22
    assert sorted(np.nonzero(~kept2[0])[0].tolist()) == [17, 22]


def test_border_drop_counts():
    s = np.zeros((2, 6, 7), dtype=np.float32)
    vol, var, n = O.krige_volume(s, None, 2, 1, ("spherical", 0.0, 1.0, 4.0))
    assert n[0, 0, 0] == 8 and n[0, 0, 3] == 12 and n[0, 3, 3] == 18
    vol, var, n = O.krige_volume(s, None, 2, 3, ("spherical", 0.0, 1.0, 4.0))
    assert n[0, 0, 0] == 2 * 16 and n[0, 2, 3] == 2 * 6 * 7


# --- P11, P12: symmetry and equivariance --------------------------------------

def test_P11_symmetries():
    rng = np.random.default_rng(6)
    s = rng.normal(size=(3, 9, 9)).astype(np.float32)
    e = (rng.random((3, 9, 9)) < 0.15).astype(np.uint8)
    vario = ("exponential", 0.01, 1.0, 5.0)
    vol, var, n = O.krige_volume(s, e, 3, 2, vario)
    for tf in (lambda a: a[:, :, ::-1], lambda a: a[:, ::-1, :], lambda a: a.transpose(0, 2, 1),
               lambda a: a[::-1]):
        v2, r2, n2 = O.krige_volume(np.ascontiguousarray(tf(s)), np.ascontiguousarray(tf(e)), 3, 2,
                                    vario)
        a, b = tf(vol), v2
        # away from the floor (its fill order is not symmetric)
        keep = tf(np.concatenate([np.repeat(n >= 5, 3, axis=0), np.ones((1, 9, 9), bool)]))
        np.testing.assert_allclose(a[keep], b[keep], atol=1e-12)
        np.testing.assert_allclose(tf(var)[keep], r2[keep], atol=1e-12)


def test_P12_equivariance():
    rng = np.random.default_rng(7)
    s = rng.normal(size=(3, 8, 8)).astype(np.float32)
    e = (rng.random((3, 8, 8)) < 0.1).astype(np.uint8)
    vol, var, _ = O.krige_volume(s, e, 4, 2, ("spherical", 0.05, 1.0, 6.0))
    s2 = (2.0 * s.astype(np.float64) - 3.0)
    vol2, _, _ = O.krige_volume(s2, e, 4, 2, ("spherical", 0.05, 1.0, 6.0))
    np.testing.assert_allclose(vol2, 2.0 * vol.astype(np.float64) - 3.0, atol=1e-5)
    vol3, var3, _ = O.krige_volume(s, e, 4, 2, ("spherical", 0.15, 3.0, 6.0))
    np.testing.assert_allclose(vol3, vol, atol=1e-12)
    np.testing.assert_allclose(var3, 3.0 * var, atol=1e-12)


def test_P13_window_condition_bounds_systems():
    kw = O.window_condition("exponential", 0.01, 1.0, 6.0, 2, 4)
    cands = np.array(O.candidates(2), dtype=np.float64)
    P = np.stack([cands[:, 0], cands[:, 1], cands[:, 2] * 4], axis=1)
    rng = np.random.default_rng(8)
    for _ in range(20):
        sub = np.sort(rng.choice(50, size=rng.integers(4, 50), replace=False))
        d = np.linalg.norm(P[sub, None] - P[None, sub], axis=2)
        ev = np.linalg.eigvalsh(O.covariance("exponential", 0.01, 1.0, 6.0, d))
        assert ev[-1] / ev[0] <= kw * (1 + 1e-12)


# --- P14: gradients -------------------------------------------------------------

def test_P14_adjoint_vs_finite_differences():
    vario = W.Variogram("exponential", 0.02, 0.8, 5.0)
    f, _ = W.gaussian_field((6, 14, 13), vario, seed=11)
    s = f.astype(np.float32)
    th = ("exponential", 0.1, 1.0, 2.0)
    L, g = O.loso_loss_grad(s, 2, th)
    assert L == pytest.approx(O.loso_loss(s, 2, th), rel=1e-13)
    fd = O.loso_fd_grad(s, 2, th, h=1e-4)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-12 * np.abs(g).max())
    # OK weights depend only on nugget/sill and range: n dL/dn + s dL/ds = 0
    assert abs(0.1 * g[0] + 1.0 * g[1]) <= 1e-12 * np.abs(g).max()


def _loso_edges(shape, seed, frac=0.2):
    return (np.random.default_rng(seed).random(shape) < frac).astype(np.uint8)


def test_P14_drift_adjoint_with_edges_vs_finite_differences():
    vario = W.Variogram("exponential", 0.02, 0.8, 5.0)
    f, _ = W.gaussian_field((5, 12, 11), vario, seed=5)
    s = f.astype(np.float32)
    e = _loso_edges(s.shape, 6)
    th = ("exponential", 0.1, 1.0, 2.0)
    for drift in ("none", "linear_z"):
        L, g = O.loso_loss_grad(s, 2, th, edges=e, drift=drift)
        assert L == pytest.approx(O.loso_loss(s, 2, th, edges=e, drift=drift), rel=1e-13)
        fd = O.loso_fd_grad(s, 2, th, h=1e-4, edges=e, drift=drift)
        np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-12 * np.abs(g).max())
        # Q and q0 do not scale with C: the weights still depend on nugget/sill
        # and range only
        assert abs(0.1 * g[0] + 1.0 * g[1]) <= 1e-12 * np.abs(g).max()


def test_P14_drift_reproduces_a_trend_across_slices():
    # a field constant in-plane and linear across the slices: with edge masks
    # the two slices keep different point sets, so ordinary kriging's weights
    # on the upper slice no longer sum to 1/2 and it misses the trend, while
    # the slice predictor reproduces it exactly
    ns, ny, nx = 5, 10, 9
    s = np.broadcast_to((3.0 + 2.0 * np.arange(ns, dtype=np.float32))[:, None, None],
                        (ns, ny, nx)).astype(np.float32)
    e = _loso_edges(s.shape, 8, 0.3)
    th = ("spherical", 0.05, 1.0, 4.0)
    L_ok = O.loso_loss(s, 2, th, edges=e)
    L_dr, g_dr = O.loso_loss_grad(s, 2, th, edges=e, drift="linear_z")
    assert L_ok > 1e-3
    assert L_dr < 1e-20 and np.abs(g_dr).max() < 1e-9


def test_P14_drift_equals_ordinary_kriging_without_masks():
    # without masks both slices keep mirror-image point sets around a target
    # half-way between them, so ordinary kriging already puts weight 1/2 on
    # each slice and the slice constraint changes nothing
    rng = np.random.default_rng(9)
    s = rng.normal(size=(4, 9, 10)).astype(np.float32)
    th = ("gaussian", 0.1, 1.0, 3.0)
    L0, g0 = O.loso_loss_grad(s, 2, th)
    L1, g1 = O.loso_loss_grad(s, 2, th, drift="linear_z")
    assert L1 == pytest.approx(L0, rel=1e-10)
    np.testing.assert_allclose(g1, g0, rtol=1e-7, atol=1e-12 * np.abs(g0).max())


@pytest.mark.parametrize("model", ["spherical", "gaussian"])
def test_P14_adjoint_other_models(model):
    rng = np.random.default_rng(12)
    s = rng.normal(size=(4, 9, 8)).astype(np.float32)
    th = (model, 0.05, 1.2, 3.5)
    L, g = O.loso_loss_grad(s, 1, th)
    fd = O.loso_fd_grad(s, 1, th, h=1e-5)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-10 * np.abs(g).max())


def test_adam_first_step_is_signed_lr():
    # with bias correction the first Adam step is -lr * sign(g) per coordinate
    def lg(th):
        return float(np.sum((th - 1.0) ** 2)), 2.0 * (th - 1.0)
    traj = O.adam_fit(lg, [0.5, 2.0, 4.0], steps=1, lr=0.05)
    u0 = np.log([0.5, 2.0, 4.0])
    u1 = np.log(traj[-1][1])
    np.testing.assert_allclose(u1 - u0, [0.05, -0.05, -0.05], rtol=1e-6)


# ---- universal kriging with a linear drift across the gap (Appendix A, p = 2) ----

def test_drift_reproduces_linear_trend_exactly():
    """Predictors 1 and the slice position: a field linear across the gap is
    reproduced exactly at every target, masked or not (the two unbiasedness
    constraints sum(w) = 1 and sum(w s_i) = t/f do it); ordinary kriging does
    not reproduce it in general."""
    n, H, W_, f, r = 4, 11, 13, 4, 2
    planes = np.array([0.3 + 0.7 * k for k in range(n)], dtype=np.float32)
    s = np.broadcast_to(planes[:, None, None], (n, H, W_)).copy()
    rng = np.random.default_rng(5)
    e = (rng.random((n, H, W_)) < 0.2).astype(np.uint8)
    for edge in (None, e):
        v, var, _ = O.krige_volume(s, edge, f, r, ("exponential", 0.01, 1.0, 6.0),
                                   drift="linear_z")
        for g in range(n - 1):
            for t in range(1, f):
                exact = float(planes[g]) + (float(planes[g + 1]) - float(planes[g])) * t / f
                np.testing.assert_allclose(v[g * f + t], exact, rtol=0, atol=1e-12)
    vo, _, _ = O.krige_volume(s, e, f, r, ("exponential", 0.01, 1.0, 6.0))
    kz = np.ones(vo.shape[0], bool)
    kz[::f] = False
    zexact = np.array([[planes[g] + (planes[g + 1] - planes[g]) * t / f for t in range(1, f)]
                       for g in range(n - 1)]).ravel()
    assert np.abs(vo[kz].reshape(-1, H * W_).mean(axis=1) - zexact).max() > 1e-3


def test_drift_variance_not_below_ordinary():
    """An extra unbiasedness constraint can only raise the minimum of the
    estimation variance: sigma^2(drift) >= sigma^2(ordinary) >= 0."""
    rng = np.random.default_rng(6)
    s = rng.normal(size=(3, 9, 10)).astype(np.float32)
    e = (rng.random(s.shape) < 0.15).astype(np.uint8)
    for vario in (("spherical", 0.0, 1.0, 4.0), ("gaussian", 0.05, 2.0, 5.0)):
        _, v0, _ = O.krige_volume(s, e, 3, 2, vario)
        _, v1, _ = O.krige_volume(s, e, 3, 2, vario, drift="linear_z")
        kz = np.ones(v0.shape[0], bool)
        kz[::3] = False
        assert (v1[kz] >= v0[kz] - 1e-12).all()
        assert (v0[kz] >= -1e-12).all()


def test_drift_solve_brute_force_optimal():
    """The drift weights minimise Q(w) = w'Cw - 2 w'c0 + sill among weights
    that satisfy both constraints: moving weight between two points of the
    same slice keeps the constraints and never lowers Q."""
    rng = np.random.default_rng(7)
    pts = np.array([[x, y, s * 2.0] for s in (0, 1) for y in (-1, 0, 1) for x in (-1, 0, 1)], float)
    pts = pts[rng.permutation(len(pts))[:11]]
    tgt = np.array([[0.2, -0.1, 0.5]])
    d = np.linalg.norm(pts[:, None] - pts[None], axis=2)
    C = O.covariance("exponential", 0.0, 1.0, 5.0, d)
    c0 = O.covariance("exponential", 0.0, 1.0, 5.0, np.linalg.norm(pts - tgt, axis=1))[:, None]
    sl = pts[:, 2] / 2.0
    Q = np.stack([np.ones(len(pts)), sl], axis=1)
    q0 = np.array([[1.0], [0.25]])
    w, ph = O.drift_solve(C[None], c0[None], Q[None], q0[None])
    w = w[0, :, 0]
    assert abs(w.sum() - 1.0) < 1e-12 and abs(w @ sl - 0.25) < 1e-12
    Qf = lambda x: x @ C @ x - 2 * x @ c0[:, 0] + 1.0
    base = Qf(w)
    for i in range(len(w)):
        for j in range(len(w)):
            if i != j and sl[i] == sl[j]:
                e_ = np.zeros_like(w)
                e_[i], e_[j] = 1e-3, -1e-3
                assert Qf(w + e_) >= base - 1e-14
    # variance formula matches Q at the optimum
    var = 1.0 - w @ c0[:, 0] - ph[0, :, 0] @ q0[:, 0]
    assert abs(var - base) < 1e-12

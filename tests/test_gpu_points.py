"""GPU point entry point (okr_krige_points): FP64 ordinary kriging of explicit
point sets against the oracle, and the closed forms and invariants of the
method (pins P1-P8) evaluated on the GPU's own outputs. Outputs are float32,
so the bars are float32 rounding of FP64 results."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


def _run(systems, vario, want_weights=True):
    """systems: list of (pts [n][3], vals [n], target [3])."""
    import torch
    import paper_2303_09523_amd as P
    counts = np.array([len(v) for _, v, _ in systems], np.int32)
    offs = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
    xyz = np.concatenate([p for p, _, _ in systems]).astype(np.float32)
    val = np.concatenate([v for _, v, _ in systems]).astype(np.float32)
    tgt = np.array([t for _, _, t in systems], np.float32)
    plan = P.Plan(4, 4, 2, 2, 1)
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    est, var, w = plan.krige_points(cu(counts), cu(offs), cu(xyz), cu(val), cu(tgt), vario,
                                    want_weights=want_weights)
    st = plan.stats()
    out = (est.cpu().numpy(), var.cpu().numpy(), None if w is None else w.cpu().numpy(), offs,
           counts, st)
    plan.close()
    return out


def _random_systems(rng, sizes, box=(12.0, 12.0, 8.0)):
    out = []
    for n in sizes:
        while True:
            pts = rng.random((n, 3)) * np.array(box)
            pts = np.round(pts * 64) / 64          # exactly representable in float32
            d = np.linalg.norm(pts[:, None] - pts[None], axis=2) + np.eye(n)
            if d.min() > 0.2:
                break
        vals = rng.normal(size=n)
        tgt = np.round(rng.random(3) * np.array(box) * 64) / 64
        out.append((pts, vals.astype(np.float32).astype(np.float64), tgt))
    return out


@pytest.mark.parametrize("model,nug,sill,rng_", [("spherical", 0.0, 1.0, 8.0),
                                                   ("exponential", 0.05, 2.0, 6.0),
                                                   ("gaussian", 0.1, 1.0, 5.0)])
def test_points_vs_oracle(model, nug, sill, rng_):
    rng = np.random.default_rng(7)
    systems = _random_systems(rng, [1, 2, 3, 5, 18, 33, 50, 64, 65, 98])
    est, var, w, offs, counts, st = _run(systems, (model, nug, sill, rng_))
    assert st["n_nonpositive_pivot"] == 0
    for i, (pts, vals, tgt) in enumerate(systems):
        e, v, wo, _ = O.krige_points(pts, vals, tgt[None], model, nug, sill, rng_)
        wg = w[offs[i]:offs[i] + counts[i]]
        scale = max(1.0, np.abs(wo).max())
        np.testing.assert_allclose(wg, wo[:, 0], rtol=0, atol=2e-6 * scale)
        assert abs(est[i] - e[0]) <= 2e-6 * max(1.0, np.abs(vals).max()) * scale
        assert abs(var[i] - v[0]) <= 2e-6 * sill


def test_point_pins_closed_forms():
    # P1: one point at distance h: w = 1, sigma^2 = 2 gamma(h)
    s1 = (np.array([[0.0, 0.0, 0.0]]), np.array([0.75]), np.array([0.0, 0.0, 2.0]))
    # P2: two points at +-1 in z from the target, spherical a = 4: w = (1/2, 1/2),
    # sigma^2 = 2 gamma(1) - gamma(2)/2 = 25/64
    s2 = (np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 2.0]]), np.array([0.25, 0.5]),
          np.array([0.0, 0.0, 1.0]))
    est, var, w, offs, counts, _ = _run([s1, s2], ("spherical", 0.0, 1.0, 4.0))
    g = O.semivariogram("spherical", 0.0, 1.0, 4.0, 2.0)
    assert w[0] == pytest.approx(1.0, abs=1e-7)
    assert est[0] == pytest.approx(0.75, abs=1e-7)
    assert var[0] == pytest.approx(2 * g, abs=1e-7)
    np.testing.assert_allclose(w[1:3], [0.5, 0.5], atol=1e-7)
    assert var[1] == 0.390625
    assert est[1] == pytest.approx(0.375, abs=1e-7)


def test_point_pins_pure_nugget():
    # P3: range below every distance: w = 1/n, z_hat = mean, sigma^2 = sill (1 + 1/n)
    n = 18
    pts = np.array([[x, y, s * 2.0] for s in (0, 1) for y in (-1, 0, 1) for x in (-1, 0, 1)],
                   float)
    vals = np.linspace(-1.0, 2.0, n)
    est, var, w, _, _, _ = _run([(pts, vals, np.array([0.5, 0.5, 1.0]))],
                                ("spherical", 0.0, 1.0, 0.9))
    np.testing.assert_allclose(w, 1.0 / n, atol=1e-7)
    assert est[0] == pytest.approx(vals.mean(), abs=1e-6)
    assert var[0] == pytest.approx(1.0 + 1.0 / n, abs=1e-6)


def test_point_invariants():
    rng = np.random.default_rng(11)
    systems = _random_systems(rng, [4, 12, 27, 50, 98])
    vario = ("exponential", 0.0, 1.0, 6.0)
    est, var, w, offs, counts, _ = _run(systems, vario)
    for i, (pts, vals, tgt) in enumerate(systems):
        wi = w[offs[i]:offs[i] + counts[i]].astype(np.float64)
        # P4 weights sum to one; P7 variance non-negative
        assert abs(wi.sum() - 1.0) <= 1e-6
        assert var[i] >= -1e-6
        # P8 the weights minimise Q(w) = w'Cw - 2 w'c0 + sill on sum(w) = 1
        d = np.linalg.norm(pts[:, None] - pts[None], axis=2)
        C = O.covariance("exponential", 0.0, 1.0, 6.0, d)
        c0 = O.covariance("exponential", 0.0, 1.0, 6.0, np.linalg.norm(pts - tgt, axis=1))
        Q = lambda x: x @ C @ x - 2 * x @ c0 + 1.0
        assert Q(wi) == pytest.approx(var[i], abs=1e-5)
        for a, b in [(0, len(wi) - 1), (len(wi) // 2, 0)]:
            if a != b:
                e = np.zeros_like(wi)
                e[a], e[b] = 1e-2, -1e-2
                assert Q(wi + e) >= Q(wi) - 1e-9
    # P5 a constant field is reproduced; P6 a target on a data point (nugget 0)
    const = [(p, np.full(len(v), 0.625), t) for p, v, t in systems]
    est_c, _, _, _, _, _ = _run(const, vario, want_weights=False)
    np.testing.assert_allclose(est_c, 0.625, atol=1e-6)
    on_pt = [(p, v, p[len(v) // 2]) for p, v, _ in systems]
    est_p, var_p, _, _, _, _ = _run(on_pt, vario, want_weights=False)
    for i, (p, v, _) in enumerate(on_pt):
        assert est_p[i] == pytest.approx(v[len(v) // 2], abs=1e-6)
        assert abs(var_p[i]) <= 1e-6


def test_point_errors_reported():
    import torch
    import paper_2303_09523_amd as P
    # coincident points with nugget 0: singular C -> NaN and counted
    s = (np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [1.0, 0.0, 0.0]]), np.array([1.0, 2.0, 3.0]),
         np.array([0.5, 0.0, 0.0]))
    est, var, w, _, _, st = _run([s], ("gaussian", 0.0, 1.0, 5.0))
    assert np.isnan(est[0]) and st["n_nonpositive_pivot"] == 1
    # a count outside 1..98: NaN output and OKR_E_SHAPE at the sync
    plan = P.Plan(4, 4, 2, 2, 1)
    cu = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    est, var, _ = plan.krige_points(cu(np.array([0, 2], np.int32)), cu(np.array([0, 0], np.int64)),
                                    cu(np.array([[0, 0, 0], [1, 0, 0]], np.float32)),
                                    cu(np.ones(2, np.float32)),
                                    cu(np.zeros((2, 3), np.float32)), ("spherical", 0.0, 1.0, 4.0))
    torch.cuda.synchronize()
    with pytest.raises(P.OkrError) as ei:
        plan.stats()
    assert ei.value.status == 2
    e = est.cpu().numpy()
    assert np.isnan(e[0]) and e[1] == pytest.approx(1.0, abs=1e-6)
    plan.close()

"""Seeded input generators: determinism, value ranges, edge fraction and the
second-order statistics of the Gaussian random field."""
import numpy as np
import pytest

import workloads as W


def test_phantom_deterministic_and_shaped():
    w = W.workload("plain_8x64")
    a, ea = W.make_inputs(w)
    b, eb = W.make_inputs(w)
    assert a.dtype == np.float32 and a.shape == (8, 64, 64)
    assert ea is None and eb is None
    np.testing.assert_array_equal(a, b)
    c, _ = W.make_inputs(w, seed=99)
    assert not np.array_equal(a, c)
    # background ~ N(0, 0.01^2); objects have intensity in [0.2, 1]
    assert a.min() > -0.1 and a.max() < 1.1
    assert (a > 0.15).mean() > 0.01


def test_sobel_edges_step():
    s = np.zeros((1, 8, 8))
    s[0, :, 4:] = 0.2            # a 0.2 step gives |G| = 0.8 next to the step
    e = W.sobel_edges(s)
    assert e.dtype == np.uint8
    assert e[0, :, 3:5].all() and not e[0, :, :3].any() and not e[0, :, 5:].any()


def test_edge_fraction_masked_workload():
    w = W.workload("edge_32x256")
    s, e = W.make_inputs(w)
    frac = e.mean()
    assert 0.005 < frac < 0.2


def test_gaussian_field_covariance():
    v = W.Variogram("exponential", 0.02, 0.8, 5.0)
    f, clipped = W.gaussian_field((16, 128, 128), v, seed=4)
    assert clipped < 1e-3
    f = f - f.mean()
    var = (f * f).mean()
    assert var == pytest.approx(0.8, rel=0.08)
    for lag in (1, 2, 4, 6):
        emp = (f[:, :, lag:] * f[:, :, :-lag]).mean()
        model = 0.78 * np.exp(-3.0 * lag / 5.0)
        assert emp == pytest.approx(model, rel=0.15, abs=0.02)


def test_postpass_volume_deterministic():
    w = W.workload("plain_8x64")
    a = W.postpass_volume(w)
    b = W.postpass_volume(w)
    assert a.dtype == np.float32 and a.shape == (w.out_slices, 64, 64)
    np.testing.assert_array_equal(a, b)
    # planes z = s*f carry the phantom of the known slices up to the noise
    clean = W.phantom_at(w, [0.0])
    assert np.abs(a[0] - clean[0]).max() < 8 * w.noise

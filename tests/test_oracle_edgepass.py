"""Pins of the edge post-pass oracle (Section 4.1.2, Algorithm 2, Appendix B):
the worked orientation window of Section 4.1.2 and the sides of Step 5 from
the paper's example (tests/golden/edge_window_example.json), properties of
the shearlet filters, orientation recovery on straight edges at every
orientation, a hand-traced chain, and a hand-computed median adjustment."""
import json
import math
import os

import numpy as np

from oracle import edgepass as E

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "edge_window_example.json")


def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def test_worked_window_example():
    g = _golden()
    out, noisy = E.window_orientations(g["window"])
    assert noisy
    assert out == g["expected"]


def test_window_rules():
    # fewer than 4 changes: unchanged
    seq = [3] * 8 + [4] * 8
    assert E.window_orientations(seq) == (seq, False)
    # ties: the tied orientation that occurs first in the window
    seq = [5, 2, 5, 2, 5, 2, 5, 2, 2, 5, 2, 5, 2, 5, 2, 5]
    out, noisy = E.window_orientations(seq)
    assert noisy and out == [5] + [5] * 14 + [5]
    seq = [2, 5, 2, 5, 2, 5, 2, 5, 5, 2, 5, 2, 5, 2, 5, 7]
    out, noisy = E.window_orientations(seq)
    assert noisy and out == [2] + [5] * 14 + [7]


def test_step5_sides_match_the_example():
    g = _golden()["step5_next_along_second_axis"]
    left, right = E.sides(*g["tangent"])
    assert sorted(map(list, left)) == sorted(g["left"])
    assert sorted(map(list, right)) == sorted(g["right"])
    # a diagonal tangent leaves 3 pixels on each side of the diagonal line
    left, right = E.sides(1, 1)
    assert sorted(left) == [(-1, 0), (-1, 1), (0, 1)]
    assert sorted(right) == [(0, -1), (1, -1), (1, 0)]


def test_filters_have_zero_mean():
    taps = E.shearlet_filters()
    assert taps.shape == (E.K, 2 * E.RADIUS + 1, 2 * E.RADIUS + 1)
    assert np.abs(taps.sum(axis=(1, 2))).max() <= 1e-13 * np.abs(taps).max()
    sh = E.shearlet_coefficients(np.full((20, 23), 3.7))
    assert np.abs(sh).max() <= 1e-12


def test_cones_are_transposes():
    """The vertical cone is the horizontal cone with the axes exchanged: for the
    same shear, its coefficients on an image are the horizontal coefficients on
    the transposed image, transposed."""
    rng = np.random.default_rng(3)
    img = rng.normal(size=(21, 26))
    sh = E.shearlet_coefficients(img)
    sht = E.shearlet_coefficients(img.T)
    pairs = [(kh, kv) for kh, (ch, sh_) in enumerate(E.SHEARS)
             for kv, (cv, sv) in enumerate(E.SHEARS) if ch == 0 and cv == 1 and sh_ == sv]
    assert len(pairs) == 3
    for kh, kv in pairs:
        np.testing.assert_allclose(sh[kv], sht[kh].T, rtol=0, atol=1e-12)


def test_straight_edges_recover_each_orientation():
    H = W = 48
    x2, x1 = np.mgrid[0:H, 0:W].astype(float)
    for k in range(E.K):
        a = math.radians(E.normal_angle(k))
        d = (x1 - 23.3) * math.cos(a) + (x2 - 24.1) * math.sin(a)
        img = (d > 0).astype(float)
        theta = np.argmax(np.abs(E.shearlet_coefficients(img)), axis=0)
        on = (np.abs(d) <= 0.75) & (x1 > 8) & (x1 < W - 8) & (x2 > 8) & (x2 < H - 8)
        assert on.sum() > 20
        assert (theta[on] == k).all(), (k, np.unique(theta[on], return_counts=True))


def test_chain_of_a_square_ring_is_traversed_clockwise():
    edge = np.zeros((6, 6), np.uint8)
    edge[1, 1:5] = edge[4, 1:5] = edge[1:5, 1] = edge[1:5, 4] = 1
    ch = E.chains(edge)
    assert ch == [[(1, 1), (1, 2), (1, 3), (1, 4), (2, 4), (3, 4), (4, 4), (4, 3), (4, 2),
                   (4, 1), (3, 1), (2, 1)]]


def test_window_median_adjustment_by_hand():
    """A straight 16-pixel chain along row 5 whose orientation alternates with
    a minority value: the representative (normal along the rows, index 6)
    takes the interior; at each minority pixel (the new edge pixel is the same
    pixel on a straight chain) the 3 pixels above and the 3 below take their
    medians (computed by hand below)."""
    out = np.zeros((12, 20), np.float32)
    out[4] = [3, 1, 4, 1, 5, 9, 2, 6, 5, 3, 5, 8, 9, 7, 9, 3, 2, 3, 8, 4]
    out[6] = [2, 7, 1, 8, 2, 8, 1, 8, 2, 8, 4, 5, 9, 0, 4, 5, 2, 3, 5, 3]
    win = [(5, 2 + m) for m in range(16)]
    th = [6, 6, 2, 6, 6, 2, 6, 6, 2, 6, 6, 2, 6, 6, 2, 6]
    emap = np.zeros((12, 20), np.uint8)
    tmap = np.zeros((12, 20), np.uint8)
    for (r, c), t in zip(win, th):
        emap[r, c] = 1
        tmap[r, c] = t
    assert E.process_window(out, emap, tmap, win, th)
    assert out[4].tolist() == [3, 1, 4, 5, 5, 5, 5, 5, 5, 5, 5, 5, 9, 9, 9, 3, 3, 3, 8, 4]
    assert out[6].tolist() == [2, 7, 1, 8, 8, 8, 2, 2, 2, 5, 5, 5, 4, 4, 4, 3, 3, 3, 5, 3]
    assert (out[5] == 0).all()
    assert [int(tmap[r, c]) for r, c in win] == [6] * 16
    assert emap.sum() == 16 and all(emap[r, c] for r, c in win)


def test_postpass_on_a_noisy_disc_is_deterministic_and_local():
    """End to end on a small image: edges lie on the disc's boundary, only
    pixels next to edge pixels change, and the result is repeatable."""
    rng = np.random.default_rng(5)
    H, W = 40, 44
    x2, x1 = np.mgrid[0:H, 0:W]
    img = (((x1 - 21.5) ** 2 + (x2 - 19.2) ** 2) < 12.3 ** 2).astype(np.float32) * 0.8
    img += rng.normal(0, 0.05, size=img.shape).astype(np.float32)
    step = np.zeros((30, 30))
    step[:, 15:] = 1.0
    gain = np.abs(E.shearlet_coefficients(step)).max()   # response to a unit step
    tau = 0.4 * 0.8 * gain
    out, emap, tmap = E.edge_postpass_image(img, tau)
    out2, emap2, tmap2 = E.edge_postpass_image(img, tau)
    assert np.array_equal(out, out2) and np.array_equal(emap, emap2)
    r = np.hypot(x1 - 21.5, x2 - 19.2)
    edge0, _, _ = E.edges_and_orientation(img, tau)
    assert edge0.sum() > 40
    assert (np.abs(r[edge0 > 0] - 12.3) <= 2.5).all()
    changed = out != img
    near = np.zeros_like(changed)
    for dr in (-2, -1, 0, 1, 2):
        for dc in (-2, -1, 0, 1, 2):
            near |= np.roll(np.roll(emap > 0, dr, 0), dc, 1)
    assert not (changed & ~near).any()

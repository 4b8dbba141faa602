"""FP64 CPU oracle of the paper's edge post-pass on the reconstructed volume.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module. The product path never
calls it, and it shares no code, tables or constants with that path.

What it computes (Section 4.1.2, Algorithm 2; Appendix B), in the paper's
order, on every 2D image of the volume along the YZ plane (image x is
I(z, y) = V[z][y][x]):

1. Shearlet transform (Appendix B): coefficients SH(I)(k, e) of the image
   with a discrete shearlet system at one (fine) scale and K shears.
2. Edges and their orientation: theta(e) = argmax_k |SH(I)(k, e)|.
3. Edge pixels are traversed clockwise along their chains; windows of 16
   consecutive chain pixels are examined.
4. A window whose orientation changes back and forth is taken as noise: its
   interior pixels take the window's representative orientation; a pixel
   whose orientation differs is replaced by the neighbour of the previous
   edge pixel in that orientation's direction.
5. At every newly selected edge pixel, the 3 neighbours on each side of the
   edge are replaced by their median.

Readings of what the paper leaves open (the HIP path implements the same
written readings, not this code):

* Shearlet system. The system of Appendix B, psi_{a,s,t}(x) =
  a^{-3/4} psi(A_a^{-1} S_s^{-1} (x - t)), A_a = diag(a, sqrt a),
  S_s = [[1, -s], [0, 1]], with a separable mother shearlet
  psi(u1, u2) = psi1(u1) phi(u2) of compact support: the odd wavelet
  psi1(u) = -u (1 - (u/10)^2)^2 for |u| < 10 (0 elsewhere) and the window
  phi(u) = (1 - (u/10)^2)^2 for |u| < 10, at the scale a = 1/4 (so
  a^{-3/4} = 2 sqrt 2 and sqrt a = 1/2), sampled at the integer offsets
  |d1|, |d2| <= 4 (9 x 9 taps, t = the pixel). Every tap is a polynomial in
  exact binary fractions times 2 sqrt 2, so two correctly rounded evaluations
  in the same operation order agree bit for bit. Image axes:
  x1 = y (columns), x2 = z (rows). Two cones: horizontal,
  psi1((x1 + s x2) / a) phi(x2 / sqrt a), s in {-1, -1/2, 0, 1/2}; vertical
  (x1 and x2 exchanged), psi1((x2 + s x1) / a) phi(x1 / sqrt a),
  s in {1, 1/2, 0, -1/2}. Orientation index k = 0..7 in that order: edge
  normals at -45, -26.6, 0, 26.6, 45, 63.4, 90, 116.6 degrees from the x1 axis
  toward x2. Coefficients are correlations, SH(k, p) = sum_d psi_k(d) I(p + d),
  with the image extended by replicating its border.
* Edges ("as in [29]"): p is an edge pixel iff M(p) = max_k |SH(k, p)| >= tau
  (a parameter) and M(p) >= M(q) for both neighbours q = p +- n(p), n(p) the
  normal of theta(p) rounded to the nearest multiple of 45 degrees
  (out-of-image neighbours do not count). The argmax takes the first maximum.
* Traversal ("move in clockwise direction"): images are scanned row by row;
  each edge pixel not yet visited starts a chain, which repeatedly moves to
  the first edge pixel not yet visited among the 8 neighbours of its last
  pixel, searched clockwise (x1 right, x2 down: E, SE, S, SW, W, NW, N, NE)
  starting three steps counter-clockwise of the last move (E for the first
  move). Windows are the chain's consecutive full groups of 16 pixels.
* Noise and "mean(theta)": a window is noisy when its orientation changes at
  least 4 times between consecutive pixels. Its representative orientation is
  the most frequent one (the worked sequence of Section 4.1.2 maps to theta_1,
  which is its most frequent value, not the mean of its indices, 1.5), ties to
  the one that occurs first in the window. The first and last pixels keep their
  orientation; the others take the representative one.
* New edge pixels: walking the window from its first pixel, a pixel whose
  orientation differs from the representative one is replaced by the previous
  (kept or new) pixel plus the edge tangent t: the representative normal
  rounded to 45 degrees, turned by 90 degrees, with the sign that points from
  the window's first toward its last pixel. Out-of-image replacements keep the
  original pixel.
* Median adjustment: around each new edge pixel e, the 8 neighbours other than
  e +- t split by the sign of the cross product t x d (d = neighbour offset)
  into two sides of 3 ("left of it" / "right of it" for t along an axis, as in
  the example of Section 4.1.2); each side whose 3 pixels are in the image is
  set to their median. Changes apply in traversal order (later medians see
  earlier changes); the edge map records the new pixels in place of the
  replaced ones.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np

SUPPORT, RADIUS = 10.0, 4   # support of psi1 and phi; taps |d| <= RADIUS
# (cone, shear): cone 0 horizontal, 1 vertical
SHEARS = [(0, -1.0), (0, -0.5), (0, 0.0), (0, 0.5), (1, 1.0), (1, 0.5), (1, 0.0), (1, -0.5)]
K = len(SHEARS)
WINDOW = 16
MIN_CHANGES = 4
# clockwise neighbour order with x1 right, x2 down: (d1, d2)
CLOCKWISE = [(1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1)]


def normal_angle(k: int) -> float:
    """Edge-normal angle of orientation k in degrees (from x1 toward x2)."""
    cone, s = SHEARS[k]
    return math.degrees(math.atan(s)) if cone == 0 else 90.0 - math.degrees(math.atan(s))


def _psi1(u: float) -> float:
    if abs(u) >= SUPPORT:
        return 0.0
    q = 1.0 - (u / SUPPORT) * (u / SUPPORT)
    return -u * (q * q)


def _phi(u: float) -> float:
    if abs(u) >= SUPPORT:
        return 0.0
    q = 1.0 - (u / SUPPORT) * (u / SUPPORT)
    return q * q


def shearlet_filters() -> np.ndarray:
    """psi_k(d) for k < K, taps [k][d2 + R][d1 + R] (Appendix B, readings above):
    a^{-3/4} psi1(u1 / a) phi(u2 / sqrt a) with (u1, u2) = S_s^{-1} d for the
    horizontal cone and the axes exchanged for the vertical one."""
    R = RADIUS
    norm = 2.0 * math.sqrt(2.0)        # a^{-3/4} at a = 1/4
    out = np.empty((K, 2 * R + 1, 2 * R + 1))
    for k, (cone, s) in enumerate(SHEARS):
        for i2 in range(2 * R + 1):
            for i1 in range(2 * R + 1):
                d1, d2 = float(i1 - R), float(i2 - R)
                if cone == 0:
                    u, v = d1 + s * d2, d2
                else:
                    u, v = d2 + s * d1, d1
                out[k, i2, i1] = norm * (_psi1(u * 4.0) * _phi(v * 2.0))
    return out


def shearlet_coefficients(img: np.ndarray) -> np.ndarray:
    """SH(k, p) [K][rows][cols]: correlation with each filter, border replicated."""
    img = np.asarray(img, dtype=np.float64)
    R = RADIUS
    pad = np.pad(img, R, mode="edge")
    H, Wd = img.shape
    taps = shearlet_filters()
    out = np.zeros((K,) + img.shape)
    for i2 in range(2 * R + 1):
        for i1 in range(2 * R + 1):
            win = pad[i2:i2 + H, i1:i1 + Wd]
            out += taps[:, i2, i1][:, None, None] * win[None]
    return out


def normal_step(k: int) -> Tuple[int, int]:
    """Normal of orientation k rounded to the nearest multiple of 45 degrees, as a
    neighbour offset (d1, d2)."""
    q = int(round(normal_angle(k) / 45.0)) % 4
    return [(1, 0), (1, 1), (0, 1), (-1, 1)][q]


def edges_and_orientation(img: np.ndarray, tau: float):
    """(edge uint8 [rows][cols], theta uint8, M float64) of one image."""
    sh = np.abs(shearlet_coefficients(img))
    theta = np.argmax(sh, axis=0).astype(np.uint8)
    M = np.max(sh, axis=0)
    H, Wd = M.shape
    edge = np.zeros((H, Wd), dtype=np.uint8)
    for r in range(H):
        for c in range(Wd):
            if M[r, c] < tau:
                continue
            d1, d2 = normal_step(int(theta[r, c]))
            ok = True
            for sgn in (1, -1):
                rr, cc = r + sgn * d2, c + sgn * d1
                if 0 <= rr < H and 0 <= cc < Wd and M[rr, cc] > M[r, c]:
                    ok = False
            edge[r, c] = 1 if ok else 0
    return edge, theta, M


def chains(edge: np.ndarray) -> List[List[Tuple[int, int]]]:
    """Edge chains as lists of (row, col), in the traversal order of the readings."""
    H, Wd = edge.shape
    visited = np.zeros_like(edge, dtype=bool)
    out = []
    for r in range(H):
        for c in range(Wd):
            if not edge[r, c] or visited[r, c]:
                continue
            chain = [(r, c)]
            visited[r, c] = True
            cr, cc, last = r, c, None
            while True:
                start = 0 if last is None else (last + 5) % 8
                moved = False
                for j in range(8):
                    dd = (start + j) % 8
                    d1, d2 = CLOCKWISE[dd]
                    nr, nc = cr + d2, cc + d1
                    if 0 <= nr < H and 0 <= nc < Wd and edge[nr, nc] and not visited[nr, nc]:
                        visited[nr, nc] = True
                        chain.append((nr, nc))
                        cr, cc, last = nr, nc, dd
                        moved = True
                        break
                if not moved:
                    break
            out.append(chain)
    return out


def representative(thetas) -> int:
    """Most frequent orientation; ties to the one occurring first in the window."""
    counts = {}
    for t in thetas:
        counts[t] = counts.get(t, 0) + 1
    best = max(counts.values())
    for t in thetas:
        if counts[t] == best:
            return int(t)
    raise ValueError("empty window")


def window_orientations(thetas):
    """The orientation sequence of one window after Step 4: unchanged unless it
    changes at least MIN_CHANGES times; then first and last keep theirs and the
    others take the representative one."""
    thetas = [int(t) for t in thetas]
    changes = sum(1 for m in range(1, len(thetas)) if thetas[m] != thetas[m - 1])
    if changes < MIN_CHANGES:
        return thetas, False
    rep = representative(thetas)
    return [thetas[0]] + [rep] * (len(thetas) - 2) + [thetas[-1]], True


def sides(t1: int, t2: int):
    """The two sides (cross product > 0 first) of 3 neighbour offsets each."""
    left, right = [], []
    for d1, d2 in CLOCKWISE:
        cr = t1 * d2 - t2 * d1
        if cr > 0:
            left.append((d1, d2))
        elif cr < 0:
            right.append((d1, d2))
    return left, right


def process_window(out, emap, tmap, win, th):
    """Steps 4 and 5 on one window of 16 chain pixels (win: (row, col) in chain
    order, th: their orientations), updating the image `out` and the edge and
    orientation maps in place. Returns whether the window was taken as noise."""
    H, Wd = out.shape
    new_th, noisy = window_orientations(th)
    if not noisy:
        return False
    rep = new_th[1]
    n1, n2 = normal_step(rep)
    t1, t2 = -n2, n1
    dr, dc = win[-1][0] - win[0][0], win[-1][1] - win[0][1]
    if t1 * dc + t2 * dr < 0:
        t1, t2 = -t1, -t2
    left, right = sides(t1, t2)
    qr, qc = win[0]
    for m in range(1, len(win) - 1):
        pr, pc = win[m]
        if th[m] == rep:
            qr, qc = pr, pc
            tmap[pr, pc] = rep
            continue
        nr, nc = qr + t2, qc + t1
        if not (0 <= nr < H and 0 <= nc < Wd):
            qr, qc = pr, pc
            tmap[pr, pc] = rep
            continue
        emap[pr, pc] = 0
        emap[nr, nc] = 1
        tmap[nr, nc] = rep
        qr, qc = nr, nc
        for side in (left, right):
            pts = [(nr + d2, nc + d1) for d1, d2 in side]
            if all(0 <= a < H and 0 <= b < Wd for a, b in pts):
                med = sorted(out[a, b] for a, b in pts)[1]
                for a, b in pts:
                    out[a, b] = med
    return True


def edge_postpass_image(img: np.ndarray, tau: float):
    """Alg. 2 on one image: (adjusted image float32, edge map, orientation map)."""
    out = np.asarray(img, dtype=np.float32).copy()
    edge, theta, _ = edges_and_orientation(img, tau)
    emap = edge.copy()
    tmap = theta.copy()
    for chain in chains(edge):
        for w0 in range(0, len(chain) - WINDOW + 1, WINDOW):
            win = chain[w0:w0 + WINDOW]
            process_window(out, emap, tmap, win, [int(theta[p]) for p in win])
    return out, emap, tmap


def edge_postpass_volume(vol: np.ndarray, tau: float):
    """Every YZ image of a volume [Z][ny][nx]: (volume float32, edges, orientations)."""
    vol = np.asarray(vol, dtype=np.float32)
    Z, ny, nx = vol.shape
    out = vol.copy()
    emap = np.zeros(vol.shape, dtype=np.uint8)
    tmap = np.zeros(vol.shape, dtype=np.uint8)
    for x in range(nx):
        o, e, t = edge_postpass_image(vol[:, :, x], tau)
        out[:, :, x] = o
        emap[:, :, x] = e
        tmap[:, :, x] = t
    return out, emap, tmap

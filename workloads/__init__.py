"""Seeded synthetic inputs for inter-slice kriging.

This module only *generates inputs*: known slices, edge masks and the
parameters of each workload. It contains none of the kriging arithmetic, so
both the FP64 oracle and the GPU path may draw their inputs from it without
sharing any of the method's code.

The paper evaluates on 512x512 T2 MRI stacks with 1-5 mm gaps (Section 5);
those studies are not available, so seeded phantoms stand in for them:

* ``phantom``: random ellipsoids plus thin high-contrast shells, sampled at the
  known slice positions z = s*f, with iid Gaussian noise.
* ``sobel_edges``: the edge mask that the edge-preserving neighbour selection
  takes as an input (uint8, 1 = edge).
* ``gaussian_field``: a stationary Gaussian random field with an exponential
  covariance, by circulant embedding (Wood & Chan 1994; Dietrich & Newsam
  1997), used for the variogram-fitting workload.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

__all__ = [
    "Variogram", "Workload", "WORKLOADS", "workload", "phantom", "phantom_at",
    "sobel_edges", "gaussian_field", "make_inputs", "EDGE_TAU", "postpass_volume",
]


@dataclasses.dataclass(frozen=True)
class Variogram:
    """Variogram parameters: ``sill`` is the total sill (Cov(0)), ``range``
    the practical range, ``nugget`` the discontinuity at the origin."""
    model: str          # "spherical" | "exponential" | "gaussian"
    nugget: float
    sill: float
    range: float


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    nslices: int        # known slices
    m: int              # slice width = height
    upsample: int       # f: output has (nslices-1)*f + 1 slices
    radius: int         # r: window (2r+1) x (2r+1) x 2
    masked: bool        # edge mask from the Sobel threshold, else none
    n_ellipsoids: int
    n_shells: int
    noise: float        # noise standard deviation on the known slices
    vario: Variogram
    seed: int
    field: bool = False  # Gaussian random field instead of a phantom

    @property
    def out_slices(self) -> int:
        return (self.nslices - 1) * self.upsample + 1

    @property
    def kriged_voxels(self) -> int:
        return (self.nslices - 1) * (self.upsample - 1) * self.m * self.m

    @property
    def systems(self) -> int:
        return (self.nslices - 1) * self.m * self.m


# The five workloads of the study. Sizes, variograms and windows follow the
# workload descriptions; unstated sizes are fixed here (f=4 and a 7x7x2
# masked window for the precision study; 8 shells for the large volume).
WORKLOADS = {
    "plain_8x64": Workload("plain_8x64", 8, 64, 2, 1, False, 3, 0, 0.01,
                           Variogram("spherical", 0.0, 1.0, 4.0), 1),
    "edge_32x256": Workload("edge_32x256", 32, 256, 4, 2, True, 10, 2, 0.02,
                            Variogram("exponential", 0.01, 1.0, 6.0), 2),
    "precision_48x384": Workload("precision_48x384", 48, 384, 4, 3, True, 10, 2, 0.02,
                                 Variogram("gaussian", 1e-4, 1.0, 5.0), 3),
    "loso_16x128": Workload("loso_16x128", 16, 128, 2, 2, False, 0, 0, 0.0,
                            Variogram("exponential", 0.02, 0.8, 5.0), 4, field=True),
    "large_160x512": Workload("large_160x512", 160, 512, 4, 3, True, 40, 8, 0.02,
                              Variogram("spherical", 0.005, 1.0, 8.0), 5),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def _draw_objects(rng: np.random.Generator, m: int, zmax: float, n_ell: int, n_shell: int):
    objs = []
    for k in range(n_ell + n_shell):
        centre = rng.uniform(0.2, 0.8, size=3) * np.array([m, m, zmax], dtype=np.float64)
        ax, ay = rng.uniform(0.08, 0.30, size=2) * m
        az = rng.uniform(0.15, 0.45) * zmax
        phi = rng.uniform(0.0, np.pi)
        inten = rng.uniform(0.2, 1.0)
        shell = k >= n_ell
        objs.append((centre, ax, ay, az, phi, 1.0 if shell else inten, shell))
    return objs


def _render(objs, m: int, zs: np.ndarray) -> np.ndarray:
    """Evaluate the phantom (max over occupying objects) at planes z in zs."""
    out = np.zeros((len(zs), m, m), dtype=np.float64)
    yy, xx = np.meshgrid(np.arange(m, dtype=np.float64), np.arange(m, dtype=np.float64),
                         indexing="ij")
    for (c, ax, ay, az, phi, inten, shell) in objs:
        pad = 1.0 if shell else 0.0   # shells extend ~0.75 voxel beyond rho = 1
        reach = max(ax, ay) + pad + 1.0
        x0, x1 = max(0, int(c[0] - reach)), min(m, int(c[0] + reach) + 2)
        y0, y1 = max(0, int(c[1] - reach)), min(m, int(c[1] + reach) + 2)
        if x0 >= x1 or y0 >= y1:
            continue
        cs, sn = np.cos(phi), np.sin(phi)
        dxs = xx[y0:y1, x0:x1] - c[0]
        dys = yy[y0:y1, x0:x1] - c[1]
        u = (cs * dxs + sn * dys) / ax
        v = (-sn * dxs + cs * dys) / ay
        uv2 = u * u + v * v
        for iz, z in enumerate(zs):
            w = (z - c[2]) / az
            if abs(w) > 1.0 + (0.75 / min(ax, ay) + 0.1 if shell else 0.0):
                continue
            rho = np.sqrt(uv2 + w * w)
            if shell:
                occ = np.abs(rho - 1.0) * min(ax, ay) <= 0.75
            else:
                occ = rho <= 1.0
            if occ.any():
                blk = out[iz, y0:y1, x0:x1]
                np.maximum(blk, np.where(occ, inten, 0.0), out=blk)
    return out


def phantom(w: Workload, seed: Optional[int] = None) -> np.ndarray:
    """Known slices, float32 [nslices][m][m], slice s sampled at z = s*f."""
    rng = np.random.default_rng(w.seed if seed is None else seed)
    zmax = float(w.upsample * (w.nslices - 1))
    objs = _draw_objects(rng, w.m, zmax, w.n_ellipsoids, w.n_shells)
    zs = np.arange(w.nslices, dtype=np.float64) * w.upsample
    clean = _render(objs, w.m, zs)
    noisy = clean + rng.normal(0.0, w.noise, size=clean.shape)
    return noisy.astype(np.float32)


def phantom_at(w: Workload, zs, seed: Optional[int] = None) -> np.ndarray:
    """Noise-free phantom at arbitrary output planes (quality reports only)."""
    rng = np.random.default_rng(w.seed if seed is None else seed)
    zmax = float(w.upsample * (w.nslices - 1))
    objs = _draw_objects(rng, w.m, zmax, w.n_ellipsoids, w.n_shells)
    return _render(objs, w.m, np.asarray(zs, dtype=np.float64))


# Edge threshold of the post-pass workloads: with the post-pass filters about
# 3% of the pixels of a noisy phantom volume are edges (Section 4.1.2 leaves
# the threshold open).
EDGE_TAU = 4.0


def postpass_volume(w: Workload, seed: Optional[int] = None) -> np.ndarray:
    """Input of the edge post-pass in place of a reconstructed volume: the
    phantom at every output plane z = 0 .. (nslices-1)*f with iid Gaussian
    noise of the workload's level, float32 [out_slices][m][m]."""
    base = w.seed if seed is None else seed
    vol = phantom_at(w, np.arange(w.out_slices, dtype=np.float64), seed=base)
    rng = np.random.default_rng(base + 7919)
    return (vol + rng.normal(0.0, w.noise, size=vol.shape)).astype(np.float32)


def sobel_edges(slices: np.ndarray, threshold: float = 0.5) -> np.ndarray:
    """Edge mask per known slice: unnormalised 3x3 Sobel in FP64 with a
    replicated border; edge iff the gradient magnitude is >= threshold."""
    s = np.asarray(slices, dtype=np.float64)
    p = np.pad(s, ((0, 0), (1, 1), (1, 1)), mode="edge")
    # p[:, 1 + dy, 1 + dx] windows for dy, dx in {-1, 0, 1}
    def sh(dy, dx):
        return p[:, 1 + dy:1 + dy + s.shape[1], 1 + dx:1 + dx + s.shape[2]]
    gx = (sh(-1, 1) + 2 * sh(0, 1) + sh(1, 1)) - (sh(-1, -1) + 2 * sh(0, -1) + sh(1, -1))
    gy = (sh(1, -1) + 2 * sh(1, 0) + sh(1, 1)) - (sh(-1, -1) + 2 * sh(-1, 0) + sh(-1, 1))
    return (np.sqrt(gx * gx + gy * gy) >= threshold).astype(np.uint8)


def gaussian_field(shape, vario: Variogram, seed: int, pad_factor: int = 2):
    """Zero-mean stationary Gaussian field on a unit grid with covariance
    (sill - nugget) * rho(h) plus an iid nugget term of variance ``nugget``.

    Circulant embedding on a torus ``pad_factor`` times larger per axis;
    negative eigenvalues are clipped and their mass is returned.
    Returns (field float64 [nz][ny][nx], clipped_fraction).
    """
    nz, ny, nx = shape
    tz, ty, tx = nz * pad_factor, ny * pad_factor, nx * pad_factor
    dz = np.minimum(np.arange(tz), tz - np.arange(tz)).astype(np.float64)
    dy = np.minimum(np.arange(ty), ty - np.arange(ty)).astype(np.float64)
    dx = np.minimum(np.arange(tx), tx - np.arange(tx)).astype(np.float64)
    h = np.sqrt(dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2)
    a = vario.range
    if vario.model == "exponential":
        rho = np.exp(-3.0 * h / a)
    elif vario.model == "gaussian":
        rho = np.exp(-3.0 * (h / a) ** 2)
    elif vario.model == "spherical":
        rho = np.where(h < a, 1.0 - 1.5 * h / a + 0.5 * (h / a) ** 3, 0.0)
    else:
        raise ValueError(vario.model)
    c = (vario.sill - vario.nugget) * rho
    lam = np.fft.fftn(c).real
    neg = -lam[lam < 0].sum()
    clipped = neg / max(np.abs(lam).sum(), 1e-300)
    lam = np.clip(lam, 0.0, None)
    rng = np.random.default_rng(seed)
    wn = rng.standard_normal((tz, ty, tx)) + 1j * rng.standard_normal((tz, ty, tx))
    y = np.fft.fftn(np.sqrt(lam / lam.size) * wn)
    field = y.real[:nz, :ny, :nx]
    field = field + rng.normal(0.0, np.sqrt(vario.nugget), size=field.shape)
    return field, clipped


def make_inputs(w: Workload, seed: Optional[int] = None):
    """(slices float32 [n][m][m], edge uint8 [n][m][m] or None)."""
    if w.field:
        f, _ = gaussian_field((w.nslices, w.m, w.m), w.vario, w.seed if seed is None else seed)
        return f.astype(np.float32), None
    s = phantom(w, seed)
    e = sobel_edges(s) if w.masked else None
    return s, e

"""FP64 CPU oracle for edge-preserved ordinary kriging along Z.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module. The product path (the
HIP library and its Python binding) never calls it, and it shares no code,
tables or constants with that path.

What it computes, in the paper's order:

* Known slices are placed into the output volume at z = s*f and padded gaps
  are filled by kriging (Algorithm 1, step 3 and the text after it).
* Each missing voxel is estimated by kriging over its neighbours in the two
  adjacent known slices (Section 4.1.2, "3D domain"), as a weighted linear sum
  whose weights minimise the estimation variance under an unbiasedness
  constraint.
* The weights and Lagrange multiplier come from the extended covariance
  system of Appendix A (the KED/universal-kriging system) with a single
  constant predictor q_1 = 1, i.e. ordinary kriging: the bordered system
  [[C, 1], [1^T, 0]] [w; mu] = [c0; 1], solved here with LAPACK (dgesv).
* The kriging (estimation-error) variance is sill - w^T c0 - mu.
* With a drift (``drift="linear_z"``) the same Appendix A system is solved with
  two predictors, q_0 = 1 and q_1 = the point's slice (0 lower, 1 upper; the
  target's value is t/f): [[C, Q], [Q^T, 0]] [w; phi] = [c0; q0], variance
  sill - w^T c0 - phi^T q0 (universal kriging with a linear trend across the
  gap). A system whose kept points all lie in one slice cannot carry that
  trend (Q loses rank) and is solved as ordinary kriging.

Readings of what the paper leaves open:

* Covariance model: GSLIB convention with practical range a and total sill;
  Cov(0) = sill, Cov(h > 0) = (sill - nugget) * rho(h).
* Distances: Euclidean in output-voxel units; known slices are f apart.
* Window: (2r+1) x (2r+1) candidates in each of the two bounding slices;
  out-of-image candidates are dropped.
* Edge rule: a candidate (dx, dy) in slice s is kept iff no pixel of its
  discrete path from the centre is an edge in that slice's mask; the path is
  p_k = (rha(k dx / L), rha(k dy / L)), k = 1..L, L = max(|dx|, |dy|), with
  rha = round half away from zero; the centre is always kept.
* Floor: with fewer than ``min_points`` kept, rejected in-image candidates are
  added in the order (dx^2 + dy^2, lower slice first, dy, dx).
* Leave-one-slice-out: known slice s is predicted from slices s-1 and s+1
  (distance 1 each) with an unmasked window; the loss is the mean squared
  error over all held-out voxels.

Parity pins: see tests/test_oracle_pins.py (closed forms, invariants, brute
force, a 50-digit second arithmetic and finite differences). Whether the
Adam fit recovers the true (nugget/sill, range) is parity unpinned.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence

import numpy as np

MODELS = ("spherical", "exponential", "gaussian")


# ----------------------------------------------------------------------------
# Covariance model (Appendix A's "covariance of residuals"; model per reading)
# ----------------------------------------------------------------------------

def correlation(model: str, h, a: float):
    """rho(h) for practical range a."""
    h = np.asarray(h, dtype=np.float64)
    if model == "spherical":
        q = h / a
        return np.where(q < 1.0, 1.0 - 1.5 * q + 0.5 * q ** 3, 0.0)
    if model == "exponential":
        return np.exp(-3.0 * h / a)
    if model == "gaussian":
        return np.exp(-3.0 * (h / a) ** 2)
    raise ValueError(model)


def covariance(model: str, nugget: float, sill: float, a: float, h):
    """Cov(h): sill at h == 0, (sill - nugget) * rho(h) elsewhere."""
    h = np.asarray(h, dtype=np.float64)
    return np.where(h == 0.0, sill, (sill - nugget) * correlation(model, h, a))


def semivariogram(model: str, nugget: float, sill: float, a: float, h):
    """gamma(h) = sill - Cov(h); gamma(0) = 0."""
    return sill - covariance(model, nugget, sill, a, h)


def covariance_derivatives(model: str, nugget: float, sill: float, a: float, h):
    """d Cov(h) / d(nugget, sill, range), stacked on a leading axis of 3."""
    h = np.asarray(h, dtype=np.float64)
    rho = correlation(model, h, a)
    if model == "spherical":
        q = h / a
        drho_da = np.where(q < 1.0, 1.5 * h / a ** 2 - 1.5 * h ** 3 / a ** 4, 0.0)
    elif model == "exponential":
        drho_da = rho * 3.0 * h / a ** 2
    elif model == "gaussian":
        drho_da = rho * 6.0 * h ** 2 / a ** 3
    else:
        raise ValueError(model)
    zero = h == 0.0
    d_nug = np.where(zero, 0.0, -rho)
    d_sill = np.where(zero, 1.0, rho)
    d_a = np.where(zero, 0.0, (sill - nugget) * drho_da)
    return np.stack([d_nug, d_sill, d_a])


# ----------------------------------------------------------------------------
# Neighbourhood: candidates, edge rule, floor
# ----------------------------------------------------------------------------

def _rha_ratio(num: int, den: int) -> int:
    """round-half-away-from-zero of num/den for den > 0, exactly."""
    q = (2 * abs(num) + den) // (2 * den)
    return q if num >= 0 else -q


def edge_path(dx: int, dy: int):
    """Pixels of the discrete path from the centre (excluded) to (dx, dy)
    (included)."""
    L = max(abs(dx), abs(dy))
    return [(_rha_ratio(k * dx, L), _rha_ratio(k * dy, L)) for k in range(1, L + 1)]


def candidates(r: int):
    """Candidate offsets in canonical order: index = s*W^2 + (dy+r)*W + (dx+r)."""
    W = 2 * r + 1
    out = []
    for s in (0, 1):
        for dy in range(-r, r + 1):
            for dx in range(-r, r + 1):
                out.append((dx, dy, s))
    assert len(out) == 2 * W * W
    return out


def floor_order(r: int):
    """Canonical indices sorted by (dx^2 + dy^2, s, dy, dx)."""
    c = candidates(r)
    keyed = sorted(range(len(c)), key=lambda i: (c[i][0] ** 2 + c[i][1] ** 2, c[i][2], c[i][1], c[i][0]))
    return keyed


def select_neighbours(edge_pair, ys, xs, r: int, min_points: int, shape):
    """Kept-candidate masks, in canonical candidate order.

    edge_pair: (lo, hi) uint8 arrays [S][H][W] holding, for each system, the
    edge masks of its lower and upper bounding slices; or None (no mask).
    shape: (H, W) of the slices.
    Returns (kept bool [S][2W^2], inimage bool [S][2W^2]).
    """
    H, Wd = shape
    ys = np.asarray(ys, dtype=np.int64)
    xs = np.asarray(xs, dtype=np.int64)
    S = ys.shape[0]
    cands = candidates(r)
    kept = np.zeros((S, len(cands)), dtype=bool)
    inimg = np.zeros((S, len(cands)), dtype=bool)
    sidx = np.arange(S)
    for ci, (dx, dy, s) in enumerate(cands):
        yy, xx = ys + dy, xs + dx
        ok = (yy >= 0) & (yy < H) & (xx >= 0) & (xx < Wd)
        inimg[:, ci] = ok
        k = ok.copy()
        if edge_pair is not None and (dx, dy) != (0, 0):
            e = edge_pair[s]
            for (px, py) in edge_path(dx, dy):
                py_ = np.clip(ys + py, 0, H - 1)
                px_ = np.clip(xs + px, 0, Wd - 1)
                k &= e[sidx, py_, px_] == 0
        kept[:, ci] = k
    # floor: add rejected in-image candidates in the fixed order
    short = np.nonzero(kept.sum(axis=1) < min_points)[0]
    order = floor_order(r)
    for i in short:
        n = int(kept[i].sum())
        for ci in order:
            if n >= min_points:
                break
            if inimg[i, ci] and not kept[i, ci]:
                kept[i, ci] = True
                n += 1
    return kept, inimg


# ----------------------------------------------------------------------------
# Ordinary kriging of one system (Appendix A with p = 1, q_1 = 1)
# ----------------------------------------------------------------------------

def bordered_solve(C, c0):
    """Solve [[C, 1], [1^T, 0]] [w; mu] = [c0; 1] (LAPACK dgesv, batched).

    C: [G][n][n]; c0: [G][n][T]. Returns (w [G][n][T], mu [G][T]).
    """
    G, n, _ = C.shape
    T = c0.shape[2]
    K = np.zeros((G, n + 1, n + 1), dtype=np.float64)
    K[:, :n, :n] = C
    K[:, :n, n] = 1.0
    K[:, n, :n] = 1.0
    rhs = np.empty((G, n + 1, T), dtype=np.float64)
    rhs[:, :n, :] = c0
    rhs[:, n, :] = 1.0
    sol = np.linalg.solve(K, rhs)
    return sol[:, :n, :], sol[:, n, :]


def drift_solve(C, c0, Q, q0):
    """Solve Appendix A's extended system [[C, Q], [Q^T, 0]] [w; phi] = [c0; q0]
    (LAPACK dgesv, batched). C [G][n][n], c0 [G][n][T], Q [G][n][p], q0 [G][p][T].
    Returns (w [G][n][T], phi [G][p][T])."""
    G, n, _ = C.shape
    p = Q.shape[2]
    T = c0.shape[2]
    K = np.zeros((G, n + p, n + p), dtype=np.float64)
    K[:, :n, :n] = C
    K[:, :n, n:] = Q
    K[:, n:, :n] = np.transpose(Q, (0, 2, 1))
    rhs = np.empty((G, n + p, T), dtype=np.float64)
    rhs[:, :n, :] = c0
    rhs[:, n:, :] = q0
    sol = np.linalg.solve(K, rhs)
    return sol[:, :n, :], sol[:, n:, :]


def krige_points(pts, vals, targets, model, nugget, sill, a):
    """Kriging of one system given explicit coordinates.

    pts [n][3], vals [n], targets [T][3] -> (est [T], var [T], w [n][T], mu [T]).
    """
    pts = np.asarray(pts, dtype=np.float64)
    targets = np.asarray(targets, dtype=np.float64)
    vals = np.asarray(vals, dtype=np.float64)
    d = np.linalg.norm(pts[:, None, :] - pts[None, :, :], axis=2)
    d0 = np.linalg.norm(pts[:, None, :] - targets[None, :, :], axis=2)
    C = covariance(model, nugget, sill, a, d)
    c0 = covariance(model, nugget, sill, a, d0)
    w, mu = bordered_solve(C[None], c0[None])
    w, mu = w[0], mu[0]
    est = vals @ w
    var = sill - np.einsum("nt,nt->t", w, c0) - mu
    return est, var, w, mu


def _systems(lo, hi, elo, ehi, ys, xs, f, targets_t, r, vario, min_points, chunk=8192,
             drift="none"):
    """Kriging of systems whose lower / upper slices are lo[i] / hi[i].

    lo, hi: float32 [S][H][W]; elo, ehi: uint8 [S][H][W] or None.
    targets_t: target heights above the lower slice (upper slice at f).
    drift: "none" (ordinary kriging) or "linear_z" (predictors 1 and slice).
    Returns (est [S][T], var [S][T], n [S], kept [S][2W^2]).
    """
    if drift not in ("none", "linear_z"):
        raise ValueError(drift)
    model, nug, sill, a = vario
    S = ys.shape[0]
    H, Wd = lo.shape[1], lo.shape[2]
    T = len(targets_t)
    cands = np.array(candidates(r), dtype=np.int64)          # (dx, dy, s)
    offs = np.stack([cands[:, 0], cands[:, 1], cands[:, 2] * f], axis=1).astype(np.float64)
    tgt = np.array([[0.0, 0.0, float(t)] for t in targets_t])
    est = np.empty((S, T)); var = np.empty((S, T))
    ns = np.empty(S, dtype=np.int64)
    kept_all = np.empty((S, len(cands)), dtype=bool)
    for c0_ in range(0, S, chunk):
        sl = slice(c0_, min(S, c0_ + chunk))
        yc, xc = ys[sl], xs[sl]
        ep = None if elo is None else (elo[sl], ehi[sl])
        kept, _ = select_neighbours(ep, yc, xc, r, min_points, (H, Wd))
        kept_all[sl] = kept
        n_sys = kept.sum(axis=1)
        ns[sl] = n_sys
        # values of every candidate (clipped for out-of-image; never used then)
        idx = np.arange(yc.shape[0])
        cv = np.empty((yc.shape[0], len(cands)), dtype=np.float64)
        for ci, (dx, dy, s) in enumerate(cands):
            src = lo[sl] if s == 0 else hi[sl]
            cv[:, ci] = src[idx, np.clip(yc + dy, 0, H - 1), np.clip(xc + dx, 0, Wd - 1)]
        for n in np.unique(n_sys):
            grp = np.nonzero(n_sys == n)[0]
            ci = np.nonzero(kept[grp])[1].reshape(len(grp), n)    # ascending per row
            P = offs[ci]                                          # [G][n][3]
            d = np.linalg.norm(P[:, :, None, :] - P[:, None, :, :], axis=3)
            d0 = np.linalg.norm(P[:, :, None, :] - tgt[None, None, :, :], axis=3)
            C = covariance(model, nug, sill, a, d)
            c0 = covariance(model, nug, sill, a, d0)
            w, mu = bordered_solve(C, c0)
            v = sill - np.einsum("gnt,gnt->gt", w, c0) - mu
            if drift == "linear_z":
                sl_pt = cands[ci][:, :, 2].astype(np.float64)        # 0 lower, 1 upper
                both = (sl_pt.min(axis=1) == 0) & (sl_pt.max(axis=1) == 1)
                if both.any():
                    b = np.nonzero(both)[0]
                    Q = np.stack([np.ones_like(sl_pt[b]), sl_pt[b]], axis=2)      # [G'][n][2]
                    q0 = np.stack([np.ones(T), np.asarray(targets_t, float) / f])  # [2][T]
                    q0 = np.broadcast_to(q0, (len(b), 2, T))
                    wd, ph = drift_solve(C[b], c0[b], Q, q0)
                    w = w.copy()
                    w[b] = wd
                    v[b] = sill - np.einsum("gnt,gnt->gt", wd, c0[b]) - np.einsum("gpt,gpt->gt", ph, q0)
            z = cv[grp[:, None], ci]                              # [G][n]
            est[c0_ + grp] = np.einsum("gn,gnt->gt", z, w)
            var[c0_ + grp] = v
    return est, var, ns, kept_all


def _vtuple(vario):
    if isinstance(vario, tuple):
        return vario
    return (vario.model, float(vario.nugget), float(vario.sill), float(vario.range))


def krige_volume(slices, edge, f: int, r: int, vario, min_points: int = 4,
                 gaps: Optional[Sequence[int]] = None, drift: str = "none"):
    """Reconstruct the volume [(n-1)f+1][H][W] and its kriging variance.

    Known slice s is copied to z = s*f with variance 0; every other voxel
    (x, y, g*f + t) is kriged from slices g and g+1. ``gaps`` restricts the
    kriging to some gaps (other kriged voxels are left NaN).
    Returns (volume, variance, n_per_system [n-1][H][W]).
    """
    vario = _vtuple(vario)
    slices = np.asarray(slices, dtype=np.float32)
    ns, H, Wd = slices.shape
    Z = (ns - 1) * f + 1
    vol = np.full((Z, H, Wd), np.nan, dtype=np.float64)
    var = np.full((Z, H, Wd), np.nan, dtype=np.float64)
    npts = np.zeros((ns - 1, H, Wd), dtype=np.int64)
    for s in range(ns):
        vol[s * f] = slices[s]
        var[s * f] = 0.0
    if f < 2:
        return vol, var, npts
    yy, xx = np.meshgrid(np.arange(H), np.arange(Wd), indexing="ij")
    ys, xs = yy.ravel(), xx.ravel()
    for g in (range(ns - 1) if gaps is None else gaps):
        S = ys.shape[0]
        lo = np.broadcast_to(slices[g], (S, H, Wd))
        hi = np.broadcast_to(slices[g + 1], (S, H, Wd))
        if edge is None:
            elo = ehi = None
        else:
            elo = np.broadcast_to(edge[g], (S, H, Wd))
            ehi = np.broadcast_to(edge[g + 1], (S, H, Wd))
        e, v, n, _ = _systems(lo, hi, elo, ehi, ys, xs, f, list(range(1, f)), r, vario, min_points,
                              drift=drift)
        for t in range(1, f):
            vol[g * f + t] = e[:, t - 1].reshape(H, Wd)
            var[g * f + t] = v[:, t - 1].reshape(H, Wd)
        npts[g] = n.reshape(H, Wd)
    return vol, var, npts


def krige_sample(slices, edge, f: int, r: int, vario, gs, ys, xs, min_points: int = 4,
                 drift: str = "none"):
    """Kriging of individual systems (g, y, x): (est [S][f-1], var [S][f-1],
    n [S], kept [S][2(2r+1)^2])."""
    vario = _vtuple(vario)
    slices = np.asarray(slices, dtype=np.float32)
    gs = np.asarray(gs, dtype=np.int64)
    ys = np.asarray(ys, dtype=np.int64)
    xs = np.asarray(xs, dtype=np.int64)
    _, H, Wd = slices.shape
    S = gs.shape[0]
    nc = 2 * (2 * r + 1) ** 2
    est = np.empty((S, f - 1)); var = np.empty((S, f - 1))
    ns = np.empty(S, dtype=np.int64)
    kept = np.empty((S, nc), dtype=bool)
    # one gap at a time, its two slices shared by every system of the gap
    for g in np.unique(gs):
        sel = np.nonzero(gs == g)[0]
        k = sel.shape[0]
        lo = np.broadcast_to(slices[g], (k, H, Wd))
        hi = np.broadcast_to(slices[g + 1], (k, H, Wd))
        if edge is None:
            elo = ehi = None
        else:
            elo = np.broadcast_to(edge[g], (k, H, Wd))
            ehi = np.broadcast_to(edge[g + 1], (k, H, Wd))
        e_, v_, n_, k_ = _systems(lo, hi, elo, ehi, ys[sel], xs[sel], f, list(range(1, f)), r,
                                  vario, min_points, drift=drift)
        est[sel], var[sel], ns[sel], kept[sel] = e_, v_, n_, k_
    return est, var, ns, kept


# ----------------------------------------------------------------------------
# Leave-one-slice-out loss and its gradient
# ----------------------------------------------------------------------------

def _loso_systems(slices, r, held):
    ns, H, Wd = slices.shape
    yy, xx = np.meshgrid(np.arange(H), np.arange(Wd), indexing="ij")
    ys = np.tile(yy.ravel(), len(held))
    xs = np.tile(xx.ravel(), len(held))
    hs = np.repeat(np.asarray(held, dtype=np.int64), H * Wd)
    return hs, ys, xs


def loso_loss(slices, r: int, vario, min_points: int = 4, edges=None, drift: str = "none"):
    """Mean over held-out slices s = 1..n-2 and all their voxels of
    (z_hat - z)^2, z_hat kriged from slices s-1 and s+1 (edge masks of those
    two slices when given; ordinary kriging or the slice predictor)."""
    vario = _vtuple(vario)
    slices = np.asarray(slices, dtype=np.float32)
    ns = slices.shape[0]
    hs, ys, xs = _loso_systems(slices, r, range(1, ns - 1))
    elo = ehi = None
    if edges is not None:
        edges = np.asarray(edges, dtype=np.uint8)
        elo, ehi = edges[hs - 1], edges[hs + 1]
    est, _, _, _ = _systems(slices[hs - 1], slices[hs + 1], elo, ehi, ys, xs, 2, [1], r, vario,
                            min_points, drift=drift)
    truth = slices[hs, ys, xs].astype(np.float64)
    return float(np.mean((est[:, 0] - truth) ** 2))


def loso_loss_grad(slices, r: int, vario, min_points: int = 4, chunk: int = 8192, edges=None,
                   drift: str = "none"):
    """Loss and its FP64 adjoint gradient d L / d(nugget, sill, range).

    Per system, with K the matrix of Appendix A's extended system (border Q:
    the constant predictor, with drift="linear_z" also the point's slice, 0
    lower and 1 upper; target row q0 = (1[, 1/2])) and lambda = [w; phi]:
    nu = K^{-1} [e z_nb; 0], e = 2 (z_hat - z) / N, and, since Q and q0 do
    not depend on the variogram,
    dL/dtheta = nu_w^T dc0/dtheta - nu_w^T (dC/dtheta) w.
    The centre column of both slices is always kept, so Q has full rank.
    """
    if drift not in ("none", "linear_z"):
        raise ValueError(drift)
    model, nug, sill, a = _vtuple(vario)
    slices = np.asarray(slices, dtype=np.float32)
    ns, H, Wd = slices.shape
    hs, ys, xs = _loso_systems(slices, r, range(1, ns - 1))
    N = hs.shape[0]
    cands = np.array(candidates(r), dtype=np.int64)
    offs = np.stack([cands[:, 0], cands[:, 1], cands[:, 2] * 2], axis=1).astype(np.float64)
    tgt = np.array([0.0, 0.0, 1.0])
    loss = 0.0
    grad = np.zeros(3)
    for c_ in range(0, N, chunk):
        sl = slice(c_, min(N, c_ + chunk))
        hc, yc, xc = hs[sl], ys[sl], xs[sl]
        ep = None
        if edges is not None:
            ep = (np.asarray(edges[hc - 1], dtype=np.uint8), np.asarray(edges[hc + 1], dtype=np.uint8))
        kept, _ = select_neighbours(ep, yc, xc, r, min_points, (H, Wd))
        n_sys = kept.sum(axis=1)
        for n in np.unique(n_sys):
            grp = np.nonzero(n_sys == n)[0]
            ci = np.nonzero(kept[grp])[1].reshape(len(grp), n)
            P = offs[ci]
            d = np.linalg.norm(P[:, :, None, :] - P[:, None, :, :], axis=3)
            d0 = np.linalg.norm(P - tgt[None, None, :], axis=2)
            C = covariance(model, nug, sill, a, d)
            c0 = covariance(model, nug, sill, a, d0)
            G = len(grp)
            dx_, dy_, s_ = cands[ci, 0], cands[ci, 1], cands[ci, 2]
            if drift == "none":
                Q = np.ones((G, n, 1))
                q0 = np.array([1.0])
            else:
                assert np.all(s_.min(axis=1) == 0) and np.all(s_.max(axis=1) == 1)
                Q = np.stack([np.ones((G, n)), s_.astype(np.float64)], axis=2)
                q0 = np.array([1.0, 0.5])
            p_ = Q.shape[2]
            K = np.zeros((G, n + p_, n + p_))
            K[:, :n, :n] = C
            K[:, :n, n:] = Q
            K[:, n:, :n] = np.transpose(Q, (0, 2, 1))
            rhs = np.zeros((G, n + p_))
            rhs[:, :n] = c0
            rhs[:, n:] = q0
            lam = np.linalg.solve(K, rhs[:, :, None])[:, :, 0]
            w = lam[:, :n]
            src_lo = slices[hc[grp] - 1]
            src_hi = slices[hc[grp] + 1]
            gi = np.arange(G)[:, None]
            yy = yc[grp][:, None] + dy_
            xx = xc[grp][:, None] + dx_
            z = np.where(s_ == 0, src_lo[gi, yy, xx], src_hi[gi, yy, xx]).astype(np.float64)
            est = np.einsum("gn,gn->g", z, w)
            truth = slices[hc[grp], yc[grp], xc[grp]].astype(np.float64)
            res = est - truth
            loss += float(np.sum(res ** 2))
            e = 2.0 * res / N
            adj_rhs = np.zeros((G, n + p_))
            adj_rhs[:, :n] = e[:, None] * z
            nu = np.linalg.solve(K, adj_rhs[:, :, None])[:, :, 0]
            nu_w = nu[:, :n]
            dC = covariance_derivatives(model, nug, sill, a, d)        # [3][G][n][n]
            dc0 = covariance_derivatives(model, nug, sill, a, d0)      # [3][G][n]
            grad += np.einsum("gn,kgn->k", nu_w, dc0)
            grad -= np.einsum("gi,kgij,gj->k", nu_w, dC, w)
    return loss / N, grad


def loso_fd_grad(slices, r: int, vario, h: float = 1e-4, min_points: int = 4, edges=None,
                 drift: str = "none"):
    """Central finite differences of loso_loss on raw (nugget, sill, range)."""
    model, nug, sill, a = _vtuple(vario)
    th = np.array([nug, sill, a], dtype=np.float64)
    g = np.zeros(3)
    for k in range(3):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        lp = loso_loss(slices, r, (model, *tp), min_points, edges, drift)
        lm = loso_loss(slices, r, (model, *tm), min_points, edges, drift)
        g[k] = (lp - lm) / (2 * h)
    return g


def adam_fit(loss_grad, theta0, steps: int = 200, lr: float = 0.05,
             betas=(0.9, 0.999), eps: float = 1e-8):
    """Adam (Kingma & Ba 2015) on u = log(theta); loss_grad(theta) returns
    (loss, dL/dtheta). Returns the trajectory [(loss, theta)], one entry per
    evaluated point, the last being the final parameters."""
    u = np.log(np.asarray(theta0, dtype=np.float64))
    m = np.zeros_like(u)
    v = np.zeros_like(u)
    traj = []
    for k in range(1, steps + 1):
        th = np.exp(u)
        L, g = loss_grad(th)
        traj.append((L, th.copy()))
        gu = g * th
        m = betas[0] * m + (1 - betas[0]) * gu
        v = betas[1] * v + (1 - betas[1]) * gu * gu
        mh = m / (1 - betas[0] ** k)
        vh = v / (1 - betas[1] ** k)
        u = u - lr * mh / (np.sqrt(vh) + eps)
    th = np.exp(u)
    L, _ = loss_grad(th)
    traj.append((L, th.copy()))
    return traj


def window_condition(model, nugget, sill, a, r: int, f: int) -> float:
    """2-norm condition number of the full-window covariance matrix; every
    system's matrix is a principal submatrix, so by Cauchy interlacing its
    condition number is bounded by this value."""
    cands = np.array(candidates(r), dtype=np.float64)
    P = np.stack([cands[:, 0], cands[:, 1], cands[:, 2] * f], axis=1)
    d = np.linalg.norm(P[:, None, :] - P[None, :, :], axis=2)
    C = covariance(model, nugget, sill, a, d)
    ev = np.linalg.eigvalsh(C)
    return float(ev[-1] / ev[0])

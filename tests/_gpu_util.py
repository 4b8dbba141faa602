"""Helpers shared by the GPU tests: run the library through its binding and
compare with the oracle under the error metric of the parity bar."""
import numpy as np


def rel_err_est(est, ref, zmax):
    """|z_hat - z*| / max(|z*|, 0.01 Zmax) per voxel."""
    return np.abs(est.astype(np.float64) - ref) / np.maximum(np.abs(ref), 0.01 * zmax)


def rel_err_var(var, ref, sill):
    return np.abs(var.astype(np.float64) - ref) / sill


def canonical_bits(kept):
    """Oracle kept masks [S][ncand] -> (lo, hi) uint64 words."""
    S, nc = kept.shape
    lo = np.zeros(S, dtype=np.uint64)
    hi = np.zeros(S, dtype=np.uint64)
    for c in range(nc):
        col = kept[:, c].astype(np.uint64)
        if c < 64:
            lo |= col << np.uint64(c)
        else:
            hi |= col << np.uint64(c - 64)
    return lo, hi


def run_gpu(slices, edge, f, r, vario, precision="fp32", algo="batched", min_points=4,
            flags=False, **plan_kw):
    import torch
    import paper_2303_09523_amd as P
    n, ny, nx = slices.shape
    st = torch.from_numpy(np.ascontiguousarray(slices)).cuda()
    et = torch.from_numpy(np.ascontiguousarray(edge)).cuda() if edge is not None else None
    plan = P.Plan(nx, ny, n, f, r, min_points, precision, algo, **plan_kw)
    vol, var, fl = plan.execute(st, vario, et, want_flags=flags)
    stats = plan.stats()
    out = (vol.cpu().numpy(), var.cpu().numpy(), None if fl is None else fl.cpu().numpy(), stats)
    plan.close()
    return out

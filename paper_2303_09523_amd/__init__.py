"""MI355X edge-preserved ordinary kriging along Z.

Fills the missing voxels between known 2D slices (Section 4.1 of the paper):
known slices are placed into the output volume and every missing voxel is
kriged from its edge-masked neighbourhood in the two adjacent known slices.
All computation happens in the HIP library (libokrig.so, C ABI in
include/okrig.h); this module only marshals torch device tensors and the
current HIP stream into those calls.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

from . import _lib
from ._lib import OkrError, load  # noqa: F401

__all__ = ["Plan", "krige", "select", "execute_noalloc", "OkrError", "load", "LosoLoss"]


def _torch():
    import torch
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _vario(model, nugget, sill, rng):
    m = _lib.MODELS[model] if isinstance(model, str) else int(model)
    return _lib.Variogram(m, float(nugget), float(sill), float(rng))


def _as_vario(v):
    if isinstance(v, _lib.Variogram):
        return v
    if isinstance(v, (tuple, list)):
        return _vario(*v)
    return _vario(v.model, v.nugget, v.sill, v.range)


def edge_filters():
    """The edge post-pass's filters as the library evaluates them (host only):
    (taps float64 [8][9][9] indexed [k][d2 + 4][d1 + 4], normals int32 [8][2]
    as (d1, d2))."""
    import numpy as np
    taps = np.zeros((8, 9, 9), dtype=np.float64)
    normals = np.zeros((8, 2), dtype=np.int32)
    _lib.check(load().okr_edge_filters(taps.ctypes.data_as(C.c_void_p),
                                       normals.ctypes.data_as(C.c_void_p)), None)
    return taps, normals


class Plan:
    """One problem shape: workspace and launch state owned by the library."""

    def __init__(self, nx: int, ny: int, nslices: int, upsample: int, radius: int,
                 min_points: int = 4, precision: str = "fp32", algo: str = "batched",
                 refine_tol: float = 0.0, refine_max: int = 1, strict: bool = False,
                 stream=None, drift: str = "none"):
        torch = _torch()
        lib = load()
        self.shape = (nslices, ny, nx)
        self.upsample = upsample
        self.radius = radius
        drifts = {"none": 0, "linear_z": 1}
        prob = _lib.Problem(nx, ny, nslices, upsample, radius, min_points,
                            _lib.PRECISIONS[precision], _lib.ALGOS[algo], refine_tol, refine_max,
                            int(strict), drifts[drift] if isinstance(drift, str) else int(drift))
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        _lib.check(lib.okr_plan_create(C.byref(prob), C.c_void_p(stream.cuda_stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load().okr_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_in(self, t, dtype, shape, name):
        torch = _torch()
        if t is None:
            return
        if not (t.is_cuda and t.dtype == dtype and tuple(t.shape) == tuple(shape)
                and t.is_contiguous()):
            raise ValueError(f"{name}: expected contiguous {dtype} {tuple(shape)} on the GPU, got "
                             f"{t.dtype} {tuple(t.shape)} on {t.device}")
        del torch

    def out_shape(self):
        n, ny, nx = self.shape
        return ((n - 1) * self.upsample + 1, ny, nx)

    def execute(self, slices, vario, edge=None, volume=None, variance=None, flags=None,
                want_variance: bool = True, want_flags: bool = False):
        """Reconstruct the volume; returns (volume, variance or None, flags or None)."""
        torch = _torch()
        self._check_in(slices, torch.float32, self.shape, "slices")
        if edge is not None:
            self._check_in(edge, torch.uint8, self.shape, "edge")
        dev = slices.device
        if volume is None:
            volume = torch.empty(self.out_shape(), dtype=torch.float32, device=dev)
        if variance is None and want_variance:
            variance = torch.empty(self.out_shape(), dtype=torch.float32, device=dev)
        if flags is None and want_flags:
            n, ny, nx = self.shape
            flags = torch.empty((max(n - 1, 0), ny, nx), dtype=torch.uint8, device=dev)
        v = _as_vario(vario)
        _lib.check(load().okr_execute(self._h, C.byref(v), _ptr(slices), _ptr(edge),
                                      _ptr(volume), _ptr(variance), _ptr(flags)), self._h)
        return volume, variance, flags

    def set_graph(self, enable: bool = True):
        """Replay okr_execute from a captured HIP graph (see okr_plan_set_graph)."""
        _lib.check(load().okr_plan_set_graph(self._h, int(bool(enable))), self._h)

    def autotune(self, slices, vario, edge=None, volume=None, variance=None) -> dict:
        """Pick the fastest launch shape on these inputs (okr_plan_autotune)."""
        torch = _torch()
        self._check_in(slices, torch.float32, self.shape, "slices")
        if edge is not None:
            self._check_in(edge, torch.uint8, self.shape, "edge")
        dev = slices.device
        if volume is None:
            volume = torch.empty(self.out_shape(), dtype=torch.float32, device=dev)
        v = _as_vario(vario)
        _lib.check(load().okr_plan_autotune(self._h, C.byref(v), _ptr(slices), _ptr(edge),
                                            _ptr(volume), _ptr(variance)), self._h)
        return self.tuning()

    def tuning(self) -> dict:
        g, u, fc = C.c_int32(), C.c_int32(), C.c_int32()
        ms = (C.c_double * 8)()
        _lib.check(load().okr_plan_get_tuning(self._h, C.byref(g), C.byref(u), ms, C.byref(fc)),
                   self._h)
        return {"grid_per_cu": g.value, "update_arith": u.value, "candidate_ms": list(ms),
                "from_cache": bool(fc.value)}

    def krige_points(self, count, offset, xyz, val, target_xyz, vario, want_weights=False):
        """FP64 ordinary kriging of explicit point sets (okr_krige_points).

        count int32 [S], offset int64 [S] (CSR), xyz float32 [T][3], val float32
        [T], target_xyz float32 [S][3]; returns (est [S], var [S], weights [T] or
        None), all CUDA float32."""
        torch = _torch()
        S = int(count.numel())
        for t, dt, nm in ((count, torch.int32, "count"), (offset, torch.int64, "offset"),
                          (xyz, torch.float32, "xyz"), (val, torch.float32, "val"),
                          (target_xyz, torch.float32, "target_xyz")):
            if not t.is_cuda or t.dtype != dt or not t.is_contiguous():
                raise ValueError(f"{nm} must be a contiguous CUDA {dt} tensor")
        est = torch.empty(S, dtype=torch.float32, device=count.device)
        var = torch.empty(S, dtype=torch.float32, device=count.device)
        w = torch.empty(val.numel(), dtype=torch.float32, device=count.device) if want_weights \
            else None
        v = _as_vario(vario)
        _lib.check(load().okr_krige_points(self._h, C.byref(v), S, _ptr(count), _ptr(offset),
                                           _ptr(xyz), _ptr(val), _ptr(target_xyz), _ptr(est),
                                           _ptr(var), _ptr(w)), self._h)
        return est, var, w

    def marching_cubes(self, volume, iso, max_tris=None, want_ids=True):
        """Triangles of the iso-surface of a volume of the plan's output shape
        (okr_marching_cubes): float32 [T][3][3] vertex coordinates (x, y, z)
        and, with want_ids, int64 [T] cube indices, both CUDA tensors. With
        max_tris None the triangles are counted first and the buffers sized
        to fit."""
        torch = _torch()
        self._check_in(volume, torch.float32, self.out_shape(), "volume")
        lib = load()
        n = C.c_int64(0)
        if max_tris is None:
            _lib.check(lib.okr_marching_cubes(self._h, _ptr(volume), C.c_float(iso), None, None,
                                              0, C.byref(n)), self._h)
            max_tris = n.value
        tris = torch.empty((max(int(max_tris), 0), 3, 3), dtype=torch.float32,
                           device=volume.device)
        ids = torch.empty((tris.shape[0],), dtype=torch.int64, device=volume.device) \
            if want_ids else None
        if tris.shape[0] > 0:
            _lib.check(lib.okr_marching_cubes(self._h, _ptr(volume), C.c_float(iso), _ptr(tris),
                                              _ptr(ids), tris.shape[0], C.byref(n)), self._h)
        T = min(n.value, tris.shape[0])
        return tris[:T], (ids[:T] if ids is not None else None)

    def edge_postpass(self, volume, tau, out=None, edge=None, orient=None, mag=None):
        """The edge post-pass (okr_edge_postpass) on a float32 volume of the
        plan's output shape: returns (out, edge, orient) CUDA tensors, the
        adjusted volume (float32; pass out=volume for an in-place pass), the
        edge map and the orientation map (uint8) after the pass; with a
        float64 tensor `mag` the coefficient magnitude M is written too."""
        torch = _torch()
        shape = self.out_shape()
        self._check_in(volume, torch.float32, shape, "volume")
        if out is None:
            out = torch.empty_like(volume)
        if edge is None:
            edge = torch.empty(shape, dtype=torch.uint8, device=volume.device)
        if orient is None:
            orient = torch.empty(shape, dtype=torch.uint8, device=volume.device)
        self._check_in(out, torch.float32, shape, "out")
        self._check_in(edge, torch.uint8, shape, "edge")
        self._check_in(orient, torch.uint8, shape, "orient")
        if mag is not None:
            self._check_in(mag, torch.float64, shape, "mag")
        _lib.check(load().okr_edge_postpass(self._h, _ptr(volume), _ptr(out), C.c_double(tau),
                                            _ptr(edge), _ptr(orient), _ptr(mag)), self._h)
        return out, edge, orient

    def select(self, edge=None):
        """Kept-candidate bitmasks [(n-1)*ny*nx][2] (int64 view of uint64) and counts."""
        torch = _torch()
        n, ny, nx = self.shape
        if edge is not None:
            self._check_in(edge, torch.uint8, self.shape, "edge")
        nsys = max(n - 1, 0) * ny * nx
        bits = torch.empty((nsys, 2), dtype=torch.int64, device="cuda")
        count = torch.empty((nsys,), dtype=torch.uint8, device="cuda")
        _lib.check(load().okr_select(self._h, _ptr(edge), _ptr(bits), _ptr(count)), self._h)
        return bits, count

    def loso_forward(self, slices, vario, edge=None, loss=None):
        torch = _torch()
        self._check_in(slices, torch.float32, self.shape, "slices")
        if loss is None:
            loss = torch.empty((), dtype=torch.float64, device=slices.device)
        v = _as_vario(vario)
        _lib.check(load().okr_loso_forward(self._h, C.byref(v), _ptr(slices), _ptr(edge),
                                           _ptr(loss)), self._h)
        self.loso_token = getattr(self, "loso_token", 0) + 1
        return loss

    def loso_backward(self, grad=None):
        torch = _torch()
        if grad is None:
            grad = torch.empty((3,), dtype=torch.float64, device="cuda")
        _lib.check(load().okr_loso_backward(self._h, _ptr(grad)), self._h)
        return grad

    def stats(self) -> dict:
        s = _lib.Stats()
        _lib.check(load().okr_stats_get(self._h, C.byref(s)), self._h)
        return {"n_systems": s.n_systems, "n_kriged": s.n_kriged, "bucket": list(s.bucket),
                "n_floor_filled": s.n_floor_filled, "n_refined": s.n_refined,
                "n_fp64_fallback": s.n_fp64_fallback,
                "n_nonpositive_pivot": s.n_nonpositive_pivot, "max_kappa_est": s.max_kappa_est,
                "n_not_converged": s.n_not_converged,
                "n_refine_unconverged": s.n_refine_unconverged, "kappa_window": s.kappa_window,
                "direct_fp64": bool(s.direct_fp64),
                "phase_ms": dict(zip(_lib.PHASES, list(s.phase_ms))),
                "phase_calls": dict(zip(_lib.PHASES, list(s.phase_calls)))}

    def set_profiling(self, enable: bool = True):
        _lib.check(load().okr_plan_set_profiling(self._h, int(enable)), self._h)


def krige(slices, vario, upsample: int, radius: int, edge=None, min_points: int = 4,
          precision: str = "fp32", algo: str = "batched", want_variance: bool = True):
    """One-shot reconstruction: (volume, variance) as CUDA tensors."""
    n, ny, nx = slices.shape
    plan = Plan(nx, ny, n, upsample, radius, min_points, precision, algo)
    vol, var, _ = plan.execute(slices, vario, edge, want_variance=want_variance)
    plan.close()
    return vol, var


def execute_noalloc(slices, vario, upsample: int, radius: int, volume, variance=None, edge=None,
                    flags=None, status=None, min_points: int = 4, precision: str = "fp32",
                    algo: str = "batched", refine_tol: float = 0.0, refine_max: int = 1,
                    strict: bool = False, drift: str = "none", stream=None):
    """okr_execute_noalloc: one reconstruction into caller tensors with the
    library's static workspace (no plan, no device allocation). status, if
    given, is a CUDA int32 tensor of one element that receives the
    device-detected status."""
    torch = _torch()
    n, ny, nx = slices.shape
    drifts = {"none": 0, "linear_z": 1}
    prob = _lib.Problem(nx, ny, n, upsample, radius, min_points, _lib.PRECISIONS[precision],
                        _lib.ALGOS[algo], refine_tol, refine_max, int(strict),
                        drifts[drift] if isinstance(drift, str) else int(drift))
    if stream is None:
        stream = torch.cuda.current_stream()
    v = _as_vario(vario)
    _lib.check(load().okr_execute_noalloc(C.byref(prob), C.c_void_p(stream.cuda_stream),
                                          C.byref(v), _ptr(slices), _ptr(edge), _ptr(volume),
                                          _ptr(variance), _ptr(flags), _ptr(status)))


def select(edge, nslices, ny, nx, radius, min_points=4):
    plan = Plan(nx, ny, nslices, 2, radius, min_points)
    out = plan.select(edge)
    plan.close()
    return out


def __getattr__(name):
    if name == "LosoLoss":
        from .autograd import LosoLoss
        return LosoLoss
    raise AttributeError(name)

"""Benchmark: kriged voxels/s of the batched edge-preserved kriging path.

One step = one okr_execute over the whole synthetic volume: placement, table
build, neighbour selection, size bucketing and the batched solve (one
persistent launch per 16-wide size class, largest first) plus the FP64 re-solve
launch. The default is the metric's operating point on the large volume: the
mixed_fp16 path (split-FP16 MFMA trailing updates with FP32 accumulation, FP32
diagonal tiles) with the FP64-residual correction of every system's estimate
and precision control at a per-voxel tolerance of 1e-5 (systems the bound
cannot certify are re-solved in FP64). Inputs are resident in HBM before
timing starts; the launch shape comes from the library's autotuner and the
timed steps replay the library's HIP graph of okr_execute.

Prints ONE JSON line. Extra keys:
  roofline          dominant kernel (the solve launches of one step):
                    algorithmic FLOP / mean time from the library's HIP events
                    over the same number of direct (non-graph) steps, against
                    the peak of the contraction's own instruction (FP16 MFMA
                    for split products), with the FP32-equivalent fraction, an
                    additive MFMA + vector-ALU bound, MFMA busy fraction and
                    HBM traffic from the committed counter summaries while the
                    kernel sources are unchanged
  cpu_baseline      the FP64 oracle on a bounded random sample of the same
                    systems, one worker and one worker per core of this host
  accuracy          the headline result vs the oracle on that sample
  batched_variants  the other operating points (read-out only, FP64, FP32),
                    each with its accuracy on the same sample
  next_rows         pattern_cache (full-window stencil and window-inverse
                    solves), marching_cubes and
                    edge_postpass, below
  plain_fp32        the per-voxel comparison kernel (FP32 with its FP64-residual
                    refinement step, at the same per-voxel 1e-5 bar), on a slab
  other_configs     the small and the edge-preserved workloads: batched FP32,
                    refined mixed and the refined plain per-voxel kernel
  precision_study   the ill-conditioned Gaussian workload in every precision
                    mode, with routing counts and per-voxel errors
  loso              leave-one-slice-out loss + adjoint gradient timing on the
                    16 x 128^2 field workload
  marching_cubes    the iso-surface of the reconstructed volume
  edge_postpass     the paper's edge post-pass on the reconstructed volume:
                    per-kernel times and the shearlet kernel's FP64 roofline
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published dense peaks (MFMA; the FP32 / FP64 vector peaks are the same)
    "fp32_tflops": 157.3, "fp64_tflops": 78.6, "fp16_tflops": 2500.0, "hbm_gbs": 8000.0,
}
# Peak of the instruction the trailing updates issue, and MFMA products per
# algorithmic product (split halves: hi*hi + hi*lo + lo*hi).
CONTRACTION = {"fp32": ("fp32_tflops", 1), "fp64": ("fp64_tflops", 1),
               "mixed_fp16": ("fp16_tflops", 3), "mixed_bf16": ("fp16_tflops", 3)}


def system_flops(n, f):
    """Algorithmic FLOP of one (column, gap) system: Cholesky of the n x n
    covariance (n^3/3), solves of its f+1 border columns ((f+1) n^2) and the
    read-out of f-1 targets."""
    return n ** 3 / 3.0 + (f + 1) * n * n + 8.0 * (f - 1) * n


def diag_flops(n, nb):
    """The part of system_flops done inside the 16 x 16 diagonal tiles (one
    Cholesky of 16^3/3 per block of the augmented matrix), which runs on the
    vector ALUs; the rest is MFMA work."""
    return ((n + nb + 15) // 16) * 16.0 ** 3 / 3.0


# Inputs of the oracle workers: set before the pool forks, so the workers
# share them without copies.
_CPU = {}


def _oracle_chunk(args):
    import oracle as O
    g, y, x = args
    s, e, f, r, vario = _CPU["inputs"]
    est, var, n, _ = O.krige_sample(s, e, f, r, vario, g, y, x)
    return est, var


def _full_oracle(w, s, e):
    """Every system of a small workload, in the sample format of cpu_baseline."""
    import numpy as np
    import oracle as O
    vario = (w.vario.model, w.vario.nugget, w.vario.sill, w.vario.range)
    idx = np.arange(w.systems)
    plane = w.m * w.m
    est, var, _, _ = O.krige_sample(s, e, w.upsample, w.radius, vario, idx // plane,
                                    (idx % plane) // w.m, idx % w.m)
    return idx, est, var


def _sample_accuracy(w, s, sample, vol_t, var_t):
    """Per-voxel and normwise errors of a volume against an oracle sample."""
    import numpy as np
    import torch
    if sample is None:
        return None
    idx, est_o, var_o = sample
    plane = w.m * w.m
    g, p = idx // plane, idx % plane
    zs = g[:, None] * w.upsample + np.arange(1, w.upsample)[None, :]
    yy, xx = (p // w.m)[:, None], (p % w.m)[:, None]
    dev = vol_t.device
    zt = torch.from_numpy(zs).to(dev)
    yt = torch.from_numpy(np.broadcast_to(yy, zs.shape).copy()).to(dev)
    xt = torch.from_numpy(np.broadcast_to(xx, zs.shape).copy()).to(dev)
    ge = vol_t[zt, yt, xt].double().cpu().numpy()
    out = {"voxels": int(ge.size)}
    zmax = float(np.abs(s).max())
    ee = np.abs(ge - est_o) / np.maximum(np.abs(est_o), 0.01 * zmax)
    out.update({"max_rel_err_est": float(ee.max()),
                "p9999_rel_err_est": float(np.percentile(ee, 99.99)),
                "normwise_est": float(np.abs(ge - est_o).max() / np.abs(est_o).max())})
    if var_t is not None:
        gv = var_t[zt, yt, xt].double().cpu().numpy()
        out["max_rel_err_var"] = float((np.abs(gv - var_o) / w.vario.sill).max())
    return out


def _time_executes(plan, st, vario, et, vol, var, reps):
    """Median and minimum of `reps` timed executes (HIP events on the plan's
    stream, after one warm-up)."""
    import torch
    plan.execute(st, vario, et, volume=vol, variance=var)
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record()
        plan.execute(st, vario, et, volume=vol, variance=var)
        a1.record()
        torch.cuda.synchronize()
        ts.append(a0.elapsed_time(a1))
    ts.sort()
    return ts[len(ts) // 2], ts[0]


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, s, e, target_s: float, seed: int = 12345):
    """The FP64 oracle on a random sample of systems: one worker, then a
    process pool with one worker per core of this process's affinity set (BLAS
    threads pinned to one per worker). Only the solves are timed."""
    import multiprocessing as mp
    import numpy as np
    # one worker per core of this process's affinity set, within the host share
    # the launcher grants (MAX_JOBS, when it sets one)
    affinity = len(os.sched_getaffinity(0))
    share = int(os.environ.get("MAX_JOBS", affinity))
    cores = max(1, min(affinity, share))
    rng = np.random.default_rng(seed)
    vario = (w.vario.model, w.vario.nugget, w.vario.sill, w.vario.range)
    plane = w.m * w.m
    _CPU["inputs"] = (s, e, w.upsample, w.radius, vario)
    # one worker: calibration sample, timed in this process
    cal = rng.choice(w.systems, 600, replace=False)
    _oracle_chunk((cal[:20] // plane, (cal[:20] % plane) // w.m, cal[:20] % w.m))
    t0 = time.perf_counter()
    _oracle_chunk((cal // plane, (cal % plane) // w.m, cal % w.m))
    one = (time.perf_counter() - t0) / len(cal)
    nsamp = int(min(max(target_s * cores / one, 2000), 400000))
    idx = np.sort(rng.choice(w.systems, nsamp, replace=False))
    chunk = max(200, nsamp // (cores * 4))
    jobs = [(sl // plane, (sl % plane) // w.m, sl % w.m)
            for sl in (idx[a:a + chunk] for a in range(0, nsamp, chunk))]
    ctx = mp.get_context("fork")   # no GPU is initialised in this process yet
    with ctx.Pool(cores) as pool:
        pool.map(_oracle_chunk, jobs[:cores])   # warm the workers
        t0 = time.perf_counter()
        res = pool.map(_oracle_chunk, jobs)
        wall = time.perf_counter() - t0
    est = np.concatenate([r[0] for r in res])
    var = np.concatenate([r[1] for r in res])
    vox = nsamp * (w.upsample - 1)
    value = vox / wall
    one_value = (w.upsample - 1) / one
    return {"value": value, "unit": "voxels/s", "cores": cores, "kind": "oracle",
            "cpu_model": _cpu_model(), "affinity_cores": affinity, "host_share": share,
            "sample": f"{nsamp} random (column, gap) systems of {w.name} "
                      f"({vox} kriged voxels), FP64 NumPy/LAPACK, {cores} processes "
                      f"(one BLAS thread each), {wall:.1f} s of solves",
            "one_worker_value": one_value,
            "time_reduction_vs_one_worker": 1.0 - one_value / value}, (idx, est, var)


def edge_cpu_baseline(vol, tau: float, target_s: float):
    """The edge post-pass oracle on whole YZ images of the volume (each image
    is independent), in this process, until about target_s seconds."""
    from oracle import edgepass as EP
    nz, ny, nx = vol.shape
    order = [(i * 97) % nx for i in range(nx)]
    done, t0 = 0, time.perf_counter()
    for x in order:
        EP.edge_postpass_image(vol[:, :, x], tau)
        done += 1
        if time.perf_counter() - t0 >= target_s:
            break
    wall = time.perf_counter() - t0
    return {"value": done * nz * ny / wall, "unit": "voxels/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} whole YZ images ({nz}x{ny}) of the reconstructed volume, "
                      f"FP64 NumPy + Python loops, one process, {wall:.1f} s"}


def edge_postpass_record(w, vol, args, reps: int = 5):
    """The paper's edge post-pass on the reconstructed volume: per-kernel
    times from the library's HIP events, the shearlet kernel's FP64 roofline
    and, unless --no-cpu, the oracle on whole sampled images."""
    import numpy as np
    import torch
    import workloads as W
    import paper_2303_09523_amd as P
    pe = P.Plan(w.m, w.m, w.nslices, w.upsample, w.radius, 4, args.precision, "batched",
                refine_max=args.refine_max)
    eout = torch.empty_like(vol)
    emap = torch.empty(vol.shape, dtype=torch.uint8, device=vol.device)
    omap = torch.empty_like(emap)
    pe.edge_postpass(vol, W.EDGE_TAU, out=eout, edge=emap, orient=omap)
    pe.set_profiling(True)
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    for _ in range(reps):
        pe.edge_postpass(vol, W.EDGE_TAU, out=eout, edge=emap, orient=omap)
    torch.cuda.synchronize()
    e_wall = (time.perf_counter() - e0) / reps * 1e3
    se = pe.stats()
    pe.close()
    eph = {k: se["phase_ms"][k] / max(1, se["phase_calls"][k])
           for k in ("edge_shear", "edge_thin", "edge_trace")}
    e_ms = sum(eph.values())
    nvox = int(vol.numel())
    # one product and one sum per nonzero tap of the eight filters
    edge_fpv = 2 * int(np.count_nonzero(P.edge_filters()[0]))
    sflops = edge_fpv * nvox
    rec = {
        "value": nvox / (e_ms * 1e-3), "unit": "voxels/s", "ms": round(e_ms, 4),
        "wall_ms": round(e_wall, 4), "voxels": nvox, "tau": W.EDGE_TAU,
        "edge_fraction": round(float(emap.float().mean().item()), 5),
        "voxels_changed": int((eout != vol).sum().item()),
        "phase_ms": {k: round(v, 4) for k, v in eph.items()},
        "timing": "library HIP events around each of the three launches",
        "roofline_shear": {
            "bound": "alu", "achieved": round(sflops / (eph["edge_shear"] * 1e-3) / 1e12, 3),
            "peak": PEAKS["fp64_tflops"], "unit": "TFLOP/s",
            "frac": round(sflops / (eph["edge_shear"] * 1e-3) / 1e12 / PEAKS["fp64_tflops"], 4),
            "flops_per_voxel": edge_fpv,
            # HBM bytes of one launch (committed counter summary, same sources)
            "traffic": _counter_summary(f"traffic_edge_shear_{w.name}.txt", EDGE_TRAFFIC_SOURCES,
                                        "shear_hbm_bytes_per_call"),
            "algorithmic_bytes": 14 * nvox}}
    if not args.no_cpu:
        rec["cpu_baseline"] = edge_cpu_baseline(vol.cpu().numpy(), W.EDGE_TAU,
                                                min(10.0, args.cpu_seconds))
    del eout, emap, omap
    print(f"# edge post-pass: {e_ms:.3f} ms ({eph})", file=sys.stderr, flush=True)
    return rec


def downdate_floor(ncand, nb, max_drop=32):
    """Smallest neighbour count the weight cache serves from the full
    window's inverse (whole 16-wide size classes 16 (NB - 1) - nb < n <=
    16 NB - nb that drop at most max_drop candidates); ncand when none."""
    for NB in range(1, 9):
        lo = max(1, 16 * (NB - 1) - nb + 1)
        if ncand - max_drop <= lo <= ncand - 1:
            return lo
    return ncand


def mcubes_record(w, s, vol, args, reps: int = 5):
    """Marching cubes of the reconstructed volume at the median of the known
    slices: library HIP-event time per call and the HBM roofline."""
    import numpy as np
    import paper_2303_09523_amd as P
    pm = P.Plan(w.m, w.m, w.nslices, w.upsample, w.radius, 4, args.precision, "batched",
                refine_max=args.refine_max)
    iso = float(np.median(s))
    tris, ids = pm.marching_cubes(vol, iso)
    ntri = int(tris.shape[0])
    pm.set_profiling(True)
    for _ in range(reps):
        pm.marching_cubes(vol, iso, max_tris=ntri)
    smc = pm.stats()
    pm.close()
    mesh_ms = smc["phase_ms"]["mesh"] / max(1, smc["phase_calls"]["mesh"])
    nz, ny, nx = vol.shape
    ncubes = (nz - 1) * (ny - 1) * (nx - 1)
    # algorithmic bytes: the volume read once, each triangle's vertices and cube id written
    mbytes = 4.0 * nz * ny * nx + 44.0 * ntri
    del tris, ids
    print(f"# marching cubes: {mesh_ms:.3f} ms, {ntri} triangles", file=sys.stderr, flush=True)
    return {
        "value": ncubes / (mesh_ms * 1e-3), "unit": "cubes/s", "ms": round(mesh_ms, 4),
        "cubes": ncubes, "triangles": ntri, "iso": iso,
        "timing": "library HIP events around the count, scan and emit launches",
        "roofline": {
            "bound": "hbm", "achieved": round(mbytes / (mesh_ms * 1e-3) / 1e9, 2),
            "peak": PEAKS["hbm_gbs"], "unit": "GB/s",
            "frac": round(mbytes / (mesh_ms * 1e-3) / 1e9 / PEAKS["hbm_gbs"], 5),
            "traffic": mesh_traffic_from_profiles(args.workload)}}


def _calibration_copy(nbytes):
    """A plain device copy of nbytes, whose FETCH_SIZE / WRITE_SIZE scale the
    counters of the kernels of the same run."""
    import torch
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    return {"copy_bytes": int(src.numel() * 4)}


def loso_record(reps: int = 3):
    """Leave-one-slice-out loss and adjoint gradient on the 16 x 128^2 field:
    times from CUDA events over `reps` calls each, and the forward's roofline
    (algorithmic FLOP of its systems, one held-out target each, against the
    FP32 MFMA peak of its trailing updates)."""
    import numpy as np
    import torch
    import workloads as W
    import paper_2303_09523_amd as P
    wl = W.workload("loso_16x128")
    sl_, _ = W.make_inputs(wl)
    slt = torch.from_numpy(sl_).cuda()
    pl = P.Plan(wl.m, wl.m, wl.nslices, 2, wl.radius, 4)
    th = ("exponential", 0.1, 1.0, 2.0)
    pl.loso_forward(slt, th)
    pl.loso_backward()
    hist = np.array(pl.stats()["bucket"], dtype=np.float64)
    torch.cuda.synchronize()
    c0 = torch.cuda.Event(enable_timing=True)
    c1 = torch.cuda.Event(enable_timing=True)
    c2 = torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(reps):
        pl.loso_forward(slt, th)
    c1.record()
    for _ in range(reps):
        pl.loso_backward()
    c2.record()
    torch.cuda.synchronize()
    fms, bms = c0.elapsed_time(c1) / reps, c1.elapsed_time(c2) / reps
    pl.close()
    nvox = (wl.nslices - 2) * wl.m * wl.m
    nn = np.arange(len(hist), dtype=np.float64)
    flops = float((hist * system_flops(nn, 2)).sum())
    return {"workload": wl.name, "held_out_voxels": nvox, "forward_ms": round(fms, 3),
            "backward_ms": round(bms, 3),
            "loss_grad_evals_per_s": round(1000.0 / (fms + bms), 2),
            "roofline_forward": {
                "bound": "mfma", "achieved": round(flops / (fms * 1e-3) / 1e12, 3),
                "peak": PEAKS["fp32_tflops"], "unit": "TFLOP/s",
                "frac": round(flops / (fms * 1e-3) / 1e12 / PEAKS["fp32_tflops"], 5),
                "flop": flops, "traffic": None}}


TRAFFIC_SOURCES = ["okrig_internal.h", "solver_core.h", "solver_refine.h", "kernels_solve.hip",
                   "kernels_mixed.hip"]


MESH_TRAFFIC_SOURCES = ["okrig_internal.h", "kernels_mcubes.hip"]
EDGE_TRAFFIC_SOURCES = ["edge_internal.h", "edge_filters.h", "kernels_edge.hip"]


def _source_hash(names) -> str:
    import hashlib
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2303_09523_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_source_hash() -> str:
    return _source_hash(TRAFFIC_SOURCES)


def _counter_summary(name, sources, key):
    """A value of a committed counter summary under profiles/, or None when
    the file is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != _source_hash(sources):
        return None
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


def mfma_busy_from_profiles(args):
    """MFMA busy fraction of the dominant solve kernel from the committed SQ
    counter summary (SQ_VALU_MFMA_BUSY_CYCLES / (4 SIMDs x SQ_BUSY_CU_CYCLES))."""
    return _counter_summary(f"sq_{args.workload}_{args.precision}_r{args.refine_max}.txt",
                            TRAFFIC_SOURCES, "mfma_busy_frac")


def traffic_from_profiles(args):
    """HBM bytes of one step's solve launches from the committed counter
    summary (profiles/traffic_<workload>_<precision>_r<refine_max>.txt)."""
    return _counter_summary(f"traffic_{args.workload}_{args.precision}_r{args.refine_max}.txt",
                            TRAFFIC_SOURCES, "solve_hbm_bytes_per_step")


def mesh_traffic_from_profiles(workload):
    """HBM bytes of one marching-cubes call on the workload's volume
    (profiles/traffic_mcubes_<workload>.txt)."""
    return _counter_summary(f"traffic_mcubes_{workload}.txt", MESH_TRAFFIC_SOURCES,
                            "mesh_hbm_bytes_per_call")


def class_counts(bucket, nb):
    """Systems per 16-wide size class NB (n + nb rounded up to 16)."""
    out = {}
    for n, c in enumerate(bucket):
        if c:
            k = (n + nb + 15) // 16
            out[k] = out.get(k, 0) + int(c)
    return {f"NB{k}": v for k, v in sorted(out.items())}


NEXT_ROWS = ("pattern_cache", "marching_cubes", "edge_postpass")
DTYPES = {"fp32": "f32", "fp64": "f64", "mixed_fp16": "f16x3+f32", "mixed_bf16": "bf16x3+f32"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large_160x512")
    ap.add_argument("--precision", default="mixed_fp16")
    ap.add_argument("--refine-max", type=int, default=1,
                    help="mixed precisions: 0 = factorisation read-out, 1 = FP64 correction")
    ap.add_argument("--refine-tol", type=float, default=1e-5,
                    help="per-voxel error tolerance of the precision control "
                         "(okr_problem.refine_tol)")
    ap.add_argument("--no-graph", action="store_true", help="direct launches instead of graph replay")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other precisions and the leave-one-slice-out timing")
    ap.add_argument("--loso-only", action="store_true",
                    help="only the leave-one-slice-out timing (for profiling its kernels)")
    ap.add_argument("--pattern-only", action="store_true",
                    help="only the pattern-cache plan, profiled per phase")
    ap.add_argument("--mcubes-only", action="store_true",
                    help="only marching cubes on the reconstructed volume")
    ap.add_argument("--edge-only", action="store_true",
                    help="only the edge post-pass on the volume of one untimed execute "
                         "(for profiling its kernels)")
    ap.add_argument("--calib-copy", type=int, default=0,
                    help="after timing, copy this many bytes device-to-device (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding the gaps over GPUs is designed, not implemented)",
              file=sys.stderr)
        sys.exit(2)

    for var_ in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[var_] = "1"   # the oracle's workers: one BLAS thread each
    import numpy as np
    import workloads as W
    w = W.workload(args.workload)
    t0 = time.time()
    s, e = W.make_inputs(w)
    print(f"# inputs {w.name}: {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    if args.loso_only:
        print(json.dumps({"loso": loso_record(reps=args.steps)}))
        return
    if args.pattern_only:
        import torch
        import paper_2303_09523_amd as P
        st = torch.from_numpy(s).cuda()
        et = torch.from_numpy(e).cuda() if e is not None else None
        pc = P.Plan(w.m, w.m, w.nslices, w.upsample, w.radius, 4, args.precision, "pattern",
                    refine_max=args.refine_max, refine_tol=args.refine_tol)
        pc.set_profiling(True)
        vol, var, _ = pc.execute(st, w.vario, et)
        pc.stats()   # reads and clears the phase clocks of the first execute
        for _ in range(args.steps):
            pc.execute(st, w.vario, et, volume=vol, variance=var)
        sc = pc.stats()
        pc.close()
        ncand = 2 * (2 * w.radius + 1) ** 2
        nlo = downdate_floor(ncand, w.upsample + 1)
        rec = {"workload": w.name, "pattern_cache": {
            "steps": args.steps,
            "full_window_systems": int(sc["bucket"][ncand]),
            "inverse_systems": int(sum(sc["bucket"][nlo:ncand])),
            "phase_ms_per_step": {k: round(v / args.steps, 3)
                                  for k, v in sc["phase_ms"].items() if v > 0}}}
        if args.calib_copy > 0:
            rec["calibration"] = _calibration_copy(args.calib_copy)
        print(json.dumps(rec))
        return
    if args.edge_only or args.mcubes_only:
        import torch
        import paper_2303_09523_amd as P
        st = torch.from_numpy(s).cuda()
        et = torch.from_numpy(e).cuda() if e is not None else None
        pk = P.Plan(w.m, w.m, w.nslices, w.upsample, w.radius, 4, args.precision, "batched",
                    refine_max=args.refine_max, refine_tol=args.refine_tol)
        vol, _, _ = pk.execute(st, w.vario, et)
        pk.close()
        if args.edge_only:
            rec = {"edge_postpass": edge_postpass_record(w, vol, args, reps=args.steps)}
        else:
            rec = {"marching_cubes": mcubes_record(w, s, vol, args, reps=args.steps)}
        if args.calib_copy > 0:
            rec["calibration"] = _calibration_copy(args.calib_copy)
        print(json.dumps({"workload": w.name, **rec}))
        return

    cpu = None
    sample = None
    if not args.no_cpu:
        cpu, sample = cpu_baseline(w, s, e, args.cpu_seconds)
        print(f"# cpu baseline: {cpu['value']:.0f} voxels/s on {cpu['cores']} cores",
              file=sys.stderr, flush=True)
    # every oracle run happens here, before the GPU is initialised (the pools fork)
    extra_inputs = {}
    if not args.no_extra:
        for name, secs, seed in (("precision_48x384", 4.0, 777), ("plain_8x64", 0.0, 0),
                                 ("edge_32x256", 3.0, 778)):
            wx = W.workload(name)
            sx, ex_ = W.make_inputs(wx)
            samp = None
            if not args.no_cpu:
                samp = cpu_baseline(wx, sx, ex_, secs, seed=seed)[1] if secs > 0 else \
                    _full_oracle(wx, sx, ex_)
            extra_inputs[name] = (wx, sx, ex_, samp)
        print("# oracle samples of the other workloads done", file=sys.stderr, flush=True)

    import torch
    import paper_2303_09523_amd as P
    dev = torch.device("cuda:0")
    st = torch.from_numpy(s).to(dev)
    et = torch.from_numpy(e).to(dev) if e is not None else None
    kriged = w.kriged_voxels
    vol = torch.empty((w.upsample * (w.nslices - 1) + 1, w.m, w.m), dtype=torch.float32,
                      device=dev)
    var = torch.empty_like(vol)

    def accuracy(vol_t, var_t):
        return _sample_accuracy(w, s, sample, vol_t, var_t)

    def timed(plan, steps, warmup):
        for _ in range(warmup):
            plan.execute(st, w.vario, et, volume=vol, variance=var)
        torch.cuda.synchronize()
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record()
        for _ in range(steps):
            plan.execute(st, w.vario, et, volume=vol, variance=var)
        a1.record()
        torch.cuda.synchronize()
        return a0.elapsed_time(a1) / steps

    # ---- the headline path: timed graph replays of whole executes ----
    plan = P.Plan(w.m, w.m, w.nslices, w.upsample, w.radius, 4, args.precision, "batched",
                  refine_max=args.refine_max, refine_tol=args.refine_tol)
    tuning = None
    if not args.no_tune:
        tuning = plan.autotune(st, w.vario, et, volume=vol, variance=var)
        print(f"# tuning {tuning}", file=sys.stderr, flush=True)
    if not args.no_graph:
        plan.set_graph(True)
    for _ in range(args.warmup):
        plan.execute(st, w.vario, et, volume=vol, variance=var)
    torch.cuda.synchronize()
    plan.stats()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_host = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        plan.execute(st, w.vario, et, volume=vol, variance=var)
    ev1.record()
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t_host
    ms = ev0.elapsed_time(ev1) / args.steps
    stats = plan.stats()
    value = kriged / (ms * 1e-3)
    acc = accuracy(vol, var)

    # ---- the dominant kernel: the same steps with per-phase HIP events ----
    plan.set_graph(False)
    plan.set_profiling(True)
    for _ in range(args.steps):
        plan.execute(st, w.vario, et, volume=vol, variance=var)
    pstats = plan.stats()
    plan.set_profiling(False)
    plan.close()
    hist = np.array(pstats["bucket"], dtype=np.float64)
    nn = np.arange(len(hist), dtype=np.float64)
    flops = float((hist * system_flops(nn, w.upsample)).sum())
    fdiag = float((hist * np.minimum(diag_flops(nn, w.upsample + 1),
                                     system_flops(nn, w.upsample))).sum())
    solve_ms = pstats["phase_ms"]["solve"] / max(1, pstats["phase_calls"]["solve"]) + \
        pstats["phase_ms"]["fallback"] / max(1, pstats["phase_calls"]["fallback"])
    achieved = flops / (solve_ms * 1e-3) / 1e12
    # The contraction's own peak: split FP16/BF16 products issue three FP16
    # MFMAs per product, priced at the FP16 dense peak; FP32 and FP64 at theirs.
    pkey, mult = CONTRACTION[args.precision]
    peak = PEAKS[pkey]
    # additive bound: the trailing updates at the MFMA peak (as issued) plus the
    # diagonal tiles at the vector-ALU peak of the same precision
    valu_peak = PEAKS["fp64_tflops"] if args.precision == "fp64" else PEAKS["fp32_tflops"]
    add_ms = ((flops - fdiag) * mult / (peak * 1e12) + fdiag / (valu_peak * 1e12)) * 1e3
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 5), "traffic": traffic_from_profiles(args),
            "kernel": "batched solve (all size-class launches and the FP64 re-solve of one step)",
            "flop_per_launch": flops, "mean_launch_ms": round(solve_ms, 4),
            "timing": "library HIP events around the solve launches, same steps without graph",
            "mfma_products_per_flop": mult,
            "frac_of_fp32_peak": round(achieved / PEAKS["fp32_tflops"], 5),
            "additive_bound_ms": round(add_ms, 3),
            "frac_of_additive_bound": round(add_ms / solve_ms, 5),
            "mfma_busy_frac": mfma_busy_from_profiles(args)}

    calib = None
    if args.calib_copy > 0:
        calib = _calibration_copy(args.calib_copy)

    # ---- the other operating points of the batched path ----
    others = {}
    loso = None
    if not args.no_extra:
        variants = [("mixed_fp16+fp64_correction", "mixed_fp16", 1), ("fp64", "fp64", 0),
                    ("fp32", "fp32", 0), ("mixed_fp16_readout", "mixed_fp16", 0)]
        for name, prec, rmax in variants:
            if prec == args.precision and rmax == args.refine_max:
                continue
            pv = P.Plan(w.m, w.m, w.nslices, w.upsample, w.radius, 4, prec, "batched",
                        refine_max=rmax)
            pv.set_graph(True)
            mv = timed(pv, 2, 1)
            sv = pv.stats()
            pv.close()
            others[name] = {"value": kriged / (mv * 1e-3), "unit": "voxels/s",
                            "ms_per_step": round(mv, 3), "dtype": DTYPES[prec] +
                            ("+f64corr" if rmax else ""),
                            "n_fp64_resolved": sv["n_fp64_fallback"],
                            "accuracy": accuracy(vol, var)}
            print(f"# {name}: {mv:.1f} ms", file=sys.stderr, flush=True)
        # the exact full-window pattern cache (a separate algorithm, not the headline)
        pc = P.Plan(w.m, w.m, w.nslices, w.upsample, w.radius, 4, args.precision, "pattern",
                    refine_max=args.refine_max)
        pc.set_graph(True)
        mc = timed(pc, 2, 1)
        acc_c = accuracy(vol, var)
        pc.set_graph(False)
        pc.set_profiling(True)
        pc.execute(st, w.vario, et, volume=vol, variance=var)
        sc = pc.stats()
        pc.close()
        ncand = 2 * (2 * w.radius + 1) ** 2
        nfull = int(sc["bucket"][ncand])
        pat_ms = sc["phase_ms"]["pattern"]
        # algorithmic bytes of a full-window system: its f-1 estimates and variances
        # written, its column of the two bounding slices read, its neighbour count
        pbytes = nfull * (8.0 * (w.upsample - 1) + 8.0 + 1.0)
        # algorithmic FLOP: the weighted sums of its f-1 targets over ncand values
        pflop = nfull * 2.0 * ncand * (w.upsample - 1)
        others["pattern_cache"] = {
            "value": kriged / (mc * 1e-3), "unit": "voxels/s", "ms_per_step": round(mc, 3),
            "dtype": DTYPES[args.precision] + " + f64 cached weights",
            "full_window_systems": nfull,
            "inverse_systems": int(sum(sc["bucket"][downdate_floor(ncand, w.upsample + 1):ncand])),
            "accuracy": acc_c,
            "phase_ms": {"pattern": round(pat_ms, 3), "solve": round(sc["phase_ms"]["solve"], 3)},
            # the pattern phase: the full window's weights, inverse and solves
            # and the stencil apply; the apply's FP64 FMAs bound it (its HBM
            # bytes take a tenth of the time). The systems from the window's
            # inverse are timed with the solve phase.
            "roofline_pattern_apply": {
                "bound": "alu", "achieved": round(pflop / (pat_ms * 1e-3) / 1e12, 2),
                "peak": PEAKS["fp64_tflops"], "unit": "TFLOP/s",
                "frac": round(pflop / (pat_ms * 1e-3) / 1e12 / PEAKS["fp64_tflops"], 4),
                "hbm_gbs": round(pbytes / (pat_ms * 1e-3) / 1e9, 1),
                "traffic": None}}
        print(f"# pattern cache: {mc:.1f} ms", file=sys.stderr, flush=True)
        others["marching_cubes"] = mcubes_record(w, s, vol, args)
        others["edge_postpass"] = edge_postpass_record(w, vol, args)
        loso = loso_record()

    # ---- precision study on the ill-conditioned Gaussian workload ----
    study = None
    if not args.no_extra:
        w3, s3, e3, samp3 = extra_inputs["precision_48x384"]
        st3 = torch.from_numpy(s3).to(dev)
        et3 = torch.from_numpy(e3).to(dev)
        v3 = torch.empty((w3.upsample * (w3.nslices - 1) + 1, w3.m, w3.m), dtype=torch.float32,
                         device=dev)
        var3 = torch.empty_like(v3)
        study = {"workload": w3.name, "variogram": [w3.vario.model, w3.vario.nugget,
                                                     w3.vario.sill, w3.vario.range],
                 "kriged_voxels": w3.kriged_voxels,
                 "timing": "median of 3 executes after one warm-up", "modes": {}}
        modes = [("fp32", "fp32", 0, 0.0), ("fp32, routed at 1e-4", "fp32", 0, 1e-4),
                 ("mixed_fp16 read-out", "mixed_fp16", 0, 0.0),
                 ("mixed_bf16 read-out", "mixed_bf16", 0, 0.0),
                 ("mixed_fp16 read-out, routed at 1e-4", "mixed_fp16", 0, 1e-4),
                 ("mixed_fp16 + fp64 correction", "mixed_fp16", 1, 0.0),
                 ("mixed_fp16 + fp64 correction, checked at 1e-4", "mixed_fp16", 1, 1e-4),
                 ("mixed_bf16 + fp64 correction", "mixed_bf16", 1, 0.0),
                 ("mixed_bf16 + fp64 correction, checked at 1e-4", "mixed_bf16", 1, 1e-4),
                 ("fp64", "fp64", 0, 0.0)]
        for name, prec, rmax, tol in modes:
            pv = P.Plan(w3.m, w3.m, w3.nslices, w3.upsample, w3.radius, 4, prec, "batched",
                        refine_max=rmax, refine_tol=tol)
            med, mn_ = _time_executes(pv, st3, w3.vario, et3, v3, var3, 3)
            sv = pv.stats()
            pv.close()
            ent = {"ms": round(med, 3), "ms_min": round(mn_, 3),
                   "n_fp64_resolved": sv["n_fp64_fallback"], "n_refined": sv["n_refined"],
                   "n_refine_unconverged": sv["n_refine_unconverged"],
                   "n_nonpositive_pivot": sv["n_nonpositive_pivot"],
                   "kappa_window": sv["kappa_window"], "max_kappa_est": sv["max_kappa_est"],
                   "direct_fp64": sv["direct_fp64"]}
            acc3 = _sample_accuracy(w3, s3, samp3, v3, None)
            if acc3:
                ent.update(acc3)
            study["modes"][name] = ent
            print(f"# precision study {name}: {ent}", file=sys.stderr, flush=True)

    # ---- the small and the edge-preserved workloads: batched, mixed, plain ----
    other_workloads = None
    if not args.no_extra:
        other_workloads = {}
        for name in ("plain_8x64", "edge_32x256"):
            wx, sx, ex_, sampx = extra_inputs[name]
            stx = torch.from_numpy(sx).to(dev)
            etx = torch.from_numpy(ex_).to(dev) if ex_ is not None else None
            vx = torch.empty((wx.upsample * (wx.nslices - 1) + 1, wx.m, wx.m), dtype=torch.float32,
                             device=dev)
            varx = torch.empty_like(vx)
            ent = {"kriged_voxels": wx.kriged_voxels, "systems": wx.systems,
                   "timing": "median of 7 graph-replayed executes after one warm-up"}
            for label, prec, algo, rmax, tol in (("batched_fp32", "fp32", "batched", 0, 0.0),
                                                 ("batched_mixed_refined", "mixed_fp16",
                                                  "batched", 1, 1e-5),
                                                 ("plain_fp32_refined", "fp32", "plain", 1, 0.0)):
                px = P.Plan(wx.m, wx.m, wx.nslices, wx.upsample, wx.radius, 4, prec, algo,
                            refine_max=rmax, refine_tol=tol)
                if algo != "plain":
                    px.set_graph(True)
                med, mn_ = _time_executes(px, stx, wx.vario, etx, vx, varx, 7)
                sx_ = px.stats()
                px.close()
                hist = np.array(sx_["bucket"], dtype=np.float64)
                nn = np.arange(len(hist), dtype=np.float64)
                fl = float((hist * system_flops(nn, wx.upsample)).sum())
                pkey, _ = CONTRACTION[prec]
                ent[label] = {"value": wx.kriged_voxels / (med * 1e-3), "unit": "voxels/s",
                              "ms": round(med, 4), "ms_min": round(mn_, 4),
                              "achieved_tflops": round(fl / (med * 1e-3) / 1e12, 4),
                              "roofline_frac": round(fl / (med * 1e-3) / 1e12 / PEAKS[pkey], 6),
                              "peak": PEAKS[pkey],
                              "n_fp64_resolved": sx_["n_fp64_fallback"],
                              "accuracy": _sample_accuracy(wx, sx, sampx, vx, varx)}
                print(f"# {name} {label}: {med:.3f} ms", file=sys.stderr, flush=True)
            other_workloads[name] = ent

    # ---- variogram fit: 200 Adam steps on the leave-one-slice-out loss ----
    fit = None
    if not args.no_extra:
        from paper_2303_09523_amd.autograd import fit_variogram
        wl = W.workload("loso_16x128")
        sl_, _ = W.make_inputs(wl)
        slt = torch.from_numpy(sl_).to(dev)
        pl = P.Plan(wl.m, wl.m, wl.nslices, 2, wl.radius, 4)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        traj = fit_variogram(pl, slt, (0.1, 1.0, 2.0), steps=200, lr=0.05, model="exponential")
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        pl.close()
        l0, th0 = traj[0]
        l1, th1 = traj[-1]
        fit = {"workload": wl.name, "steps": 200, "seconds": round(tf, 3),
               "loss_start": l0, "loss_end": l1,
               "theta_end": [float(x) for x in th1],
               "nugget_over_sill_end": float(th1[0] / th1[1]), "range_end": float(th1[2]),
               "truth": {"nugget_over_sill": 0.02 / 0.8, "range": 5.0}}
        print(f"# fit: {fit}", file=sys.stderr, flush=True)

    plain = None
    if not args.no_plain:
        # a slab of 9 known slices from the middle of the stack (8 gaps); the
        # per-voxel kernel shares nothing between voxels, so its rate on a slab
        # is its rate on the volume up to the slab's mix of neighbour counts
        sub = min(w.nslices, 9)
        z0 = (w.nslices - sub) // 2
        pp = P.Plan(w.m, w.m, sub, w.upsample, w.radius, 4, "fp32", "plain")
        ss = st[z0:z0 + sub].contiguous()
        es = et[z0:z0 + sub].contiguous() if et is not None else None
        pv = torch.empty(pp.out_shape(), dtype=torch.float32, device=dev)
        pvar = torch.empty_like(pv)
        pp.execute(ss, w.vario, es, volume=pv, variance=pvar)
        torch.cuda.synchronize()
        a0 = torch.cuda.Event(enable_timing=True)
        a1 = torch.cuda.Event(enable_timing=True)
        a0.record()
        pp.execute(ss, w.vario, es, volume=pv, variance=pvar)
        a1.record()
        torch.cuda.synchronize()
        pms = a0.elapsed_time(a1)
        pvox = (sub - 1) * (w.upsample - 1) * w.m * w.m
        plain = {"value": pvox / (pms * 1e-3), "unit": "voxels/s", "ms": round(pms, 2),
                 "slab": f"known slices {z0}..{z0 + sub - 1} ({pvox} kriged voxels)",
                 "batched_over_plain": round(value / (pvox / (pms * 1e-3)), 2)}
        pp.close()

    out = {
        "metric": "kriged voxels/sec, batched mixed vs plain FP32 at <=1e-5 rel err; % roofline",
        "value": value, "unit": "voxels/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPES.get(args.precision, args.precision) + ("+f64corr" if args.refine_max and
                                                               args.precision.startswith("mixed")
                                                               else ""),
        "data": "synthetic",
        "config": {"workload": w.name, "known_slices": w.nslices, "slice": f"{w.m}x{w.m}",
                   "upsample": w.upsample, "window": f"{2 * w.radius + 1}x{2 * w.radius + 1}x2",
                   "edge_mask": w.masked, "variogram": [w.vario.model, w.vario.nugget,
                                                         w.vario.sill, w.vario.range],
                   "kriged_voxels": kriged, "systems": w.systems,
                   "precision": args.precision, "refine_max": args.refine_max,
                   "graph": not args.no_graph, "tuning": tuning},
        "roofline": roof,
        "cpu_baseline": cpu,
        "accuracy": acc,
        "plain_fp32": plain,
        "batched_variants": {k: v for k, v in others.items() if k not in NEXT_ROWS},
        # the rows beyond the path: pattern cache, marching cubes and
        # the paper's edge post-pass
        "next_rows": {k: others[k] for k in NEXT_ROWS if k in others},
        "loso": loso,
        "variogram_fit": fit,
        "precision_study": study,
        "other_configs": other_workloads,
        "calibration": calib,
        "phases_ms_per_step": {k: round(v / args.steps, 4) for k, v in pstats["phase_ms"].items()},
        "solver_stats": dict({k: stats[k] for k in ("n_systems", "n_refined", "n_fp64_fallback",
                                                    "n_nonpositive_pivot", "n_not_converged",
                                                    "max_kappa_est")},
                             systems_per_size_class=class_counts(stats["bucket"], w.upsample + 1)),
        "host_wall_s": round(t_host, 3),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()

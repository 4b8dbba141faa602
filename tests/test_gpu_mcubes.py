"""GPU marching cubes (okr_marching_cubes) against the oracle: bit-exact
triangle lists (vertex coordinates and cube indices, in order) on random
fields covering all 256 corner configurations, on a kriged volume, across
workgroup runs of a long row, with NaNs, for empty and degenerate shapes and
a too-small output buffer; at the large workload's full size the triangle
total against the oracle's per-configuration counts and sampled cubes
recomputed one by one."""
import numpy as np
import pytest

from oracle import mcubes as M
import workloads as W

pytestmark = pytest.mark.gpu


def _plan(n, ny, nx, f):
    import paper_2303_09523_amd as P
    return P.Plan(nx, ny, n, f, 1)


def _configs(vol, iso):
    v = vol >= iso
    cfg = np.zeros(tuple(s - 1 for s in vol.shape), np.int32)
    for c in range(8):
        x, y, z = c & 1, (c >> 1) & 1, (c >> 2) & 1
        cfg |= v[z:z + v.shape[0] - 1, y:y + v.shape[1] - 1, x:x + v.shape[2] - 1].astype(np.int32) << c
    return cfg


def _gpu(plan, vol, iso, **kw):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(vol)).cuda()
    tris, ids = plan.marching_cubes(t, iso, **kw)
    return tris.cpu().numpy(), (ids.cpu().numpy() if ids is not None else None)


@pytest.mark.parametrize("seed", [0, 1])
def test_random_field_all_configurations(seed):
    n, ny, nx, f = 5, 23, 37, 4
    plan = _plan(n, ny, nx, f)
    shape = plan.out_shape()
    rng = np.random.default_rng(seed)
    vol = rng.standard_normal(shape).astype(np.float32)
    iso = 0.05
    assert len(np.unique(_configs(vol, iso))) == 256
    print(f"random field {shape} seed {seed}", flush=True)
    tg, ig = _gpu(plan, vol, iso)
    to, io = M.marching_cubes(vol, iso)
    assert tg.shape == to.shape and tg.shape[0] > 1000
    np.testing.assert_array_equal(ig, io)
    np.testing.assert_array_equal(tg, to)
    plan.close()


def test_kriged_volume():
    import torch
    import paper_2303_09523_amd as P
    w = W.workload("edge_32x256")
    s, e = W.make_inputs(w)
    s, e = s[:3, :48, :40].copy(), (e[:3, :48, :40].copy() if e is not None else None)
    n, ny, nx = s.shape
    plan = P.Plan(nx, ny, n, w.upsample, w.radius, 4, "mixed_fp16")
    vol, _, _ = plan.execute(torch.from_numpy(s).cuda(), w.vario,
                             torch.from_numpy(e).cuda() if e is not None else None)
    v = vol.cpu().numpy()
    iso = float(np.median(v))
    tris, ids = plan.marching_cubes(vol, iso)
    to, io = M.marching_cubes(v, iso)
    assert to.shape[0] > 100
    np.testing.assert_array_equal(ids.cpu().numpy(), io)
    np.testing.assert_array_equal(tris.cpu().numpy(), to)
    plan.close()


def test_long_rows_and_nan():
    n, ny, nx, f = 2, 3, 2301, 2   # rows of 2300 cubes: three workgroup runs
    plan = _plan(n, ny, nx, f)
    rng = np.random.default_rng(7)
    vol = rng.standard_normal(plan.out_shape()).astype(np.float32)
    vol[1, 1, 1000:1030] = np.nan
    vol[0, 2, 2047:2050] = np.inf
    tg, ig = _gpu(plan, vol, 0.0)
    to, io = M.marching_cubes(vol, 0.0)
    np.testing.assert_array_equal(ig, io)
    np.testing.assert_array_equal(tg, to)
    assert np.isnan(tg).any()
    plan.close()


def test_empty_degenerate_and_capacity():
    from paper_2303_09523_amd import OkrError
    import torch
    plan = _plan(3, 6, 7, 2)
    vol = np.random.default_rng(3).standard_normal(plan.out_shape()).astype(np.float32)
    tg, ig = _gpu(plan, vol, 100.0)                    # nothing inside
    assert tg.shape == (0, 3, 3) and ig.shape == (0,)
    tg, ig = _gpu(plan, vol, -100.0)                   # everything inside
    assert tg.shape == (0, 3, 3)
    to, io = M.marching_cubes(vol, 0.2)
    tg, ig = _gpu(plan, vol, 0.2, want_ids=False)
    assert ig is None
    np.testing.assert_array_equal(tg, to)
    # a buffer of 10 triangles: the first 10, the total reported, OKR_E_CAPACITY
    t = torch.from_numpy(vol).cuda()
    with pytest.raises(OkrError) as ex:
        plan.marching_cubes(t, 0.2, max_tris=10)
    assert ex.value.status == 8
    import ctypes as C
    from paper_2303_09523_amd import _lib
    buf = torch.full((10, 3, 3), -7.0, dtype=torch.float32, device="cuda")
    n = C.c_int64(0)
    st = _lib.load().okr_marching_cubes(plan._h, t.data_ptr(), C.c_float(0.2), buf.data_ptr(),
                                        None, 10, C.byref(n))
    assert st == 8 and n.value == to.shape[0]
    np.testing.assert_array_equal(buf.cpu().numpy(), to[:10])
    plan.close()
    one = _plan(1, 5, 5, 2)                            # a single plane: no cubes
    tg, ig = _gpu(one, np.zeros(one.out_shape(), np.float32), 0.0)
    assert tg.shape == (0, 3, 3)
    one.close()


def test_full_size_headline_volume():
    import torch
    import paper_2303_09523_amd as P
    w = W.workload("large_160x512")
    s, e = W.make_inputs(w)
    print("large_160x512 marching cubes", flush=True)
    plan = P.Plan(w.m, w.m, w.nslices, w.upsample, w.radius, 4, "mixed_fp16", refine_max=0)
    vol, _, _ = plan.execute(torch.from_numpy(s).cuda(), w.vario,
                             torch.from_numpy(e).cuda() if e is not None else None)
    v = vol.cpu().numpy()
    iso = float(np.median(s))
    tris, ids = plan.marching_cubes(vol, iso)
    ids = ids.cpu().numpy()
    # total against the oracle's triangles per configuration
    per_cfg = np.array([len(M.cube_triangles([(c >> i) & 1 for i in range(8)]))
                        for c in range(256)], np.int64)
    hist = np.bincount(_configs(v, np.float32(iso)).ravel(), minlength=256)
    assert tris.shape[0] == int(hist @ per_cfg)
    assert np.all(np.diff(ids) >= 0)
    # sampled cubes, one by one
    rng = np.random.default_rng(11)
    pick = np.unique(rng.choice(ids, 1500, replace=False))
    lo = np.searchsorted(ids, pick, side="left")
    hi = np.searchsorted(ids, pick, side="right")
    sel = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)])
    tg = tris[torch.from_numpy(sel).cuda()].cpu().numpy()
    to, io = M.marching_cubes_cubes(v, iso, pick)
    np.testing.assert_array_equal(ids[sel], io)
    np.testing.assert_array_equal(tg, to)
    plan.close()

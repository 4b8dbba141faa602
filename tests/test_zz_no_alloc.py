"""okr_execute_noalloc (the entry point for callers that cannot allocate)
against okr_execute on the same problems: two calls in a row, the second on a
smaller input, each compared bit for bit with a plan's execute (the same
kernels), plus its size limit and its device status word."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _inputs(n, m, f, r, seed):
    w = W.Workload("noalloc", n, m, f, r, True, 6, 2, 0.02, W.Variogram("spherical", 0, 1, 4), seed)
    s = W.phantom(w)
    return s, W.sobel_edges(s)


def _via_plan(st, et, f, r, vario, precision, refine_max, refine_tol):
    import torch
    import paper_2303_09523_amd as P
    n, ny, nx = st.shape
    plan = P.Plan(nx, ny, n, f, r, 4, precision, refine_max=refine_max, refine_tol=refine_tol)
    vol, var, fl = plan.execute(st, vario, et, want_flags=True)
    plan.stats()
    plan.close()
    torch.cuda.synchronize()
    return vol.cpu().numpy(), var.cpu().numpy(), fl.cpu().numpy()


@pytest.mark.parametrize("precision,refine_max,refine_tol", [("mixed_fp16", 1, 1e-5),
                                                             ("fp32", 0, 0.0)])
def test_noalloc_matches_execute_twice(precision, refine_max, refine_tol):
    import torch
    import paper_2303_09523_amd as P
    vario = ("spherical", 0.005, 1.0, 8.0)
    # the first call larger than the second: the second must not see the first's state
    for n, m, f, r, seed in ((5, 96, 4, 3, 31), (3, 40, 3, 2, 32)):
        s, e = _inputs(n, m, f, r, seed)
        st = torch.from_numpy(s).cuda()
        et = torch.from_numpy(e).cuda()
        print(f"noalloc {precision} shape {s.shape} f={f} r={r}", flush=True)
        vol = torch.full(((n - 1) * f + 1, m, m), float("nan"), dtype=torch.float32, device="cuda")
        var = torch.full_like(vol, float("nan"))
        flags = torch.zeros((n - 1, m, m), dtype=torch.uint8, device="cuda")
        status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        P.execute_noalloc(st, vario, f, r, vol, var, et, flags, status, precision=precision,
                          refine_max=refine_max, refine_tol=refine_tol)
        torch.cuda.synchronize()
        v0, w0, f0 = _via_plan(st, et, f, r, vario, precision, refine_max, refine_tol)
        assert int(status.item()) == 0
        np.testing.assert_array_equal(vol.cpu().numpy(), v0)
        np.testing.assert_array_equal(var.cpu().numpy(), w0)
        np.testing.assert_array_equal(flags.cpu().numpy(), f0)


def test_noalloc_rejects_problems_beyond_its_workspace():
    import torch
    import paper_2303_09523_amd as P
    st = torch.zeros((3, 1024, 1024), dtype=torch.float32, device="cuda")   # 2 x 2^20 systems
    vol = torch.empty((5, 1024, 1024), dtype=torch.float32, device="cuda")
    with pytest.raises(P.OkrError) as ei:
        P.execute_noalloc(st, ("spherical", 0.0, 1.0, 4.0), 2, 1, vol)
    assert ei.value.status == 2


def test_noalloc_reports_nonfinite_input_on_its_status_word():
    import torch
    import paper_2303_09523_amd as P
    s = np.zeros((2, 8, 8), np.float32)
    s[1, 3, 3] = np.inf
    st = torch.from_numpy(s).cuda()
    vol = torch.empty((3, 8, 8), dtype=torch.float32, device="cuda")
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    P.execute_noalloc(st, ("spherical", 0.0, 1.0, 4.0), 2, 1, vol, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == 3

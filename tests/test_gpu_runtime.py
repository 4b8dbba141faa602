"""GPU checks of the launch runtime: graph capture and replay of okr_execute,
and the autotuner's launch-shape choice. Both must leave the results of the
direct launches unchanged."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from _gpu_util import rel_err_est

pytestmark = pytest.mark.gpu


def _inputs(seed=21, n=4, ny=40, nx=44, f=4, r=3):
    w = W.Workload("rt", n, max(ny, nx), f, r, True, 6, 2, 0.02,
                   W.Variogram("spherical", 0, 1, 4), seed)
    s = W.phantom(w)[:, :ny, :nx].copy()
    e = W.sobel_edges(s)
    rng = np.random.default_rng(seed + 1)
    e = np.maximum(e, (rng.random(e.shape) < 0.1).astype(np.uint8))
    return s, e


@pytest.mark.parametrize("precision", ["fp32", "mixed_fp16"])
def test_graph_replay_matches_direct_launches(precision):
    import torch
    import paper_2303_09523_amd as P
    s, e = _inputs()
    n, ny, nx = s.shape
    f, r = 4, 3
    vario = ("spherical", 0.005, 1.0, 8.0)
    st = torch.from_numpy(s).cuda()
    et = torch.from_numpy(e).cuda()
    direct = P.Plan(nx, ny, n, f, r, precision=precision)
    v_ref, w_ref, f_ref = direct.execute(st, vario, et, want_flags=True)
    torch.cuda.synchronize()
    direct.close()
    plan = P.Plan(nx, ny, n, f, r, precision=precision)
    plan.set_graph(True)
    vol = torch.empty_like(v_ref)
    var = torch.empty_like(w_ref)
    fl = torch.empty_like(f_ref)
    for rep in range(4):
        vol.fill_(float("nan"))
        var.fill_(float("nan"))
        fl.fill_(255)
        plan.execute(st, vario, et, volume=vol, variance=var, flags=fl)
        torch.cuda.synchronize()
        junk = torch.randn(1 << 16, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(vol, v_ref), rep
        assert torch.equal(var, w_ref), rep
        assert torch.equal(fl, f_ref), rep
        del junk
    # other buffers or another variogram: re-captured, still equal to direct launches
    vol2 = torch.empty_like(v_ref)
    plan.execute(st, vario, et, volume=vol2, variance=var, flags=fl)
    torch.cuda.synchronize()
    assert torch.equal(vol2, v_ref)
    vario2 = ("exponential", 0.01, 1.0, 6.0)
    plan.execute(st, vario2, et, volume=vol2, variance=var)
    torch.cuda.synchronize()
    d2 = P.Plan(nx, ny, n, f, r, precision=precision)
    v2, _, _ = d2.execute(st, vario2, et)
    torch.cuda.synchronize()
    assert torch.equal(vol2, v2)
    d2.close()
    plan.close()


def test_autotune_keeps_results():
    import torch
    import paper_2303_09523_amd as P
    s, e = _inputs(seed=23)
    n, ny, nx = s.shape
    f, r = 4, 3
    vario = ("spherical", 0.005, 1.0, 8.0)
    st = torch.from_numpy(s).cuda()
    et = torch.from_numpy(e).cuda()
    ref = P.Plan(nx, ny, n, f, r, precision="fp32")
    v_ref, w_ref, _ = ref.execute(st, vario, et)
    torch.cuda.synchronize()
    ref.close()
    plan = P.Plan(nx, ny, n, f, r, precision="fp32")
    t = plan.autotune(st, vario, et)
    print("fp32 tuning", t, flush=True)
    assert 1 <= t["grid_per_cu"] <= 4
    assert all(m > 0 for m in t["candidate_ms"][:4])
    v, w, _ = plan.execute(st, vario, et)
    torch.cuda.synchronize()
    # the launch shape only changes which wave takes which system
    assert torch.equal(v, v_ref) and torch.equal(w, w_ref)
    plan.close()
    # a second plan with the same key takes the cached shape without timing
    again = P.Plan(nx, ny, n, f, r, precision="fp32")
    t2 = again.autotune(st, vario, et)
    print("fp32 tuning again", t2, flush=True)
    assert t2["from_cache"]
    assert (t2["grid_per_cu"], t2["update_arith"]) == (t["grid_per_cu"], t["update_arith"])
    assert t2["candidate_ms"] == t["candidate_ms"]
    again.close()
    # mixed: the tuned update arithmetic still meets the refined bar
    vo, _, _ = O.krige_volume(s, e, f, r, vario)
    plan = P.Plan(nx, ny, n, f, r, precision="mixed_fp16")
    t = plan.autotune(st, vario, et)
    print("mixed tuning", t, flush=True)
    assert t["update_arith"] in (0, 1)
    v, _, _ = plan.execute(st, vario, et)
    vn = v.cpu().numpy()
    kz = np.ones(vn.shape[0], bool)
    kz[::f] = False
    assert rel_err_est(vn[kz], vo[kz], np.abs(s).max()).max() <= 1e-5
    plan.close()


def test_allocation_failures_are_reported(monkeypatch):
    """A forced device allocation failure (OKR_FAIL_ALLOC) makes plan creation
    and the lazily allocated leave-one-slice-out workspace return OKR_E_OOM
    with nothing left half-built; the same calls succeed once it is lifted."""
    import torch
    import paper_2303_09523_amd as P
    s, e = _inputs()
    n, ny, nx = s.shape
    monkeypatch.setenv("OKR_FAIL_ALLOC", "1")
    with pytest.raises(P.OkrError) as ei:
        P.Plan(nx, ny, n, 4, 3)
    assert ei.value.status == 5
    monkeypatch.delenv("OKR_FAIL_ALLOC")
    plan = P.Plan(nx, ny, n, 2, 2)
    st = torch.from_numpy(s).cuda()
    monkeypatch.setenv("OKR_FAIL_ALLOC", "1")
    with pytest.raises(P.OkrError) as ei:
        plan.loso_forward(st, ("exponential", 0.1, 1.0, 2.0))
    assert ei.value.status == 5
    monkeypatch.delenv("OKR_FAIL_ALLOC")
    loss = plan.loso_forward(st, ("exponential", 0.1, 1.0, 2.0))
    grad = plan.loso_backward()
    plan.close()
    assert np.isfinite(float(loss)) and torch.isfinite(grad).all()

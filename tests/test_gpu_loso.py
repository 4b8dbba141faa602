"""GPU leave-one-slice-out loss and adjoint gradient against the FP64 oracle,
finite differences of the GPU loss, bitwise repeatability and Adam
trajectories."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _field(n, ny, nx, seed=11):
    v = W.Variogram("exponential", 0.02, 0.8, 5.0)
    f, _ = W.gaussian_field((n, ny, nx), v, seed=seed)
    return f.astype(np.float32)


def _plan(s, r=2):
    import paper_2303_09523_amd as P
    n, ny, nx = s.shape
    return P.Plan(nx, ny, n, 2, r, 4)


@pytest.mark.parametrize("model,theta", [("exponential", (0.1, 1.0, 2.0)),
                                         ("spherical", (0.05, 1.2, 4.5)),
                                         ("gaussian", (0.2, 1.0, 3.0))])
def test_loso_loss_and_grad_vs_oracle(model, theta):
    import torch
    s = _field(6, 23, 21)
    L_o, g_o = O.loso_loss_grad(s, 2, (model, *theta))
    plan = _plan(s)
    st = torch.from_numpy(s).cuda()
    loss = plan.loso_forward(st, (model, *theta))
    grad = plan.loso_backward()
    L, g = float(loss.item()), grad.cpu().numpy()
    plan.close()
    print(f"{model}: loss {L:.10e} vs {L_o:.10e}; grad {g} vs {g_o}", flush=True)
    assert abs(L - L_o) <= 1e-9 * abs(L_o)
    np.testing.assert_allclose(g, g_o, rtol=1e-4, atol=1e-6 * np.abs(g_o).max())


@pytest.mark.parametrize("drift", ["none", "linear_z"])
@pytest.mark.parametrize("r", [2, 3])
def test_loso_edges_and_drift_vs_oracle(r, drift):
    """Edge masks on both neighbouring slices (so the kept sets differ and the
    floor fills some systems), ordinary kriging and the slice predictor."""
    import torch
    import paper_2303_09523_amd as P
    s = _field(5, 26, 23, seed=13)
    e = (np.random.default_rng(14).random(s.shape) < 0.2).astype(np.uint8)
    th = ("spherical", 0.05, 1.0, 4.5)
    L_o, g_o = O.loso_loss_grad(s, r, th, edges=e, drift=drift)
    n, ny, nx = s.shape
    plan = P.Plan(nx, ny, n, 2, r, 4, drift=drift)
    print(f"loso r={r} drift={drift}", flush=True)
    loss = plan.loso_forward(torch.from_numpy(s).cuda(), th, torch.from_numpy(e).cuda())
    grad = plan.loso_backward()
    L, g = float(loss.item()), grad.cpu().numpy()
    plan.close()
    print(f"loss {L:.10e} vs {L_o:.10e}; grad {g} vs {g_o}", flush=True)
    assert abs(L - L_o) <= 1e-9 * abs(L_o)
    np.testing.assert_allclose(g, g_o, rtol=1e-4, atol=1e-6 * np.abs(g_o).max())


def test_loso_drift_reproduces_a_trend_across_slices():
    """A field constant in-plane and linear across the slices, with masks:
    ordinary kriging misses the trend, the slice predictor reproduces it."""
    import torch
    import paper_2303_09523_amd as P
    ns, ny, nx = 5, 19, 17
    s = np.broadcast_to((3.0 + 2.0 * np.arange(ns, dtype=np.float32))[:, None, None],
                        (ns, ny, nx)).astype(np.float32)
    e = (np.random.default_rng(8).random(s.shape) < 0.3).astype(np.uint8)
    th = ("spherical", 0.05, 1.0, 4.0)
    st, et = torch.from_numpy(s).cuda(), torch.from_numpy(e).cuda()
    out = {}
    for drift in ("none", "linear_z"):
        plan = P.Plan(nx, ny, ns, 2, 2, 4, drift=drift)
        out[drift] = float(plan.loso_forward(st, th, et).item())
        plan.close()
    L_ok = O.loso_loss(s, 2, th, edges=e)
    print(out, L_ok, flush=True)
    assert abs(out["none"] - L_ok) <= 1e-9 * L_ok and L_ok > 1e-3
    assert out["linear_z"] < 1e-10


def test_loso_grad_vs_gpu_finite_differences():
    import torch
    s = _field(5, 20, 22, seed=3)
    plan = _plan(s)
    st = torch.from_numpy(s).cuda()
    th = np.array([0.1, 1.0, 2.0])
    plan.loso_forward(st, ("exponential", *th))
    g = plan.loso_backward().cpu().numpy()
    fd = np.zeros(3)
    h = 1e-4
    for k in range(3):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        lp = float(plan.loso_forward(st, ("exponential", *tp)).item())
        lm = float(plan.loso_forward(st, ("exponential", *tm)).item())
        fd[k] = (lp - lm) / (2 * h)
    plan.close()
    print("adjoint", g, "fd", fd, flush=True)
    np.testing.assert_allclose(g, fd, rtol=1e-4, atol=1e-6 * np.abs(fd).max())
    # only nugget/sill and range matter: n dL/dn + s dL/ds = 0
    assert abs(th[0] * g[0] + th[1] * g[1]) <= 1e-5 * np.abs(g).max()


def test_loso_bitwise_repeatable():
    import torch
    s = _field(6, 31, 29, seed=5)
    plan = _plan(s)
    st = torch.from_numpy(s).cuda()
    out = []
    for _ in range(2):
        L = plan.loso_forward(st, ("exponential", 0.05, 0.9, 4.0)).cpu().numpy()
        g = plan.loso_backward().cpu().numpy()
        out.append((L.tobytes(), g.tobytes()))
    plan.close()
    assert out[0] == out[1]


def test_loso_backward_requires_forward():
    import torch
    import paper_2303_09523_amd as P
    s = _field(4, 9, 9)
    plan = _plan(s)
    with pytest.raises(P.OkrError):
        plan.loso_backward()
    plan.close()


@pytest.mark.parametrize("between", ["autotune", "select", "execute"])
def test_loso_backward_refused_after_other_work(between):
    """A call that rewrites the selection, permutation or counters between
    the forward and the backward makes the backward an argument error (it
    returns before any launch)."""
    import torch
    import paper_2303_09523_amd as P
    s = _field(5, 12, 11)
    st = torch.from_numpy(s).cuda()
    plan = _plan(s)
    th = ("exponential", 0.1, 1.0, 2.0)
    plan.loso_forward(st, th)
    if between == "autotune":
        plan.autotune(st, th)
    elif between == "select":
        plan.select()
    else:
        plan.execute(st, th)
    with pytest.raises(P.OkrError):
        plan.loso_backward()
    # a new forward makes the pair valid again
    plan.loso_forward(st, th)
    g = plan.loso_backward()
    torch.cuda.synchronize()
    assert np.all(np.isfinite(g.cpu().numpy()))
    plan.close()


def test_loso_autograd_refuses_a_stale_forward():
    import torch
    from paper_2303_09523_amd.autograd import LosoLoss
    s = _field(5, 12, 11)
    st = torch.from_numpy(s).cuda()
    plan = _plan(s)
    t1 = torch.tensor([0.1, 1.0, 2.0], dtype=torch.float64, requires_grad=True)
    t2 = torch.tensor([0.2, 1.0, 3.0], dtype=torch.float64, requires_grad=True)
    l1 = LosoLoss.apply(t1, plan, st, None, "exponential")
    l2 = LosoLoss.apply(t2, plan, st, None, "exponential")
    with pytest.raises(RuntimeError):
        l1.backward()
    l2.backward()
    assert torch.isfinite(t2.grad).all()
    plan.close()


def test_adam_trajectory_vs_oracle():
    import torch
    from paper_2303_09523_amd.autograd import fit_variogram
    s = _field(5, 18, 17, seed=7)
    plan = _plan(s)
    st = torch.from_numpy(s).cuda()
    steps = 25
    traj = fit_variogram(plan, st, (0.1, 1.0, 2.0), steps=steps, lr=0.05)
    plan.close()
    ref = O.adam_fit(lambda th: O.loso_loss_grad(s, 2, ("exponential", *th)), (0.1, 1.0, 2.0),
                     steps=steps, lr=0.05)
    (Lg, tg), (Lr, tr) = traj[-1], ref[-1]
    print("gpu", Lg, tg, "oracle", Lr, tr, flush=True)
    assert abs(Lg - Lr) <= 1e-4 * abs(Lr)
    np.testing.assert_allclose(tg, tr, rtol=1e-3)


@pytest.mark.slow
def test_loso_full_size_vs_oracle():
    """The differentiation workload at full size (16 slices of 128x128)."""
    import torch
    w = W.workload("loso_16x128")
    s, _ = W.make_inputs(w)
    th = ("exponential", 0.1, 1.0, 2.0)
    L_o, g_o = O.loso_loss_grad(s, 2, th)
    plan = _plan(s)
    st = torch.from_numpy(s).cuda()
    L = float(plan.loso_forward(st, th).item())
    g = plan.loso_backward().cpu().numpy()
    plan.close()
    print(f"full: loss {L:.10e} vs {L_o:.10e}; grad {g} vs {g_o}", flush=True)
    assert abs(L - L_o) <= 1e-9 * abs(L_o)
    np.testing.assert_allclose(g, g_o, rtol=1e-4)


@pytest.mark.slow
def test_loso_full_size_drift_with_masks_vs_oracle():
    """The differentiation workload at full size with the slice predictor and
    edge masks (10 % of the pixels) on every slice."""
    import torch
    import paper_2303_09523_amd as P
    w = W.workload("loso_16x128")
    s, _ = W.make_inputs(w)
    e = (np.random.default_rng(21).random(s.shape) < 0.1).astype(np.uint8)
    th = ("exponential", 0.1, 1.0, 2.0)
    L_o, g_o = O.loso_loss_grad(s, w.radius, th, edges=e, drift="linear_z")
    n, ny, nx = s.shape
    plan = P.Plan(nx, ny, n, 2, w.radius, 4, drift="linear_z")
    print("loso_16x128 drift with masks", flush=True)
    L = float(plan.loso_forward(torch.from_numpy(s).cuda(), th, torch.from_numpy(e).cuda()).item())
    g = plan.loso_backward().cpu().numpy()
    plan.close()
    print(f"full drift: loss {L:.10e} vs {L_o:.10e}; grad {g} vs {g_o}", flush=True)
    assert abs(L - L_o) <= 1e-9 * abs(L_o)
    np.testing.assert_allclose(g, g_o, rtol=1e-4)


@pytest.mark.slow
def test_full_fit_trajectory_vs_golden():
    """The 200-step Adam fit of the variogram on the 16 x 128^2 field workload
    (exponential model from (0.1, 1.0, 2.0), lr 0.05) against the FP64
    oracle's trajectory stored by tests/golden/make_loso_fit.py: final loss
    within 1e-4 relative, nugget/sill and range within 1e-2 relative."""
    import json
    import os
    import torch
    import workloads as W
    from paper_2303_09523_amd.autograd import fit_variogram
    import paper_2303_09523_amd as P
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "loso_fit_16x128.json")))
    w = W.workload(gold["workload"])
    s, _ = W.make_inputs(w)
    plan = P.Plan(w.m, w.m, w.nslices, 2, w.radius, 4)
    traj = fit_variogram(plan, torch.from_numpy(s).cuda(), tuple(gold["theta0"]),
                         steps=gold["steps"], lr=gold["lr"], model=gold["model"])
    plan.close()
    assert len(traj) == len(gold["loss"]) == gold["steps"] + 1
    Lg, tg = traj[-1]
    Lr, tr = gold["loss"][-1], np.array(gold["theta"][-1])
    print("gpu", Lg, tg, "oracle", Lr, tr, flush=True)
    assert abs(Lg - Lr) <= 1e-4 * abs(Lr)
    assert abs(tg[0] / tg[1] - tr[0] / tr[1]) <= 1e-2 * abs(tr[0] / tr[1])
    assert abs(tg[2] - tr[2]) <= 1e-2 * abs(tr[2])
    # the loss falls along the whole trajectory as the oracle's does
    assert abs(traj[0][0] - gold["loss"][0]) <= 1e-6 * abs(gold["loss"][0])

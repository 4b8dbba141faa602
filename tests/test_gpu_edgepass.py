"""GPU edge post-pass (okr_edge_postpass) against the oracle, bit for bit:
the adjusted volume, the edge and orientation maps after the pass and the
coefficient magnitude M, on noisy phantoms of ragged shapes (images narrower
and wider than a wave, columns across bitmap words), on noise with a low
threshold (many re-routed windows), in place, with the bitmaps too large for
LDS, and at the large workload's full size on whole sampled images (every
YZ image is independent)."""
import numpy as np
import pytest

from oracle import edgepass as E
import workloads as W

pytestmark = pytest.mark.gpu


def _plan(n, ny, nx, f):
    import paper_2303_09523_amd as P
    return P.Plan(nx, ny, n, f, 1)


def _oracle_images(vol, tau, xs):
    """Oracle result of the YZ images x in xs: (out, edge, orient, M), each
    [Z][ny][len(xs)]."""
    outs, edges, thetas, mags = [], [], [], []
    for x in xs:
        img = vol[:, :, x]
        o, e, t = E.edge_postpass_image(img, tau)
        _, _, m = E.edges_and_orientation(img, tau)
        outs.append(o)
        edges.append(e)
        thetas.append(t)
        mags.append(m)
    st = lambda a: np.stack(a, axis=-1)   # noqa: E731
    return st(outs), st(edges), st(thetas), st(mags)


def _gpu(plan, vol, tau, inplace=False):
    import torch
    v = torch.from_numpy(np.ascontiguousarray(vol)).cuda()
    mag = torch.empty(v.shape, dtype=torch.float64, device="cuda")
    out, edge, orient = plan.edge_postpass(v, tau, out=v if inplace else None, mag=mag)
    return (out.cpu().numpy(), edge.cpu().numpy(), orient.cpu().numpy(), mag.cpu().numpy())


def _rerouted(vol, tau, xs):
    """Noisy windows the oracle finds in images xs."""
    n = 0
    for x in xs:
        e, th, _ = E.edges_and_orientation(vol[:, :, x], tau)
        for c in E.chains(e):
            for w0 in range(0, len(c) - E.WINDOW + 1, E.WINDOW):
                n += E.window_orientations([int(th[p]) for p in c[w0:w0 + E.WINDOW]])[1]
    return n


def _assert_same(got, ref, what=""):
    names = ("out", "edge", "orient", "mag")
    for g, r, name in zip(got, ref, names):
        assert g.shape == r.shape, (name, g.shape, r.shape)
        if g.dtype.kind == "f":
            same = g.view(np.uint32 if g.dtype == np.float32 else np.uint64) == \
                r.astype(g.dtype).view(np.uint32 if g.dtype == np.float32 else np.uint64)
        else:
            same = g == r
        if not same.all():
            idx = np.argwhere(~same)[:5]
            raise AssertionError(f"{what} {name}: {int((~same).sum())} differ, first {idx.tolist()}")


def _phantom(n, m, f, seed, noise=0.02):
    w = W.Workload("edge_pass", n, m, f, 1, False, 6, 2, noise,
                   W.Variogram("spherical", 0.0, 1.0, 4.0), seed)
    return w, W.postpass_volume(w)


@pytest.mark.parametrize("n,ny,nx,f,seed", [
    (5, 45, 70, 4, 11),     # images wider than a wave; 2 bitmap words per row
    (4, 33, 3, 3, 12),      # 3 images; 33 + 2 padding bits -> 2 words
    (9, 96, 64, 2, 13),     # exactly one wave of images; 3 words
    (3, 130, 129, 4, 14),   # ragged: 129 images, 5 words
])
def test_phantom_bit_exact(n, ny, nx, f, seed):
    w = W.Workload("edge_pass", n, max(ny, nx), f, 1, False, 6, 2, 0.02,
                   W.Variogram("spherical", 0.0, 1.0, 4.0), seed)
    vol = W.postpass_volume(w)[:, :ny, :nx].copy()
    print(f"edge post-pass phantom {vol.shape} seed {seed}", flush=True)
    plan = _plan(n, ny, nx, f)
    got = _gpu(plan, vol, W.EDGE_TAU)
    plan.close()
    ref = _oracle_images(vol, W.EDGE_TAU, range(nx))
    assert ref[1].any()
    _assert_same(got, ref, "phantom")


def test_noise_many_rerouted_windows():
    rng = np.random.default_rng(5)
    n, ny, nx, f = 6, 48, 20, 4
    Z = (n - 1) * f + 1
    vol = rng.normal(0.0, 1.0, size=(Z, ny, nx)).astype(np.float32)
    tau = 30.0
    print(f"edge post-pass noise {vol.shape}", flush=True)
    assert _rerouted(vol, tau, range(nx)) >= 10
    plan = _plan(n, ny, nx, f)
    got = _gpu(plan, vol, tau)
    ref = _oracle_images(vol, tau, range(nx))
    assert (ref[0] != vol).any()     # medians were applied
    _assert_same(got, ref, "noise")
    # a second call on the same plan gives the same bits
    again = _gpu(plan, vol, tau)
    plan.close()
    _assert_same(again, ref, "noise (second call)")


def test_in_place_and_threshold_extremes():
    n, ny, nx, f = 4, 40, 24, 4
    w, vol = _phantom(n, 40, f, 21)
    vol = vol[:, :ny, :nx].copy()
    print(f"edge post-pass in place {vol.shape}", flush=True)
    plan = _plan(n, ny, nx, f)
    got = _gpu(plan, vol, W.EDGE_TAU, inplace=True)
    _assert_same(got, _oracle_images(vol, W.EDGE_TAU, range(nx)), "in place")
    # a threshold above every M: no edges, volume unchanged
    out, edge, orient, mag = _gpu(plan, vol, 1e30)
    assert not edge.any() and np.array_equal(out, vol)
    # threshold 0: every local maximum along its normal is an edge
    got = _gpu(plan, vol, 0.0)
    plan.close()
    _assert_same(got, _oracle_images(vol, 0.0, range(nx)), "tau 0")


def test_constant_volume_has_no_edges():
    n, ny, nx, f = 3, 20, 10, 4
    vol = np.full(((n - 1) * f + 1, ny, nx), 0.25, np.float32)
    plan = _plan(n, ny, nx, f)
    out, edge, orient, mag = _gpu(plan, vol, 1e-9)
    plan.close()
    assert not edge.any() and np.array_equal(out, vol)
    assert np.abs(mag).max() < 1e-12


@pytest.mark.parametrize("n,ny,nx,f", [(1, 7, 5, 4), (2, 1, 4, 3), (2, 2, 1, 2)])
def test_degenerate_shapes(n, ny, nx, f):
    rng = np.random.default_rng(n * 100 + ny)
    Z = (n - 1) * f + 1
    vol = rng.normal(0.0, 1.0, size=(Z, ny, nx)).astype(np.float32)
    print(f"edge post-pass degenerate {vol.shape}", flush=True)
    plan = _plan(n, ny, nx, f)
    got = _gpu(plan, vol, 1.0)
    plan.close()
    _assert_same(got, _oracle_images(vol, 1.0, range(nx)), "degenerate")


def test_bitmaps_beyond_lds():
    # (Z + 2) * ceil((ny + 2) / 32) * 4 bytes > 64 KB: traced in global memory
    n, ny, nx, f = 509, 290, 3, 4
    Z = (n - 1) * f + 1
    assert (Z + 2) * ((ny + 2 + 31) // 32) * 4 > 65536
    w = W.Workload("edge_pass_tall", n, ny, f, 1, False, 30, 6, 0.02,
                   W.Variogram("spherical", 0.0, 1.0, 4.0), 31)
    vol = np.ascontiguousarray(W.postpass_volume(w)[:, :ny, :nx])
    print(f"edge post-pass tall {vol.shape}", flush=True)
    plan = _plan(n, ny, nx, f)
    got = _gpu(plan, vol, W.EDGE_TAU)
    plan.close()
    ref = _oracle_images(vol, W.EDGE_TAU, range(nx))
    assert _rerouted(vol, W.EDGE_TAU, range(nx)) > 0
    _assert_same(got, ref, "tall")


def test_full_size_sampled_images():
    import torch
    w = W.workload("large_160x512")
    vol = W.postpass_volume(w)
    print(f"edge post-pass full size {vol.shape}", flush=True)
    plan = _plan(w.nslices, w.m, w.m, w.upsample)
    v = torch.from_numpy(vol).cuda()
    mag = torch.empty(v.shape, dtype=torch.float64, device="cuda")
    out, edge, orient = plan.edge_postpass(v, W.EDGE_TAU, mag=mag)
    out2, edge2, orient2 = plan.edge_postpass(v, W.EDGE_TAU)
    plan.close()
    assert torch.equal(out, out2) and torch.equal(edge, edge2) and torch.equal(orient, orient2)
    xs = [0, 137, 300, 511]
    got = (out[:, :, xs].cpu().numpy(), edge[:, :, xs].cpu().numpy(),
           orient[:, :, xs].cpu().numpy(), mag[:, :, xs].cpu().numpy())
    ref = _oracle_images(vol, W.EDGE_TAU, xs)
    print(f"  sampled images {xs}: {int(ref[1].sum())} edge pixels, "
          f"{int((ref[0] != vol[:, :, xs]).sum())} voxels changed", flush=True)
    _assert_same(got, ref, "full size")
    # properties on the whole volume: orientations in range, a few percent
    # of the pixels are edges
    e = edge.cpu().numpy()
    assert int(orient.max()) <= 7
    assert e.mean() > 0.005

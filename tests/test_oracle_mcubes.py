"""Pins of the marching-cubes oracle (Appendix C) against geometry and
topology: closed forms for single cubes and planes, watertight manifold
meshes with the Euler characteristic of the sphere, torus and two spheres,
enclosed volume and area against the analytic values, and closed,
consistently oriented surfaces on random fields (ambiguous faces included)."""
import math

import numpy as np
import pytest

from oracle import mcubes as M


def _closed_and_oriented(faces):
    """Every directed edge of the welded mesh has exactly one reverse."""
    directed = {}
    for f in faces:
        for i in range(3):
            a, b = f[i], f[(i + 1) % 3]
            directed[(a, b)] = directed.get((a, b), 0) + 1
    for (a, b), m in directed.items():
        if m != 1 or directed.get((b, a), 0) != 1:
            return False
    return True


def _boundary_free(faces):
    """The oriented triangles form a closed chain: every directed edge occurs
    as often as its reverse (no hole, no orientation flip). Unlike
    _closed_and_oriented this allows two polygons of neighbouring cubes that
    both cross their shared face twice to meet along a fan diagonal lying in
    that face."""
    directed = {}
    for f in faces:
        for i in range(3):
            a, b = f[i], f[(i + 1) % 3]
            directed[(a, b)] = directed.get((a, b), 0) + 1
    return all(directed.get((b, a), 0) == m for (a, b), m in directed.items())


def _euler(faces):
    verts = set(v for f in faces for v in f)
    edges = set()
    for f in faces:
        for i in range(3):
            a, b = f[i], f[(i + 1) % 3]
            edges.add((a, b) if a < b else (b, a))
    return len(verts) - len(edges) + len(faces)


def test_every_configuration_partitions_its_crossing_edges():
    for cfg in range(256):
        inside = [(cfg >> c) & 1 for c in range(8)]
        crossing = set()
        for e in range(12):
            lo, hi, _ = M.edge_corners(e)
            if inside[lo] != inside[hi]:
                crossing.add(e)
        polys = M.cube_polygons(inside)
        used = [e for p in polys for e in p]
        assert sorted(used) == sorted(crossing), cfg
        assert all(len(p) >= 3 for p in polys)
        assert [p[0] for p in polys] == sorted(min(p) for p in polys)
        tris = M.cube_triangles(inside)
        assert len(tris) == sum(len(p) - 2 for p in polys)
        # complementary configurations cross the same edges
        comp = [1 - v for v in inside]
        assert sorted(e for p in M.cube_polygons(comp) for e in p) == sorted(crossing)


def test_single_corner_closed_form():
    vol = np.zeros((2, 2, 2), np.float32)
    vol[0, 0, 0] = 1.0
    tris, ids = M.marching_cubes(vol, 0.5)
    assert tris.shape == (1, 3, 3) and list(ids) == [0]
    got = sorted(map(tuple, tris[0].tolist()))
    assert got == sorted([(0.5, 0.0, 0.0), (0.0, 0.5, 0.0), (0.0, 0.0, 0.5)])
    n = np.cross(tris[0, 1] - tris[0, 0], tris[0, 2] - tris[0, 0])
    assert n @ np.ones(3) > 0   # away from the inside corner


def test_interpolation_closed_form():
    # one edge along y from A = 0.2 (outside) to B = 1.7 (inside), iso 1.1
    vol = np.zeros((2, 2, 2), np.float32)
    vol[:, 1, :] = np.float32(1.7)
    vol[:, 0, :] = np.float32(0.2)
    tris, _ = M.marching_cubes(vol, 1.1)
    t = (np.float32(1.1) - np.float32(0.2)) / (np.float32(1.7) - np.float32(0.2))
    assert tris.shape == (2, 3, 3)
    assert np.all(tris[:, :, 1] == np.float32(0.0) + t)
    # normal from inside (y = 1) to outside (y = 0)
    for tri in tris:
        assert np.cross(tri[1] - tri[0], tri[2] - tri[0])[1] < 0


def test_plane():
    nz, ny, nx = 5, 4, 6
    vol = np.broadcast_to(np.arange(nz, dtype=np.float32)[:, None, None], (nz, ny, nx))
    tris, ids = M.marching_cubes(vol, 2.5)
    assert tris.shape[0] == 2 * (ny - 1) * (nx - 1)
    assert np.all(tris[:, :, 2] == np.float32(2.5))
    assert abs(M.mesh_area(tris) - (ny - 1) * (nx - 1)) < 1e-9
    n = np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0])
    assert np.all(n[:, 2] < 0)   # inside is z >= 2.5
    assert np.all(np.diff(ids) >= 0)


def test_checkerboard_cube_separates_inside_corners():
    inside = [0] * 8
    for c in (0, 3, 5, 6):
        inside[c] = 1
    polys = M.cube_polygons(inside)
    assert len(polys) == 4 and all(len(p) == 3 for p in polys)
    for p in polys:   # each triangle surrounds one inside corner: its three edges share it
        common = None
        for e in p:
            lo, hi, _ = M.edge_corners(e)
            common = {lo, hi} if common is None else common & {lo, hi}
        assert len(common) == 1 and inside[common.pop()] == 1


def _sphere(n, c, R):
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    return (R - np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)).astype(np.float32)


def test_sphere_closed_volume_area():
    R = 5.0
    vol = _sphere(16, (7.5, 7.3, 7.1), R)
    faces = M.mesh_topology(vol, 0.0)
    assert _closed_and_oriented(faces)
    assert _euler(faces) == 2
    tris, _ = M.marching_cubes(vol, 0.0)
    V = M.mesh_volume(tris)
    assert V > 0
    assert abs(V / (4.0 / 3.0 * math.pi * R ** 3) - 1.0) < 0.03
    assert abs(M.mesh_area(tris) / (4.0 * math.pi * R ** 2) - 1.0) < 0.05


def test_torus_and_two_spheres_euler():
    n = 20
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    c = (9.6, 9.4, 9.7)
    q = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2) - 5.5
    torus = (2.2 - np.sqrt(q ** 2 + (z - c[2]) ** 2)).astype(np.float32)
    faces = M.mesh_topology(torus, 0.0)
    assert _closed_and_oriented(faces)
    assert _euler(faces) == 0
    two = np.maximum(_sphere(n, (5.3, 5.6, 9.2), 3.1), _sphere(n, (14.4, 13.9, 9.6), 3.3))
    faces = M.mesh_topology(two, 0.0)
    assert _closed_and_oriented(faces)
    assert _euler(faces) == 4


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_random_fields_closed_and_oriented(seed):
    rng = np.random.default_rng(seed)
    vol = rng.standard_normal((9, 8, 10)).astype(np.float32)
    vol[0] = vol[-1] = -10.0
    vol[:, 0] = vol[:, -1] = -10.0
    vol[:, :, 0] = vol[:, :, -1] = -10.0
    faces = M.mesh_topology(vol, 0.1)
    assert len(faces) > 50
    assert _boundary_free(faces)
    tris, _ = M.marching_cubes(vol, 0.1)
    assert M.mesh_volume(tris) > 0


def test_nan_corners_are_outside_and_empty_shapes():
    vol = np.full((2, 2, 2), np.nan, np.float32)
    tris, ids = M.marching_cubes(vol, 0.0)
    assert tris.shape == (0, 3, 3)
    for shape in [(1, 5, 5), (5, 1, 5), (5, 5, 1), (0, 3, 3)]:
        tris, ids = M.marching_cubes(np.zeros(shape, np.float32), 0.0)
        assert tris.shape == (0, 3, 3) and ids.shape == (0,)

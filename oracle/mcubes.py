"""CPU oracle for marching cubes on the reconstructed volume.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module. The product path never
calls it, and it shares no code or tables with that path: the library builds
its case table with its own code, this module derives every cube's polygons
directly from the corner signs.

What it computes (Appendix C): the volume is divided into unit cubes between
neighbouring voxels; each cube's eight corners are classified against the
threshold; where a cube's corners disagree, the surface crosses the cube's
edges at points found by linear interpolation, and the crossing points are
joined into triangles.

Readings of what the paper leaves open (the definition implemented here):

* Threshold: a parameter ``iso``; a corner is inside when its value >= iso
  (NaN is outside). Coordinates are voxel indices (x, y, z), z counting the
  output planes.
* Numbering: corner c = x + 2y + 4z of the cube (x, y, z in {0, 1}); edge
  e = 4a + u + 2w runs along axis a (0 = x, 1 = y, 2 = z) from the corner with
  bit a clear to the one with bit a set, u and w being its coordinates on the
  other two axes in increasing axis order.
* Crossing point on an edge from corner value A (lower end) to B:
  t = (iso - A) / (B - A), in float32, added to the float32 coordinate of the
  lower end along the edge's axis.
* Faces: on each cube face the crossing edges are paired into segments. With
  two crossings the pair is obvious; with four (diagonal corners alike) each
  segment cuts off one inside corner. A shared face is paired identically by
  both cubes, so the surface has no holes.
* Polygons: the segments chain into closed cycles (each crossing edge lies on
  two faces). A cycle is oriented so that its normal points from inside to
  outside: the vector area of the cycle through the edge midpoints has a
  positive dot product with the sum of the cycle edges' inside-to-outside
  directions.
* Triangles: each cycle is a fan from its lowest edge id, following the
  orientation; a cube's polygons are taken in order of their lowest edge id,
  cubes in order of the linear index (z * (ny-1) + y) * (nx-1) + x.
* Smoothing after marching cubes (the paper cites one) is not specified and
  not done.
"""
import numpy as np

__all__ = ["corner_xyz", "edge_corners", "cube_polygons", "cube_triangles",
           "marching_cubes", "marching_cubes_cubes", "mesh_topology", "mesh_volume",
           "mesh_area", "vertex_key"]


def corner_xyz(c):
    """Corner c -> (x, y, z) in {0, 1}^3."""
    return (c & 1, (c >> 1) & 1, (c >> 2) & 1)


def _other_axes(a):
    return [b for b in range(3) if b != a]


def edge_corners(e):
    """Edge e -> (lower corner, upper corner, axis)."""
    a, k = divmod(e, 4)
    u, w = k & 1, k >> 1
    b0, b1 = _other_axes(a)
    lo = (u << b0) | (w << b1)
    return lo, lo | (1 << a), a


def _edge_between(c0, c1):
    """The cube edge joining corners c0 and c1 (which differ in one bit)."""
    d = c0 ^ c1
    a = d.bit_length() - 1
    lo = min(c0, c1)
    b0, b1 = _other_axes(a)
    u, w = (lo >> b0) & 1, (lo >> b1) & 1
    return 4 * a + u + 2 * w


def _faces():
    """Each face as its four corners in cyclic order."""
    out = []
    for a in range(3):
        b0, b1 = _other_axes(a)
        for s in (0, 1):
            ring = []
            for (p, q) in ((0, 0), (1, 0), (1, 1), (0, 1)):
                ring.append((s << a) | (p << b0) | (q << b1))
            out.append(ring)
    return out


def _face_segments(ring, inside):
    """Pairs of crossing edges on one face (the face rule of the header)."""
    cross = []   # (position around the ring, edge)
    for i in range(4):
        c0, c1 = ring[i], ring[(i + 1) % 4]
        if inside[c0] != inside[c1]:
            cross.append((i, _edge_between(c0, c1)))
    if len(cross) == 2:
        return [(cross[0][1], cross[1][1])]
    if len(cross) == 4:
        segs = []
        for j in range(4):
            i, e = cross[j]
            i2, e2 = cross[(j + 1) % 4]
            shared = ring[(i + 1) % 4]   # corner between consecutive ring edges i and i+1
            if inside[shared]:
                segs.append((e, e2))
        assert len(segs) == 2
        return segs
    assert not cross
    return []


def _midpoint(e):
    lo, hi, a = edge_corners(e)
    p = np.array(corner_xyz(lo), dtype=np.float64)
    p[a] += 0.5
    return p


def cube_polygons(inside):
    """Oriented polygons (lists of edge ids) of a cube whose corner c is inside
    when inside[c] is true; polygons sorted by their lowest edge id, each
    starting at its lowest edge id."""
    inside = [bool(v) for v in inside]
    adj = {}
    for ring in _faces():
        for e0, e1 in _face_segments(ring, inside):
            adj.setdefault(e0, []).append(e1)
            adj.setdefault(e1, []).append(e0)
    for e, nb in adj.items():
        assert len(nb) == 2, (e, nb)
    polys, seen = [], set()
    for start in sorted(adj):
        if start in seen:
            continue
        cyc, prev, cur = [start], None, start
        seen.add(start)
        while True:
            a, b = adj[cur]
            nxt = b if a == prev else a
            if nxt == start:
                break
            cyc.append(nxt)
            seen.add(nxt)
            prev, cur = cur, nxt
        # orientation: normal from inside to outside
        area = np.zeros(3)
        for i in range(len(cyc)):
            area += np.cross(_midpoint(cyc[i]), _midpoint(cyc[(i + 1) % len(cyc)]))
        out_dir = np.zeros(3)
        for e in cyc:
            lo, hi, a = edge_corners(e)
            out_dir[a] += 1.0 if inside[lo] else -1.0   # from the inside end to the outside end
        if float(area @ out_dir) < 0.0:
            cyc = [cyc[0]] + cyc[1:][::-1]
        polys.append(cyc)
    return polys


def cube_triangles(inside):
    """Triangles (edge-id triples) of one cube configuration."""
    tris = []
    for cyc in cube_polygons(inside):
        for i in range(1, len(cyc) - 1):
            tris.append((cyc[0], cyc[i], cyc[i + 1]))
    return tris


def _vertex(vol, x, y, z, e, iso):
    lo, hi, a = edge_corners(e)
    l = corner_xyz(lo)
    h = corner_xyz(hi)
    A = vol[z + l[2], y + l[1], x + l[0]]
    B = vol[z + h[2], y + h[1], x + h[0]]
    with np.errstate(invalid="ignore", divide="ignore"):
        t = (np.float32(iso) - A) / (B - A)
    p = [np.float32(x + l[0]), np.float32(y + l[1]), np.float32(z + l[2])]
    p[a] = np.float32(p[a] + t)
    return p


def marching_cubes_cubes(vol, iso, cubes):
    """Triangles of the listed cubes (linear indices), in the listed order:
    float32 [T, 3, 3] vertex coordinates (x, y, z) and int64 [T] cube ids."""
    vol = np.asarray(vol, dtype=np.float32)
    nz, ny, nx = vol.shape
    iso = np.float32(iso)
    memo = {}
    verts, ids = [], []
    for cid in cubes:
        cid = int(cid)
        x = cid % (nx - 1)
        y = (cid // (nx - 1)) % (ny - 1)
        z = cid // ((nx - 1) * (ny - 1))
        cfg = 0
        for c in range(8):
            cx, cy, cz = corner_xyz(c)
            if vol[z + cz, y + cy, x + cx] >= iso:
                cfg |= 1 << c
        if cfg not in memo:
            memo[cfg] = cube_triangles([(cfg >> c) & 1 for c in range(8)])
        for tri in memo[cfg]:
            verts.append([_vertex(vol, x, y, z, e, iso) for e in tri])
            ids.append(cid)
    if not verts:
        return np.zeros((0, 3, 3), np.float32), np.zeros(0, np.int64)
    return np.asarray(verts, dtype=np.float32), np.asarray(ids, dtype=np.int64)


def marching_cubes(vol, iso):
    """All triangles of a volume [nz, ny, nx] (see marching_cubes_cubes)."""
    nz, ny, nx = np.asarray(vol).shape
    if nz < 2 or ny < 2 or nx < 2:
        return np.zeros((0, 3, 3), np.float32), np.zeros(0, np.int64)
    return marching_cubes_cubes(vol, iso, range((nz - 1) * (ny - 1) * (nx - 1)))


# ---- mesh checks (used by the pins) ----

def vertex_key(cid, e, nx, ny):
    """A crossing point's identity independent of the cube that emits it: the
    global grid edge (lower voxel, axis)."""
    x = cid % (nx - 1)
    y = (cid // (nx - 1)) % (ny - 1)
    z = cid // ((nx - 1) * (ny - 1))
    lo, hi, a = edge_corners(e)
    cx, cy, cz = corner_xyz(lo)
    return (x + cx, y + cy, z + cz, a)


def mesh_topology(vol, iso):
    """Welded mesh of the volume: (faces as vertex-key triples, set of
    directed edges with multiplicity)."""
    vol = np.asarray(vol, dtype=np.float32)
    nz, ny, nx = vol.shape
    faces = []
    for cid in range((nz - 1) * (ny - 1) * (nx - 1)):
        x = cid % (nx - 1)
        y = (cid // (nx - 1)) % (ny - 1)
        z = cid // ((nx - 1) * (ny - 1))
        inside = []
        for c in range(8):
            cx, cy, cz = corner_xyz(c)
            inside.append(vol[z + cz, y + cy, x + cx] >= iso)
        for tri in cube_triangles(inside):
            faces.append(tuple(vertex_key(cid, e, nx, ny) for e in tri))
    return faces


def mesh_volume(tris):
    """Signed enclosed volume (divergence theorem) of a triangle soup."""
    t = np.asarray(tris, dtype=np.float64)
    return float(np.einsum("ij,ij->i", t[:, 0], np.cross(t[:, 1], t[:, 2])).sum() / 6.0)


def mesh_area(tris):
    t = np.asarray(tris, dtype=np.float64)
    return float(0.5 * np.linalg.norm(np.cross(t[:, 1] - t[:, 0], t[:, 2] - t[:, 0]), axis=1).sum())

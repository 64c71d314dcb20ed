"""Pins of the oracle's marching cubes (the mesh extraction of Sec. III and
Sec. VI): closed forms of area and enclosed volume, exact planes, topology
(every edge of a closed surface shared by two triangles, Euler
characteristic 2 for a sphere and 0 for a torus), outward orientation, and
watertightness across cells on random fields (the ambiguous-face rule must
agree between neighbours)."""
import math

import numpy as np
import pytest

import oracle


def _weld(tri):
    """Vertices shared by exact coordinates -> (V, F) index form."""
    v = tri.reshape(-1, 3)
    uniq, inv = np.unique(v, axis=0, return_inverse=True)
    return uniq, inv.reshape(-1, 3)


def _edge_counts(F):
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    e = np.sort(e, axis=1)
    _, cnt = np.unique(e, axis=0, return_counts=True)
    return e, cnt


def _area_volume(tri):
    a, b, c = tri[:, 0].astype(np.float64), tri[:, 1].astype(np.float64), tri[:, 2].astype(np.float64)
    cr = np.cross(b - a, c - a)
    area = 0.5 * np.linalg.norm(cr, axis=1).sum()
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0  # divergence theorem
    return area, vol


def _field(res, lo, hi, f):
    p = oracle.grid_points(res, lo, hi).astype(np.float64)
    return f(p[:, 0], p[:, 1], p[:, 2]).astype(np.float32)


def test_case_table_basics():
    assert len(oracle.mc_case(0)) == 0 and len(oracle.mc_case(255)) == 0
    t = oracle.mc_case(1)  # corner 0 inside: one triangle on its three edges 0 (x), 4 (y), 8 (z)
    assert t.shape == (1, 3) and sorted(t[0]) == [0, 4, 8]
    ends = {0: (0, 1), 2: (4, 5), 4: (0, 2), 6: (4, 6), 8: (0, 4)}
    crossing_ok = True
    for m in range(256):
        tris = oracle.mc_case(m)
        used = set(tris.reshape(-1).tolist())
        # exactly the edges whose two corners differ carry vertices
        edges_x = [(c, c | 1) for c in (0, 2, 4, 6)]
        edges_y = [(c, c | 2) for c in (0, 1, 4, 5)]
        edges_z = [(c, c | 4) for c in (0, 1, 2, 3)]
        want = {e for e, (a, b) in enumerate(edges_x + edges_y + edges_z)
                if ((m >> a) & 1) != ((m >> b) & 1)}
        crossing_ok &= used == want
        assert len(tris) <= 5
    assert crossing_ok


@pytest.mark.parametrize("res", [24, 48])
def test_sphere_area_volume_topology(res):
    r = 0.6
    lo, hi = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    g = _field(res, lo, hi, lambda x, y, z: r - np.sqrt((x - 0.05) ** 2 + (y + 0.03) ** 2 + z ** 2))
    tri = oracle.marching_cubes(g, res, 0.0, lo, hi)
    V, F = _weld(tri)
    _, cnt = _edge_counts(F)
    assert (cnt == 2).all()  # closed
    E = cnt.size
    assert len(V) - E + len(F) == 2  # sphere
    area, vol = _area_volume(tri)
    h = 2.0 / res
    assert abs(area - 4 * math.pi * r * r) < 0.02 * 4 * math.pi * r * r
    assert abs(vol - 4 / 3 * math.pi * r ** 3) < 0.02 * 4 / 3 * math.pi * r ** 3
    assert vol > 0  # outward normals
    rad = np.linalg.norm(V.astype(np.float64) - [0.05, -0.03, 0.0], axis=1)
    assert np.abs(rad - r).max() < h * h  # linear interpolation of a smooth field


def test_torus_topology():
    res, R0, r0 = 40, 0.55, 0.22
    lo, hi = (-1.0, -1.0, -0.5), (1.0, 1.0, 0.5)
    g = _field(res, lo, hi, lambda x, y, z: r0 * r0 - ((np.sqrt(x * x + y * y) - R0) ** 2 + z * z))
    tri = oracle.marching_cubes(g, res, 0.0, lo, hi)
    V, F = _weld(tri)
    _, cnt = _edge_counts(F)
    assert (cnt == 2).all()
    assert len(V) - cnt.size + len(F) == 0  # genus 1
    area, vol = _area_volume(tri)
    assert abs(vol - 2 * math.pi ** 2 * R0 * r0 * r0) < 0.03 * 2 * math.pi ** 2 * R0 * r0 * r0


def test_plane_is_exact():
    res = 16
    lo, hi = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)
    g = _field(res, lo, hi, lambda x, y, z: 0.3 - z + 0.0 * x)  # inside below z = 0.3
    tri = oracle.marching_cubes(g, res, 0.0, lo, hi)
    assert np.abs(tri[..., 2] - 0.3).max() < 2e-7
    area, _ = _area_volume(tri)
    assert abs(area - 4.0) < 1e-5
    n = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
    assert (n[:, 2] > 0).all()  # pointing from inside (below) to outside (above)


def test_random_field_watertight_inside_the_grid():
    rng = np.random.default_rng(3)
    res = 12
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    g = rng.standard_normal((res + 1) ** 3).astype(np.float32)
    tri = oracle.marching_cubes(g, res, 0.0, lo, hi)
    V, F = _weld(tri)
    e, _ = _edge_counts(F)
    uniq, cnt = np.unique(e, axis=0, return_counts=True)
    on_border = np.zeros(len(uniq), bool)
    for a in range(3):
        for b in (0.0, 1.0):
            on_border |= (V[uniq[:, 0], a] == b) & (V[uniq[:, 1], a] == b)
    assert (cnt[~on_border] == 2).all()  # every inner edge shared by two triangles
    assert (cnt[on_border] == 1).all()


def test_object_mesh_in_world_frame():
    """The world transform of the object mesh: Rz(yaw) x + t of the
    object-frame triangles (FP64)."""
    cfg = oracle.make_config(L=2, nmin=4, nmax=8, log2T=8, N=32)
    o = oracle.OracleContext(cfg)
    oid = o.add_object(3, np.array([1.0, -2.0, 0.5], np.float32), 0.7,
                       np.array([0.5, 0.4, 0.3], np.float32))
    ob = o.objects[oid]
    rng = np.random.default_rng(0)
    ob.params[:] = rng.standard_normal(ob.params.size) * 2.0
    world, local = o.extract_mesh(oid, res=8, iso=1.0)
    assert len(local) > 0
    c, s = math.cos(ob.yaw), math.sin(ob.yaw)
    x = local[..., 0].astype(np.float64)
    y = local[..., 1].astype(np.float64)
    assert np.allclose(world[..., 0], c * x - s * y + 1.0)
    assert np.allclose(world[..., 1], s * x + c * y - 2.0)
    assert np.all(np.abs(local) <= ob.half + 1e-7)


# ------------------------------------------------------------------ box from points (Eq. 1, PCA, Eq. 4)
def _box_cloud(t0, yaw0, half0, n, seed):
    """Points filling a yawed box: its 8 corners and random interior points,
    mirrored through the box axes (a centrally and axially symmetric cloud)."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1, 1, (n, 3))
    s = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)], float)
    local = np.concatenate([s] + [u * f for f in s]) * half0
    c, sn = math.cos(yaw0), math.sin(yaw0)
    R = np.array([[c, -sn, 0], [sn, c, 0], [0, 0, 1]])
    return local @ R.T + t0


@pytest.mark.parametrize("yaw0", [-0.7, -0.2, 0.0, 0.4, 0.75])
def test_box_from_symmetric_cloud_is_exact(yaw0):
    t0 = np.array([1.5, -0.4, 0.35])
    half0 = np.array([0.6, 0.25, 0.35])  # long axis along the box x
    t, yaw, half = oracle.box_from_points(_box_cloud(t0, yaw0, half0, 300, 7))
    assert np.allclose(t, t0, atol=1e-12)       # Eq. 1: midpoint of the world extremes
    assert abs(yaw - yaw0) < 1e-9                # PCA axis of a symmetric box cloud
    assert np.allclose(half, half0, atol=1e-9)   # Eq. 4 with the corners present


def test_box_yaw_is_folded_and_axis_swaps():
    t0 = np.zeros(3)
    half0 = np.array([0.6, 0.25, 0.35])
    _, y1, h1 = oracle.box_from_points(_box_cloud(t0, 0.3 + math.pi, half0, 200, 1))
    assert abs(y1 - 0.3) < 1e-9 and np.allclose(h1, half0, atol=1e-9)
    # long axis along y: the principal axis is the box y axis, so yaw turns by pi/2
    # and the extents swap
    half1 = np.array([0.25, 0.6, 0.35])
    _, y2, h2 = oracle.box_from_points(_box_cloud(t0, 0.2, half1, 200, 2))
    assert abs(y2 - (0.2 - math.pi / 2)) < 1e-9
    assert np.allclose(h2, [0.6, 0.25, 0.35], atol=1e-9)


def test_box_from_one_point():
    t, yaw, half = oracle.box_from_points(np.array([[0.3, 0.2, 0.1]]))
    assert np.allclose(t, [0.3, 0.2, 0.1]) and yaw == 0.0 and np.allclose(half, 0.0)
    with pytest.raises(ValueError):
        oracle.box_from_points(np.zeros((0, 3)))

"""Meshing on the GPU (marching cubes, Sec. III / Sec. VI) against the oracle:
the triangles of a given grid bit for bit and in order; an object's mesh
from its own density grid, object frame and world frame."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2304_05735_amd as pk
from tests.tiny import random_params

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _ctx():
    return pk.Context(pk.default_config(n_levels=4, base_res=8, max_res=32, log2_table_size=10,
                                        samples_per_ray=32, autotune=0))


@pytest.mark.parametrize("kind,res", [("sphere", 1), ("sphere", 17), ("sphere", 64),
                                      ("random", 23), ("torus", 40)])
def test_marching_cubes_matches_oracle_bit_for_bit(kind, res):
    _say("mc", kind, res)
    rng = np.random.default_rng(res)
    lo = np.array([-1.0, -0.8, -0.6], np.float32)
    hi = np.array([0.9, 1.1, 0.7], np.float32)
    p = oracle.grid_points(res, lo, hi).astype(np.float64)
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    if kind == "sphere":
        g = 0.7 - np.sqrt(x * x + y * y + z * z)
    elif kind == "torus":
        g = 0.04 - ((np.sqrt(x * x + y * y) - 0.5) ** 2 + z * z)
    else:
        g = rng.standard_normal(p.shape[0])
    g = g.astype(np.float32)
    ctx = _ctx()
    tri = ctx.marching_cubes(g, res, 0.0, lo, hi)
    ref = oracle.marching_cubes(g, res, 0.0, lo, hi)
    assert tri.shape == ref.shape
    assert np.array_equal(tri, ref)
    # device buffers give the same
    td = ctx.marching_cubes(torch.from_numpy(g).cuda(), res, 0.0, lo, hi)
    assert np.array_equal(td.cpu().numpy(), ref)


def test_count_only_and_truncated_output():
    res = 20
    lo, hi = np.zeros(3, np.float32), np.ones(3, np.float32)
    p = oracle.grid_points(res, lo, hi).astype(np.float64)
    g = (0.4 - np.linalg.norm(p - 0.5, axis=1)).astype(np.float32)
    ctx = _ctx()
    ref = oracle.marching_cubes(g, res, 0.0, lo, hi)
    import ctypes as C
    n = C.c_int64(0)
    gg = np.ascontiguousarray(g)
    assert pk.lib().romap_marching_cubes(ctx.h, pk._ptr(gg), res, 0.0, pk._ptr(lo), pk._ptr(hi),
                                         None, 0, C.byref(n), 0) == 0
    assert n.value == len(ref)
    out = np.full((10, 9), -7.0, np.float32)
    assert pk.lib().romap_marching_cubes(ctx.h, pk._ptr(gg), res, 0.0, pk._ptr(lo), pk._ptr(hi),
                                         pk._ptr(out), 7, C.byref(n), 0) == 0
    assert n.value == len(ref)
    assert np.array_equal(out[:7], ref[:7].reshape(7, 9)) and (out[7:] == -7.0).all()
    assert pk.lib().romap_marching_cubes(ctx.h, pk._ptr(gg), 0, 0.0, pk._ptr(lo), pk._ptr(hi),
                                         None, 0, C.byref(n), 0) == pk.ROMAP_E_INVALID_ARG


def test_object_mesh_object_and_world_frame():
    """extract_mesh = the object's density on its box corners (the same
    values as query_density) meshed by the oracle's marching cubes, then
    the box pose."""
    _say("object mesh")
    ctx = _ctx()
    t = np.array([0.4, -1.2, 0.3], np.float32)
    yaw = 0.6
    half = np.array([0.5, 0.35, 0.25], np.float32)
    oid = ctx.add_object(5, t, yaw, half)
    p = random_params(ctx.object_info(oid).n_grid_params, 8, seed=3)
    ctx.set_params(oid, (p * 3.0).astype(np.float32))
    res, iso = 24, 1.2
    pts = oracle.grid_points(res, -half, half)
    sig = ctx.query_density(oid, pts)
    local = ctx.extract_mesh(oid, res, iso, world=False)
    ref = oracle.marching_cubes(sig, res, iso, -half, half)
    assert len(ref) > 50
    assert np.array_equal(local, ref)
    world = ctx.extract_mesh(oid, res, iso, world=True)
    c, s = math.cos(np.float32(yaw)), math.sin(np.float32(yaw))
    R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
    want = local.astype(np.float64) @ R.T + t
    assert np.abs(world - want).max() < 1e-5 * (1 + np.abs(want).max())

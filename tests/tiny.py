"""Tiny seeded workloads shared by the oracle pins and the GPU parity tests.

Only inputs live here (cameras, images, masks, depth, parameter draws): no
arithmetic of the method.
"""
import math

import numpy as np

import scenes


def tiny_scene(W=24, H=20, n_views=3, seed=0):
    """Two spheres (instance 1 = trained object, 2 = occluder) seen from a few
    cameras; sparse depth on some object pixels.  All three ray classes occur."""
    prims = [scenes.Primitive("sphere", np.array([0.0, 0.0, 0.0]), np.array([0.3]), 0.0, 1),
             scenes.Primitive("sphere", np.array([0.35, -0.5, 0.1]), np.array([0.15]), 0.0, 2,
                              np.array([1.0, 2.0, 3.0]))]
    sc = scenes.Scene(prims)
    rng = np.random.default_rng(seed)
    frames = []
    for k in range(n_views):
        ang = 2 * math.pi * k / n_views + 0.3
        eye = (1.6 * math.cos(ang), 1.6 * math.sin(ang), 0.4 + 0.2 * k)
        cam = scenes.camera(scenes.look_at(eye, (0, 0, 0)), W, H, 0.9 * W, 0.9 * W, W / 2 + 0.25,
                            H / 2 - 0.25)
        rgb, mask, dz = sc.render(cam)
        depth = np.zeros_like(dz)
        obj = np.flatnonzero(mask.reshape(-1) == 1)
        pick = rng.choice(obj, max(1, obj.size // 4), replace=False)
        depth.reshape(-1)[pick] = dz.reshape(-1)[pick]
        frames.append((cam, scenes.to_u8(rgb), mask, depth))
    box = dict(instance=1, t=np.array([0.02, -0.01, 0.0], np.float32), yaw=0.2,
               half=np.array([0.36, 0.33, 0.35], np.float32))
    return frames, box


def random_params(n_grid, din, seed=0, grid_scale=0.5, layers=1):
    """Grid U(-s, s); MLP Glorot-uniform.  Layout: grid, W1 (64 x din), layers - 1
    matrices 64 x 64 (density MLP), W2 (16 x 64), W3 (64 x 15), W4 (3 x 64)."""
    rng = np.random.default_rng(seed)
    grid = rng.uniform(-grid_scale, grid_scale, n_grid)
    mats = []
    for (o, i) in [(64, din)] + [(64, 64)] * (layers - 1) + [(16, 64), (64, 15), (3, 64)]:
        lim = math.sqrt(6.0 / (o + i))
        mats.append(rng.uniform(-lim, lim, o * i))
    return np.concatenate([grid] + mats)

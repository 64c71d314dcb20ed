"""Oracle pins of the deeper density MLPs (the model-size study of Table 4:
density MLPs of 1, 2 and 3 hidden layers of 64).

The forward of a deeper MLP is pinned by two invariants that hold for any
ReLU network and that a dropped layer, a transposed or mis-offset matrix
would break: identity hidden-to-hidden matrices reduce it to the one-layer
model (ReLU outputs are non-negative), and permuting the hidden units of a
layer (rows of the matrix that makes them, columns of the one that reads
them) changes nothing.  The backward is pinned by central finite
differences and directional derivatives of the forward.
"""
import math

import numpy as np
import pytest

import oracle
from tests.tiny import random_params, tiny_scene

H = 64


def _split(p, din, layers):
    """W1, [Wh...], W2, W3, W4 views of an MLP parameter vector."""
    o = 0
    W1 = p[o:o + H * din].reshape(H, din)
    o += H * din
    Wh = []
    for _ in range(layers - 1):
        Wh.append(p[o:o + H * H].reshape(H, H))
        o += H * H
    W2 = p[o:o + 16 * H].reshape(16, H)
    o += 16 * H
    W3 = p[o:o + H * 15].reshape(H, 15)
    o += H * 15
    W4 = p[o:o + 3 * H].reshape(3, H)
    assert o + 3 * H == p.size
    return W1, Wh, W2, W3, W4


def _ctx(layers, N=8, lambda_density=0.01):
    frames, box = tiny_scene(n_views=3)
    cfg = oracle.make_config(L=2, nmin=16, nmax=32, log2T=8, N=N, lambda_density=lambda_density)
    ctx = oracle.OracleContext(cfg, alpha_deg=25.0, nthreads=1, mlp_layers=layers)
    oid = ctx.add_object(box["instance"], box["t"], box["yaw"], box["half"])
    for cam, rgb, mask, depth in frames:
        ctx.add_keyframe(cam, rgb, mask, depth)
    return ctx, oid


def test_parameter_counts():
    for din in (4, 16, 32):
        base = oracle.mlp_params(din, 1)
        assert base == 64 * din + 16 * 64 + 64 * 15 + 3 * 64
        assert oracle.mlp_params(din, 2) == base + 4096
        assert oracle.mlp_params(din, 3) == base + 8192
    with pytest.raises(ValueError):
        oracle.levels(2, 16, 32, 8, mlp_layers=4)


@pytest.mark.parametrize("layers", [2, 3])
def test_identity_hidden_layers_reduce_to_one_layer(layers):
    """Wh = I: every hidden layer repeats the first (ReLU outputs are >= 0),
    so the outputs are the one-layer model's, bit for bit."""
    rng = np.random.default_rng(3)
    din = 16
    p1 = random_params(0, din, seed=4)
    W1, _, W2, W3, W4 = _split(p1, din, 1)
    pk = np.concatenate([W1.ravel()] + [np.eye(H).ravel()] * (layers - 1)
                        + [W2.ravel(), W3.ravel(), W4.ravel()])
    for _ in range(10):
        e = rng.standard_normal(din)
        a = oracle.mlp_forward(din, p1, e, 1)
        b = oracle.mlp_forward(din, pk, e, layers)
        assert np.array_equal(a["y"], b["y"]) and np.array_equal(a["rgb"], b["rgb"])
        assert a["sigma"] == b["sigma"]
        for k in range(layers):
            assert np.array_equal(b["h1"][64 * k:64 * (k + 1)], a["h1"])


@pytest.mark.parametrize("layers", [2, 3])
def test_identity_layers_give_the_one_layer_loss_and_gradient(layers):
    """Whole training step: with identity hidden-to-hidden matrices the loss
    and the gradient of every parameter shared with the one-layer model are
    the one-layer model's."""
    c1, o1 = _ctx(1)
    ck, ok = _ctx(layers)
    Pg = oracle.grid_params(c1.objects[o1].lv)
    p1 = random_params(Pg, 4, seed=8, grid_scale=1.0)
    grid, mlp = p1[:Pg], p1[Pg:]
    W1, _, W2, W3, W4 = _split(mlp, 4, 1)
    pk = np.concatenate([grid, W1.ravel()] + [np.eye(H).ravel()] * (layers - 1)
                        + [W2.ravel(), W3.ravel(), W4.ravel()])
    l1, g1, _ = c1.loss_and_grad(o1, 0, 40, params=p1)
    lk, gk, _ = ck.loss_and_grad(ok, 0, 40, params=pk)
    assert l1 == lk
    s1 = _split(g1[Pg:], 4, 1)
    sk = _split(gk[Pg:], 4, layers)
    assert np.array_equal(g1[:Pg], gk[:Pg])
    for a, b in ((s1[0], sk[0]), (s1[2], sk[2]), (s1[3], sk[3]), (s1[4], sk[4])):
        assert np.allclose(a, b, rtol=1e-13, atol=1e-15)
    assert np.abs(np.concatenate([w.ravel() for w in sk[1]])).max() > 0


@pytest.mark.parametrize("layers", [2, 3])
def test_hidden_unit_permutation_invariance(layers):
    """Relabelling the units of any hidden layer (rows of the matrix that
    produces them, columns of the matrix that reads them) leaves the outputs
    unchanged up to summation order."""
    rng = np.random.default_rng(5)
    din = 8
    p = random_params(0, din, seed=6, layers=layers)
    W1, Wh, W2, W3, W4 = _split(p.copy(), din, layers)
    mats = [W1] + Wh + [W2]  # mats[k] produces hidden layer k (k < layers), mats[-1] reads the last
    for k in range(layers):
        perm = rng.permutation(H)
        mats[k] = mats[k][perm, :]
        mats[k + 1] = mats[k + 1][:, perm]
    q = np.concatenate([m.ravel() for m in mats] + [W3.ravel(), W4.ravel()])
    assert not np.array_equal(p, q)
    for _ in range(10):
        e = rng.standard_normal(din)
        a = oracle.mlp_forward(din, p, e, layers)
        b = oracle.mlp_forward(din, q, e, layers)
        assert np.allclose(a["y"], b["y"], rtol=1e-12, atol=1e-13)
        assert np.allclose(a["rgb"], b["rgb"], rtol=1e-12)


@pytest.mark.parametrize("layers", [2, 3])
def test_deep_gradient_matches_finite_differences(layers):
    """Central differences on every hidden-to-hidden weight of one output
    unit, a random sample of all other parameters, and three random
    directions through all of them."""
    ctx, oid = _ctx(layers)
    o = ctx.objects[oid]
    Pg = oracle.grid_params(o.lv)
    p = random_params(Pg, 4, seed=11, grid_scale=1.0, layers=layers)
    B = 24
    loss, g, _ = ctx.loss_and_grad(oid, 0, B, params=p)
    rng = np.random.default_rng(12)
    wh0 = Pg + 64 * 4  # first hidden-to-hidden matrix
    picks = set(range(wh0 + 64 * 7, wh0 + 64 * 8))                  # row 7 of Wh_1
    picks |= set(range(wh0 + 4096 * (layers - 1) - 64, wh0 + 4096 * (layers - 1)))  # last row of the last Wh
    picks |= set(rng.choice(p.size, 300, replace=False).tolist())
    scale = np.abs(g).max()
    for i in sorted(picks):
        h = 1e-6 * max(1.0, abs(p[i]))
        pp = p.copy()
        pp[i] += h
        lp, _, _ = ctx.loss_and_grad(oid, 0, B, params=pp, want_grad=False)
        pp[i] -= 2 * h
        lm, _, _ = ctx.loss_and_grad(oid, 0, B, params=pp, want_grad=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * scale + 1e-5 * abs(g[i]), (i, fd, g[i])
    assert np.count_nonzero(g[wh0:wh0 + 4096 * (layers - 1)]) > 100
    for _ in range(3):
        v = rng.standard_normal(p.size)
        v /= np.linalg.norm(v)
        h = 1e-6
        lp, _, _ = ctx.loss_and_grad(oid, 0, B, params=p + h * v, want_grad=False)
        lm, _, _ = ctx.loss_and_grad(oid, 0, B, params=p - h * v, want_grad=False)
        assert math.isclose((lp - lm) / (2 * h), float(g @ v), rel_tol=1e-6)


@pytest.mark.parametrize("layers", [2, 3])
def test_deep_gradient_mass_bounds_gradient(layers):
    ctx, oid = _ctx(layers)
    o = ctx.objects[oid]
    p = random_params(oracle.grid_params(o.lv), 4, seed=21, grid_scale=1.0, layers=layers)
    mass = np.zeros(p.size)
    _, g, _ = ctx.loss_and_grad(oid, 0, 32, params=p, mass=mass)
    assert (mass >= np.abs(g) * (1 - 1e-12)).all()
    assert (g[mass == 0] == 0).all()

"""Pins of the oracle's BF16 mode (the GPU path's BF16 MLP: every operand of an
MLP contraction rounded to BF16, everything else FP64).

- the rounding itself equals torch's FP32 -> bfloat16 conversion (a library
  routine), ties to even and subnormals included;
- the BF16 forward equals numpy matmuls on operands rounded by torch;
- the BF16 gradient stays within the rounding's reach of the FP32-mode
  gradient (which central differences pin), and differs from it;
- the allowance of the BF16 rounding decisions bounds what rounding error in
  the operands (up to 3e-6 relative, more than FP32 sums of these lengths
  can make) changes in the loss and in every gradient entry.
"""
import numpy as np
import pytest
import torch

import oracle
from tests.tiny import random_params, tiny_scene


def _torch_bf16(x):
    t = torch.tensor(np.asarray(x, np.float32), dtype=torch.float32)
    return t.to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)


def test_bf16_rounding_equals_torch_conversion():
    rng = np.random.default_rng(3)
    x = np.concatenate([
        rng.standard_normal(20000) * 10.0 ** rng.uniform(-30, 30, 20000),
        rng.uniform(-1, 1, 2000) * 2.0 ** -130,            # FP32 subnormals
        np.array([1.0, -1.0, 0.0, 2.0 ** -126, 3.0 * 2.0 ** -133]),
    ]).astype(np.float32)
    # exact ties between neighbouring BF16 values: both parities
    base = _torch_bf16(rng.uniform(0.5, 1.0, 500))
    ties = (base + 2.0 ** -9).astype(np.float32)            # halfway at [0.5, 1)
    x = np.concatenate([x, ties, -ties])
    want = _torch_bf16(x)
    got = np.array([oracle.bf16(float(v)) for v in x])
    assert np.array_equal(got, want)


def test_bf16_gap_is_the_distance_to_the_rounding_boundary():
    rng = np.random.default_rng(4)
    for x in rng.standard_normal(3000) * 10.0 ** rng.uniform(-5, 5, 3000):
        g = oracle.bf16_gap(x)
        r = oracle.bf16(x)
        # just inside the gap the rounding is unchanged, just beyond it, on
        # the side of the boundary, it moves to the neighbour
        assert oracle.bf16(x + 0.5 * g) == r and oracle.bf16(x - 0.5 * g) == r
        moved = [oracle.bf16(x + s * g * (1 + 1e-6)) for s in (1.0, -1.0)]
        assert any(m != r for m in moved)
    assert oracle.bf16_gap(1.0 + 2.0 ** -8) == 0.0  # a midpoint


@pytest.mark.parametrize("layers", [1, 3])
def test_bf16_mlp_forward_equals_numpy_on_rounded_operands(layers):
    rng = np.random.default_rng(5)
    din = 32
    mlp = random_params(0, din, seed=6, layers=layers).astype(np.float32).astype(np.float64)
    e = rng.uniform(-2, 2, din)
    out = oracle.mlp_forward(din, mlp, e, layers=layers, bf16=True)
    o = 0
    W1 = mlp[o:o + 64 * din].reshape(64, din); o += 64 * din
    Wh = []
    for _ in range(layers - 1):
        Wh.append(mlp[o:o + 4096].reshape(64, 64)); o += 4096
    W2 = mlp[o:o + 1024].reshape(16, 64); o += 1024
    W3 = mlp[o:o + 960].reshape(64, 15); o += 960
    W4 = mlp[o:o + 192].reshape(3, 64)
    b = _torch_bf16
    h = np.maximum(b(W1) @ b(e), 0.0)
    hs = [h]
    for W in Wh:
        h = np.maximum(b(W) @ b(h), 0.0)
        hs.append(h)
    y = b(W2) @ b(h)
    h2 = np.maximum(b(W3) @ b(y[1:]), 0.0)
    rgb = 1.0 / (1.0 + np.exp(-(b(W4) @ b(h2))))
    assert np.allclose(out["h1"], np.concatenate(hs), rtol=1e-13, atol=1e-15)
    assert np.allclose(out["y"], y, rtol=1e-13, atol=1e-15)
    assert np.isclose(out["sigma"], np.exp(min(y[0], 15.0)), rtol=1e-13)
    assert np.allclose(out["h2"], h2, rtol=1e-13, atol=1e-15)
    assert np.allclose(out["rgb"], rgb, rtol=1e-13)
    # and it is not the FP32 forward
    f = oracle.mlp_forward(din, mlp, e, layers=layers)
    assert not np.allclose(out["y"], f["y"], rtol=1e-6)


def _pair(L, nmin, nmax, lt, N, seed=1):
    frames, box = tiny_scene(W=32, H=24, n_views=3)
    ctx = {}
    for bf in (False, True):
        cfg = oracle.make_config(L=L, nmin=nmin, nmax=nmax, log2T=lt, N=N)
        o = oracle.OracleContext(cfg, bf16=bf)
        oid = o.add_object(box["instance"], box["t"], box["yaw"], box["half"])
        for cam, rgb, mask, depth in frames:
            o.add_keyframe(cam, rgb, mask, depth)
        p = random_params(oracle.grid_params(o.objects[oid].lv), 2 * L, seed=seed)
        o.objects[oid].params[:] = p.astype(np.float32).astype(np.float64)
        ctx[bf] = (o, oid)
    return ctx


@pytest.mark.parametrize("case", [(2, 16, 32, 8, 32), (8, 16, 128, 12, 32)])
def test_bf16_gradient_is_the_fp32_gradient_within_rounding_reach(case):
    """Each operand moves by at most 2^-8 of itself (half a BF16 unit), so
    the BF16-mode gradient differs from the FP32-mode gradient (pinned by
    central differences) by rounding-sized amounts: norm-wise between 1e-5
    and 2^-4 per tensor (a grid contribution passes about eight roundings;
    measured 0.2-3.5 %), never by a dropped, sign-flipped or transposed
    term (an O(1) change)."""
    ctx = _pair(*case)
    B = 256
    (of, i), (ob, j) = ctx[False], ctx[True]
    lf, gf, _ = of.loss_and_grad(i, 0, B)
    lb, gb, _ = ob.loss_and_grad(j, 0, B)
    assert abs(lb - lf) <= 2.0 ** -6 * abs(lf)
    lv = of.objects[i].lv
    P_grid = oracle.grid_params(lv)
    din = 2 * case[0]
    cuts = [0, P_grid, P_grid + 64 * din, P_grid + 64 * din + 1024, P_grid + 64 * din + 1984,
            gf.size]
    for a, b in zip(cuts[:-1], cuts[1:]):
        rel = np.linalg.norm(gb[a:b] - gf[a:b]) / np.linalg.norm(gf[a:b])
        assert 1e-5 < rel < 2.0 ** -4, (a, b, rel)


@pytest.mark.parametrize("case", [(2, 16, 32, 8, 32), (8, 16, 128, 12, 32),
                                  (16, 16, 1024, 14, 64)])
def test_bf16_allowance_bounds_operand_rounding_error(case):
    """Every rounded operand moved by up to rel |x| before rounding (rel up to
    3e-6) changes the loss and every gradient entry by no more than the
    allowance the oracle derives for its BF16 decisions (plus 1e-9 of the
    entry's magnitude for the FP64 sums' own reordering)."""
    ctx = _pair(*case, seed=2)
    o, oid = ctx[True]
    B = 256
    P = o.n_params(oid)
    mass, amb, bam, la = np.zeros(P), np.zeros(P), np.zeros(P), np.zeros(1)
    l0, g0, _ = o.loss_and_grad(oid, 0, B, mass=mass, ambiguous=amb, loss_allow=la,
                                bf16_allow=bam)
    assert la[0] > 0 and bam.max() > 0
    amb = amb + bam
    try:
        for rel in (3e-7, 1e-6, 3e-6):
            oracle.set_bf16_jitter(rel)
            l1, g1, _ = o.loss_and_grad(oid, 0, B)
            assert abs(l1 - l0) <= la[0] + 1e-12 * abs(l0)
            d = np.abs(g1 - g0)
            bad = d > amb + 1e-9 * mass
            assert not bad.any(), (rel, np.flatnonzero(bad)[:5])
            assert (d > 0).any()
    finally:
        oracle.set_bf16_jitter(0.0)


def test_fp32_mode_has_no_bf16_allowance():
    ctx = _pair(2, 16, 32, 8, 32)
    o, oid = ctx[False]
    la = np.zeros(1)
    P = o.n_params(oid)
    bam = np.ones(P)
    o.loss_and_grad(oid, 0, 128, mass=np.zeros(P), ambiguous=np.zeros(P), loss_allow=la,
                    bf16_allow=bam)
    assert la[0] == 0.0 and not bam.any()

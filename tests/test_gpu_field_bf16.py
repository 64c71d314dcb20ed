"""The autograd surface and the BF16 MLP path against the oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2304_05735_amd as pk
import scenes
from paper_2304_05735_amd.field import RomapField
from tests.gpu_common import (assert_bf16_close, assert_fwd_close, assert_grad_close,
                              bf16_reference, make_pair, tensor_cuts)
from tests.tiny import random_params, tiny_scene

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pixel_rays(o, cam, half, W, H):
    M, c = oracle.object_frame(cam["T_wc"], o.t, o.yaw)
    rays = []
    for v in range(H):
        for u in range(W):
            ro, rd = oracle.pixel_ray(M, c, cam["fx"], cam["fy"], cam["cx"], cam["cy"], u, v)
            hit, tn, tf = oracle.slab(ro, rd, half)
            rays.append(list(ro) + list(rd) + ([tn, tf] if hit else [0.0, 0.0]))
    return np.array(rays, np.float32)


@pytest.mark.parametrize("L,lt,N", [(2, 8, 32), (16, 14, 64)])
def test_autograd_field_matches_oracle(L, lt, N):
    _say("field autograd", L, lt, N)
    frames, box = tiny_scene(W=32, H=24, n_views=2)
    nmax = {2: 32, 8: 128}.get(L, 1024)
    cfg = pk.default_config(n_levels=L, base_res=16, max_res=nmax, log2_table_size=lt,
                            samples_per_ray=N, autotune=0)
    rctx = pk.Context(cfg, stream=torch.cuda.current_stream())
    o = oracle.OracleContext(oracle.make_config(L=L, nmin=16, nmax=nmax, log2T=lt, N=N))
    gid = rctx.add_object(1, box["t"], box["yaw"], box["half"])
    oid = o.add_object(1, box["t"], box["yaw"], box["half"])
    ob = o.objects[oid]
    p = random_params(oracle.grid_params(ob.lv), 2 * L, seed=41).astype(np.float32)
    rctx.set_params(gid, p)
    ob.params[:] = p.astype(np.float64)
    cam = scenes.camera(scenes.look_at((1.2, -1.0, 0.6), (0, 0, 0)), 24, 18, 20.0)
    rays_np = _pixel_rays(ob, cam, ob.half, 24, 18)
    field = RomapField(rctx, gid)
    rays = torch.from_numpy(rays_np).cuda()
    rgb, depth, tend = field(rays)
    orgb, odepth, otend, _ = o.field(oid, rays_np)
    torch.cuda.synchronize()
    assert_fwd_close(rgb.detach().cpu().numpy(), orgb, what="rgb")
    assert_fwd_close(depth.detach().cpu().numpy(), odepth, what="depth")
    assert_fwd_close(tend.detach().cpu().numpy(), otend, what="tend")
    rng = np.random.default_rng(42)
    a = rng.standard_normal((rays_np.shape[0], 3)).astype(np.float32)
    b = rng.standard_normal(rays_np.shape[0]).astype(np.float32)
    c = rng.standard_normal(rays_np.shape[0]).astype(np.float32)
    loss = (rgb * torch.from_numpy(a).cuda()).sum() + (depth * torch.from_numpy(b).cuda()).sum() \
        + (tend * torch.from_numpy(c).cuda()).sum()
    loss.backward()
    torch.cuda.synchronize()
    mass, allow = np.zeros(p.size), np.zeros(p.size)
    _, _, _, og = o.field(oid, rays_np, d_rgb=a, d_depth=b, d_tend=c, grad=True, mass=mass,
                          ambiguous=allow)
    err = assert_grad_close(field.params.grad.cpu().numpy(), og, mass, allow, what="field grad",
                            cuts=tensor_cuts(o, oid))
    _say(f"  field grad rel err {err:.2e}")
    # a torch optimiser can drive the library's field
    opt = torch.optim.Adam(field.parameters(), lr=1e-3)
    opt.step()
    assert not torch.equal(field.params.detach().cpu(), torch.from_numpy(p))


@pytest.mark.parametrize("N", [32, 64, 128])
def test_long_corner_chains_match_oracle(N):
    """Short ray segments (from a hundredth of a finest-level cell to a few
    coarse cells) put many consecutive samples of a ray in one cell, or in
    cells that touch, on most levels: the binning's shared-corner merge then
    sums chains of up to a whole wave of lanes (every step of its doubling;
    at 128 samples a ray's chains also meet the boundary between its two
    waves).  Outputs and parameter gradient of the field match the oracle."""
    _say("long corner chains", N)
    L, lt, nmax = 16, 16, 1024
    cfg = pk.default_config(n_levels=L, base_res=16, max_res=nmax, log2_table_size=lt,
                            samples_per_ray=N, autotune=0)
    rctx = pk.Context(cfg, stream=torch.cuda.current_stream())
    o = oracle.OracleContext(oracle.make_config(L=L, nmin=16, nmax=nmax, log2T=lt, N=N))
    t, yaw, half = np.zeros(3, np.float32), 0.1, np.array([0.4, 0.3, 0.35], np.float32)
    gid = rctx.add_object(1, t, yaw, half)
    oid = o.add_object(1, t, yaw, half)
    ob = o.objects[oid]
    p = random_params(oracle.grid_params(ob.lv), 2 * L, seed=43).astype(np.float32)
    rctx.set_params(gid, p)
    ob.params[:] = p.astype(np.float64)
    rng = np.random.default_rng(44)
    n = 192
    org = rng.uniform(-0.9, 0.9, (n, 3)) * half
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d[:16] = np.eye(3)[rng.integers(0, 3, 16)]  # some along an axis: runs on one cell row
    span = np.exp(rng.uniform(np.log(2e-5), np.log(0.2), n))
    rays_np = np.concatenate([org, d, np.zeros((n, 1)), span[:, None]], 1).astype(np.float32)
    field = RomapField(rctx, gid)
    rays = torch.from_numpy(rays_np).cuda()
    rgb, depth, tend = field(rays)
    orgb, odepth, otend, _ = o.field(oid, rays_np)
    torch.cuda.synchronize()
    assert_fwd_close(rgb.detach().cpu().numpy(), orgb, what="rgb")
    assert_fwd_close(depth.detach().cpu().numpy(), odepth, what="depth")
    assert_fwd_close(tend.detach().cpu().numpy(), otend, what="tend")
    a = rng.standard_normal((n, 3)).astype(np.float32)
    b = rng.standard_normal(n).astype(np.float32)
    c = rng.standard_normal(n).astype(np.float32)
    loss = (rgb * torch.from_numpy(a).cuda()).sum() + (depth * torch.from_numpy(b).cuda()).sum() \
        + (tend * torch.from_numpy(c).cuda()).sum()
    loss.backward()
    torch.cuda.synchronize()
    mass, allow = np.zeros(p.size), np.zeros(p.size)
    _, _, _, og = o.field(oid, rays_np, d_rgb=a, d_depth=b, d_tend=c, grad=True, mass=mass,
                          ambiguous=allow)
    err = assert_grad_close(field.params.grad.cpu().numpy(), og, mass, allow,
                            what="field grad, long chains", cuts=tensor_cuts(o, oid))
    _say(f"  field grad rel err {err:.2e}")


def test_bf16_mlp_error_against_fp64():
    """BF16 MFMA MLP (FP32 accumulate, FP32 grid, transmittance and Adam):
    rendered colour, loss and gradient errors against the FP64 oracle."""
    _say("bf16 errors")
    frames, box = tiny_scene(W=32, H=24, n_views=3)
    B = 512
    g, o, gid = make_pair(16, 16, 1024, 14, 64, B, frames, box, precision=pk.PREC_BF16)
    ob = o.objects[gid]
    p = random_params(oracle.grid_params(ob.lv), 32, seed=51).astype(np.float32)
    g.set_params(gid, p)
    ob.params[:] = p.astype(np.float64)
    cam = scenes.camera(scenes.look_at((1.3, -0.9, 0.7), (0, 0, 0)), 40, 30, 36.0)
    rgb, depth, opac = g.render(gid, cam)
    orgb, _, oopac = o.render(gid, cam, 40, 30)
    cerr = np.abs(rgb - orgb)
    _say(f"  BF16 colour error vs FP64: max {cerr.max():.3e} rms {np.sqrt((cerr ** 2).mean()):.3e}; "
         f"opacity max {np.abs(opac - oopac).max():.3e}")
    assert cerr.max() < 3e-2 and np.sqrt((cerr ** 2).mean()) < 5e-3
    gl = g.loss_and_grad([gid])[0]
    gg = g.get_params(gid, pk.GRAD)
    ol, og, _ = o.loss_and_grad(gid, 0, B)
    rel = np.linalg.norm(gg - og) / np.linalg.norm(og)
    _say(f"  BF16 loss {gl:.6f} vs FP64 {ol:.6f} (rel {abs(gl - ol) / ol:.2e}); grad rel {rel:.2e}")
    assert abs(gl - ol) <= 2e-2 * abs(ol)
    assert rel < 0.1
    st = g.train(5, [gid])
    assert np.isfinite(st.loss_mean)


@pytest.mark.parametrize("L,lt,N,B", [(2, 8, 32, 256), (16, 14, 64, 512), (8, 12, 64, 384),
                                      (16, 14, 128, 256)])
def test_bf16_step_matches_bf16_oracle(L, lt, N, B):
    """The BF16 MLP step (BF16 operands, FP32 accumulation) against the
    oracle's BF16 mode entry by entry: FP32 bounds, plus per entry what the
    BF16 rounding decisions near a midpoint can move, per tensor three times
    the spread that FP32-sized operand perturbations make.  The cases cover
    the backward's pairs of 16-sample blocks with 16 and 32 MLP inputs, one
    and two pairs per ray with the encodings kept in registers, and four
    pairs per ray with the encodings read again (128 samples)."""
    _say("bf16 step vs bf16 oracle", L, lt, N)
    frames, box = tiny_scene(W=32, H=24, n_views=3)
    nmax = {2: 32, 8: 128}.get(L, 1024)
    g, o, gid = make_pair(L, 16, nmax, lt, N, B, frames, box, precision=pk.PREC_BF16,
                          bf16_oracle=True)
    ob = o.objects[gid]
    p = random_params(oracle.grid_params(ob.lv), 2 * L, seed=52).astype(np.float32)
    g.set_params(gid, p)
    ob.params[:] = p.astype(np.float64)
    gl = float(g.loss_and_grad([gid])[0])
    ref = bf16_reference(o, gid, 0, B)
    assert_bf16_close(gl, g.get_params(gid, pk.GRAD), ref, what="BF16 step")


def _err(a, b):
    d = np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64))
    return float(d.max()), float(np.sqrt((d ** 2).mean())), float(np.abs(b).max())


def test_errors_against_fp64():
    """Every result of the path in FP32 and with the BF16 MLP against the FP64
    oracle, on 16 levels x 2^14, 64 samples, trained-scale parameters:
    encodings e (4000 points), densities sigma (4000 points), a rendered
    frame's colour, depth and T_end (1200 rays through the differentiable
    surface), one step's loss and gradient per tensor.  Prints max and rms
    error and the reference's largest magnitude; FP32 is held to its parity
    bars, BF16 to the rendered-colour bound (3e-2 max, 5e-3 rms)."""
    frames, box = tiny_scene(W=32, H=24, n_views=3)
    B = 512
    rows = []
    for prec in (pk.PREC_FP32, pk.PREC_BF16):
        name = "BF16" if prec else "FP32"
        g, o, gid = make_pair(16, 16, 1024, 14, 64, B, frames, box, precision=prec)
        ob = o.objects[gid]
        p = random_params(oracle.grid_params(ob.lv), 32, seed=53).astype(np.float32)
        g.set_params(gid, p)
        ob.params[:] = p.astype(np.float64)
        rng = np.random.default_rng(54)
        pts = rng.random((4000, 3)).astype(np.float32)
        _, feat = g.debug_encode(gid, pts)
        oe = np.stack([oracle.encode(ob.lv, q, ob.params)[2] for q in pts])
        rows.append((name, "e", *_err(feat.reshape(4000, -1), oe)))
        xyz = ((pts * 2.0 - 1.0) * ob.half).astype(np.float32)
        sig = g.query_density(gid, xyz)
        osig = o.query_density(gid, xyz)
        rows.append((name, "sigma", *_err(sig, osig)))
        cam = scenes.camera(scenes.look_at((1.3, -0.9, 0.7), (0, 0, 0)), 40, 30, 36.0)
        rays_np = _pixel_rays(ob, cam, ob.half, 40, 30)
        rgb, depth, tend = g.field_forward(gid, torch.from_numpy(rays_np).cuda())
        torch.cuda.synchronize()
        orgb, odepth, otend, _ = o.field(gid, rays_np)
        rows.append((name, "C", *_err(rgb.cpu().numpy(), orgb)))
        rows.append((name, "D", *_err(depth.cpu().numpy(), odepth)))
        rows.append((name, "T_end", *_err(tend.cpu().numpy(), otend)))
        gl = float(g.loss_and_grad([gid])[0])
        ol, og, _ = o.loss_and_grad(gid, 0, B)
        rows.append((name, "loss", *_err([gl], [ol])))
        gg = g.get_params(gid, pk.GRAD)
        for tname, a, b in tensor_cuts(o, gid):
            mx, rms, ref = _err(gg[a:b], og[a:b])
            nrel = np.linalg.norm(gg[a:b] - og[a:b]) / np.linalg.norm(og[a:b])
            rows.append((name, f"grad {tname} (norm-wise {nrel:.1e})", mx, rms, ref))
        if prec == pk.PREC_FP32:
            assert_fwd_close(rgb.cpu().numpy(), orgb, what="FP32 colour")
            assert_fwd_close(tend.cpu().numpy(), otend, what="FP32 T_end")
            assert_fwd_close([gl], [ol], what="FP32 loss")
        else:
            cerr = np.abs(rgb.cpu().numpy() - orgb)
            assert cerr.max() < 3e-2 and np.sqrt((cerr ** 2).mean()) < 5e-3
        del g
    _say("  precision  result  max|err|  rms err  max|ref|")
    for r in rows:
        _say(f"  {r[0]} {r[1]}: {r[2]:.2e} {r[3]:.2e} {r[4]:.2e}")

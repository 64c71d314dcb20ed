"""The autograd surface and the BF16 MLP path against the oracle."""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2304_05735_amd as pk
import scenes
from paper_2304_05735_amd.field import RomapField
from tests.gpu_common import assert_fwd_close, assert_grad_close, make_pair
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
    nmax = 32 if L == 2 else 1024
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
    err = assert_grad_close(field.params.grad.cpu().numpy(), og, mass, allow, what="field grad")
    _say(f"  field grad rel err {err:.2e}")
    # a torch optimiser can drive the library's field
    opt = torch.optim.Adam(field.parameters(), lr=1e-3)
    opt.step()
    assert not torch.equal(field.params.detach().cpu(), torch.from_numpy(p))


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

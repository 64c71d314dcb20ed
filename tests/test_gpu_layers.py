"""Density MLPs of 2 and 3 hidden layers (the model-size study of Table 4)
on the GPU path against the oracle: loss, gradient, the fused Adam step,
rendering and density queries, in FP32 and with the BF16 MLP."""
import sys

import numpy as np
import pytest

import oracle
import paper_2304_05735_amd as pk
import scenes
from tests.gpu_common import (assert_fwd_close, assert_grad_close, make_pair, oracle_grad,
                              tensor_cuts)
from tests.tiny import random_params, tiny_scene

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tiny():
    return tiny_scene(W=32, H=24, n_views=3)


def _same_params(g, o, gid, layers, seed):
    ob = o.objects[gid]
    p = random_params(oracle.grid_params(ob.lv), 2 * ob.lv.L, seed=seed, layers=layers)
    p32 = p.astype(np.float32)
    g.set_params(gid, p32)
    ob.params[:] = p32.astype(np.float64)
    return p32


@pytest.mark.parametrize("layers", [2, 3])
@pytest.mark.parametrize("case", ["L2_T8_N32", "L16_T16_N64"])
def test_deep_mlp_loss_and_gradient_parity(tiny, layers, case):
    _say("deep mlp parity", layers, case)
    frames, box = tiny
    L, lt, N = {"L2_T8_N32": (2, 8, 32), "L16_T16_N64": (16, 16, 64)}[case]
    nmax = 32 if L == 2 else 1024
    B = 192
    g, o, gid = make_pair(L, 16, nmax, lt, N, B, frames, box, mlp_layers=layers)
    assert g.object_info(gid).n_mlp_params == oracle.mlp_params(2 * L, layers)
    _same_params(g, o, gid, layers, seed=L + lt + layers)
    gl = g.loss_and_grad([gid])[0]
    gg = g.get_params(gid, pk.GRAD)
    ol, og, mass, allow, _ = oracle_grad(o, gid, 0, B)
    assert_fwd_close([gl], [ol], rtol=1e-5, what="loss")
    Pg = oracle.grid_params(o.objects[gid].lv)
    err = assert_grad_close(gg, og, mass, allow, what="grad", cuts=tensor_cuts(o, gid))
    wh = slice(Pg + 64 * 2 * L, Pg + 64 * 2 * L + 4096 * (layers - 1))
    assert np.count_nonzero(og[wh]) > 1000
    _say(f"  loss {gl:.6g} vs {ol:.6g}; largest tensor grad rel err {err:.2e}")


@pytest.mark.parametrize("layers", [2, 3])
def test_deep_mlp_adam_step_matches_oracle(tiny, layers):
    _say("deep mlp adam", layers)
    frames, box = tiny
    g, o, gid = make_pair(2, 16, 32, 8, 32, 64, frames, box, mlp_layers=layers)
    _same_params(g, o, gid, layers, seed=7)
    gl = g.loss_and_grad([gid])[0]
    gg = g.get_params(gid, pk.GRAD).astype(np.float64)
    p0 = g.get_params(gid).astype(np.float64)
    m, v = np.zeros(p0.size), np.zeros(p0.size)
    st = g.train(1, [gid])
    assert abs(st.loss_mean - gl) <= 1e-6 * abs(gl)
    oracle.adam(p0, gg, m, v, 1, 1e-2, 0.9, 0.99, 1e-15)
    assert_fwd_close(g.get_params(gid), p0, rtol=2e-6, atol=2e-8, what="params after step")
    assert_fwd_close(g.get_params(gid, pk.ADAM_V), v, rtol=1e-5, atol=1e-30, what="v")
    assert np.abs(g.get_params(gid, pk.GRAD)).max() == 0.0


@pytest.mark.parametrize("layers", [2, 3])
def test_deep_mlp_render_and_density_parity(tiny, layers):
    _say("deep mlp render", layers)
    frames, box = tiny
    g, o, gid = make_pair(8, 16, 128, 12, 64, 64, frames, box, mlp_layers=layers)
    _same_params(g, o, gid, layers, seed=3)
    cam = scenes.camera(scenes.look_at((1.3, -0.9, 0.7), (0, 0, 0)), 40, 30, 36.0)
    rgb, depth, opac = g.render(gid, cam)
    orgb, odepth, oopac = o.render(gid, cam, 40, 30)
    assert (oopac > 0.05).sum() > 50
    assert_fwd_close(rgb, orgb, what="rgb")
    assert_fwd_close(depth, odepth, what="depth")
    assert_fwd_close(opac, oopac, rtol=1e-5, atol=2e-7, what="opacity")
    rng = np.random.default_rng(9)
    xyz = (rng.uniform(-1.1, 1.1, (4000, 3)) * box["half"]).astype(np.float32)
    assert_fwd_close(g.query_density(gid, xyz), o.query_density(gid, xyz), what="sigma")


def test_identity_hidden_layers_reproduce_one_layer_on_gpu(tiny):
    """FP32 MFMA with identity hidden-to-hidden matrices multiplies by 1 and
    adds zeros: the 3-layer step gives the 1-layer loss and shared gradients
    bit for bit (64 rays: one accumulation workgroup per table region, whose
    fixed-point sums do not depend on order)."""
    _say("identity layers")
    frames, box = tiny
    g1, o1, i1 = make_pair(2, 16, 32, 8, 32, 64, frames, box, mlp_layers=1)
    g3, o3, i3 = make_pair(2, 16, 32, 8, 32, 64, frames, box, mlp_layers=3)
    Pg = oracle.grid_params(o1.objects[i1].lv)
    p1 = random_params(Pg, 4, seed=12).astype(np.float32)
    eye = np.eye(64, dtype=np.float32).ravel()
    p3 = np.concatenate([p1[:Pg + 256], eye, eye, p1[Pg + 256:]])
    g1.set_params(i1, p1)
    g3.set_params(i3, p3)
    l1 = g1.loss_and_grad([i1])[0]
    l3 = g3.loss_and_grad([i3])[0]
    assert l1 == l3
    a, b = g1.get_params(i1, pk.GRAD), g3.get_params(i3, pk.GRAD)
    assert np.array_equal(a[:Pg + 256], b[:Pg + 256])
    assert np.array_equal(a[Pg + 256:], b[Pg + 256 + 8192:])


def test_deep_mlp_bf16_error_against_fp64(tiny):
    """BF16 MFMA for the deeper MLP (FP32 accumulation): colour, loss and
    gradient error against the FP64 oracle stay at the one-layer BF16 level."""
    _say("deep mlp bf16")
    frames, box = tiny
    B = 512
    g, o, gid = make_pair(16, 16, 1024, 14, 64, B, frames, box, precision=pk.PREC_BF16,
                          mlp_layers=3)
    _same_params(g, o, gid, 3, seed=51)
    cam = scenes.camera(scenes.look_at((1.3, -0.9, 0.7), (0, 0, 0)), 40, 30, 36.0)
    rgb, _, _ = g.render(gid, cam)
    orgb, _, _ = o.render(gid, cam, 40, 30)
    cerr = np.abs(rgb - orgb)
    _say(f"  colour error max {cerr.max():.3e} rms {np.sqrt((cerr ** 2).mean()):.3e}")
    assert cerr.max() < 3e-2 and np.sqrt((cerr ** 2).mean()) < 5e-3
    gl = g.loss_and_grad([gid])[0]
    gg = g.get_params(gid, pk.GRAD)
    ol, og, _ = o.loss_and_grad(gid, 0, B)
    rel = np.linalg.norm(gg - og) / np.linalg.norm(og)
    _say(f"  loss {gl:.6f} vs {ol:.6f}; grad rel {rel:.2e}")
    assert abs(gl - ol) <= 2e-2 * abs(ol)
    assert rel < 0.1
    st = g.train(5, [gid])
    assert np.isfinite(st.loss_mean)


def test_mlp_layers_out_of_range_is_rejected():
    for bad in (0, 4):
        with pytest.raises(pk.RomapError):
            pk.Context(pk.default_config(mlp_layers=bad))


def test_deep_mlp_occupancy_refresh_follows_density(tiny):
    """The occupancy refresh thresholds the density of the deeper MLP at the
    cell centres (bits match the oracle's density wherever it is not within
    1e-4 of the threshold)."""
    _say("deep mlp occupancy")
    frames, box = tiny
    g, o, gid = make_pair(8, 16, 128, 12, 64, 64, frames, box, mlp_layers=2)
    _same_params(g, o, gid, 2, seed=17)
    ob = o.objects[gid]
    cells = (np.arange(64) + 0.5) / 64.0
    z, y, x = np.meshgrid(cells, cells, cells, indexing="ij")
    xyz = (np.stack([x, y, z], -1).reshape(-1, 3) * (2.0 * ob.half) - ob.half).astype(np.float32)
    dens = o.query_density(gid, xyz)
    thr = float(np.median(dens))
    g.update_occupancy(gid, thr)
    gb = np.unpackbits(g.get_occupancy(gid), bitorder="little").astype(bool)
    sure = np.abs(dens - thr) > 1e-4 * thr
    assert sure.sum() > 200000
    assert np.array_equal(gb[sure], (dens > thr)[sure])

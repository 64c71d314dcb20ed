"""GPU path vs the CPU oracle, element by element, on the same seeded inputs.

Integer work (ray draws, classes, hash indices) and the FP32 position path are
compared bit for bit; FP32 forward outputs to 1e-5 relative; gradients to
1e-4.  Every test calls the library through the C ABI.
"""
import math
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


def _set_same_params(g, o, gid, seed=0, grid_scale=0.5):
    ob = o.objects[gid]
    p = random_params(oracle.grid_params(ob.lv), 2 * ob.lv.L, seed=seed, grid_scale=grid_scale)
    p32 = p.astype(np.float32)
    g.set_params(gid, p32)
    ob.params[:] = p32.astype(np.float64)
    return p32


# ------------------------------------------------------------------ encoding
@pytest.mark.parametrize("lt", [19, 12, 8])
def test_hash_indices_bit_exact_and_features(tiny, lt):
    _say("encode parity log2T", lt)
    frames, box = tiny
    g, o, gid = make_pair(16, 16, 1024, lt, 64, 256, frames, box)
    p32 = _set_same_params(g, o, gid, seed=lt, grid_scale=1.0)
    rng = np.random.default_rng(lt)
    pts = rng.random((3000, 3)).astype(np.float32)
    pts[:100] = np.round(pts[:100] * 16) / 16  # exact vertices of the coarse levels
    pts[100:120] = 0.0
    pts[120:140] = 1.0
    idx, feat = g.debug_encode(gid, pts)
    ob = o.objects[gid]
    G = ob.params
    for i in range(pts.shape[0]):
        oi, ow, oe = oracle.encode(ob.lv, pts[i], G)
        assert np.array_equal(idx[i], oi), i
        # 1e-5 relative + 1e-7, plus the FP32 rounding of a sum of eight
        # products where it cancels: 4 units of 2^-24 of the sum of |terms|
        mag = np.zeros(2 * ob.lv.L)
        for l in range(ob.lv.L):
            at = ob.lv.off[l] + 2 * oi[l].astype(np.int64)
            mag[2 * l] = np.sum(np.abs(ow[l]) * np.abs(G[at]))
            mag[2 * l + 1] = np.sum(np.abs(ow[l]) * np.abs(G[at + 1]))
        err = np.abs(feat[i].reshape(-1).astype(np.float64) - oe)
        bound = 1e-5 * np.abs(oe) + 1e-7 + 4 * 2.0 ** -24 * mag
        assert (err <= bound).all(), (i, err.max(), np.flatnonzero(err > bound))


# ------------------------------------------------------------------ rays
@pytest.mark.parametrize("N", [32, 64, 128])
def test_ray_draws_and_sample_positions_bit_exact(tiny, N):
    _say("ray parity N", N)
    frames, box = tiny
    B = 1500
    g, o, gid = make_pair(2, 16, 32, 8, N, B, frames, box)
    kfuv, cls, rf, pos = g.debug_rays(gid, B)
    _, _, rays = o.loss_and_grad(gid, 0, B, rays=True, want_grad=False)
    ob = o.objects[gid]
    seen = set()
    for r in range(B):
        ra = rays[r]
        assert (kfuv[r, 0], kfuv[r, 1], kfuv[r, 2]) == (ra.kf, ra.u, ra.v), r
        want_cls = ra.cls if ra.hit else -1
        assert cls[r] == want_cls, r
        seen.add(int(cls[r]))
        if not ra.hit:
            continue
        assert np.array_equal(rf[r, 0:3], np.array(ra.o, np.float32))
        assert np.array_equal(rf[r, 3:6], np.array(ra.d, np.float32))
        assert rf[r, 6] == np.float32(ra.tn)
        _, dist, opos = oracle.sample_positions(ra.o, ra.d, ob.half, ra.tn, ra.tf, N)
        delta, _, _ = oracle.sample_positions(ra.o, ra.d, ob.half, ra.tn, ra.tf, N)
        assert rf[r, 7] == np.float32(delta)
        tgt = np.array(ra.Crand if ra.cls == 2 else ra.C, np.float32)
        assert np.array_equal(rf[r, 8:11], tgt)
        if ra.has_depth:
            assert rf[r, 15] == 1.0 and rf[r, 11] == np.float32(ra.D)
        assert np.array_equal(pos[r], opos), r
    assert {0, 1, 2} <= seen


# ------------------------------------------------------------------ one step
@pytest.mark.parametrize("prec_case", ["L2_T8_N32", "L8_T12_N32", "L16_T19_N64", "L16_T15_N128",
                                       "L16_T14_N64_lambda2_0"])
def test_step_loss_and_gradient_parity(tiny, prec_case):
    """One step's loss and gradient; the last case drops the density term of
    the background rays (lambda_2 = 0, the loss ablation of Fig. 8)."""
    _say("step parity", prec_case)
    frames, box = tiny
    L, lt, N = {"L2_T8_N32": (2, 8, 32), "L8_T12_N32": (8, 12, 32), "L16_T19_N64": (16, 19, 64),
                "L16_T15_N128": (16, 15, 128), "L16_T14_N64_lambda2_0": (16, 14, 64)}[prec_case]
    nmax = {2: 32, 8: 128, 16: 1024}[L]
    B = 192
    kw = {"lambda_density": 0.0} if prec_case.endswith("lambda2_0") else {}
    g, o, gid = make_pair(L, 16, nmax, lt, N, B, frames, box, **kw)
    assert o.cfg.lambda_density == (0.0 if kw else np.float32(0.01))
    _set_same_params(g, o, gid, seed=L + lt)
    gl = g.loss_and_grad([gid])[0]
    gg = g.get_params(gid, pk.GRAD)
    ol, og, mass, allow, rays = oracle_grad(o, gid, 0, B, rays=True)
    assert sum(1 for r in rays if r.hit and r.cls == 1) > 10
    assert sum(1 for r in rays if r.hit and r.cls == 2) > 10
    assert_fwd_close([gl], [ol], rtol=1e-5, what="loss")
    err = assert_grad_close(gg, og, mass, allow, what="grad", cuts=tensor_cuts(o, gid))
    _say(f"  loss {gl:.6g} vs {ol:.6g}; largest tensor grad rel err {err:.2e}")


def test_every_launch_shape_of_the_autotuner(tiny):
    """The shapes the autotuner chooses among (4, 8, 16, 32 rays per work
    item of the field kernel; gather blocks of 128, 256, 512 samples), each
    forced, on 16 levels x 64 samples with a ray count that leaves a ragged
    last work item: loss within 1e-5 and gradient within 1e-4 (per tensor
    and per entry) of the oracle, in a training step's launch (loss_and_grad
    launches as a step of these objects does)."""
    _say("launch shapes")
    frames, box = tiny
    B = 203
    g, o, gid = make_pair(16, 16, 1024, 14, 64, B, frames, box)
    _set_same_params(g, o, gid, seed=77)
    ol, og, mass, allow, _ = oracle_grad(o, gid, 0, B)
    cuts = tensor_cuts(o, gid)
    for rpi in (4, 8, 16, 32):
        for blk in (128, 256, 512):
            g.debug_tiles(rpi, blk)
            gl = g.loss_and_grad([gid])[0]
            gg = g.get_params(gid, pk.GRAD)
            assert_fwd_close([gl], [ol], what=f"loss {rpi}x{blk}")
            assert_grad_close(gg, og, mass, allow, what=f"grad {rpi} rays/item, block {blk}",
                              cuts=cuts)
    with pytest.raises(pk.RomapError):
        g.debug_tiles(12, 256)
    with pytest.raises(pk.RomapError):
        g.debug_tiles(8, 64)


def test_loss_and_grad_leaves_state_untouched(tiny):
    frames, box = tiny
    g, o, gid = make_pair(2, 16, 32, 8, 32, 128, frames, box)
    _set_same_params(g, o, gid)
    a = g.loss_and_grad([gid])[0]
    b = g.loss_and_grad([gid])[0]
    assert g.object_info(gid).step == 0
    assert abs(a - b) <= 1e-6 * abs(a)


# ------------------------------------------------------------------ Adam
@pytest.mark.parametrize("B", [64, 512])
def test_dense_adam_matches_oracle(tiny, B):
    """Adam is applied inside the gradient kernels of a training step (the
    MLP's in the reduction, the table's where each region is summed).  Each
    step's gradient is first taken with loss_and_grad (same draw, no step
    advance); the training step must then move p, m and v exactly as the
    oracle's dense Adam does with that gradient, zero-gradient entries
    included.  With B = 512 the coarse table's region is summed by several
    workgroups (the shared-region finishing path)."""
    _say("adam parity", B)
    frames, box = tiny
    g, o, gid = make_pair(2, 16, 32, 8, 32, B, frames, box)
    p0 = _set_same_params(g, o, gid)
    P = p0.size
    p = p0.astype(np.float64)
    m = np.zeros(P)
    v = np.zeros(P)
    for k in (1, 2, 3):
        g.loss_and_grad([gid])
        gk = g.get_params(gid, pk.GRAD).astype(np.float64)
        assert np.count_nonzero(gk) > P // 4
        g.train(1, [gid])
        oracle.adam(p, gk, m, v, k, 1e-2, 0.9, 0.99, 1e-15)
        gp = g.get_params(gid)
        assert_fwd_close(gp, p, rtol=2e-6, atol=2e-8, what=f"params after step {k}")
        assert_fwd_close(g.get_params(gid, pk.ADAM_M), m, rtol=1e-5, atol=1e-10, what="m")
        assert_fwd_close(g.get_params(gid, pk.ADAM_V), v, rtol=1e-5, atol=1e-14, what="v")
    assert g.object_info(gid).step == 3
    assert np.abs(g.get_params(gid, pk.GRAD)).max() == 0.0


# ------------------------------------------------------------------ training steps
def test_training_steps_track_oracle(tiny):
    _say("train parity")
    frames, box = tiny
    B = 256
    g, o, gid = make_pair(8, 16, 128, 12, 32, B, frames, box)
    _set_same_params(g, o, gid, grid_scale=0.1)
    gl = []
    for _ in range(4):
        st = g.train(1, [gid])
        gl.append(st.loss_mean)
    ol = o.train(gid, 4, B)
    # the first loss is evaluated at identical parameters
    assert_fwd_close([gl[0]], [ol[0]], rtol=1e-5, what="loss step 0")
    # later steps differ only by FP32 rounding carried through Adam
    assert_fwd_close(gl, ol, rtol=2e-2, what="loss curve")


# ------------------------------------------------------------------ render / query
def test_render_and_density_parity(tiny):
    _say("render parity")
    frames, box = tiny
    g, o, gid = make_pair(8, 16, 128, 12, 64, 64, frames, box)
    _set_same_params(g, o, gid, seed=3)
    cam = scenes.camera(scenes.look_at((1.3, -0.9, 0.7), (0, 0, 0)), 40, 30, 36.0)
    rgb, depth, opac = g.render(gid, cam)
    orgb, odepth, oopac = o.render(gid, cam, 40, 30)
    assert (oopac > 0.05).sum() > 100
    assert_fwd_close(rgb, orgb, what="rgb")
    assert_fwd_close(depth, odepth, what="depth")
    assert_fwd_close(opac, oopac, rtol=1e-5, atol=2e-7, what="opacity")
    rng = np.random.default_rng(9)
    xyz = (rng.uniform(-1.1, 1.1, (4000, 3)) * box["half"]).astype(np.float32)
    assert_fwd_close(g.query_density(gid, xyz), o.query_density(gid, xyz), what="sigma")


# ------------------------------------------------------------------ many objects, one launch
def test_batched_objects_match_per_object_oracle():
    """Three objects with uneven tables and ray counts in one launch per phase."""
    _say("batched parity")
    wl = scenes.room_scene(n_obj=3, n_views=8, W=160, H=120, seed=1, room=4.0)
    cfg = pk.default_config(samples_per_ray=32, autotune=0)
    g = pk.Context(cfg)
    ocfg = oracle.make_config(N=32)
    o = oracle.OracleContext(ocfg)
    rays = [300, 77, 1024]
    lts = [15, 19, 16]
    ids = []
    for ob, lt in zip(wl.objects, lts):
        ids.append(g.add_object(ob.instance, ob.t, ob.yaw, ob.half, lt))
        o.add_object(ob.instance, ob.t, ob.yaw, ob.half, lt)
    for cam, rgb, mask, depth in wl.frames:
        g.add_keyframe(cam, rgb, mask, depth)
        o.add_keyframe(cam, rgb, mask, depth)
    for i in ids:
        assert o.objects[i].kfs, "object never seen"
        _set_same_params(g, o, i, seed=10 + i)
    gl = g.loss_and_grad(ids, rays)
    for k, i in enumerate(ids):
        ol, og, mass, allow, _ = oracle_grad(o, i, 0, rays[k])
        assert_fwd_close([gl[k]], [ol], what=f"loss obj {i}")
        assert_grad_close(g.get_params(i, pk.GRAD), og, mass, allow, what=f"grad obj {i}",
                          cuts=tensor_cuts(o, i))


@pytest.mark.parametrize("streams", [1, 2])
def test_degenerate_batches(streams):
    """Ray counts of 1, 2 and 65 (a single ray, a ragged tail of one
    workgroup) batched with each other: loss and gradient match the oracle,
    and a training step of that batch (split over two streams when asked)
    applies Adam with exactly that gradient.  An empty object list and zero
    steps do nothing; ray counts outside [1, 2^22] are rejected."""
    _say("degenerate batches", streams)
    wl = scenes.room_scene(n_obj=3, n_views=8, W=160, H=120, seed=1, room=4.0)
    g = pk.Context(pk.default_config(samples_per_ray=32, autotune=0, streams=streams))
    assert scenes._gpu_open()  # later scene builds in this process render serially
    o = oracle.OracleContext(oracle.make_config(N=32))
    ids = []
    for ob, lt in zip(wl.objects, (12, 14, 13)):
        ids.append(g.add_object(ob.instance, ob.t, ob.yaw, ob.half, lt))
        o.add_object(ob.instance, ob.t, ob.yaw, ob.half, lt)
    for cam, rgb, mask, depth in wl.frames:
        g.add_keyframe(cam, rgb, mask, depth)
        o.add_keyframe(cam, rgb, mask, depth)
    p0 = [_set_same_params(g, o, i, seed=30 + i).astype(np.float64) for i in ids]
    rays = [1, 2, 65]
    for bad in ([0, 2, 65], [1, -3, 65], [1, 2, (1 << 22) + 1]):
        with pytest.raises(pk.RomapError) as e:
            g.train(1, ids, rays=bad)
        assert e.value.code == pk.ROMAP_E_INVALID_ARG
    st = g.train(1, [])
    assert st.rays_trained == 0
    g.train(0, ids, rays=rays)
    assert all(g.object_info(i).step == 0 for i in ids)
    gl = g.loss_and_grad(ids, rays)
    grads = []
    for k, i in enumerate(ids):
        ol, og, mass, allow, _ = oracle_grad(o, i, 0, rays[k])
        assert_fwd_close([gl[k]], [ol], what=f"loss obj {i} ({rays[k]} rays)")
        gg = g.get_params(i, pk.GRAD)
        assert_grad_close(gg, og, mass, allow, what=f"grad obj {i} ({rays[k]} rays)",
                          cuts=tensor_cuts(o, i))
        grads.append(gg.astype(np.float64))
    st = g.train(1, ids, rays=rays)
    assert st.rays_trained == sum(rays) and math.isfinite(st.loss_mean)
    for k, i in enumerate(ids):
        assert g.object_info(i).step == 1
        p = p0[k]
        m, v = np.zeros(p.size), np.zeros(p.size)
        oracle.adam(p, grads[k], m, v, 1, 1e-2, 0.9, 0.99, 1e-15)
        assert_fwd_close(g.get_params(i), p, rtol=2e-6, atol=2e-8, what=f"params obj {i}")


# ------------------------------------------------------------------ full size of the workload
def test_full_size_workload_sampled():
    """16 levels x 2^19, 4096 rays x 64 samples: every position bit-exact on a
    sample of rays, the loss and the full gradient against the oracle."""
    _say("full-size parity")
    wl = scenes.torus_scene(n_views=6)
    ob = wl.objects[0]
    B = 4096
    frames = wl.frames
    box = dict(instance=ob.instance, t=ob.t, yaw=ob.yaw, half=ob.half)
    g, o, gid = make_pair(16, 16, 1024, 19, 64, B, frames, box)
    # trained-like parameters: the library's own initialisation
    p = g.get_params(gid)
    o.objects[gid].params[:] = p.astype(np.float64)
    kfuv, cls, rf, pos = g.debug_rays(gid, B)
    _, _, rays = o.loss_and_grad(gid, 0, B, rays=True, want_grad=False)
    for r in range(0, B, 37):
        ra = rays[r]
        assert (kfuv[r, 1], kfuv[r, 2]) == (ra.u, ra.v)
        if ra.hit:
            _, _, opos = oracle.sample_positions(ra.o, ra.d, ob.half, ra.tn, ra.tf, 64)
            assert np.array_equal(pos[r], opos), r
    gl = g.loss_and_grad([gid])[0]
    gg = g.get_params(gid, pk.GRAD)
    ol, og, mass, allow, _ = oracle_grad(o, gid, 0, B)
    assert_fwd_close([gl], [ol], what="loss")
    assert_grad_close(gg, og, mass, allow, what="grad", cuts=tensor_cuts(o, gid))


def test_largest_table_and_resolution(tiny):
    """The largest accepted table (2^24 entries) and finest resolution
    (2^16 cells per axis) on two levels, one dense (16^3 cells) and one
    hashed: every corner index bit for bit, loss and gradient against the
    oracle, and one fused Adam step over all of its 2^25 grid parameters."""
    _say("largest table")
    frames, box = tiny
    B = 256
    g, o, gid = make_pair(2, 16, 1 << 16, 24, 32, B, frames, box)
    p0 = _set_same_params(g, o, gid, seed=24, grid_scale=1.0).astype(np.float64)
    ob = o.objects[gid]
    assert ob.lv.L == 2 and oracle.grid_params(ob.lv) > (1 << 24)
    rng = np.random.default_rng(24)
    pts = rng.random((2000, 3)).astype(np.float32)
    pts[:20] = 1.0
    idx, feat = g.debug_encode(gid, pts)
    for i in range(pts.shape[0]):
        oi, _, oe = oracle.encode(ob.lv, pts[i], ob.params)
        assert np.array_equal(idx[i], oi), i
        assert_fwd_close(feat[i].reshape(-1), oe, rtol=1e-5, atol=1e-6, what=f"feat {i}")
    assert idx.max() >= (1 << 23)
    gl = g.loss_and_grad([gid])[0]
    gg = g.get_params(gid, pk.GRAD)
    ol, og, mass, allow, _ = oracle_grad(o, gid, 0, B)
    assert_fwd_close([gl], [ol], what="loss")
    assert_grad_close(gg, og, mass, allow, what="grad", cuts=tensor_cuts(o, gid))
    g.train(1, [gid])
    m, v = np.zeros(p0.size), np.zeros(p0.size)
    oracle.adam(p0, gg.astype(np.float64), m, v, 1, 1e-2, 0.9, 0.99, 1e-15)
    assert_fwd_close(g.get_params(gid), p0, rtol=2e-6, atol=2e-8, what="params after step")


def test_largest_object():
    """Sixteen hashed levels of 2^24 entries (256 to 2^16 cells per axis):
    2^29 grid parameters, so the object's gradient and Adam moments start at
    byte offsets of 2^31 and beyond.  Corner indices bit for bit at sampled
    points, loss and full gradient of a small batch against the oracle."""
    _say("largest object")
    frames, box = tiny_scene(W=32, H=24, n_views=3)
    B = 64
    g, o, gid = make_pair(16, 256, 1 << 16, 24, 32, B, frames, box)
    ob = o.objects[gid]
    Pg = oracle.grid_params(ob.lv)
    assert Pg == 1 << 29
    _set_same_params(g, o, gid, seed=29, grid_scale=1.0)
    pts = np.random.default_rng(29).random((300, 3)).astype(np.float32)
    idx, feat = g.debug_encode(gid, pts)
    for i in range(pts.shape[0]):
        oi, _, oe = oracle.encode(ob.lv, pts[i], ob.params)
        assert np.array_equal(idx[i], oi), i
        assert_fwd_close(feat[i].reshape(-1), oe, rtol=1e-5, atol=1e-6, what=f"feat {i}")
    gl = g.loss_and_grad([gid])[0]
    gg = g.get_params(gid, pk.GRAD)
    ol, og, mass, allow, _ = oracle_grad(o, gid, 0, B)
    assert_fwd_close([gl], [ol], what="loss")
    assert_grad_close(gg, og, mass, allow, what="grad", cuts=tensor_cuts(o, gid))
    assert np.count_nonzero(gg[Pg - (1 << 25):Pg]) > 0  # the finest level is reached


# ------------------------------------------------------------------ ABI contract
def test_abi_errors_and_no_partial_state(tiny):
    frames, box = tiny
    g = pk.Context(pk.default_config(n_levels=2, base_res=16, max_res=32, log2_table_size=8,
                                     samples_per_ray=32))
    with pytest.raises(pk.RomapError) as e:
        g.add_object(1, box["t"], box["yaw"], [0.3, -1.0, 0.3])
    assert e.value.code == pk.ROMAP_E_INVALID_ARG
    with pytest.raises(pk.RomapError) as e:
        g.add_object(1, box["t"], box["yaw"], box["half"], log2T=30)
    assert e.value.code == pk.ROMAP_E_INVALID_ARG
    gid = g.add_object(1, box["t"], box["yaw"], box["half"])
    with pytest.raises(pk.RomapError) as e:
        g.add_object(1, box["t"], box["yaw"], box["half"])
    assert e.value.code == pk.ROMAP_E_INVALID_ARG
    with pytest.raises(pk.RomapError) as e:
        g.train(1, [gid])
    assert e.value.code == pk.ROMAP_E_STATE
    with pytest.raises(pk.RomapError) as e:
        g.train(1, [5])
    assert e.value.code == pk.ROMAP_E_NOT_FOUND
    cam, rgb, mask, depth = frames[0]
    bad = dict(cam, fx=-1.0)
    with pytest.raises(pk.RomapError):
        g.add_keyframe(bad, rgb, mask, depth)
    assert g.object_info(gid).n_keyframes == 0
    g.add_keyframe(cam, rgb, mask, depth)
    assert g.object_info(gid).n_keyframes == 1
    with pytest.raises(pk.RomapError):
        g.set_params(gid, np.zeros(3, np.float32))
    with pytest.raises(pk.RomapError) as e:  # 2^22 rays x 32 samples is the largest step
        g.train(1, [gid], rays=[(1 << 22) + 1])
    assert e.value.code == pk.ROMAP_E_INVALID_ARG
    g128 = pk.Context(pk.default_config(n_levels=2, base_res=16, max_res=32, log2_table_size=8,
                                        samples_per_ray=128, rays_per_step=64))
    g128.add_object(1, box["t"], box["yaw"], box["half"])
    with pytest.raises(pk.RomapError) as e:  # 2^20 + 1 rays x 128 samples > 2^27
        g128.train(1, [0], rays=[(1 << 20) + 1])
    assert e.value.code == pk.ROMAP_E_INVALID_ARG
    with pytest.raises(pk.RomapError) as e:  # 2^20 x 128 is accepted (then: no keyframe)
        g128.train(1, [0], rays=[1 << 20])
    assert e.value.code == pk.ROMAP_E_STATE
    st = g.train(2, [gid])
    assert math.isfinite(st.loss_mean) and st.rays_trained == 2 * 4096
    assert g.object_info(gid).step == 2


def test_checkpoint_roundtrip_continues_identically(tiny, tmp_path):
    frames, box = tiny
    cfg = dict(n_levels=8, base_res=16, max_res=128, log2_table_size=12, samples_per_ray=32,
               rays_per_step=256, autotune=0)
    a = pk.Context(pk.default_config(**cfg))
    gid = a.add_object(1, box["t"], box["yaw"], box["half"])
    for cam, rgb, mask, depth in frames:
        a.add_keyframe(cam, rgb, mask, depth)
    a.train(3, [gid])
    path = tmp_path / "ck.bin"
    a.save(path)
    b = pk.Context(pk.default_config(**cfg))
    b.load(path)
    assert np.array_equal(a.get_params(gid), b.get_params(0))
    assert np.array_equal(a.get_params(gid, pk.ADAM_V), b.get_params(0, pk.ADAM_V))
    assert b.object_info(0).step == 3 and b.object_info(0).n_keyframes == len(frames)
    # the next draw is the same: identical rays, positions
    ka, ca, ra, pa = a.debug_rays(gid, 256)
    kb, cb, rb, pb = b.debug_rays(0, 256)
    assert np.array_equal(ka, kb) and np.array_equal(pa, pb)
    la = a.loss_and_grad([gid])[0]
    lb = b.loss_and_grad([0])[0]
    assert abs(la - lb) <= 1e-6 * abs(la)


def test_checkpoint_with_a_corrupt_rectangle_is_rejected(tiny, tmp_path):
    """A keyframe reference whose candidate rectangle leaves its keyframe (or
    is empty) makes load fail with E_INVALID_ARG; nothing is trained after
    it (the ray draw would read outside the keyframe's pixels)."""
    import struct
    frames, box = tiny
    cfg = dict(n_levels=8, base_res=16, max_res=128, log2_table_size=12, samples_per_ray=32,
               rays_per_step=256, autotune=0)
    a = pk.Context(pk.default_config(**cfg))
    gid = a.add_object(1, box["t"], box["yaw"], box["half"])
    for cam, rgb, mask, depth in frames:
        a.add_keyframe(cam, rgb, mask, depth)
    path = tmp_path / "ck.bin"
    a.save(path)
    raw = bytearray(path.read_bytes())
    # one object: its keyframe references (5 int32 each) precede its
    # parameters and Adam moments (3 x P rounded up to 64 floats)
    P = a.get_params(gid).size
    nref = a.object_info(gid).n_keyframes
    first = len(raw) - 3 * 4 * (-(-P // 64) * 64) - 20 * nref
    kf, x0, y0, w, h = struct.unpack_from("<5i", raw, first)
    W, H = frames[kf][1].shape[1], frames[kf][1].shape[0]
    for k, v in [(1, -1), (2, -1), (3, 0), (4, 0), (3, W - x0 + 1), (4, H - y0 + 1),
                 (3, 2 ** 31 - 1)]:
        bad = bytearray(raw)
        struct.pack_into("<i", bad, first + 4 * k, v)
        p2 = tmp_path / f"bad{k}_{v}.bin"
        p2.write_bytes(bytes(bad))
        b = pk.Context(pk.default_config(**cfg))
        with pytest.raises(pk.RomapError) as e:
            b.load(p2)
        assert e.value.code == pk.ROMAP_E_INVALID_ARG, (k, v)
        del b
    b = pk.Context(pk.default_config(**cfg))  # the untouched file still loads
    b.load(path)
    assert np.array_equal(a.get_params(gid), b.get_params(0))


# ------------------------------------------------------------------ occupancy skip
def test_occupancy_skip_parity(tiny):
    _say("occupancy parity")
    frames, box = tiny
    B = 256
    g, o, gid = make_pair(8, 16, 128, 12, 64, B, frames, box)
    _set_same_params(g, o, gid, seed=7, grid_scale=1.0)
    ob = o.objects[gid]
    cells = (np.arange(64) + 0.5) / 64.0
    z, y, x = np.meshgrid(cells, cells, cells, indexing="ij")
    xyz = (np.stack([x, y, z], -1).reshape(-1, 3) * (2.0 * ob.half) - ob.half).astype(np.float32)
    dens = o.query_density(gid, xyz)
    thr = float(np.median(dens))
    bits = np.packbits(dens > thr, bitorder="little")
    g.set_occupancy(gid, bits)
    o.set_occupancy(gid, bits)
    assert np.array_equal(g.get_occupancy(gid), bits)
    gl = g.loss_and_grad([gid])[0]
    gg = g.get_params(gid, pk.GRAD)
    ol, og, mass, allow, _ = oracle_grad(o, gid, 0, B)
    assert_fwd_close([gl], [ol], what="loss with occupancy")
    assert_grad_close(gg, og, mass, allow, what="grad with occupancy", cuts=tensor_cuts(o, gid))
    cam = scenes.camera(scenes.look_at((1.3, -0.9, 0.7), (0, 0, 0)), 40, 30, 36.0)
    rgb, _, opac = g.render(gid, cam)
    orgb, _, oopac = o.render(gid, cam, 40, 30)
    assert_fwd_close(rgb, orgb, what="rgb with occupancy")
    assert_fwd_close(opac, oopac, rtol=1e-5, atol=2e-7, what="opacity with occupancy")
    # refresh rule: bit = density at the cell centre > threshold
    g.update_occupancy(gid, thr)
    gb = np.unpackbits(g.get_occupancy(gid), bitorder="little").astype(bool)
    sure = np.abs(dens - thr) > 1e-4 * thr
    assert np.array_equal(gb[sure], (dens > thr)[sure])
    g.set_occupancy(gid, None)
    with pytest.raises(pk.RomapError):
        g.get_occupancy(gid)


@pytest.mark.parametrize("N", [64, 128])
def test_occupancy_gaps_on_merged_levels(tiny, N):
    """On coarse levels the binning sums the records of corners that
    consecutive samples of a ray share, along chains of samples.  A sample
    skipped by the occupancy test must end every chain through it (a merge
    whose sums reached across such a gap once counted the samples after it
    twice, first seen on the 128-object stream).  Here a checkerboard of
    occupancy cells (every other 64^3 cell off) puts gaps inside nearly every
    chain of 16 levels x 2^19 (merged up to N_l = 4 x samples per ray, dense
    and hashed levels): loss and gradient match the oracle."""
    _say("occupancy gaps on merged levels", N)
    frames, box = tiny
    B = 256
    g, o, gid = make_pair(16, 16, 1024, 19, N, B, frames, box)
    _set_same_params(g, o, gid, seed=8, grid_scale=1.0)
    c = np.arange(64)
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    on = ((x + y + z) % 2 == 0).reshape(-1)
    bits = np.packbits(on, bitorder="little")
    g.set_occupancy(gid, bits)
    o.set_occupancy(gid, bits)
    gl = g.loss_and_grad([gid])[0]
    gg = g.get_params(gid, pk.GRAD)
    ol, og, mass, allow, _ = oracle_grad(o, gid, 0, B)
    assert_fwd_close([gl], [ol], what="loss with occupancy gaps")
    assert_grad_close(gg, og, mass, allow, what="grad with occupancy gaps",
                      cuts=tensor_cuts(o, gid))


# ------------------------------------------------------------------ gradient bins that overflow
@pytest.mark.parametrize("B", [48, 512])
def test_bin_overflow_path_matches_oracle(tiny, B):
    """Bins capped at 64 records: nearly every record takes the overflow path
    (atomics into the gradient, merged by the region's accumulation; with
    B = 48 the region has one accumulation workgroup, with B = 512 several).
    The gradient still matches the oracle, and a training step still applies
    Adam with that gradient."""
    _say("bin overflow", B)
    frames, box = tiny
    g, o, gid = make_pair(2, 16, 32, 8, 32, B, frames, box)
    _set_same_params(g, o, gid, seed=9)
    g.debug_bin_capacity(64)
    gl = g.loss_and_grad([gid])[0]
    gg = g.get_params(gid, pk.GRAD)
    ol, og, mass, allow, _ = oracle_grad(o, gid, 0, B)
    assert_fwd_close([gl], [ol], what="loss")
    assert_grad_close(gg, og, mass, allow, what="grad (overflow)", cuts=tensor_cuts(o, gid))
    p0 = g.get_params(gid).astype(np.float64)
    P = p0.size
    m, v = np.zeros(P), np.zeros(P)
    g.train(1, [gid])
    oracle.adam(p0, gg.astype(np.float64), m, v, 1, 1e-2, 0.9, 0.99, 1e-15)
    assert_fwd_close(g.get_params(gid), p0, rtol=2e-6, atol=2e-8, what="params after step")
    assert np.abs(g.get_params(gid, pk.GRAD)).max() == 0.0
    g.debug_bin_capacity(0)


# ------------------------------------------------------------------ graph replay
def test_graph_replay_equals_eager_steps(tiny):
    """The captured step graph (used for calls of >= 8 steps, and replayed by
    later calls of the same shapes) advances exactly like eager launches: with
    one accumulation workgroup per region every sum is order-independent, so
    parameters and Adam moments agree bit for bit after 10 + 10 steps."""
    _say("graph replay")
    frames, box = tiny
    ctxs = []
    for graph in (1, 0):
        g, o, gid = make_pair(2, 16, 32, 8, 32, 64, frames, box, use_graph=graph)
        _set_same_params(g, o, gid, seed=21)
        st1 = g.train(10, [gid])
        st2 = g.train(10, [gid])
        ctxs.append((g, gid, st1.loss_mean, st2.loss_mean))
    (ga, ia, la1, la2), (gb, ib, lb1, lb2) = ctxs
    assert ga.object_info(ia).step == gb.object_info(ib).step == 20
    for kind in (pk.PARAMS, pk.ADAM_M, pk.ADAM_V):
        assert np.array_equal(ga.get_params(ia, kind), gb.get_params(ib, kind)), kind
    assert la1 == lb1 and la2 == lb2


def test_profiled_steps_match_and_count_records(tiny):
    """Profiled steps (one event pair per phase, records counted) advance the
    state exactly as unprofiled ones, and the counted gradient records stay
    within 8 per sample and level; on a coarse dense level, where runs of
    samples in one cell are merged, there are fewer."""
    _say("profiled steps")
    frames, box = tiny
    B, N, L = 64, 32, 2
    res = {}
    for nmin, nmax, log2T in ((16, 32, 8), (4, 8, 12)):
        for prof in (1, 0):
            g, o, gid = make_pair(L, nmin, nmax, log2T, N, B, frames, box,
                                  profile_phases=prof, use_graph=0)
            _set_same_params(g, o, gid, seed=5)
            g.train(3, [gid])
            res[(nmin, prof)] = (g.get_params(gid, pk.PARAMS), g.get_params(gid, pk.ADAM_V),
                                 g.step_records() if prof else None)
        for k in (0, 1):
            assert np.array_equal(res[(nmin, 1)][k], res[(nmin, 0)][k])
    hashed, merged = res[(16, 1)][2], res[(4, 1)][2]
    assert 0 < hashed <= 8 * B * N * L
    assert 0 < merged < 8 * B * N * L


def test_two_stream_step_equals_one_stream():
    """A batched step split in two halves on two streams (graph replay and
    eager) advances every object exactly as the one-stream step: the halves
    share no object and no scratch, and with one accumulation workgroup per
    table region every sum is order-independent."""
    _say("two streams")
    wl = scenes.room_scene(n_obj=3, n_views=8, W=160, H=120, seed=1, room=4.0)
    rays = [300, 77, 256]
    lts = [15, 19, 16]
    res = []
    for streams in (2, 1):
        g = pk.Context(pk.default_config(samples_per_ray=32, autotune=0, streams=streams))
        ids = [g.add_object(ob.instance, ob.t, ob.yaw, ob.half, lt)
               for ob, lt in zip(wl.objects, lts)]
        for cam, rgb, mask, depth in wl.frames:
            g.add_keyframe(cam, rgb, mask, depth)
        st1 = g.train(10, ids, rays)  # captured graph of 4 steps: 2 launches, 2 eager steps
        st2 = g.train(8, ids, rays)   # its replay: 2 launches
        st3 = g.train(2, ids, rays[::-1][:2] + [rays[2]])  # new shapes: eager
        res.append((g, ids, [st1.loss_mean, st2.loss_mean, st3.loss_mean]))
    (ga, ia, la), (gb, ib, lb) = res
    assert la == lb
    for i, j in zip(ia, ib):
        assert ga.object_info(i).step == gb.object_info(j).step == 20
        for kind in (pk.PARAMS, pk.ADAM_M, pk.ADAM_V):
            assert np.array_equal(ga.get_params(i, kind), gb.get_params(j, kind)), (i, kind)


def test_mfma_rate_probe():
    """The matrix-core rate probe returns a positive rate below the datasheet
    peaks (2.5 PFLOP/s BF16 and 157.3 TFLOP/s FP32 dense, with 10 % margin)."""
    bf = pk.debug_mfma_rate(pk.PREC_BF16)
    f32 = pk.debug_mfma_rate(pk.PREC_FP32)
    _say(f"measured MFMA rate: BF16 {bf:.0f} TFLOP/s, FP32 {f32:.1f} TFLOP/s")
    assert 0 < bf < 2750 and 0 < f32 < 173
    with pytest.raises(pk.RomapError):
        pk.debug_mfma_rate(7)

"""The allocation-free forward (romap_field_forward_noalloc) against the
allocating one (romap_field_forward), through the C ABI, with the FP32 and
the BF16 MLP: the same colours,
depths and transmittances bit for bit (both run the same kernels in the same
launch shape; the parity bar of a forward output, 1e-5 relative, is implied),
on two calls in a row (the second smaller, so it reads what the first left
in the shared scratch array only where it writes first), and a call beyond
the scratch array's size is rejected."""
import numpy as np
import pytest
import torch

import oracle
import paper_2304_05735_amd as pk
from tests.tiny import random_params

pytestmark = pytest.mark.gpu


def _rays(rng, n, half):
    """n object-frame rays (origin, unit direction, t_near, t_far) from points
    around the box towards points inside it; about a tenth miss it."""
    half = np.asarray(half, np.float32)
    out = np.zeros((n, 8), np.float32)
    for r in range(n):
        o = rng.normal(size=3)
        o = (2.5 * o / np.linalg.norm(o) * half.max()).astype(np.float32)
        tgt = (rng.uniform(-1.2, 1.2, 3) * half).astype(np.float32)
        d = tgt - o
        d = (d / np.linalg.norm(d)).astype(np.float32)
        hit, tn, tf = oracle.slab(o, d, half)
        out[r, :3], out[r, 3:6] = o, d
        out[r, 6:8] = (tn, tf) if hit else (0.0, 0.0)
    return out


@pytest.mark.parametrize("N,prec", [(64, pk.PREC_FP32), (128, pk.PREC_FP32), (64, pk.PREC_BF16)])
def test_noalloc_forward_equals_allocating_forward(N, prec):
    torch.cuda.set_device(0)
    L = 16
    cfg = pk.default_config(n_levels=L, base_res=16, max_res=1024, log2_table_size=14,
                            samples_per_ray=N, autotune=0, precision=prec)
    g = pk.Context(cfg, stream=torch.cuda.current_stream())
    half = np.array([0.4, 0.3, 0.25], np.float32)
    gid = g.add_object(1, np.zeros(3, np.float32), 0.3, half)
    ng = g.object_info(gid).n_grid_params
    g.set_params(gid, random_params(ng, 2 * L, seed=61).astype(np.float32))
    rng = np.random.default_rng(62)
    # about 8100 rays fill the 64 MiB scratch at 64 samples, 4000 at 128
    n_big = 7000 if N == 64 else 3500
    for n in (n_big, 701):
        rays = torch.from_numpy(_rays(rng, n, half)).cuda()
        rgb, depth, tend = g.field_forward(gid, rays)
        rgb2 = torch.full_like(rgb, float("nan"))
        depth2 = torch.full_like(depth, float("nan"))
        tend2 = torch.full_like(tend, float("nan"))
        g.field_forward_noalloc(gid, rays, rgb2, depth2, tend2)
        torch.cuda.synchronize()
        for a, b, what in ((rgb, rgb2, "rgb"), (depth, depth2, "depth"), (tend, tend2, "T_end")):
            a, b = a.cpu().numpy(), b.cpu().numpy()
            assert np.isfinite(b).all(), what
            assert np.array_equal(a, b), (n, what, float(np.abs(a - b).max()))
        assert (tend2 < 1.0).any() and (tend2 == 1.0).any()  # hits and misses
    # an output of the wrong size is refused by the binding, before the library
    with pytest.raises(ValueError):
        g.field_forward_noalloc(gid, rays, rgb2[:-1], depth2, tend2)
    # beyond the scratch array: rejected before any launch, outputs untouched
    n_over = 9000 if N == 64 else 4600
    rays = torch.from_numpy(_rays(rng, n_over, half)).cuda()
    out = [torch.full((n_over, 3), 7.0, device="cuda"), torch.full((n_over,), 7.0, device="cuda"),
           torch.full((n_over,), 7.0, device="cuda")]
    with pytest.raises(pk.RomapError) as e:
        g.field_forward_noalloc(gid, rays, *out)
    assert e.value.code == pk.ROMAP_E_INVALID_ARG
    torch.cuda.synchronize()
    assert all(bool((t == 7.0).all()) for t in out)

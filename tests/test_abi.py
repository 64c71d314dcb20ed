"""C-ABI library checks that need no GPU: it loads and exports every symbol
that include/romap.h declares."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2304_05735_amd", "libromap.so")
HEADER = os.path.join(ROOT, "include", "romap.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:romap_status|const char\*|int32_t)\s+(romap_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for verb in ("romap_create", "romap_add_object", "romap_add_keyframe", "romap_train",
                 "romap_render", "romap_query_density", "romap_field_forward",
                 "romap_field_backward"):
        assert verb in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libromap.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libromap.so not built")
def test_binding_names_match_header():
    import paper_2304_05735_amd as pk
    assert sorted(pk.EXPORTS) == declared_symbols()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libromap.so not built")
def test_default_config_and_create_validation_without_gpu():
    """Host-only calls: defaults, and argument checks that fail before any HIP call."""
    import paper_2304_05735_amd as pk
    cfg = pk.default_config()
    assert (cfg.n_levels, cfg.base_res, cfg.max_res, cfg.log2_table_size) == (16, 16, 1024, 19)
    assert cfg.samples_per_ray == 64 and cfg.rays_per_step == 4096
    assert abs(cfg.lambda_depth - 0.5) < 1e-7 and abs(cfg.lambda_density - 0.01) < 1e-9
    assert abs(cfg.alpha_deg - 25.0) < 1e-6
    assert cfg.mlp_layers == 1 and cfg.streams == 2
    L = pk.lib()
    h = ctypes.c_void_p()
    for field, bad in [("n_levels", 17), ("samples_per_ray", 48), ("log2_table_size", 30),
                       ("precision", 5), ("rays_per_step", 0), ("mlp_layers", 0),
                       ("mlp_layers", 4), ("streams", 0), ("streams", 3), ("use_graph", 3),
                       ("use_graph", -1)]:
        c = pk.default_config(**{field: bad})
        assert L.romap_create(ctypes.byref(c), None, ctypes.byref(h)) == pk.ROMAP_E_INVALID_ARG
        assert L.romap_last_error(None)
    # rays x samples of one object at most 2^27 (int32 record counts per region)
    for N, rays in [(32, (1 << 22) + 1), (64, (1 << 21) + 1), (128, (1 << 20) + 1)]:
        c = pk.default_config(samples_per_ray=N, rays_per_step=rays)
        assert L.romap_create(ctypes.byref(c), None, ctypes.byref(h)) == pk.ROMAP_E_INVALID_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="libromap.so not built")
def test_library_mc_table_equals_oracle_table():
    """The library's marching-cubes case table (host code) equals the
    oracle's case by case, triangle by triangle.  Both are built from the same
    face rules, so this checks the library's transcription of them (the
    bit-for-bit triangle comparison needs the same table); what pins the
    table itself are the oracle's geometric tests (area, volume, Euler
    characteristic, watertight surfaces)."""
    import oracle
    import paper_2304_05735_amd as pk
    for m in range(256):
        assert np.array_equal(pk.mc_case(m), oracle.mc_case(m)), m


@pytest.mark.skipif(not os.path.exists(LIB), reason="libromap.so not built")
def test_box_from_points_matches_oracle():
    """The library's box producer (host code) against the oracle's on yawed,
    noisy, uneven point clouds (the float32 input rounded once on both sides)."""
    import math
    import oracle
    import paper_2304_05735_amd as pk
    rng = np.random.default_rng(11)
    for trial in range(20):
        half = rng.uniform(0.1, 1.0, 3)
        yaw = rng.uniform(-1.5, 1.5)
        t = rng.uniform(-3, 3, 3)
        loc = rng.uniform(-1, 1, (rng.integers(5, 400), 3)) * half
        c, s = math.cos(yaw), math.sin(yaw)
        pts = (loc @ np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]]).T + t).astype(np.float32)
        gt, gy, gh = pk.box_from_points(pts)
        ot, oy, oh = oracle.box_from_points(pts.astype(np.float64))
        assert np.allclose(gt, ot, rtol=1e-6, atol=1e-6)
        assert abs(gy - oy) < 1e-6
        assert np.allclose(gh, oh, rtol=1e-5, atol=1e-6)
    with pytest.raises(pk.RomapError):
        pk.box_from_points(np.zeros((0, 3), np.float32))

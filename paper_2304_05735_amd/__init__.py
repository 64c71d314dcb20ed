"""Python binding of libromap, the MI355X (gfx950) training path for RO-MAP's
per-object radiance fields (arXiv 2304.05735, Sec. V).

Argument marshalling only: every step of the path runs in the HIP kernels of
``libromap.so``.  The names mirror ``include/romap.h``.  PyTorch is imported
first so that the library binds to the same HIP runtime as torch (device
memory and streams are shared with it).  There is no CPU fallback: loading
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (HIP runtime shared with torch)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libromap.so")

ROMAP_OK = 0
ROMAP_E_INVALID_ARG = -1
ROMAP_E_OUT_OF_MEMORY = -2
ROMAP_E_NOT_FOUND = -3
ROMAP_E_HIP = -4
ROMAP_E_NUMERIC = -5
ROMAP_E_STATE = -6
PREC_FP32, PREC_BF16 = 0, 1
BATCH_ALL, BATCH_PER_OBJECT = 0, 1
PARAMS, ADAM_M, ADAM_V, GRAD = 0, 1, 2, 3
PHASES = ("raygen", "encode_fwd", "pack", "field", "reduce", "bin_scatter", "bin_acc",
          "bin_finish")


class romap_config(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("base_res", C.c_int32), ("max_res", C.c_int32),
                ("log2_table_size", C.c_int32), ("samples_per_ray", C.c_int32),
                ("rays_per_step", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("lambda_depth", C.c_float),
                ("lambda_density", C.c_float), ("alpha_deg", C.c_float),
                ("bbox_margin_pct", C.c_int32), ("precision", C.c_int32),
                ("batch_mode", C.c_int32), ("use_graph", C.c_int32), ("autotune", C.c_int32),
                ("profile_phases", C.c_int32), ("mlp_layers", C.c_int32), ("streams", C.c_int32),
                ("seed", C.c_uint64)]


class romap_box(C.Structure):
    _fields_ = [("t", C.c_float * 3), ("yaw", C.c_float), ("half", C.c_float * 3)]


class romap_camera(C.Structure):
    _fields_ = [("T_wc", C.c_float * 12), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("width", C.c_int32), ("height", C.c_int32)]


class romap_train_stats(C.Structure):
    _fields_ = [("loss_mean", C.c_float), ("rays_trained", C.c_int64), ("seconds", C.c_float),
                ("n_objects_nan", C.c_int32)]


class romap_object_info(C.Structure):
    _fields_ = [("instance_id", C.c_int32), ("log2_table_size", C.c_int32),
                ("n_grid_params", C.c_int64), ("n_mlp_params", C.c_int64),
                ("n_keyframes", C.c_int32), ("step", C.c_int32), ("n_candidates", C.c_int64),
                ("active", C.c_int32), ("level_res", C.c_int32 * 16),
                ("level_hashed", C.c_int32 * 16)]


class RomapError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"romap error {code}: {msg}")
        self.code = code


_lib = None
EXPORTS = ["romap_default_config", "romap_create", "romap_destroy", "romap_last_error",
           "romap_add_object", "romap_set_object_active", "romap_get_object_info",
           "romap_add_keyframe", "romap_train", "romap_loss_and_grad", "romap_render",
           "romap_query_density", "romap_get_params", "romap_set_params", "romap_save",
           "romap_load", "romap_debug_rays", "romap_debug_encode", "romap_field_forward",
           "romap_field_forward_noalloc",
           "romap_field_backward", "romap_get_phase_times", "romap_sync", "romap_set_occupancy",
           "romap_update_occupancy", "romap_get_occupancy", "romap_marching_cubes",
           "romap_extract_mesh", "romap_mc_case", "romap_box_from_points",
           "romap_debug_bin_capacity", "romap_get_step_records", "romap_debug_tiles",
           "romap_debug_mfma_rate"]


def lib():
    """The loaded libromap (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2304_05735_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        i32, i64 = C.c_int32, C.c_int64
        sig = {
            "romap_default_config": [C.POINTER(romap_config)],
            "romap_create": [C.POINTER(romap_config), P, C.POINTER(P)],
            "romap_destroy": [P],
            "romap_add_object": [P, i32, C.POINTER(romap_box), i32, C.POINTER(i32)],
            "romap_set_object_active": [P, i32, i32],
            "romap_get_object_info": [P, i32, C.POINTER(romap_object_info)],
            "romap_add_keyframe": [P, C.POINTER(romap_camera), P, P, P, C.POINTER(i32),
                                   C.POINTER(i32)],
            "romap_train": [P, P, i32, i32, P, C.POINTER(romap_train_stats)],
            "romap_loss_and_grad": [P, P, i32, P, P],
            "romap_render": [P, i32, C.POINTER(romap_camera), P, P, P, i32],
            "romap_query_density": [P, i32, P, i64, P, i32],
            "romap_get_params": [P, i32, i32, P, i64, C.POINTER(i64)],
            "romap_set_params": [P, i32, i32, P, i64],
            "romap_save": [P, C.c_char_p],
            "romap_load": [P, C.c_char_p],
            "romap_debug_rays": [P, i32, i32, P, P, P, P],
            "romap_debug_encode": [P, i32, P, i64, P, P],
            "romap_field_forward": [P, i32, P, P, i32, P, P, P],
            "romap_field_forward_noalloc": [P, i32, P, P, i32, P, P, P],
            "romap_field_backward": [P, i32, P, P, i32, P, P, P, P],
            "romap_get_phase_times": [P, P, C.POINTER(i32)],
            "romap_sync": [P],
            "romap_set_occupancy": [P, i32, P],
            "romap_update_occupancy": [P, i32, C.c_float],
            "romap_get_occupancy": [P, i32, P],
            "romap_marching_cubes": [P, P, i32, C.c_float, P, P, P, i64, C.POINTER(i64), i32],
            "romap_extract_mesh": [P, i32, i32, C.c_float, i32, P, i64, C.POINTER(i64), i32],
            "romap_mc_case": [i32, P],
            "romap_debug_bin_capacity": [P, i32],
            "romap_debug_tiles": [P, i32, i32],
            "romap_debug_mfma_rate": [i32, C.POINTER(C.c_double)],
            "romap_get_step_records": [P, C.POINTER(C.c_double)],
            "romap_box_from_points": [P, i64, C.POINTER(romap_box)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = i32
        L.romap_last_error.argtypes = [P]
        L.romap_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def default_config(**kw) -> romap_config:
    cfg = romap_config()
    lib().romap_default_config(C.byref(cfg))
    for k, v in kw.items():
        if not hasattr(cfg, k):
            raise KeyError(k)
        setattr(cfg, k, v)
    return cfg


def make_camera(cam: dict) -> romap_camera:
    c = romap_camera()
    c.T_wc[:] = [float(x) for x in np.asarray(cam["T_wc"], np.float32).reshape(12)]
    c.fx, c.fy, c.cx, c.cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    c.width, c.height = int(cam["W"]), int(cam["H"])
    return c


def box_from_points(xyz):
    """Box of a world point cloud (Eq. 1, PCA yaw, Eq. 4): (t, yaw, half)."""
    xyz = np.ascontiguousarray(xyz, np.float32).reshape(-1, 3)
    b = romap_box()
    rc = lib().romap_box_from_points(_ptr(xyz), xyz.shape[0], C.byref(b))
    if rc != 0:
        raise RomapError(rc, "box_from_points: empty or NULL input")
    return (np.array(b.t[:], np.float32), float(b.yaw), np.array(b.half[:], np.float32))


def debug_mfma_rate(precision=None) -> float:
    """Sustained MFMA rate of the current device in TFLOP/s (BF16 by default)."""
    x = C.c_double(0.0)
    p = PREC_BF16 if precision is None else int(precision)
    rc = lib().romap_debug_mfma_rate(p, C.byref(x))
    if rc != 0:
        raise RomapError(rc, "debug_mfma_rate failed")
    return float(x.value)


def mc_case(m: int):
    """The library's marching-cubes case m: (n, 3) edge triples (host only)."""
    t = np.zeros(16, np.int8)
    n = lib().romap_mc_case(int(m), _ptr(t))
    return t[:3 * n].reshape(n, 3).astype(np.int64)


class Context:
    """Owns one romap_ctx.  Methods map one-to-one onto the C ABI."""

    def __init__(self, cfg: romap_config | None = None, stream=None, **kw):
        self.cfg = cfg if cfg is not None else default_config(**kw)
        h = C.c_void_p()
        st = None if stream is None else C.c_void_p(stream.cuda_stream)
        self._check(lib().romap_create(C.byref(self.cfg), st, C.byref(h)), None)
        self.h = h

    def _check(self, rc, h="self"):
        if rc != ROMAP_OK:
            hh = self.h if h == "self" else None
            raise RomapError(rc, lib().romap_last_error(hh).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().romap_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- verbs
    def add_object(self, instance, t, yaw, half, log2T=0) -> int:
        b = romap_box()
        b.t[:] = [float(x) for x in np.asarray(t, np.float32)]
        b.yaw = float(np.float32(yaw))
        b.half[:] = [float(x) for x in np.asarray(half, np.float32)]
        oid = C.c_int32()
        self._check(lib().romap_add_object(self.h, int(instance), C.byref(b), int(log2T),
                                           C.byref(oid)))
        return oid.value

    def set_active(self, oid, active=True):
        self._check(lib().romap_set_object_active(self.h, int(oid), int(bool(active))))

    def object_info(self, oid) -> romap_object_info:
        info = romap_object_info()
        self._check(lib().romap_get_object_info(self.h, int(oid), C.byref(info)))
        return info

    def add_keyframe(self, cam: dict, rgb, mask, depth=None):
        c = make_camera(cam)
        rgb = np.ascontiguousarray(rgb, np.uint8)
        mask = np.ascontiguousarray(mask, np.int32)
        dep = None if depth is None else np.ascontiguousarray(depth, np.float32)
        kid, nacc = C.c_int32(), C.c_int32()
        self._check(lib().romap_add_keyframe(self.h, C.byref(c), _ptr(rgb), _ptr(mask), _ptr(dep),
                                             C.byref(kid), C.byref(nacc)))
        return kid.value, nacc.value

    def train(self, n_steps, object_ids=None, rays=None, stats=True):
        ids = None if object_ids is None else np.ascontiguousarray(object_ids, np.int32)
        ry = None if rays is None else np.ascontiguousarray(rays, np.int32)
        n = 0 if ids is None else ids.size
        st = romap_train_stats()
        self._check(lib().romap_train(self.h, _ptr(ids), n, int(n_steps), _ptr(ry),
                                      C.byref(st) if stats else None))
        return st if stats else None

    def loss_and_grad(self, object_ids, rays=None):
        ids = np.ascontiguousarray(object_ids, np.int32)
        ry = None if rays is None else np.ascontiguousarray(rays, np.int32)
        losses = np.zeros(ids.size, np.float32)
        self._check(lib().romap_loss_and_grad(self.h, _ptr(ids), ids.size, _ptr(ry),
                                              _ptr(losses)))
        return losses

    def render(self, oid, cam: dict):
        c = make_camera(cam)
        H, W = int(cam["H"]), int(cam["W"])
        rgb = np.zeros((H, W, 3), np.float32)
        depth = np.zeros((H, W), np.float32)
        opac = np.zeros((H, W), np.float32)
        self._check(lib().romap_render(self.h, int(oid), C.byref(c), _ptr(rgb), _ptr(depth),
                                       _ptr(opac), 0))
        return rgb, depth, opac

    def debug_bin_capacity(self, slots: int):
        """Cap every gradient bin at `slots` records (0 = sized capacity)."""
        self._check(lib().romap_debug_bin_capacity(self.h, int(slots)))

    def debug_tiles(self, rays_per_item: int, gather_block: int):
        """Launch shape of the field and gather kernels when autotune is off."""
        self._check(lib().romap_debug_tiles(self.h, int(rays_per_item), int(gather_block)))

    def marching_cubes(self, grid, res, iso, lo, hi):
        """Marching cubes on a (res+1)^3 grid (x fastest; numpy or a device
        tensor): (n, 3, 3) triangles (numpy, or a tensor on the grid's device)."""
        lo = np.ascontiguousarray(lo, np.float32)
        hi = np.ascontiguousarray(hi, np.float32)
        n = C.c_int64(0)
        if isinstance(grid, torch.Tensor):
            g = grid.contiguous().float()
            self._check(lib().romap_marching_cubes(self.h, _ptr(g), int(res), float(iso), _ptr(lo),
                                                   _ptr(hi), None, 0, C.byref(n), 1))
            out = torch.empty((max(n.value, 1), 3, 3), dtype=torch.float32, device=g.device)
            self._check(lib().romap_marching_cubes(self.h, _ptr(g), int(res), float(iso), _ptr(lo),
                                                   _ptr(hi), _ptr(out), n.value, C.byref(n), 1))
            return out[:n.value]
        g = np.ascontiguousarray(grid, np.float32).reshape(-1)
        self._check(lib().romap_marching_cubes(self.h, _ptr(g), int(res), float(iso), _ptr(lo),
                                               _ptr(hi), None, 0, C.byref(n), 0))
        out = np.zeros((max(n.value, 1), 3, 3), np.float32)
        self._check(lib().romap_marching_cubes(self.h, _ptr(g), int(res), float(iso), _ptr(lo),
                                               _ptr(hi), _ptr(out), n.value, C.byref(n), 0))
        return out[:n.value]

    def extract_mesh(self, oid, res=64, iso=10.0, world=True, max_tris=None):
        """An object's mesh: (n, 3, 3) triangles, world frame by default."""
        n = C.c_int64(0)
        if max_tris is None:
            self._check(lib().romap_extract_mesh(self.h, int(oid), int(res), float(iso), int(world),
                                                 None, 0, C.byref(n), 0))
            max_tris = n.value
        out = np.zeros((max(max_tris, 1), 3, 3), np.float32)
        self._check(lib().romap_extract_mesh(self.h, int(oid), int(res), float(iso), int(world),
                                             _ptr(out), int(max_tris), C.byref(n), 0))
        return out[:min(n.value, max_tris)]

    def query_density(self, oid, xyz):
        if isinstance(xyz, torch.Tensor):
            sig = torch.empty(xyz.shape[0], dtype=torch.float32, device=xyz.device)
            self._check(lib().romap_query_density(self.h, int(oid), _ptr(xyz), xyz.shape[0],
                                                  _ptr(sig), 1))
            return sig
        xyz = np.ascontiguousarray(xyz, np.float32).reshape(-1, 3)
        sig = np.zeros(xyz.shape[0], np.float32)
        self._check(lib().romap_query_density(self.h, int(oid), _ptr(xyz), xyz.shape[0],
                                              _ptr(sig), 0))
        return sig

    def n_params(self, oid) -> int:
        n = C.c_int64()
        self._check(lib().romap_get_params(self.h, int(oid), PARAMS, None, 0, C.byref(n)))
        return n.value

    def get_params(self, oid, kind=PARAMS):
        n = self.n_params(oid)
        buf = np.zeros(n, np.float32)
        self._check(lib().romap_get_params(self.h, int(oid), int(kind), _ptr(buf), n, None))
        return buf

    def set_params(self, oid, buf, kind=PARAMS):
        buf = np.ascontiguousarray(buf, np.float32)
        self._check(lib().romap_set_params(self.h, int(oid), int(kind), _ptr(buf), buf.size))

    def save(self, path):
        self._check(lib().romap_save(self.h, str(path).encode()))

    def load(self, path):
        self._check(lib().romap_load(self.h, str(path).encode()))

    def debug_rays(self, oid, n_rays):
        N = self.cfg.samples_per_ray
        kfuv = np.zeros((n_rays, 3), np.int32)
        cls = np.zeros(n_rays, np.int32)
        rf = np.zeros((n_rays, 16), np.float32)
        pos = np.zeros((n_rays, N, 3), np.float32)
        self._check(lib().romap_debug_rays(self.h, int(oid), int(n_rays), _ptr(kfuv), _ptr(cls),
                                           _ptr(rf), _ptr(pos)))
        return kfuv, cls, rf, pos

    def debug_encode(self, oid, p):
        p = np.ascontiguousarray(p, np.float32).reshape(-1, 3)
        L = self.cfg.n_levels
        idx = np.zeros((p.shape[0], L, 8), np.uint32)
        feat = np.zeros((p.shape[0], L, 2), np.float32)
        self._check(lib().romap_debug_encode(self.h, int(oid), _ptr(p), p.shape[0], _ptr(idx),
                                             _ptr(feat)))
        return idx, feat

    def field_forward(self, oid, rays, params=None):
        n = rays.shape[0]
        dev = rays.device
        rgb = torch.empty(n, 3, device=dev)
        depth = torch.empty(n, device=dev)
        tend = torch.empty(n, device=dev)
        self._check(lib().romap_field_forward(self.h, int(oid), _ptr(params), _ptr(rays), n,
                                              _ptr(rgb), _ptr(depth), _ptr(tend)))
        return rgb, depth, tend

    def field_forward_noalloc(self, oid, rays, rgb, depth, tend, params=None):
        """romap_field_forward into caller-given device tensors, with no
        device allocation (the library's fixed scratch array)."""
        n = rays.shape[0]
        for t, shape in ((rays, (n, 8)), (rgb, (n, 3)), (depth, (n,)), (tend, (n,))):
            if (not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32
                    or tuple(t.shape) != shape or not t.is_contiguous()):
                raise ValueError(f"field_forward_noalloc: expected a contiguous float32 device "
                                 f"tensor of shape {shape}")
        self._check(lib().romap_field_forward_noalloc(self.h, int(oid), _ptr(params), _ptr(rays),
                                                      rays.shape[0], _ptr(rgb), _ptr(depth),
                                                      _ptr(tend)))

    def field_backward(self, oid, rays, d_rgb, d_depth, d_tend, params=None):
        n = rays.shape[0]
        P = self.n_params(oid)
        out = torch.empty(P, device=rays.device)
        self._check(lib().romap_field_backward(self.h, int(oid), _ptr(params), _ptr(rays), n,
                                               _ptr(d_rgb), _ptr(d_depth), _ptr(d_tend),
                                               _ptr(out)))
        return out

    def set_occupancy(self, oid, bits):
        b = None if bits is None else np.ascontiguousarray(bits, np.uint8)
        assert b is None or b.size == 32768
        self._check(lib().romap_set_occupancy(self.h, int(oid), _ptr(b)))

    def update_occupancy(self, oid, threshold):
        self._check(lib().romap_update_occupancy(self.h, int(oid), float(threshold)))

    def get_occupancy(self, oid):
        b = np.zeros(32768, np.uint8)
        self._check(lib().romap_get_occupancy(self.h, int(oid), _ptr(b)))
        return b

    def step_records(self) -> float:
        """Gradient records per step over the last profiled romap_train."""
        x = C.c_double(0.0)
        self._check(lib().romap_get_step_records(self.h, C.byref(x)))
        return x.value

    def phase_times(self):
        """Average ms per kernel over the steps of the last profiled train call."""
        ms = np.zeros(len(PHASES), np.float32)
        n = C.c_int32()
        self._check(lib().romap_get_phase_times(self.h, _ptr(ms), C.byref(n)))
        return dict(zip(PHASES, (float(x) for x in ms))), n.value

    def sync(self):
        self._check(lib().romap_sync(self.h))

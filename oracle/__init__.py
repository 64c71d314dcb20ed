"""CPU oracle for RO-MAP's per-object radiance-field training step.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU
baseline leg of ``bench.py`` may import this package.  It shares no code with
the GPU library (``paper_2304_05735_amd``) and the product path never calls it.

``romap_oracle.c`` holds the arithmetic (FP64 values, FP32 position/index
path).  This module wraps it with ctypes and keeps the host-side bookkeeping
of the method in plain Python: the object registry, the keyframe sets with the
incremental update rule of Eq. 5 (Sec. V-A "Data"), and dense Adam state.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "romap_oracle.c")
_LIB = os.path.join(_HERE, "libromap_oracle.so")

MAX_LEVELS = 16
HIDDEN = 64
GEO = 15
DOUT = 16


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP32 path needs -ffp-contract=off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fno-fast-math",
             "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Config(C.Structure):
    _fields_ = [("L", C.c_int32), ("nmin", C.c_int32), ("nmax", C.c_int32), ("log2T", C.c_int32),
                ("N", C.c_int32), ("margin_pct", C.c_int32),
                ("lambda_depth", C.c_double), ("lambda_density", C.c_double),
                ("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("seed", C.c_uint64)]


class Levels(C.Structure):
    _fields_ = [("L", C.c_int32), ("N", C.c_int32 * MAX_LEVELS), ("T", C.c_int64 * MAX_LEVELS),
                ("hashed", C.c_int32 * MAX_LEVELS), ("off", C.c_int64 * (MAX_LEVELS + 1)),
                ("mlp_layers", C.c_int32), ("mlp_bf16", C.c_int32)]


class Keyframe(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("mask", C.c_void_p), ("depth", C.c_void_p),
                ("W", C.c_int32), ("H", C.c_int32),
                ("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float),
                ("M", C.c_float * 9), ("c", C.c_float * 3),
                ("x0", C.c_int32), ("y0", C.c_int32), ("w", C.c_int32), ("h", C.c_int32)]


class Ray(C.Structure):
    _fields_ = [("kf", C.c_int32), ("u", C.c_int32), ("v", C.c_int32), ("cls", C.c_int32),
                ("hit", C.c_int32), ("has_depth", C.c_int32),
                ("C", C.c_float * 3), ("Crand", C.c_float * 3), ("D", C.c_float),
                ("o", C.c_float * 3), ("d", C.c_float * 3), ("tn", C.c_float), ("tf", C.c_float),
                ("delta", C.c_float),
                ("Chat", C.c_double * 3), ("Dhat", C.c_double), ("Tend", C.c_double),
                ("loss", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.c_void_p
        _lib.or_grid_params.restype = C.c_int64
        _lib.or_mlp_params.restype = C.c_int64
        _lib.or_mlp_params.argtypes = [C.c_int, C.c_int]
        _lib.or_make_levels.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(Levels)]
        _lib.or_slab.argtypes = [P, P, P, P, P]
        _lib.or_sample_positions.argtypes = [P, P, P, C.c_float, C.c_float, C.c_int, P, P, P]
        _lib.or_pixel_ray.argtypes = [P, P, C.c_float, C.c_float, C.c_float, C.c_float,
                                      C.c_int, C.c_int, P, P]
        _lib.or_object_frame.argtypes = [P, P, C.c_float, P, P]
        _lib.or_encode.argtypes = [C.POINTER(Levels), P, P, P, P, P]
        _lib.or_mlp_forward.argtypes = [C.c_int, C.c_int, C.c_int, P, P, P, P, P, P, P, P]
        _lib.or_bf16.argtypes = [C.c_double]
        _lib.or_bf16.restype = C.c_double
        _lib.or_bf16_gap.argtypes = [C.c_double]
        _lib.or_bf16_gap.restype = C.c_double
        _lib.or_bf16_set_jitter.argtypes = [C.c_double]
        _lib.or_set_tie_jitter.argtypes = [C.c_double]
        _lib.or_set_jitter_seed.argtypes = [C.c_uint64]
        _lib.or_composite.argtypes = [C.c_int, P, P, P, C.c_double, C.c_int, P, P, P, P, P]
        _lib.or_candidate_rect.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, P]
        _lib.or_draw_ray.argtypes = [C.POINTER(Config), C.c_int, C.c_int, C.c_int, C.c_int,
                                     C.POINTER(Keyframe), C.c_int, C.POINTER(Ray)]
        _lib.or_object_step.argtypes = [C.POINTER(Config), C.POINTER(Levels), C.c_int, C.c_int, P,
                                        C.c_int, C.POINTER(Keyframe), C.c_int, C.c_int, P, P, P, P,
                                        P, P, P, P, P, C.POINTER(Ray), C.c_int]
        _lib.or_adam.argtypes = [C.c_int64, P, P, P, P, C.c_int, C.c_double, C.c_double,
                                 C.c_double, C.c_double]
        _lib.or_render.argtypes = [C.POINTER(Config), C.POINTER(Levels), P, C.POINTER(Keyframe), P,
                                   P, P, P, P, P, C.c_int]
        _lib.or_query_density.argtypes = [C.POINTER(Levels), P, P, C.c_int64, P, P]
        _lib.or_philox4x32_10.argtypes = [P, P, P]
        _lib.or_box_from_points.argtypes = [P, C.c_int64, P, P, P]
        _lib.or_box_from_points.restype = C.c_int
        _lib.or_mc_case.argtypes = [C.c_int, P]
        _lib.or_mc_case.restype = C.c_int
        _lib.or_marching_cubes.argtypes = [P, C.c_int, C.c_float, P, P, P, C.c_int64]
        _lib.or_marching_cubes.restype = C.c_int64
        _lib.or_field.argtypes = [C.POINTER(Config), C.POINTER(Levels), P, P, C.c_int, P, P, P, P,
                                  P, P, P, P, P, P, P, C.c_int]
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def box_from_points(xyz):
    """Box (t, yaw, half) of a world point cloud: Eq. 1, PCA yaw, Eq. 4."""
    xyz = np.ascontiguousarray(xyz, np.float64).reshape(-1, 3)
    t = np.zeros(3)
    yaw = np.zeros(1)
    half = np.zeros(3)
    if lib().or_box_from_points(_p(xyz), xyz.shape[0], _p(t), _p(yaw), _p(half)) != 0:
        raise ValueError("empty point cloud")
    return t, float(yaw[0]), half


def mc_case(m: int):
    """Triangles of marching-cubes case m: (n, 3) edge numbers."""
    t = np.zeros(16, np.int8)
    n = lib().or_mc_case(int(m), _p(t))
    return t[:3 * n].reshape(n, 3).astype(np.int64)


def grid_points(res, lo, hi):
    """Corner positions of a res^3 cell grid, x fastest, as the mesher forms
    them: lo + (hi - lo) * (i / res) in FP32."""
    lo = np.asarray(lo, np.float32)
    hi = np.asarray(hi, np.float32)
    f = (np.arange(res + 1, dtype=np.float32) / np.float32(res)).astype(np.float32)
    ax = [(lo[a] + (hi[a] - lo[a]) * f).astype(np.float32) for a in range(3)]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return np.stack([x, y, z], -1).reshape(-1, 3)


def marching_cubes(grid, res, iso, lo, hi):
    """Marching cubes on a (res+1)^3 grid (x fastest): (n, 3, 3) triangles."""
    grid = np.ascontiguousarray(grid, np.float32).reshape(-1)
    assert grid.size == (res + 1) ** 3
    lo = np.asarray(lo, np.float32)
    hi = np.asarray(hi, np.float32)
    n = lib().or_marching_cubes(_p(grid), int(res), float(np.float32(iso)), _p(lo), _p(hi), None, 0)
    out = np.zeros((max(n, 1), 9), np.float32)
    lib().or_marching_cubes(_p(grid), int(res), float(np.float32(iso)), _p(lo), _p(hi), _p(out), n)
    return out[:n].reshape(n, 3, 3)


# --------------------------------------------------------------------------
# thin wrappers around single C functions (used by the pin tests)

def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def levels(L, nmin, nmax, log2T, mlp_layers=1, bf16=False) -> Levels:
    """Level table of an object's grid; mlp_layers = hidden layers of its
    density MLP (1, 2 or 3); bf16: the MLP's BF16 mode (operands of every
    contraction rounded to BF16, see bf16())."""
    if mlp_layers not in (1, 2, 3):
        raise ValueError("mlp_layers must be 1, 2 or 3")
    lv = Levels()
    if lib().or_make_levels(L, nmin, nmax, log2T, C.byref(lv)) != 0:
        raise ValueError("bad level parameters")
    lv.mlp_layers = mlp_layers
    lv.mlp_bf16 = 1 if bf16 else 0
    return lv


def grid_params(lv: Levels) -> int:
    return int(lv.off[lv.L])


def mlp_params(din: int, layers: int = 1) -> int:
    return int(lib().or_mlp_params(din, layers))


def object_frame(Twc, t, yaw):
    Twc = np.ascontiguousarray(Twc, np.float32).reshape(12)
    t = np.ascontiguousarray(t, np.float32)
    M = np.zeros(9, np.float32)
    c = np.zeros(3, np.float32)
    lib().or_object_frame(_p(Twc), _p(t), C.c_float(yaw), _p(M), _p(c))
    return M, c


def pixel_ray(M, c, fx, fy, cx, cy, u, v):
    M = np.ascontiguousarray(M, np.float32)
    c = np.ascontiguousarray(c, np.float32)
    o = np.zeros(3, np.float32)
    d = np.zeros(3, np.float32)
    lib().or_pixel_ray(_p(M), _p(c), fx, fy, cx, cy, int(u), int(v), _p(o), _p(d))
    return o, d


def slab(o, d, half):
    o = np.ascontiguousarray(o, np.float32)
    d = np.ascontiguousarray(d, np.float32)
    h = np.ascontiguousarray(half, np.float32)
    tn = np.zeros(1, np.float32)
    tf = np.zeros(1, np.float32)
    hit = lib().or_slab(_p(o), _p(d), _p(h), _p(tn), _p(tf))
    return bool(hit), float(tn[0]), float(tf[0])


def sample_positions(o, d, half, tn, tf, N):
    o = np.ascontiguousarray(o, np.float32)
    d = np.ascontiguousarray(d, np.float32)
    h = np.ascontiguousarray(half, np.float32)
    delta = np.zeros(1, np.float32)
    dist = np.zeros(N, np.float32)
    pos = np.zeros((N, 3), np.float32)
    lib().or_sample_positions(_p(o), _p(d), _p(h), tn, tf, N, _p(delta), _p(dist), _p(pos))
    return float(delta[0]), dist, pos


def encode(lv: Levels, p, grid):
    p = np.ascontiguousarray(p, np.float32)
    grid = np.ascontiguousarray(grid, np.float64)
    L = lv.L
    idx = np.zeros(8 * L, np.uint32)
    w = np.zeros(8 * L, np.float64)
    e = np.zeros(2 * L, np.float64)
    lib().or_encode(C.byref(lv), _p(p), _p(grid), _p(idx), _p(w), _p(e))
    return idx.reshape(L, 8), w.reshape(L, 8), e


def bf16(x) -> float:
    """x rounded to BF16 (8 significant bits, nearest, ties to even)."""
    return float(lib().or_bf16(float(x)))


def bf16_gap(x) -> float:
    """Distance from x to the nearest midpoint between BF16 values."""
    return float(lib().or_bf16_gap(float(x)))


def set_bf16_jitter(rel: float) -> None:
    """Tests only: move every rounded BF16 operand (not the weights) by at most
    rel |x| before it is rounded, imitating a computation with rounding
    error; 0 switches it off."""
    lib().or_bf16_set_jitter(float(rel))


def set_tie_jitter(rel: float) -> None:
    """Tests only: move every ReLU pre-activation by at most rel times the sum
    of |terms| that form it before its branch is taken, imitating a
    computation with rounding error; 0 switches it off."""
    lib().or_set_tie_jitter(float(rel))


def set_jitter_seed(seed: int) -> None:
    """Tests only: another deterministic perturbation for both jitters."""
    lib().or_set_jitter_seed(int(seed))


def mlp_forward(din, mlp, e, layers=1, bf16=False):
    """h1: the density MLP's hidden activations, 64 per layer.  bf16: the BF16
    mode (weights and every layer's input rounded where a contraction reads
    them)."""
    mlp = np.ascontiguousarray(mlp, np.float64)
    e = np.ascontiguousarray(e, np.float64)
    assert mlp.size >= mlp_params(din, layers)
    h1 = np.zeros(HIDDEN * layers)
    y = np.zeros(DOUT)
    h2 = np.zeros(HIDDEN)
    sigma = np.zeros(1)
    rgb = np.zeros(3)
    rgbc = np.zeros(3)
    lib().or_mlp_forward(din, layers, 1 if bf16 else 0, _p(mlp), _p(e), _p(h1), _p(y), _p(h2),
                         _p(sigma), _p(rgb), _p(rgbc))
    return dict(h1=h1, y=y, h2=h2, sigma=float(sigma[0]), rgb=rgb, rgb_complement=rgbc)


def composite(sigma, rgb, dist, delta, background=False, crand=(0.0, 0.0, 0.0)):
    sigma = np.ascontiguousarray(sigma, np.float64)
    rgb = np.ascontiguousarray(rgb, np.float64).reshape(-1, 3)
    dist = np.ascontiguousarray(dist, np.float64)
    N = sigma.shape[0]
    cr = np.ascontiguousarray(crand, np.float64)
    Cout = np.zeros(3)
    D = np.zeros(1)
    Tend = np.zeros(1)
    w = np.zeros(N)
    lib().or_composite(N, _p(sigma), _p(rgb), _p(dist), float(delta), int(background), _p(cr),
                       _p(Cout), _p(D), _p(Tend), _p(w))
    return Cout, float(D[0]), float(Tend[0]), w


def candidate_rect(mask, instance, margin_pct=10):
    mask = np.ascontiguousarray(mask, np.int32)
    H, W = mask.shape
    rect = np.zeros(4, np.int32)
    ok = lib().or_candidate_rect(_p(mask), W, H, int(instance), int(margin_pct), _p(rect))
    return tuple(int(x) for x in rect) if ok else None


def adam(p, g, m, v, k, lr, b1, b2, eps):
    """In-place dense Adam on float64 arrays; k is the step number (1 first)."""
    lib().or_adam(p.size, _p(p), _p(g), _p(m), _p(v), int(k), lr, b1, b2, eps)


# --------------------------------------------------------------------------
# object / keyframe bookkeeping (same semantics as the GPU library's C ABI)

def host_threads() -> int:
    """Host threads the oracle uses by default: every core this process may
    run on."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


def make_config(L=16, nmin=16, nmax=1024, log2T=19, N=64, margin_pct=10, lambda_depth=0.5,
                lambda_density=0.01, lr=1e-2, beta1=0.9, beta2=0.99, eps=1e-15, seed=0) -> Config:
    return Config(L, nmin, nmax, log2T, N, margin_pct, lambda_depth, lambda_density, lr, beta1,
                  beta2, eps, seed)


class _Kf:
    """Keyframe as stored by the oracle: owned numpy copies of the images."""

    def __init__(self, cam, rgb, mask, depth):
        self.Twc = np.ascontiguousarray(cam["T_wc"], np.float32).reshape(12)
        self.fx, self.fy, self.cx, self.cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
        self.rgb = np.ascontiguousarray(rgb, np.uint8)
        self.mask = np.ascontiguousarray(mask, np.int32)
        self.depth = None if depth is None else np.ascontiguousarray(depth, np.float32)
        self.H, self.W = self.mask.shape
        self.centre = self.Twc.reshape(3, 4)[:, 3].astype(np.float64)


class _Obj:
    def __init__(self, instance, t, yaw, half, log2T, lv, params):
        self.instance = int(instance)
        self.t = np.asarray(t, np.float32)
        self.yaw = float(np.float32(yaw))
        self.half = np.asarray(half, np.float32)
        self.log2T = log2T
        self.lv = lv
        self.params = params
        self.m = np.zeros_like(params)
        self.v = np.zeros_like(params)
        self.grad = np.zeros_like(params)
        self.k = 0
        self.kfs: list[tuple[_Kf, tuple]] = []  # (keyframe, candidate rect)
        self.occ = None  # 64^3 occupancy bits (32768 bytes) or None
        self.last_centre = None


class OracleContext:
    """Plain CPU counterpart of the GPU library's context (same verbs)."""

    def __init__(self, cfg: Config, alpha_deg: float = 25.0, nthreads: int | None = None,
                 mlp_layers: int = 1, bf16: bool = False):
        self.cfg = cfg
        self.mlp_layers = mlp_layers
        self.bf16 = bf16
        self.alpha_deg = alpha_deg
        self.nthreads = nthreads or host_threads()
        self.objects: list[_Obj] = []
        self.keyframes: list[_Kf] = []

    # register object with box and table size (Sec. V: a new model per new instance)
    def add_object(self, instance, t, yaw, half, log2T=None, params=None) -> int:
        log2T = self.cfg.log2T if log2T is None else log2T
        lv = levels(self.cfg.L, self.cfg.nmin, self.cfg.nmax, log2T, self.mlp_layers, self.bf16)
        P = grid_params(lv) + mlp_params(2 * self.cfg.L, self.mlp_layers)
        p = np.zeros(P) if params is None else np.array(params, np.float64)
        assert p.size == P
        self.objects.append(_Obj(instance, t, yaw, half, log2T, lv, p))
        return len(self.objects) - 1

    def n_params(self, oid) -> int:
        return self.objects[oid].params.size

    # add posed keyframe + mask; Eq. 5 decides per object whether it joins its set
    def add_keyframe(self, cam, rgb, mask, depth=None) -> int:
        kf = _Kf(cam, rgb, mask, depth)
        self.keyframes.append(kf)
        accepted = 0
        for o in self.objects:
            rect = candidate_rect(kf.mask, o.instance, self.cfg.margin_pct)
            if rect is None:
                continue  # the object is not observed in this image
            if o.last_centre is not None:
                a = o.last_centre - o.t.astype(np.float64)
                b = kf.centre - o.t.astype(np.float64)
                cosang = float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))
                alpha = math.degrees(math.acos(max(-1.0, min(1.0, cosang))))
                if not alpha > self.alpha_deg:
                    continue
            o.kfs.append((kf, rect))
            o.last_centre = kf.centre
            accepted += 1
        return accepted

    def _kf_array(self, o: _Obj):
        arr = (Keyframe * len(o.kfs))()
        for i, (kf, rect) in enumerate(o.kfs):
            M, c = object_frame(kf.Twc, o.t, o.yaw)
            k = arr[i]
            k.rgb = kf.rgb.ctypes.data
            k.mask = kf.mask.ctypes.data
            k.depth = kf.depth.ctypes.data if kf.depth is not None else None
            k.W, k.H = kf.W, kf.H
            k.fx, k.fy, k.cx, k.cy = kf.fx, kf.fy, kf.cx, kf.cy
            k.M[:] = M
            k.c[:] = c
            k.x0, k.y0, k.w, k.h = rect
        return arr

    def loss_and_grad(self, oid, step, B, rays=False, params=None, want_grad=True, mass=None,
                      ambiguous=None, margin=None, loss_allow=None, bf16_allow=None):
        """Loss of one step and dL/dparams (no optimiser update).  mass: an array
        of the parameter count that receives the magnitude of every gradient
        entry, the same backward on absolute values, which bounds to first order
        how far rounding (in any order of summation) can move the entry.
        ambiguous: an array of the parameter count that receives, for every
        decision (ReLU branch, density clamp) that lies within 1e-5 relative
        of its tie, the change of its sample's contributions under the other
        branch (first order), and for rays whose depth-error sign ties, twice
        the magnitude of their samples' contributions: how far other branch
        choices can move each entry.
        margin: a 1-element array that receives the smallest relative distance
        of a decision from its tie in the step.
        loss_allow (BF16 mode): a 1-element array that receives the bound of
        the change of the loss under the other choice of every ambiguous BF16
        rounding; bf16_allow (BF16 mode) the same bound for every gradient
        entry."""
        o = self.objects[oid]
        if not o.kfs:
            raise RuntimeError("object has no keyframes")
        kfa = self._kf_array(o)
        p = o.params if params is None else np.ascontiguousarray(params, np.float64)
        grad = np.zeros_like(p) if want_grad else None
        loss = np.zeros(1)
        ray_buf = (Ray * B)() if rays else None
        rc = lib().or_object_step(C.byref(self.cfg), C.byref(o.lv), oid, o.instance, _p(o.half),
                                  len(o.kfs), kfa, int(step), int(B), _p(p),
                                  None if o.occ is None else _p(o.occ),
                                  _p(grad) if want_grad else None,
                                  _p(mass) if (want_grad and mass is not None) else None,
                                  None if ambiguous is None else _p(ambiguous),
                                  None if bf16_allow is None else _p(bf16_allow),
                                  None if margin is None else _p(margin),
                                  _p(loss), None if loss_allow is None else _p(loss_allow),
                                  ray_buf, self.nthreads)
        if rc != 0:
            raise RuntimeError("oracle step failed")
        return float(loss[0]), grad, ray_buf

    def train(self, oid, n_steps, B):
        """n_steps of draw / render / loss / backward / dense Adam."""
        o = self.objects[oid]
        losses = []
        for _ in range(n_steps):
            loss, g, _ = self.loss_and_grad(oid, o.k, B)
            o.k += 1
            o.grad[:] = g
            adam(o.params, o.grad, o.m, o.v, o.k, self.cfg.lr, self.cfg.beta1, self.cfg.beta2,
                 self.cfg.eps)
            losses.append(loss)
        return losses

    def render(self, oid, cam, W, H, rgb_allow=None):
        """rgb_allow (BF16 mode): an (H, W, 3) array that receives the bound of
        the change of each colour under the other choice of every ambiguous
        BF16 rounding."""
        o = self.objects[oid]
        kf = Keyframe()
        M, c = object_frame(np.asarray(cam["T_wc"], np.float32), o.t, o.yaw)
        kf.W, kf.H = W, H
        kf.fx, kf.fy, kf.cx, kf.cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
        kf.M[:] = M
        kf.c[:] = c
        rgb = np.zeros((H, W, 3))
        depth = np.zeros((H, W))
        opac = np.zeros((H, W))
        lib().or_render(C.byref(self.cfg), C.byref(o.lv), _p(o.half), C.byref(kf), _p(o.params),
                        None if o.occ is None else _p(o.occ), _p(rgb), _p(depth), _p(opac),
                        None if rgb_allow is None else _p(rgb_allow), self.nthreads)
        return rgb, depth, opac

    def field(self, oid, rays, params=None, d_rgb=None, d_depth=None, d_tend=None, grad=False,
              mass=None, ambiguous=None, bf16_allow=None):
        """rays: (n, 8) float32 object-frame rays (o, d, t_near, t_far).  Returns
        rgb, depth, T_end and, with grad, d(sum d_rgb.C + d_depth D + d_tend T_end)/dparams."""
        o = self.objects[oid]
        rays = np.ascontiguousarray(rays, np.float32).reshape(-1, 8)
        n = rays.shape[0]
        p = o.params if params is None else np.ascontiguousarray(params, np.float64)
        rgb, depth, tend = np.zeros((n, 3)), np.zeros(n), np.zeros(n)
        g = np.zeros(p.size) if grad else None
        cv = lambda a: None if a is None else np.ascontiguousarray(a, np.float64)
        dr, dd, dt = cv(d_rgb), cv(d_depth), cv(d_tend)
        lib().or_field(C.byref(self.cfg), C.byref(o.lv), _p(o.half), _p(p), n, _p(rays), _p(rgb),
                       _p(depth), _p(tend), None if dr is None else _p(dr),
                       None if dd is None else _p(dd), None if dt is None else _p(dt),
                       None if g is None else _p(g),
                       None if (g is None or mass is None) else _p(mass),
                       None if (g is None or ambiguous is None) else _p(ambiguous),
                       None if (g is None or bf16_allow is None) else _p(bf16_allow),
                       self.nthreads)
        return rgb, depth, tend, g

    def set_occupancy(self, oid, bits):
        """64^3 occupancy bitfield (32768 bytes, bit x + 64 y + 4096 z) or None."""
        self.objects[oid].occ = None if bits is None else np.ascontiguousarray(bits, np.uint8)

    def occupancy_from_density(self, oid, threshold):
        """Bits of the cells whose centre density exceeds threshold."""
        o = self.objects[oid]
        g = (np.arange(64, dtype=np.float64) + 0.5) / 64.0
        z, y, x = np.meshgrid(g, g, g, indexing="ij")
        p = np.stack([x, y, z], -1).reshape(-1, 3)
        xyz = (p * (2.0 * o.half) - o.half).astype(np.float32)
        sig = self.query_density(oid, xyz)
        return np.packbits(sig > threshold, bitorder="little")

    def extract_mesh(self, oid, res=64, iso=10.0):
        """Density on the (res+1)^3 corners of the object's box (FP64 model,
        rounded to FP32), marching cubes in the object frame, then the box
        pose: world = Rz(yaw) x + t (FP64).  Returns (world, object-frame)
        triangle arrays."""
        o = self.objects[oid]
        half = np.asarray(o.half, np.float32)
        pts = grid_points(res, -half, half)
        sig = self.query_density(oid, pts).astype(np.float32)
        tri = marching_cubes(sig, res, iso, -half, half)
        c, s = np.cos(float(o.yaw)), np.sin(float(o.yaw))
        R = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
        world = tri.astype(np.float64) @ R.T + np.asarray(o.t, np.float64)
        return world, tri

    def query_density(self, oid, xyz):
        o = self.objects[oid]
        xyz = np.ascontiguousarray(xyz, np.float32).reshape(-1, 3)
        sig = np.zeros(xyz.shape[0])
        lib().or_query_density(C.byref(o.lv), _p(o.half), _p(o.params), xyz.shape[0], _p(xyz),
                               _p(sig))
        return sig

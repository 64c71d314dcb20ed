"""Seeded synthetic scenes: the stand-in for the paper's datasets.

The paper evaluates on Cube-Diorama, Replica and real D455 sequences, none of
which is available here.  This module builds analytic scenes of the same
structure instead (several objects on a floor, a posed RGB stream, per-pixel
instance masks, sparse depth), at the image sizes and object counts of the
workloads being measured.  It holds no arithmetic of the method itself:
intersections are analytic (sphere, yawed box) or bracketed and bisected
(torus), and the ground-truth colour of a constant-density primitive is the
exact emission-absorption integral, evaluated with the substitution
u = 1 - exp(-sigma s) and Gauss-Legendre nodes in u.

Conventions shared with the method's inputs (not its arithmetic): world +z is
up; cameras are pinhole with x right, y down, z forward, pixel centres at
+0.5; ``T_wc`` is the 3x4 camera-to-world pose; masks are int32 with 0 =
background and instance ids >= 1; sparse depth is camera z, 0 where absent.
"""
from __future__ import annotations

import math
import multiprocessing as mp
import os
from dataclasses import dataclass, field

import numpy as np

DENSITY = 50.0
_GL_X, _GL_W = np.polynomial.legendre.leggauss(8)
_GL_X = 0.5 * (_GL_X + 1.0)
_GL_W = 0.5 * _GL_W


def look_at(eye, target, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Camera-to-world 3x4 pose with OpenCV axes looking from eye at target."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    x = np.cross(f, np.asarray(up, np.float64))
    if np.linalg.norm(x) < 1e-9:
        x = np.cross(f, np.array([0.0, 1.0, 0.0]))
    x /= np.linalg.norm(x)
    y = np.cross(f, x)
    T = np.zeros((3, 4))
    T[:, 0], T[:, 1], T[:, 2], T[:, 3] = x, y, f, eye
    return T.astype(np.float32)


def camera(T_wc, W, H, fx, fy=None, cx=None, cy=None) -> dict:
    return dict(T_wc=np.asarray(T_wc, np.float32), W=int(W), H=int(H), fx=float(fx),
                fy=float(fx if fy is None else fy), cx=float(W / 2 if cx is None else cx),
                cy=float(H / 2 if cy is None else cy))


# ---------------------------------------------------------------------------
# primitives: each returns up to two (t_in, t_out) segments per ray

@dataclass
class Primitive:
    kind: str                      # "sphere" | "box" | "torus"
    center: np.ndarray
    size: np.ndarray               # sphere (r,), box half (3,), torus (R, r)
    yaw: float = 0.0
    instance: int = 1
    phase: np.ndarray = field(default_factory=lambda: np.zeros(3))

    def bound_half(self) -> np.ndarray:
        """Half extents of the primitive's box in its own (yawed) frame."""
        if self.kind == "sphere":
            return np.array([self.size[0]] * 3)
        if self.kind == "box":
            return np.asarray(self.size, np.float64)
        R, r = self.size
        return np.array([R + r, R + r, r])

    def bound_radius(self) -> float:
        return float(np.linalg.norm(self.bound_half()))

    def albedo(self, x: np.ndarray) -> np.ndarray:
        """Procedural colour 0.5 + 0.5 sin(6x + ph, 6y + 1 + ph, 6z + 2 + ph), world coords."""
        return 0.5 + 0.5 * np.sin(6.0 * x + np.array([0.0, 1.0, 2.0]) + self.phase)

    def _local(self, o, d):
        c, s = math.cos(self.yaw), math.sin(self.yaw)
        Rt = np.array([[c, s, 0.0], [-s, c, 0.0], [0.0, 0.0, 1.0]])
        return (o - self.center) @ Rt.T, d @ Rt.T

    def segments(self, o: np.ndarray, d: np.ndarray):
        """o, d: (n, 3) world rays (unit d).  Returns t_in, t_out of shape (n, 2); inf = none."""
        n = o.shape[0]
        tin = np.full((n, 2), np.inf)
        tout = np.full((n, 2), np.inf)
        lo, ld = self._local(o, d)
        if self.kind == "sphere":
            r = self.size[0]
            b = np.sum(ld * lo, 1)
            cc = np.sum(lo * lo, 1) - r * r
            disc = b * b - cc
            ok = disc > 0
            sq = np.sqrt(np.where(ok, disc, 0.0))
            t0, t1 = -b - sq, -b + sq
            ok &= t1 > 0
            tin[ok, 0] = np.maximum(t0[ok], 0.0)
            tout[ok, 0] = t1[ok]
            return tin, tout
        h = self.bound_half()
        with np.errstate(divide="ignore", invalid="ignore"):
            inv = 1.0 / ld
            ta = (-h - lo) * inv
            tb = (h - lo) * inv
        t0 = np.nanmax(np.minimum(ta, tb), 1)
        t1 = np.nanmin(np.maximum(ta, tb), 1)
        t0 = np.maximum(t0, 0.0)
        ok = t1 > t0
        if self.kind == "box":
            tin[ok, 0] = t0[ok]
            tout[ok, 0] = t1[ok]
            return tin, tout
        # torus about the local z axis: bracket sign changes, then bisect
        R, r = self.size
        idx = np.nonzero(ok)[0]
        if idx.size == 0:
            return tin, tout
        a, b = t0[idx], t1[idx]
        steps = 64
        ts = a[:, None] + (b - a)[:, None] * (np.arange(steps + 1) / steps)[None, :]
        rows_all = np.arange(idx.size)

        def inside_at(t, rows):
            p = lo[idx[rows]] + t[:, None] * ld[idx[rows]]
            q = np.sqrt(p[:, 0] ** 2 + p[:, 1] ** 2) - R
            return q * q + p[:, 2] ** 2 - r * r < 0

        px = lo[idx, 0][:, None] + ts * ld[idx, 0][:, None]
        py = lo[idx, 1][:, None] + ts * ld[idx, 1][:, None]
        pz = lo[idx, 2][:, None] + ts * ld[idx, 2][:, None]
        q = np.sqrt(px * px + py * py) - R
        inside = q * q + pz * pz - r * r < 0
        enter = ~inside[:, :-1] & inside[:, 1:]
        leave = inside[:, :-1] & ~inside[:, 1:]
        K = np.arange(steps)[None, :]

        def first(m):
            return np.where(m.any(1), np.argmax(m, 1), -1)

        def refine(k, entering):
            """bisect bracket [ts[k], ts[k+1]] of every row with k >= 0."""
            out = np.full(idx.size, np.nan)
            rows = rows_all[k >= 0]
            if rows.size == 0:
                return out
            lo_t, hi_t = ts[rows, k[rows]], ts[rows, k[rows] + 1]
            for _ in range(30):
                mid = 0.5 * (lo_t + hi_t)
                ins = inside_at(mid, rows)
                move_hi = ins if entering else ~ins
                hi_t = np.where(move_hi, mid, hi_t)
                lo_t = np.where(move_hi, lo_t, mid)
            out[rows] = 0.5 * (lo_t + hi_t)
            return out

        start_in = inside[:, 0]
        e1 = np.where(start_in, -1, first(enter))
        has1 = start_in | (e1 >= 0)
        x1 = np.where(has1, first(leave & (K > e1[:, None])), -1)
        e2 = np.where(has1 & (x1 >= 0), first(enter & (K > x1[:, None])), -1)
        x2 = np.where(e2 >= 0, first(leave & (K > e2[:, None])), -1)
        t_e1 = np.where(start_in, a, refine(e1, True))
        t_x1 = np.where(x1 >= 0, refine(x1, False), b)
        t_e2 = refine(e2, True)
        t_x2 = np.where(x2 >= 0, refine(x2, False), b)
        sel = np.nonzero(has1)[0]
        tin[idx[sel], 0] = t_e1[sel]
        tout[idx[sel], 0] = t_x1[sel]
        sel = np.nonzero(e2 >= 0)[0]
        tin[idx[sel], 1] = t_e2[sel]
        tout[idx[sel], 1] = t_x2[sel]
        return tin, tout


@dataclass
class Scene:
    prims: list

    def render(self, cam: dict):
        """Ground-truth rgb (H, W, 3) float, instance mask (H, W) int32, camera-z depth."""
        W, H = cam["W"], cam["H"]
        T = np.asarray(cam["T_wc"], np.float64).reshape(3, 4)
        u, v = np.meshgrid(np.arange(W), np.arange(H))
        xc = (u + 0.5 - cam["cx"]) / cam["fx"]
        yc = (v + 0.5 - cam["cy"]) / cam["fy"]
        dc = np.stack([xc, yc, np.ones_like(xc)], -1).reshape(-1, 3)
        dc /= np.linalg.norm(dc, axis=1, keepdims=True)
        d = dc @ T[:, :3].T
        npix = d.shape[0]
        o_all = np.broadcast_to(T[:, 3], d.shape)
        Rcw = T[:, :3].T
        # per primitive: pixels inside the projection of its bounding cube
        # (all pixels if the cube reaches behind the camera), then the exact
        # bounding-sphere test on those pixels only
        cands = []
        for p in self.prims:
            rad = p.bound_radius()
            corners = p.center + rad * np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1)
                                                  for sz in (-1, 1)], np.float64)
            pc = (corners - T[:, 3]) @ Rcw.T
            if (pc[:, 2] <= 1e-3).any():
                sel = np.arange(npix)
            else:
                uu = pc[:, 0] / pc[:, 2] * cam["fx"] + cam["cx"]
                vv = pc[:, 1] / pc[:, 2] * cam["fy"] + cam["cy"]
                u0, u1 = max(int(np.floor(uu.min())) - 1, 0), min(int(np.ceil(uu.max())) + 1, W - 1)
                v0, v1 = max(int(np.floor(vv.min())) - 1, 0), min(int(np.ceil(vv.max())) + 1, H - 1)
                if u1 < u0 or v1 < v0:
                    cands.append(np.zeros(0, np.int64))
                    continue
                ug, vg = np.meshgrid(np.arange(u0, u1 + 1), np.arange(v0, v1 + 1))
                sel = (vg * W + ug).reshape(-1)
            oc = T[:, 3] - p.center
            b = d[sel] @ oc
            disc = b * b - (float(oc @ oc) - rad ** 2)
            ok = (disc > 0) & (-b + np.sqrt(np.maximum(disc, 0)) > 0)
            cands.append(sel[ok])
        active = (np.unique(np.concatenate(cands)) if cands else np.zeros(0, np.int64))
        pos_in_active = np.full(npix, -1, np.int64)
        pos_in_active[active] = np.arange(active.size)
        rgb_full = np.zeros((npix, 3))
        mask_full = np.zeros(npix, np.int32)
        depth_full = np.zeros(npix, np.float32)
        d = d[active]
        dc = dc[active]
        o = o_all[active]
        n = active.size
        segs_in, segs_out, segs_p = [], [], []
        for pi, p in enumerate(self.prims):
            cand = pos_in_active[cands[pi]]
            if cand.size == 0:
                continue
            ti, to = p.segments(o[cand], d[cand])
            for s in range(2):
                ok = np.isfinite(ti[:, s]) & (to[:, s] > ti[:, s])
                if not ok.any():
                    continue
                full_in = np.full(n, np.inf)
                full_out = np.full(n, np.inf)
                full_in[cand[ok]] = ti[ok, s]
                full_out[cand[ok]] = to[ok, s]
                segs_in.append(full_in)
                segs_out.append(full_out)
                segs_p.append(pi)
        rgb = np.zeros((n, 3))
        mask = np.zeros(n, np.int32)
        depth = np.zeros(n, np.float32)
        if segs_in:
            tin = np.stack(segs_in, 1)
            tout = np.stack(segs_out, 1)
            pid = np.array(segs_p)
            order = np.argsort(tin, 1)
            tin = np.take_along_axis(tin, order, 1)
            tout = np.take_along_axis(tout, order, 1)
            pids = pid[order]
            trans = np.ones(n)
            first = np.isfinite(tin[:, 0])
            mask[first] = np.array([self.prims[k].instance for k in pids[first, 0]], np.int32)
            depth[first] = (tin[first, 0] * dc[first, 2]).astype(np.float32)
            for s in range(tin.shape[1]):
                rows = np.nonzero(np.isfinite(tin[:, s]) & (trans > 1e-7))[0]
                if rows.size == 0:
                    continue
                length = tout[rows, s] - tin[rows, s]
                U = -np.expm1(-DENSITY * length)
                col = np.zeros((rows.size, 3))
                for k in np.unique(pids[rows, s]):
                    sel = pids[rows, s] == k
                    rr = rows[sel]
                    # points at opacity fractions u = U * x_j along the chord
                    uu = U[sel][:, None] * _GL_X[None, :]
                    sdist = -np.log1p(-uu) / DENSITY
                    pts = o[rr][:, None, :] + (tin[rr, s][:, None] + sdist)[..., None] * d[rr][:, None, :]
                    alb = self.prims[k].albedo(pts)
                    col[sel] = U[sel][:, None] * np.einsum("j,njc->nc", _GL_W, alb)
                rgb[rows] += trans[rows, None] * col
                trans[rows] *= np.exp(-DENSITY * length)
        rgb_full[active] = rgb
        mask_full[active] = mask
        depth_full[active] = depth
        return rgb_full.reshape(H, W, 3), mask_full.reshape(H, W), depth_full.reshape(H, W)


def to_u8(rgb: np.ndarray) -> np.ndarray:
    return np.clip(np.rint(np.clip(rgb, 0.0, 1.0) * 255.0), 0, 255).astype(np.uint8)


# ---------------------------------------------------------------------------
# workloads

@dataclass
class ObjectSpec:
    instance: int
    t: np.ndarray
    yaw: float
    half: np.ndarray
    log2T: int


@dataclass
class Workload:
    name: str
    scene: Scene
    cameras: list
    objects: list          # ObjectSpec
    frames: list = field(default_factory=list)  # (cam, rgb u8, mask, depth or None)
    rays: dict = field(default_factory=dict)    # instance -> rays per step
    eval_views: list = field(default_factory=list)


def _fibonacci_cameras(n, radius, W, H, f):
    cams = []
    for k in range(n):
        z = 1.0 - (2 * k + 1) / n
        phi = k * math.pi * (3.0 - math.sqrt(5.0))
        rxy = math.sqrt(max(0.0, 1.0 - z * z))
        eye = radius * np.array([rxy * math.cos(phi), rxy * math.sin(phi), z])
        cams.append(camera(look_at(eye, (0, 0, 0)), W, H, f))
    return cams


def _render_one(args):
    scene, cam = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):  # one BLAS thread per worker process
        rgb, mask, depth = scene.render(cam)
    return to_u8(rgb), mask, depth


def _gpu_open() -> bool:
    """True once this process holds the GPU driver open (/dev/kfd among its
    file descriptors): the GPU runtime then has threads of its own, and a
    forked child can inherit a lock one of them held and crash or hang."""
    try:
        fds = os.listdir("/proc/self/fd")
    except OSError:
        return False
    for fd in fds:
        try:
            if os.readlink(f"/proc/self/fd/{fd}") == "/dev/kfd":
                return True
        except OSError:
            pass
    return False


def _render_frames(wl: Workload, depth_frac=0.0, seed=0, workers=None):
    rng = np.random.default_rng(seed)
    wl.frames = []
    jobs = [(wl.scene, cam) for cam in wl.cameras]
    workers = workers or min(16, os.cpu_count() or 1)
    if workers > 1 and len(jobs) > 2 and not _gpu_open():
        ctx = mp.get_context("fork")
        pool = ctx.Pool(workers)
        try:
            outs = pool.map(_render_one, jobs)
            pool.close()  # let the workers exit on their own (no SIGTERM)
        except BaseException:
            pool.terminate()
            raise
        finally:
            pool.join()
    else:
        outs = [_render_one(j) for j in jobs]
    for cam, (rgb, mask, dz) in zip(wl.cameras, outs):
        depth = None
        if depth_frac > 0:
            depth = np.zeros_like(dz)
            wanted = {o.instance for o in wl.objects}
            for inst in np.unique(mask):
                if int(inst) not in wanted:
                    continue
                pix = np.flatnonzero(mask.reshape(-1) == inst)
                if pix.size:
                    take = rng.choice(pix, max(1, int(round(depth_frac * pix.size))), replace=False)
                    depth.reshape(-1)[take] = dz.reshape(-1)[take]
        wl.frames.append((cam, rgb, mask, depth))
    return wl


def sphere_scene() -> Workload:
    """One sphere (r 0.3, density 50) in the unit cube; 8 posed 64x64 views."""
    sph = Primitive("sphere", np.zeros(3), np.array([0.3]), instance=1)
    cams = _fibonacci_cameras(8, 1.5, 64, 64, 64.0)
    obj = ObjectSpec(1, np.zeros(3, np.float32), 0.0, np.full(3, 0.5, np.float32), 12)
    wl = Workload("1 object (sphere), L8 T2^12, 256 rays x 32 samples", Scene([sph]), cams, [obj])
    wl.rays = {1: 256}
    _render_frames(wl)
    wl.eval_views = list(range(len(cams)))
    return wl


def torus_scene(n_views=50, W=640, H=480) -> Workload:
    """Sphere, yawed box and torus; the torus (instance 3) is the trained object."""
    prims = [
        Primitive("sphere", np.array([-0.7, 0.0, 0.3]), np.array([0.3]), 0.0, 1,
                  np.array([0.3, 0.6, 0.9])),
        Primitive("box", np.array([0.7, 0.0, 0.3]), np.array([0.25, 0.2, 0.3]), math.radians(30), 2,
                  np.array([1.1, 0.2, 2.0])),
        Primitive("torus", np.array([0.0, 0.7, 0.1]), np.array([0.3, 0.1]), 0.0, 3,
                  np.array([2.2, 1.4, 0.5])),
    ]
    f = (W / 2) / math.tan(math.radians(30))
    cams = []
    for k in range(n_views):
        ang = 2 * math.pi * k / n_views
        eye = (2.5 * math.cos(ang), 2.5 * math.sin(ang), 0.6 if k % 2 == 0 else 1.2)
        cams.append(camera(look_at(eye, (0, 0, 0.2)), W, H, f))
    tor = prims[2]
    obj = ObjectSpec(3, tor.center.astype(np.float32), 0.0,
                     (tor.bound_half() * 1.1).astype(np.float32), 19)
    wl = Workload(f"1 object (torus of 3 primitives), L16 T2^19, 4096 rays x 64 samples, {W}x{H}",
                  Scene(prims), cams, [obj])
    wl.rays = {3: 4096}
    _render_frames(wl, depth_frac=0.005)
    wl.eval_views = list(range(0, n_views, 10))
    return wl


def room_scene(n_obj=24, n_views=60, W=640, H=480, seed=0, room=8.0) -> Workload:
    """n_obj primitives of log-uniform size on a floor, a circle of cameras."""
    rng = np.random.default_rng(seed)
    prims = []
    kinds = ["sphere", "box", "torus"]
    placed = []
    for i in range(n_obj):
        kind = kinds[i % 3]
        edge = math.exp(rng.uniform(math.log(0.1), math.log(2.0)))
        yaw = float(rng.uniform(0, 2 * math.pi))
        if kind == "sphere":
            size = np.array([edge / 2])
        elif kind == "box":
            size = np.array([edge / 2, edge / 2 * rng.uniform(0.5, 1.0), edge / 2 * rng.uniform(0.5, 1.0)])
        else:
            size = np.array([edge * 0.35, edge * 0.12])
        p = Primitive(kind, np.zeros(3), size, yaw, i + 1, rng.uniform(0, 2 * math.pi, 3))
        rad = p.bound_radius()
        half_room = room / 2
        for _ in range(2000):
            xy = rng.uniform(-half_room + rad, half_room - rad, 2) if rad < half_room else np.zeros(2)
            if all(np.linalg.norm(xy - q[0]) > rad + q[1] for q in placed):
                break
        placed.append((xy, rad))
        p.center = np.array([xy[0], xy[1], p.bound_half()[2]])
        prims.append(p)
    f = (W / 2) / math.tan(math.radians(30))
    cams = []
    for k in range(n_views):
        ang = 2 * math.pi * k / n_views
        eye = (5.0 * math.cos(ang), 5.0 * math.sin(ang), 1.5)
        cams.append(camera(look_at(eye, (0, 0, 0.3)), W, H, f))
    objs = []
    vols = [float(np.prod(2 * p.bound_half())) for p in prims]
    for p, V in zip(prims, vols):
        e = 15 + 4 * (math.log(V) - math.log(1e-3)) / (math.log(8.0) - math.log(1e-3))
        log2T = int(min(19, max(15, round(e))))
        objs.append(ObjectSpec(p.instance, p.center.astype(np.float32), float(np.float32(p.yaw)),
                               (p.bound_half() * 1.1).astype(np.float32), log2T))
    wl = Workload(f"{n_obj} objects, L16 T2^15..2^19, 64 samples per ray, {W}x{H}", Scene(prims),
                  cams, objs)
    _render_frames(wl, depth_frac=0.005, seed=seed)
    counts = {o.instance: 0 for o in objs}
    for (_, _, mask, _) in wl.frames:
        ids, cnt = np.unique(mask, return_counts=True)
        for i, c in zip(ids, cnt):
            if i in counts:
                counts[i] += int(c)
    mx = max(max(counts.values()), 1)
    wl.rays = {k: int(min(8192, max(256, round(8192 * v / mx)))) for k, v in counts.items()}
    wl.eval_views = list(range(0, n_views, n_views // 5))
    return wl


def stream_scene(n_obj=128, n_frames=300, W=640, H=480, seed=5, room=14.0) -> Workload:
    """Incremental mapping stream: n_obj primitives in a room, a camera moving
    on a loop through the room at 25 frames per second, looking ahead and
    slightly inward.  Objects are meant to be registered when first seen."""
    rng = np.random.default_rng(seed)
    kinds = ["sphere", "box", "torus"]
    prims, placed = [], []
    half_room = room / 2
    for i in range(n_obj):
        kind = kinds[i % 3]
        edge = math.exp(rng.uniform(math.log(0.15), math.log(1.0)))
        yaw = float(rng.uniform(0, 2 * math.pi))
        if kind == "sphere":
            size = np.array([edge / 2])
        elif kind == "box":
            size = np.array([edge / 2, edge / 2 * rng.uniform(0.5, 1.0), edge / 2 * rng.uniform(0.5, 1.0)])
        else:
            size = np.array([edge * 0.35, edge * 0.12])
        p = Primitive(kind, np.zeros(3), size, yaw, i + 1, rng.uniform(0, 2 * math.pi, 3))
        rad = p.bound_radius()
        for _ in range(4000):
            xy = rng.uniform(-half_room + rad, half_room - rad, 2)
            if 3.0 < np.linalg.norm(xy) and all(np.linalg.norm(xy - q[0]) > rad + q[1] + 0.1
                                                for q in placed):
                break
        placed.append((xy, rad))
        p.center = np.array([xy[0], xy[1], p.bound_half()[2]])
        prims.append(p)
    f = (W / 2) / math.tan(math.radians(35))
    cams = []
    for k in range(n_frames):
        ang = 2 * math.pi * k / n_frames
        eye = np.array([2.2 * math.cos(ang), 2.2 * math.sin(ang), 1.4])
        look = eye + np.array([-math.sin(ang + 0.5), math.cos(ang + 0.5), -0.35])
        cams.append(camera(look_at(eye, look), W, H, f))
    objs = [ObjectSpec(p.instance, p.center.astype(np.float32), float(np.float32(p.yaw)),
                       (p.bound_half() * 1.1).astype(np.float32), 19) for p in prims]
    wl = Workload(f"{n_obj}-object stream, {n_frames} frames at 25 Hz, L16 T2^19, "
                  f"N 128, 64^3 occupancy, {W}x{H}", Scene(prims), cams, objs)
    _render_frames(wl, depth_frac=0.005, seed=seed)
    return wl


def psnr(pred: np.ndarray, gt: np.ndarray, mask: np.ndarray) -> float:
    """PSNR over the channels of the masked pixels."""
    sel = mask.astype(bool)
    if not sel.any():
        return float("nan")
    mse = float(np.mean((pred[sel] - gt[sel]) ** 2))
    return -10.0 * math.log10(max(mse, 1e-12))

"""Throughput benchmark of the per-object radiance-field training step.

Prints one JSON line: trained rays/s (draw, forward, loss, backward, dense
Adam) summed over all objects of the workload, measured on the batched path
(all objects per launch, one hipGraph per step), with the roofline of the
dominant kernel, the plain path (FP32, one launch per object per phase, no
graph) beside it, PSNR of both after training, and the CPU oracle timed on a
bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload objects24|objects24-fp32|torus1|stream128]

The default workload is the 24-object batched BF16 one (the metric's).  HBM
traffic per launch comes from rocprofv3 counter runs of this script, turned
into a committed summary by

    python bench.py --pmc-summary <rocprofv3 output dir> --workload <name>

(`<dir>/fetch` holds a FETCH_SIZE run, `<dir>/write` a WRITE_SIZE run, both
with --copy-probe so that a plain 512 MiB copy calibrates the counters).  The
summary records a hash of the kernel source: once the kernels change, the
traffic is reported as null until the counters are taken again.

Inputs are seeded synthetic scenes (the paper's datasets are not available).
Only one GPU is used; --gpus above 1 exits with a message.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "trained rays/s (fwd+bwd+Adam) all objects, batched BF16 vs plain FP32 @ equal PSNR"
HBM_PEAK_GBS = 8000.0     # MI355X HBM3E
BF16_PEAK_TFLOPS = 2500.0  # dense
FP32_MFMA_PEAK_TFLOPS = 157.3


KERNEL_SRC = os.path.join(ROOT, "paper_2304_05735_amd", "csrc", "romap_kernels.hip")
# kernels of each timed phase (the phase's duration covers all of them)
PHASE_KERNELS = {
    "raygen": ["k_raygen"], "encode_fwd": ["k_encode_fwd"], "pack": ["k_pack"],
    "field": ["k_field"], "reduce": ["k_reduce"], "bin_scatter": ["k_bin_scatter"],
    "bin_acc": ["k_bin_acc"], "bin_finish": ["k_bin_finish"],
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def build_workload(name, frames=300):
    import scenes
    if name == "torus1":
        return scenes.torus_scene()
    if name in ("objects24", "objects24-fp32"):
        return scenes.room_scene(n_obj=24)
    if name == "stream128":
        return scenes.stream_scene(n_frames=frames)
    raise SystemExit(f"unknown workload {name}")


def run_stream(wl, args):
    """Incremental mapping stream: keyframes arrive one by one (25 Hz in the
    scene's timeline); an object is registered on the first frame where its
    mask has >= 200 pixels; objects seen in the last 50 frames are active;
    each frame trains every active object for 4 steps of 2^16 rays in total
    (2^18 rays per frame), split in proportion to the mask pixels seen so far
    (at least 64 each), with
    the BF16 MLP and 128 samples per ray; the occupancy bitfield of an object
    is refreshed every 25 frames once it has trained for 25 frames."""
    import numpy as np
    import paper_2304_05735_amd as pk
    import scenes
    cfg = pk.default_config(samples_per_ray=128, precision=pk.PREC_BF16, batch_mode=pk.BATCH_ALL,
                            use_graph=1, autotune=0, streams=STREAMS)
    ctx = pk.Context(cfg)
    spec = {o.instance: o for o in wl.objects}
    oid_of, first, last_seen, pix, has_kf = {}, {}, {}, {}, {}
    budget, steps_per_frame = 1 << 16, 4
    frame_ms, train_ms, kf_ms, psnr_log = [], [], [], []
    rays_trained = 0
    for f, (cam, rgb, mask, depth) in enumerate(wl.frames):
        ids, counts = np.unique(mask, return_counts=True)
        if f % 50 == 49 and oid_of:  # PSNR on this frame before it is used (novel view)
            vis = sorted(((c, int(i)) for i, c in zip(ids, counts) if int(i) in oid_of), reverse=True)[:6]
            vals = []
            for c, inst in vis:
                pred, _, _ = ctx.render(oid_of[inst], cam)
                vals.append(scenes.psnr(pred, rgb / 255.0, mask == inst))
            psnr_log.append((f, round(float(np.mean(vals)), 3) if vals else None, len(vals)))
        ctx.sync()
        t0 = time.perf_counter()
        for inst, cnt in zip(ids, counts):
            inst = int(inst)
            if inst == 0 or inst not in spec:
                continue
            if inst not in oid_of and cnt >= 200:
                ob = spec[inst]
                oid_of[inst] = ctx.add_object(inst, ob.t, ob.yaw, ob.half, ob.log2T)
                first[inst], pix[inst], has_kf[inst] = f, 0, False
            if inst in oid_of:
                last_seen[inst] = f
                pix[inst] += int(cnt)
                has_kf[inst] = True
        tk = time.perf_counter()
        ctx.add_keyframe(cam, rgb, mask, depth)
        ctx.sync()
        kf_ms.append((time.perf_counter() - tk) * 1e3)
        active = [i for i in oid_of if f - last_seen[i] <= 50 and has_kf[i]]
        if active:
            w = np.array([pix[i] for i in active], np.float64)
            r = np.maximum(64, np.floor(budget * w / w.sum())).astype(np.int32)
            t1 = time.perf_counter()
            ctx.train(steps_per_frame, [oid_of[i] for i in active], r, stats=False)
            rays_trained += int(r.sum()) * steps_per_frame
            for i in active:
                if f - first[i] >= 25 and (f - first[i]) % 25 == 0:
                    ctx.update_occupancy(oid_of[i], 0.05)
            ctx.sync()
            train_ms.append((time.perf_counter() - t1) * 1e3)
        frame_ms.append((time.perf_counter() - t0) * 1e3)
        if f % 25 == 0:
            log(f"frame {f}: {len(oid_of)} objects, {len(active)} active, "
                f"{frame_ms[-1]:.2f} ms")
    fm = np.array(frame_ms)
    tm = np.array(train_ms)
    return dict(frames=len(frame_ms), objects_registered=len(oid_of),
                ms_per_frame_mean=round(float(fm.mean()), 3),
                ms_per_frame_p50=round(float(np.percentile(fm, 50)), 3),
                ms_per_frame_p95=round(float(np.percentile(fm, 95)), 3),
                frames_over_40ms=int((fm > 40.0).sum()),
                keyframe_ms_mean=round(float(np.mean(kf_ms)), 3),
                train_rays_per_s=round(rays_trained / (tm.sum() * 1e-3), 1) if tm.size else None,
                psnr_over_time=psnr_log)


STREAMS = 2  # --streams: 1 for profiler runs (one launch per kernel and phase)


def make_ctx(wl, precision, batch_mode, use_graph, autotune=1, profile=0, **kw):
    import paper_2304_05735_amd as pk
    N = 64
    kw.setdefault("streams", STREAMS)
    cfg = pk.default_config(samples_per_ray=N, precision=precision, batch_mode=batch_mode,
                            use_graph=use_graph, autotune=autotune, profile_phases=profile, **kw)
    ctx = pk.Context(cfg)
    ids = []
    for ob in wl.objects:
        ids.append(ctx.add_object(ob.instance, ob.t, ob.yaw, ob.half, ob.log2T))
    ctx.sync()
    t0 = time.perf_counter()
    for cam, rgb, mask, depth in wl.frames:
        ctx.add_keyframe(cam, rgb, mask, depth)
    ctx.sync()
    ctx.keyframe_seconds = time.perf_counter() - t0  # host buffers -> HBM, all frames
    keep, rays = [], []
    for i, ob in zip(ids, wl.objects):
        if ctx.object_info(i).n_keyframes > 0:
            keep.append(i)
            rays.append(wl.rays[ob.instance])
    return ctx, keep, rays


def timed_steps(ctx, ids, rays, warmup, steps):
    if warmup:
        ctx.train(warmup, ids, rays, stats=False)
    ctx.sync()
    t0 = time.perf_counter()
    ctx.train(steps, ids, rays, stats=False)
    ctx.sync()
    return time.perf_counter() - t0


def mean_psnr(ctx, wl, ids):
    import scenes
    vals = []
    for v in wl.eval_views:
        cam, rgb, mask, _ = wl.frames[v]
        for i, ob in zip(ids, wl.objects):
            m = mask == ob.instance
            if m.sum() < 50:
                continue
            pred, _, _ = ctx.render(i, cam)
            vals.append(scenes.psnr(pred, rgb / 255.0, m))
    return float(sum(vals) / max(len(vals), 1))


def psnr_curve(ctx, wl, ids, rays, steps, chunk):
    """PSNR on the held-out views after every `chunk` training steps."""
    curve = []
    done = 0
    while done < steps:
        n = min(chunk, steps - done)
        ctx.train(n, ids, rays, stats=False)
        done += n
        curve.append((done, mean_psnr(ctx, wl, ids)))
    return curve


def equal_psnr(wl, ids, rays, prec, steps, chunk, ms_batched, ms_plain):
    """Batched path vs the plain FP32 path from the same initialisation, PSNR
    on the held-out views every `chunk` steps.  The common target is the lower
    of the two final PSNRs less 0.1 dB (both curves reach it); each path's
    time to the target is its first evaluated step count at or above it times
    its measured time per step, and the speedup is the ratio of the two."""
    import paper_2304_05735_amd as pk
    qa, _, _ = make_ctx(wl, prec, pk.BATCH_ALL, 1)
    ca = psnr_curve(qa, wl, ids, rays, steps, chunk)
    del qa
    qb, _, _ = make_ctx(wl, pk.PREC_FP32, pk.BATCH_PER_OBJECT, 0)
    cb = psnr_curve(qb, wl, ids, rays, steps, chunk)
    del qb
    pa, pb = ca[-1][1], cb[-1][1]
    target = min(pa, pb) - 0.1
    sa = next(k for k, v in ca if v >= target)
    sb = next(k for k, v in cb if v >= target)
    return dict(steps=steps, psnr_batched=round(pa, 3), psnr_plain_fp32=round(pb, 3),
                target_psnr=round(target, 3), steps_batched_to_target=sa,
                steps_plain_to_target=sb,
                speedup_at_equal_psnr=round((sb * ms_plain) / (sa * ms_batched), 3),
                curve_batched=[(k, round(v, 3)) for k, v in ca],
                curve_plain_fp32=[(k, round(v, 3)) for k, v in cb])


def mesh_timing(ctx, ids, res=64, iso=10.0, reps=3):
    """Marching cubes of every object at res^3 (Sec. VI: 64^3 per object):
    density on the box corners, mesh, world placement, triangles copied to
    the host; wall time per object (best of reps, after one untimed call)."""
    import numpy as np
    per, ntri = [], []
    for i in ids:
        ctx.extract_mesh(i, res, iso)
        best = 1e9
        for _ in range(reps):
            t0 = time.perf_counter()
            tri = ctx.extract_mesh(i, res, iso)
            best = min(best, time.perf_counter() - t0)
        per.append(best * 1e3)
        ntri.append(len(tri))
    return dict(res=res, iso=iso, objects=len(ids), ms_per_object_mean=round(float(np.mean(per)), 4),
                ms_per_object_max=round(float(np.max(per)), 4),
                triangles_mean=int(np.mean(ntri)),
                paper_ms_per_object_rtx4090=2.84)


def table_sweep(wl, steps=200, warmup=20):
    """Table 4's model-size study on one object: time per step (graph, FP32
    and BF16) of 4096 rays x 32 samples (the paper's N) and of 4096 x 64, for
    T = 2^14 .. 2^20 with the one-hidden-layer density MLP, and for T = 2^16
    with density MLPs of 2 and 3 hidden layers, on the single-object scene."""
    import paper_2304_05735_amd as pk
    ob = wl.objects[0]
    rows = []
    models = [(lt, 1) for lt in (14, 16, 18, 20)] + [(16, 2), (16, 3)]
    for N in (32, 64):
        for prec in (pk.PREC_FP32, pk.PREC_BF16):
            for lt, layers in models:
                cfg = pk.default_config(samples_per_ray=N, precision=prec, use_graph=1, autotune=1,
                                        mlp_layers=layers)
                ctx = pk.Context(cfg)
                i = ctx.add_object(ob.instance, ob.t, ob.yaw, ob.half, lt)
                for cam, rgb, mask, depth in wl.frames:
                    ctx.add_keyframe(cam, rgb, mask, depth)
                dt = timed_steps(ctx, [i], [4096], warmup, steps)
                rows.append(dict(N=N, precision="bf16" if prec else "fp32", log2T=lt,
                                 mlp_layers=layers, ms_per_step=round(dt / steps * 1e3, 4)))
                log("table sweep", rows[-1])
                del ctx
    return dict(rows=rows, paper_rtx4090_ms={"2^14": 0.658, "2^16": 0.706, "2^18": 0.921,
                                              "2^20": 1.495, "2^16, 2 layers": 0.862,
                                              "2^16, 3 layers": 1.052})


def density_ablation(wl, ids, rays, prec, steps):
    """The loss ablation of the paper's Fig. 8 on this workload: training with
    and without the density term of the background rays (lambda_2 = 0.01 vs
    0).  Reported per setting: PSNR on the objects' pixels of the held-out
    views, and the mean rendered opacity over the pixels of those views that
    do not belong to the rendered object (mass floating in its box's empty
    space, which the term is meant to remove)."""
    import numpy as np
    import paper_2304_05735_amd as pk
    import scenes
    out = {}
    for lam in (0.01, 0.0):
        ctx, _, _ = make_ctx(wl, prec, pk.BATCH_ALL, 1, lambda_density=lam)
        ctx.train(steps, ids, rays, stats=False)
        ps, fl = [], []
        for v in wl.eval_views:
            cam, rgb, mask, _ = wl.frames[v]
            for i, ob in zip(ids, wl.objects):
                m = mask == ob.instance
                if m.sum() < 50:
                    continue
                pred, _, opac = ctx.render(i, cam)
                ps.append(scenes.psnr(pred, rgb / 255.0, m))
                fl.append(float(np.mean(opac[~m])))
        out[f"lambda2={lam}"] = {"psnr": round(float(np.mean(ps)), 3),
                                 "empty_space_opacity": float(np.mean(fl))}
        del ctx
    out["steps"] = steps
    return out


def algorithmic_bytes(ctx, ids, rays, phase):
    """Algorithmic bytes of one step of a kernel (all its launches).  The
    binning kernels' records are the counted ones (fewer than 8 per sample
    and level where runs of samples in one cell are merged)."""
    L, N = ctx.cfg.n_levels, ctx.cfg.samples_per_ray
    S = sum(rays) * N
    grid = sum(ctx.object_info(i).n_grid_params for i in ids)
    rec = ctx.step_records()
    if phase == "encode_fwd":   # 8 corners x 8 B gathered + 8 B written, per sample and level
        return S * L * (64 + 8)
    if phase == "bin_scatter":  # 8 B adjoint read per sample and level + 10 B per record written
        return S * L * 8 + 10 * rec
    if phase == "bin_acc":      # 10 B per record read; Adam on the table: p, m, v read and written
        return 10 * rec + 24 * grid
    if phase == "field":        # encodings read twice (forward, recompute), adjoints written
        return S * L * 8 * 3
    return 0


def field_flops(ctx, rays):
    """MLP flops of the field kernel: forward 2*4224, recompute 2*4224,
    adjoint 2*2*4224 (input and weight gradients) per sample."""
    S = sum(rays) * ctx.cfg.samples_per_ray
    return S * 4224 * 2 * 4


def kernel_src_hash():
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.txt")


def _kernel_key(name):
    """'void k_field<0, 64, 32>(StepArgs)' -> 'k_field'"""
    n = name.replace("void ", "").strip()
    for sep in ("<", "("):
        n = n.split(sep)[0]
    return n.strip()


def pmc_summary(d, workload, steps):
    """Writes the per-launch HBM traffic of each kernel from a FETCH_SIZE and a
    WRITE_SIZE rocprofv3 run (KiB per dispatch), each counter scaled by what it
    reads for the 512 MiB copies of --copy-probe."""
    import csv
    import statistics
    per = {}
    factor = {}
    for cname, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        rows = list(csv.DictReader(open(os.path.join(d, sub, "run_counter_collection.csv"))))
        copies = [float(r["Counter_Value"]) for r in rows
                  if r["Counter_Name"] == cname and "copyBuffer" in r["Kernel_Name"]
                  and float(r["Counter_Value"]) > 100000]
        if not copies:
            raise SystemExit(f"no 512 MiB copy dispatch in {sub}: run with --copy-probe")
        factor[cname] = 524288.0 / statistics.median(copies)
        for r in rows:
            if r["Counter_Name"] != cname or not r["Kernel_Name"].lstrip("void ").startswith("k_"):
                continue
            k = _kernel_key(r["Kernel_Name"])
            per.setdefault(k, {}).setdefault(cname, []).append(float(r["Counter_Value"]))
    out = [f"# HBM traffic per dispatch, workload {workload}",
           f"# rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) -d <dir>/fetch (write) -o run -f csv "
           f"-- python3 bench.py --steps {steps} --warmup 5 --only-headline --copy-probe "
           f"--streams 1 --workload {workload}",
           f"# then: python bench.py --pmc-summary <dir> --workload {workload}",
           f"# calibration (512 MiB copy): FETCH_SIZE x {factor['FETCH_SIZE']:.4f}, "
           f"WRITE_SIZE x {factor['WRITE_SIZE']:.4f}",
           f"kernel_source_sha256_16 {kernel_src_hash()}",
           "# kernel dispatches fetch_KiB_raw write_KiB_raw hbm_bytes_calibrated"]
    for k in sorted(per):
        f = per[k].get("FETCH_SIZE", [0.0])
        w = per[k].get("WRITE_SIZE", [0.0])
        fm, wm = sum(f) / len(f), sum(w) / len(w)
        byt = (fm * factor["FETCH_SIZE"] + wm * factor["WRITE_SIZE"]) * 1024.0
        out.append(f"{k} {len(f)} {fm:.1f} {wm:.1f} {byt:.0f}")
    path = traffic_file(workload)
    with open(path, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print("\n".join(out))
    log("wrote", path)


def copy_bandwidth(nbytes=1 << 30, reps=10):
    """Device-to-device copy rate (GB/s, bytes read + written) of a plain
    tensor copy: the achievable HBM bandwidth the roofline is also quoted
    against (besides the datasheet peak)."""
    import torch
    src = torch.ones(nbytes // 4, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def traffic_of(workload, kernels):
    """Calibrated HBM bytes per step of the given kernels from the committed
    counter summary, or None if it is missing or the kernels changed since."""
    path = traffic_file(workload)
    if not os.path.exists(path):
        return None
    tab, src = {}, None
    for line in open(path):
        if line.startswith("kernel_source_sha256_16"):
            src = line.split()[1]
        elif line.strip() and not line.startswith("#"):
            k, _, _, _, b = line.split()
            tab[k] = float(b)
    if src != kernel_src_hash():
        return None
    return sum(tab.get(k, 0.0) for k in kernels)


def cpu_baseline(wl, seconds_target=15.0):
    """The oracle as it stands on the host cores, on a bounded sample: as many
    full 4096-ray steps of the first object as fit in ~seconds_target."""
    import oracle
    ob = wl.objects[0]
    cfg = oracle.make_config(N=64, log2T=ob.log2T)
    o = oracle.OracleContext(cfg)
    oid = o.add_object(ob.instance, ob.t, ob.yaw, ob.half, ob.log2T)
    for cam, rgb, mask, depth in wl.frames:
        o.add_keyframe(cam, rgb, mask, depth)
    B = wl.rays[ob.instance]
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < seconds_target and steps < 50:
        o.train(oid, 1, B)
        steps += 1
    dt = time.perf_counter() - t0
    return dict(value=steps * B / dt, unit="rays/s", cores=o.nthreads, kind="oracle",
                sample=f"{steps} full training steps x {B} rays x 64 samples of object "
                       f"instance {ob.instance} (FP64, {o.nthreads} threads)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="objects24",
                    choices=("objects24", "objects24-fp32", "torus1", "stream128"))
    ap.add_argument("--psnr-steps", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-psnr", action="store_true")
    ap.add_argument("--table-sweep", action="store_true",
                    help="time one object for T = 2^14..2^20 and for 2- and 3-layer density MLPs "
                         "(the paper's Table 4 study) and exit")
    ap.add_argument("--ablation-density", action="store_true",
                    help="also train with lambda_2 = 0 and report PSNR and empty-space opacity")
    ap.add_argument("--psnr-chunk", type=int, default=250)
    ap.add_argument("--only-headline", action="store_true",
                    help="time the batched path only (for profiler runs)")
    ap.add_argument("--frames", type=int, default=300, help="frames of the stream128 workload")
    ap.add_argument("--streams", type=int, default=2, choices=(1, 2),
                    help="streams of a batched step (1 for profiler runs: kernel traces and "
                         "counters then describe one launch per kernel and phase)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 512 MiB three times (calibrates the HBM byte counters)")
    ap.add_argument("--pmc-summary", metavar="DIR",
                    help="write the HBM traffic summary from rocprofv3 counter runs and exit")
    args = ap.parse_args()
    global STREAMS
    STREAMS = args.streams
    if args.pmc_summary:
        pmc_summary(args.pmc_summary, args.workload, args.steps)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the path is the "
              "single-GPU share of the workload; sharding across GPUs is not built.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2304_05735_amd as pk
    # the scene renders in forked worker processes: build it before this
    # process opens the GPU (afterwards it would render serially)
    log("workload", "torus1 (table sweep)" if args.table_sweep else args.workload)
    t = time.perf_counter()
    wl = build_workload("torus1" if args.table_sweep else args.workload, args.frames)
    log(f"scene ready in {time.perf_counter() - t:.1f}s: {len(wl.objects)} objects, "
        f"{len(wl.frames)} frames")
    assert torch.cuda.is_available(), "no GPU visible"
    if args.copy_probe:
        src = torch.ones(128 << 20, device="cuda")  # 512 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 3 x 512 MiB copied")
        del src, dst
    if args.table_sweep:
        print(json.dumps({"table_sweep": table_sweep(wl)}), flush=True)
        return
    if args.workload == "stream128":
        st = run_stream(wl, args)
        log("stream", json.dumps(st))
        out = {"metric": METRIC, "value": st["train_rays_per_s"], "unit": "rays/s", "n_gpus": 1,
               "steps": None, "warmup": 0, "ms_per_step": None, "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "bf16-mfma/fp32",
               "data": "synthetic", "config": {"workload": wl.name}, "stream": st}
        print(json.dumps(out), flush=True)
        return
    prec = pk.PREC_BF16 if args.workload == "objects24" else pk.PREC_FP32
    # ---- headline: batched path, one hipGraph per step
    ctx, ids, rays = make_ctx(wl, prec, pk.BATCH_ALL, 1)
    rays_per_step = sum(rays)
    # RGB8, int32 mask, float depth where given
    kf_bytes = sum(rgb.shape[0] * rgb.shape[1] * (3 + 4 + (4 if depth is not None else 0))
                   for _, rgb, _, depth in wl.frames)
    keyframes = {"frames": len(wl.frames), "ms": round(ctx.keyframe_seconds * 1e3, 3),
                 "MB": round(kf_bytes / 1e6, 1),
                 "GB_per_s": round(kf_bytes / ctx.keyframe_seconds / 1e9, 2)}
    log("keyframes", json.dumps(keyframes))
    log(f"{len(ids)} trained objects, {rays_per_step} rays/step")
    dt = timed_steps(ctx, ids, rays, args.warmup, args.steps)
    value = rays_per_step * args.steps / dt
    ms_step = dt / args.steps * 1e3
    log(f"batched: {ms_step:.4f} ms/step, {value / 1e6:.3f} M rays/s")
    mesh = None
    if not args.only_headline:
        mesh = mesh_timing(ctx, ids)
        log("mesh", json.dumps(mesh))
    if args.only_headline:
        print(json.dumps({"value": value, "ms_per_step": ms_step}), flush=True)
        return
    # ---- per-kernel durations (HIP events on the context stream, same kernels)
    pctx, _, _ = make_ctx(wl, prec, pk.BATCH_ALL, 0, profile=1)
    pctx.train(args.warmup, ids, rays, stats=False)
    pctx.train(args.steps, ids, rays, stats=False)
    phases, nph = pctx.phase_times()
    log("phase ms:", json.dumps({k: round(v, 5) for k, v in phases.items()}))
    dominant = max(phases, key=phases.get)
    byt = algorithmic_bytes(pctx, ids, rays, dominant)
    achieved = byt / (phases[dominant] * 1e-3) / 1e9 if phases[dominant] > 0 else 0.0
    traffic = traffic_of(args.workload, PHASE_KERNELS[dominant])
    copy_gbs = copy_bandwidth()
    log(f"copy bandwidth {copy_gbs:.0f} GB/s")
    roofline = dict(bound="hbm", kernel=dominant, kernels=PHASE_KERNELS[dominant],
                    achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
                    copy_gbs=round(copy_gbs, 1), frac_of_copy=round(achieved / copy_gbs, 4),
                    traffic=None if traffic is None else int(traffic),
                    avg_ms=round(phases[dominant], 5), algorithmic_bytes=int(byt),
                    phase_ms={k: round(v, 5) for k, v in phases.items()})
    fl = field_flops(pctx, rays)
    peak_f = BF16_PEAK_TFLOPS if prec == pk.PREC_BF16 else FP32_MFMA_PEAK_TFLOPS
    mlp = dict(kernel="field", tflops=round(fl / (phases["field"] * 1e-3) / 1e12, 2),
               peak=peak_f, frac=round(fl / (phases["field"] * 1e-3) / 1e12 / peak_f, 4))
    del pctx
    # ---- plain path: FP32, one launch per object per phase, no graph
    plain_ctx, _, _ = make_ctx(wl, pk.PREC_FP32, pk.BATCH_PER_OBJECT, 0)
    dtp = timed_steps(plain_ctx, ids, rays, args.warmup, args.steps)
    plain = rays_per_step * args.steps / dtp
    log(f"plain FP32 per-object: {dtp / args.steps * 1e3:.4f} ms/step, {plain / 1e6:.3f} M rays/s")
    del plain_ctx
    quality = None
    if not args.no_psnr:
        quality = equal_psnr(wl, ids, rays, prec, args.psnr_steps, args.psnr_chunk, ms_step,
                             dtp / args.steps * 1e3)
        log("psnr", json.dumps(quality))
    ablation = None
    if args.ablation_density:
        ablation = density_ablation(wl, ids, rays, prec, args.psnr_steps)
        log("ablation", json.dumps(ablation))
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(wl)
        log("cpu", cpu)
    dtype = "bf16-mfma/fp32" if prec == pk.PREC_BF16 else "fp32"
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": wl.name, "objects": len(ids), "rays_per_step": rays_per_step,
                   "samples_per_ray": 64, "levels": 16, "batched": True, "graph": True},
        "roofline": roofline,
        "mlp_mfma": mlp,
        "plain_fp32": {"value": round(plain, 1), "unit": "rays/s",
                       "speedup": round(value / plain, 3)},
        "quality": quality,
        "ablation_density": ablation,
        "mesh": mesh,
        "cpu_baseline": cpu,
        "keyframe_upload": keyframes,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

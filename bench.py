"""Benchmark: one training step of the layered-mesh renderer on one MI355X.

Step = rasterise every layer in every view from scratch (visibility), shade
and blend the image (forward), and the texture adjoint of the RGB L2 loss
against a seeded target (backward, fused loss gradient), including zeroing
the texture gradients.  Workload: the k = 7 displaced-shell scene (101,760
triangles per layer, 1024^2 RGBA f32 textures) seen from 64 ring views at
1024 x 1024.  Inputs are seeded synthetic data already resident in HBM.

Prints one JSON line.  Metric: shaded pixel-layers per second, where the
number of shaded pixel-layers is the number of covered visibility slots
(implementation independent: visibility is bit-exact).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "shaded px·layers/s fwd+bwd (k=7, 1024², 64 views); % HBM peak"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def byte_model(scene, n_views, P_v, U, fused=True):
    """Algorithmic bytes per launch of each phase (byte model)."""
    k = scene.k
    P = n_views * P_v
    G = sum(12 * m.n_vert + 8 * m.n_vert + 12 * m.n_tri for m in scene.layers)
    tex_bytes = sum(16 * int(u) for u in U)
    grad_planes = sum(16 * t.shape[0] * t.shape[1] for t in scene.textures)
    return {
        "raster": 8 * k * P + G * n_views,                     # one key store per slot + geometry per view
        "shade_fwd": 0 if fused else 8 * k * P + 16 * P + tex_bytes + G,
        # keys, target, image (fused), texels, gradient read-modify-write, geometry
        "shade_bwd": 8 * k * P + 16 * P + (16 * P if fused else 0) + tex_bytes + 2 * grad_planes + G,
        "grad_zero": grad_planes,
    }


def counter_traffic(kernel: str):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter summary, if its sources match."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel)
    except Exception:
        return None
    if not rec:
        return None
    h = hashlib.sha256()
    for f in sorted(os.listdir(os.path.join(ROOT, "paper_2409_02482_amd", "csrc"))):
        h.update(open(os.path.join(ROOT, "paper_2409_02482_amd", "csrc", f), "rb").read())
    if rec.get("csrc_sha256") != h.hexdigest():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(scene, n_threads, per_thread=3):
    """The oracle as it stands, views spread over threads (ctypes releases the GIL)."""
    import concurrent.futures as cf

    import oracle as O
    cams = scene.cameras[:n_threads * per_thread]

    def one(v):
        cam = scene.cameras[v]
        vis = O.raster_layers(scene.layers, cam)
        O.shade(scene.layers, scene.textures, cam, vis)
        O.backward(scene.layers, scene.textures, cam, vis, target=scene.targets[v])
        return int((vis != np.uint64(0xFFFFFFFFFFFFFFFF)).sum())

    O.build(force=False)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(n_threads) as ex:
        covered = sum(ex.map(one, range(len(cams))))
    dt = time.perf_counter() - t0
    return {"value": covered / dt, "unit": "px*layers/s", "cores": n_threads, "kind": "oracle",
            "sample": f"{len(cams)} of the 64 views (full 1024x1024, k=7), raster+shade+adjoint (L2), "
                      f"{per_thread} views per thread on {n_threads} threads, {dt:.1f} s wall"}


SH_METRIC = ("shaded px·layers/s fwd, baked SH degree 3 (k=7, 1024², 64 views, 8-bit 2048² mixed-resolution "
             "textures); % HBM peak")


def sh_cpu_baseline(scene, sh, n_threads, per_thread=2):
    """The oracle's baked-SH forward (raster + shade) on a bounded sample of views, one per thread."""
    import concurrent.futures as cf

    import oracle as O
    cams = scene.cameras[:n_threads * per_thread]

    def one(v):
        cam = scene.cameras[v]
        vis = O.raster_layers(scene.layers, cam)
        O.shade_sh(scene.layers, sh, cam, vis)
        return int((vis != np.uint64(0xFFFFFFFFFFFFFFFF)).sum())

    O.build(force=False)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(n_threads) as ex:
        covered = sum(ex.map(one, range(len(cams))))
    dt = time.perf_counter() - t0
    return {"value": covered / dt, "unit": "px*layers/s", "cores": n_threads, "kind": "oracle",
            "sample": f"{len(cams)} of the {len(scene.cameras)} views (full size, k={scene.k}), raster + baked SH "
                      f"shading, {per_thread} view(s) per thread on {n_threads} threads, {dt:.1f} s wall"}


def calibration_copy(mib):
    """One plain device-to-device copy of mib MiB (reads and writes mib MiB): the HBM counter reference."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"[bench] calibration copy of {mib} MiB done")
    del a, b


def run_sh(args):
    """Forward rendering of the baked representation: raster + vs_render_sh per step."""
    import torch

    import paper_2409_02482_amd as P
    import scenes as S
    log("[bench] building scene (baked SH textures)")
    scene = S.make_config(6, n_views=args.views, resolution=(args.res, args.res), with_targets=False)
    k, nv, dev = scene.k, len(scene.cameras), "cuda"
    sh = [S.sh_texture(60, l, 2048, 2048, degree=3, opaque=(l == k - 1)) for l in range(k)]
    layers = P.Layers(scene.layers, dev)
    views = P.Views(scene.cameras, dev)
    sh_dev = [(torch.from_numpy(t.data).to(dev), t.width, t.height) for t in sh]
    out = torch.empty(views.total_pixels, 4, dtype=torch.float32, device=dev)
    vis = torch.empty(k * views.total_pixels, dtype=torch.int64, device=dev)
    ws = P.alloc_workspace(layers, views, args.bin, dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        P.raster(layers, views, vis, ws, bin=args.bin)
        if ev is not None:
            ev[1].record(stream)
        P.render_sh(layers, sh_dev, views, vis, ws, degree=3, out=out)
        if ev is not None:
            ev[2].record(stream)

    log("[bench] warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    covered = int((vis != -1).sum().item())
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for st in range(args.steps):
        step(evs[st])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phase = np.array([[evs[st][i].elapsed_time(evs[st][i + 1]) for i in range(2)] for st in range(args.steps)])
    ms_phase = phase.mean(0)
    ms_wall = wall / args.steps * 1e3
    P_v = views.total_pixels / nv
    G = sum(12 * m.n_vert + 8 * m.n_vert + 12 * m.n_tri for m in scene.layers)
    tex_bytes = sum(int(t.data.nbytes) for t in sh)
    bm = {"raster": 8 * k * views.total_pixels + G * nv,
          # keys, image, every coefficient byte once (all texels are seen by the 64 ring views), geometry
          "shade_sh": 8 * k * views.total_pixels + 16 * views.total_pixels + tex_bytes + G}
    names = ["raster", "shade_sh"]
    dom = int(np.argmax(ms_phase))
    achieved = bm[names[dom]] / (ms_phase[dom] * 1e-3) / 1e9
    res = {
        "metric": SH_METRIC, "value": covered / (ms_wall * 1e-3), "unit": "px*layers/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_wall, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"k={k} displaced shells ({scene.layers[0].n_tri:,} tris/layer), {nv} ring views at "
                               f"{args.res}x{args.res}, SH degree 3 in 8 bits, levels 2048^2..256^2, raster + "
                               "baked SH shading", "views": nv, "k": k, "pixels": views.total_pixels,
                   "covered_px_layers": covered, "bin": args.bin, "sh_texture_bytes": tex_bytes},
        "phases_ms": {n: float(m) for n, m in zip(names, ms_phase)},
        "roofline": {"bound": "hbm", "kernel": names[dom], "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(names[dom])},
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        n = max(1, min(args.cpu_threads, os.cpu_count() or 1, nv))
        res["cpu_baseline"] = sh_cpu_baseline(scene, sh, n)
    print(json.dumps(res), flush=True)


KSDF_METRIC = "rays/s, k-SDF volume rendering fwd (k=7, 64+32 samples/ray, 256^3 fields, 8 views at 512^2)"
FP_PEAK_TFLOPS = 78.6    # fp64 FMA (and unpacked fp32 FMA): 256 CUs x 64 lanes x 2 flops x 2.4 GHz


def ksdf_flops_per_ray(k, n, m, steps):
    """Algorithmic floating-point operations of one ray with samples (counted from the method's steps).

    march: per step the midpoint (2) and three voxel coordinates (4 each);
    SDF lookup: three cell coordinates (2 each) and 8 corners (weight 2 + accumulate 2);
    RGBA lookup: cell coordinates (6) and 8 corners (weight 2 + 4 channels x 2);
    SDF gradient: cell coordinates (6), per axis 4 grid lines (difference, two weight products,
    accumulate) and a scale (3);
    interval weight per sample and surface: argument (2), logistic CDF (3), a_i (3), T_i and w_i (2);
    per interval of the final samples: position (6), normal (gradient, normalise 9, dot 5),
    alpha_w (4), per surface accumulation of C and A (10).
    """
    N = n + m
    sdf, rgba, grad = 6 + 8 * 4, 6 + 8 * 10, 6 + 3 * 4 * 4 + 3
    flops = steps * 14
    flops += N * (6 + sdf)                                   # sample positions and their SDF
    flops += (n + (n + m // 2) + N) * k * 10                 # weights of both importance rounds and the final pass
    flops += (N - 1) * (6 + rgba + grad + 9 + 5 + 4 + 10 * k)
    return flops


def ksdf_cpu_baseline(grids, oopts, occ_np, cams, n_rays):
    """The oracle on a bounded random sample of the workload's rays (single process, NumPy)."""
    import threadpoolctl

    from oracle import ksdf as K
    rng = np.random.default_rng(70)
    per = n_rays // len(cams)
    with threadpoolctl.threadpool_limits(1):
        t0 = time.perf_counter()
        for cam in cams:
            o, d = K.camera_rays(cam)
            pick = rng.choice(o.shape[0], per, replace=False)
            K.render_rays(grids, oopts, occ_np, o[pick], d[pick])
        dt = time.perf_counter() - t0
    return {"value": per * len(cams) / dt, "unit": "rays/s", "cores": 1, "kind": "oracle",
            "sample": f"{per * len(cams)} random rays ({per} per view) of the {len(cams)} views, occupancy grid "
                      f"given, one NumPy thread, {dt:.1f} s wall"}


def run_ksdf(args):
    """k-SDF volume-rendering forward: occupancy grid + vs_ksdf_render per step."""
    import math

    import torch

    import paper_2409_02482_amd as P
    import scenes as S
    log("[bench] building k-SDF fields")
    k, n, m, steps, res = 7, 64, 32, 1024, 512
    beta = math.exp(7.0)
    grids = S.ksdf_grids(5, 256, 128)
    cams = S.ring_cameras(5, 8, [(res, res)] * 8)
    dev = "cuda"
    field = P.KsdfField(torch.from_numpy(grids.sdf).to(dev), grids.sdf_res,
                        torch.from_numpy(grids.rgba.reshape(-1, 4)).to(dev), grids.rgba_res, grids.lo, grids.hi)
    offs = S.ksdf_offsets(k, beta)
    opts = P.ksdf_opts(offs, beta, occ_res=256, n_uniform=n, n_importance=m, march_steps=steps)
    views = P.Views(cams, dev)
    occ = P.ksdf_occupancy(field, opts)
    out = torch.empty(views.total_pixels, 4, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        P.ksdf_occupancy(field, opts, occ)
        if ev is not None:
            ev[1].record(stream)
        P.ksdf_render(field, opts, occ, views, out=out)
        if ev is not None:
            ev[2].record(stream)

    log("[bench] warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    _, _, smp = P.ksdf_render(field, opts, occ, views, samples=True)
    sampled = int((smp[:, 0] >= 0).sum().item())
    del smp
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for st in range(args.steps):
        step(evs[st])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    phase = np.array([[evs[st][i].elapsed_time(evs[st][i + 1]) for i in range(2)] for st in range(args.steps)])
    ms_phase = phase.mean(0)
    ms_wall = wall / args.steps * 1e3
    rays = views.total_pixels
    fl = ksdf_flops_per_ray(k, n, m, steps) * sampled
    achieved = fl / (ms_phase[1] * 1e-3) / 1e12
    res_ = {
        "metric": KSDF_METRIC, "value": rays / (ms_wall * 1e-3), "unit": "rays/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_wall, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": f"k-SDF (k={k} shells of the displaced sphere, offsets pi/(sqrt(3) beta), beta=e^7), "
                               f"SDF grid 256^3, RGBA grid 128^3, occupancy 256^3, {n} uniform + {m} importance "
                               f"samples, {steps} march steps, 8 ring views at {res}x{res}; occupancy + render",
                   "views": len(cams), "k": k, "rays": rays, "rays_with_samples": sampled,
                   "samples_per_ray": n + m},
        "phases_ms": {"occupancy": float(ms_phase[0]), "render": float(ms_phase[1])},
        "samples_per_s": sampled * (n + m) / (ms_wall * 1e-3),
        "roofline": {"bound": "alu", "kernel": "ksdf_render", "achieved": achieved, "peak": FP_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP_PEAK_TFLOPS, "traffic": counter_traffic("ksdf_render"),
                     "flops_per_ray": ksdf_flops_per_ray(k, n, m, steps)},
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        from oracle import ksdf as K
        oopts = K.KsdfOpts(offsets=offs, beta=beta, occ_res=256, n_uniform=n, n_importance=m, march_steps=steps)
        occ_np = K.occupancy(grids, oopts)
        res_["cpu_baseline"] = ksdf_cpu_baseline(grids, oopts, occ_np, cams, 48000)
    print(json.dumps(res_), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--views", type=int, default=64)
    ap.add_argument("--res", type=int, default=1024)
    ap.add_argument("--bin", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=8)
    ap.add_argument("--unfused", action="store_true", help="separate forward shading pass before the adjoint")
    ap.add_argument("--workload", default="metric", choices=["metric", "cfg4", "sh", "ksdf"],
                    help="metric: k=7, 64 views at 1024^2; cfg4: k=9, 299,208 tris/layer, 64 mixed-size views; "
                         "sh: the metric scene rendered forward with baked 8-bit SH textures (degree 3, 2048^2 base); "
                         "ksdf: k-SDF volume rendering of the implicit stage (8 views at 512^2)")
    ap.add_argument("--graph", action="store_true", help="replay the step from a captured HIP graph")
    ap.add_argument("--autotune", action="store_true", help="pick the raster bin size with vs_autotune")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="run one plain device copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only; --gpus must be 1 (views would shard across GPUs, "
              "with one all-reduce of the texture gradients per step)", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        calibration_copy(args.calibrate_copy)
    if args.workload == "sh":
        return run_sh(args)
    if args.workload == "ksdf":
        return run_ksdf(args)

    import torch

    import paper_2409_02482_amd as P
    import scenes as S

    log("[bench] building scene")
    if args.workload == "cfg4":
        scene = S.make_config(4, n_views=args.views)
    else:
        scene = S.make_config(6, n_views=args.views, resolution=(args.res, args.res))
    k = scene.k
    nv = len(scene.cameras)
    dev = "cuda"
    layers = P.Layers(scene.layers, dev)
    views = P.Views(scene.cameras, dev)
    tex = [torch.from_numpy(t).to(dev) for t in scene.textures]
    target = torch.from_numpy(np.concatenate([t.reshape(-1, 4) for t in scene.targets])).to(dev)
    grads = [torch.zeros_like(t) for t in tex]
    out = torch.empty(views.total_pixels, 4, dtype=torch.float32, device=dev)
    vis = torch.empty(k * views.total_pixels, dtype=torch.int64, device=dev)
    ws = P.alloc_workspace(layers, views, 8 if args.autotune else args.bin, dev)
    if args.autotune:
        args.bin = P.autotune(layers, views, vis, ws)
        log(f"[bench] autotuned bin size {args.bin}")
    loss_scale = 1.0 / (views.total_pixels * 3)
    stream = torch.cuda.current_stream()

    sse = torch.zeros(1, dtype=torch.float64, device=dev)

    def step(ev=None):
        # fused (default): the adjoint kernel recomputes the blend, writes the image and the SSE, and
        # scatters the texture gradient; unfused: a separate forward shading pass writes the image.
        if ev is not None:
            ev[0].record(stream)
        P.raster(layers, views, vis, ws, bin=args.bin)
        if ev is not None:
            ev[1].record(stream)
        if args.unfused:
            P.render(layers, tex, views, vis, ws, out=out)
        if ev is not None:
            ev[2].record(stream)
        for g in grads:
            g.zero_()
        sse.zero_()
        if ev is not None:
            ev[3].record(stream)
        P.render_backward(layers, tex, views, vis, ws, grad_tex=grads, target=target, loss_scale=loss_scale,
                          out=None if args.unfused else out, sse=sse)
        if ev is not None:
            ev[4].record(stream)

    log("[bench] warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    graph = None
    if args.graph:
        # the whole step (raster, gradient reset, fused shade + adjoint) as one graph on torch's stream
        side = torch.cuda.Stream()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            step()
        torch.cuda.synchronize()
    st = P.read_status(ws)
    covered = int((vis != -1).sum().item())
    # distinct texels read per layer (for the byte model): the texels that received a gradient
    U = [int((g != 0).any(dim=-1).sum().item()) for g in grads]
    log(f"[bench] covered slots {covered} status {st}")

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    if graph is not None:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(args.steps):
            graph.replay()
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        # phase split from one eager step (graph replays are timed as a whole)
        step(evs[0])
        torch.cuda.synchronize()
        phase = np.array([[evs[0][i].elapsed_time(evs[0][i + 1]) for i in range(4)]])
        graph_ms = e0.elapsed_time(e1) / args.steps
    else:
        t0 = time.perf_counter()
        for s in range(args.steps):
            step(evs[s])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        phase = np.array([[evs[s][i].elapsed_time(evs[s][i + 1]) for i in range(4)] for s in range(args.steps)])
    ms_phase = phase.mean(0)
    ms_step = float(phase.sum(1).mean())
    ms_wall = wall / args.steps * 1e3
    P_v = views.total_pixels / nv
    bm = byte_model(scene, nv, P_v, U, fused=not args.unfused)
    names = ["raster", "shade_fwd", "grad_zero", "shade_bwd"]
    dom = int(np.argmax(ms_phase))
    dom_name = names[dom]
    achieved = bm[dom_name] / (ms_phase[dom] * 1e-3) / 1e9
    value = covered / (ms_wall * 1e-3)
    tri_total = sum(m.n_tri for m in scene.layers) * nv
    res = {
        "metric": METRIC,
        "value": value,
        "unit": "px*layers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"k={k} displaced shells ({scene.layers[0].n_tri:,} tris/layer), {nv} ring views "
                                + (f"at {args.res}x{args.res}" if args.workload == "metric" else
                                   "of mixed size 512^2..1920x1080")
                                + ", 1024^2 f32 RGBA textures, raster+shade+adjoint (L2)"),
                   "views": nv, "k": k, "pixels": views.total_pixels, "covered_px_layers": covered,
                   "bin": args.bin, "fused_fwd_bwd": not args.unfused, "graph": bool(args.graph)},
        "phases_ms": {n: float(m) for n, m in zip(names, ms_phase)},
        "triangles_per_s": tri_total / (ms_phase[0] * 1e-3),
        "alg_bytes_per_step": int(sum(bm[n] for n in names)),
        "alg_frac_of_peak_step": sum(bm[n] for n in names) / (ms_wall * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(dom_name)},
    }
    if graph is not None:
        res["graph_ms_per_step"] = graph_ms
    if not args.no_cpu_baseline and args.workload == "metric":
        log("[bench] cpu baseline (oracle)")
        n = max(1, min(args.cpu_threads, os.cpu_count() or 1, nv))
        res["cpu_baseline"] = cpu_baseline(scene, n)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

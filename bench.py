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
CFG4_METRIC = ("shaded px·layers/s fwd+bwd (k=9, 299,208 tris/layer, 64 views of mixed size 512²..1920x1080); "
               "% HBM peak")
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def byte_model(scene, n_views, P_v, U, fused=True):
    """Algorithmic bytes per launch of each phase: keys, images, targets, touched texels, gradient planes, mesh."""
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


def csrc_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2409_02482_amd", "csrc")
    for f in sorted(os.listdir(d)):
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def profile_record(name: str, workload: str, kernel: str):
    """Record ``<workload>/<kernel>`` of the committed summary profiles/<name>, if the kernel sources are still
    the ones the counters were taken on (else None)."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{workload}/{kernel}")
    except Exception:
        return None
    if not rec or rec.get("csrc_sha256") != csrc_sha256():
        return None
    return rec


def counter_traffic(workload: str, kernel: str):
    """HBM bytes per launch of a kernel in a workload from the committed rocprofv3 counter summaries, if the
    kernel sources are still the ones the counters were taken on."""
    rec = profile_record("traffic.json", workload, kernel)
    return None if rec is None else rec.get("bytes_per_launch")


def issue_rate(workload: str, kernel: str):
    """VALU issue share of a kernel from the committed SQ counter summary (same source rule as the traffic):
    SQ_INSTS_VALU x 4 cycles / (kernel duration x 2.4 GHz x 1024 SIMDs), the share of the chip's VALU issue
    cycles the kernel's instructions occupy at the nominal clock."""
    rec = profile_record("sq_counters.json", workload, kernel)
    if rec is None:
        return None
    return {"valu_insts_per_wave": rec["valu_insts_per_wave"], "valu_issue_frac": rec["valu_issue_frac"],
            "formula": "SQ_INSTS_VALU*4/(duration*2.4e9*1024)"}


def host_threads() -> int:
    """Host cores this process may use, capped at 16 (the CPU share of one GPU on the benchmark hosts)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def measured_copy_peak(mib=1024, reps=5):
    """Best device-to-device copy rate (read + write bytes per second, GB/s) of mib MiB, timed with events."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return 2.0 * n * 4 / (best * 1e-3) / 1e9


def cpu_baseline(scene, n_threads, per_thread=2):
    """The oracle as it stands: one view timed step by step on one thread, then views spread over n_threads
    threads (ctypes releases the GIL)."""
    import concurrent.futures as cf

    import oracle as O
    O.build(force=False)
    cam = scene.cameras[0]
    t0 = time.perf_counter()
    vis = O.raster_layers(scene.layers, cam)
    t1 = time.perf_counter()
    O.shade(scene.layers, scene.textures, cam, vis)
    t2 = time.perf_counter()
    O.backward(scene.layers, scene.textures, cam, vis, target=scene.targets[0])
    t3 = time.perf_counter()
    single = {"raster_s": t1 - t0, "shade_s": t2 - t1, "backward_s": t3 - t2, "total_s": t3 - t0,
              "px_layers": int((vis != np.uint64(0xFFFFFFFFFFFFFFFF)).sum())}
    cams = scene.cameras[1:1 + n_threads * per_thread]

    def one(v):
        cam = scene.cameras[v]
        vis = O.raster_layers(scene.layers, cam)
        O.shade(scene.layers, scene.textures, cam, vis)
        O.backward(scene.layers, scene.textures, cam, vis, target=scene.targets[v])
        return int((vis != np.uint64(0xFFFFFFFFFFFFFFFF)).sum())

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(n_threads) as ex:
        covered = sum(ex.map(one, range(1, 1 + len(cams))))
    dt = time.perf_counter() - t0
    return {"value": covered / dt, "unit": "px*layers/s", "cores": n_threads, "kind": "oracle",
            "sample": f"{len(cams)} of the 64 views (full 1024x1024, k=7), raster+shade+adjoint (L2), "
                      f"{per_thread} views per thread on {n_threads} threads (the host cores available, at most "
                      f"16), {dt:.1f} s wall",
            "single_thread_per_view": single,
            "single_thread_px_layers_per_s": single["px_layers"] / single["total_s"]}


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


def calibration_gather(mib):
    """Counter reference of a gather: mib MiB read once in a random order of 64-byte rows (index_select)
    and written contiguously, plus 8 bytes of index per row."""
    import torch
    rows = mib * (1 << 20) // 64
    a = torch.ones(rows, 16, dtype=torch.float32, device="cuda")
    idx = torch.randperm(rows, device="cuda", generator=torch.Generator(device="cuda").manual_seed(3))
    torch.cuda.synchronize()
    b = torch.index_select(a, 0, idx)
    torch.cuda.synchronize()
    log(f"[bench] calibration gather of {mib} MiB ({rows} rows of 64 B) done")
    del a, b, idx


def small_configs(P, S, torch):
    """Configurations 1-3 (one view each): latency per step, shaded px*layers/s, triangles/s (sum of k T over
    the raster phase) and the algorithmic-byte share of the HBM peak, all timed with events."""
    out = {}
    for cid, bwd in ((1, False), (2, False), (3, True)):
        sc = S.make_config(cid)
        k = sc.k
        layers = P.Layers(sc.layers)
        views = P.Views(sc.cameras)
        tex = [torch.from_numpy(t).cuda() for t in sc.textures]
        vis = torch.empty(k * views.total_pixels, dtype=torch.int64, device="cuda")
        ws = P.alloc_workspace(layers, views)
        img = torch.empty(views.total_pixels, 4, dtype=torch.float32, device="cuda")
        grads = [torch.zeros_like(t) for t in tex]
        tgt = (torch.from_numpy(sc.targets[0].reshape(-1, 4)).cuda() if bwd else None)
        ones = torch.ones(views.total_pixels, 4, dtype=torch.float32, device="cuda")

        def step():
            P.raster(layers, views, vis, ws)
            if bwd:
                P.render_backward(layers, tex, views, vis, ws, grad_tex=grads, target=tgt, out=img,
                                  loss_scale=1.0 / views.total_pixels)
            else:
                P.render(layers, tex, views, vis, ws, out=img)

        for _ in range(3):
            step()
        # texels a forward read touches = texels a unit upstream gradient reaches
        g1 = P.render_backward(layers, tex, views, vis, ws, grad_rgba=ones)
        U = [int((g != 0).any(dim=-1).sum().item()) for g in g1]
        covered = int((vis != -1).sum().item())
        reps = 20
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(reps)]
        for r in range(reps):
            ev[r][0].record()
            P.raster(layers, views, vis, ws)
            ev[r][1].record()
            if bwd:
                P.render_backward(layers, tex, views, vis, ws, grad_tex=grads, target=tgt, out=img,
                                  loss_scale=1.0 / views.total_pixels)
            else:
                P.render(layers, tex, views, vis, ws, out=img)
            ev[r][2].record()
        torch.cuda.synchronize()
        ph = np.array([[ev[r][0].elapsed_time(ev[r][1]), ev[r][1].elapsed_time(ev[r][2])] for r in range(reps)])
        ms_r, ms_s = np.median(ph[:, 0]), np.median(ph[:, 1])
        ms = ms_r + ms_s
        bm = byte_model(sc, 1, views.total_pixels, U, fused=True)
        alg = bm["raster"] + (bm["shade_bwd"] if bwd else
                              8 * k * views.total_pixels + 16 * views.total_pixels + sum(16 * u for u in U))
        out[f"cfg{cid}"] = {
            "what": ("k=3 icosphere shells, 256^2, forward" if cid == 1 else
                     "k=7 displaced shells (101,760 tris/layer), 1024^2, forward" if cid == 2 else
                     "k=7 displaced shells, 1024^2, forward + adjoint of the RGB L2 loss"),
            "latency_ms": float(ms), "raster_ms": float(ms_r), "shade_ms": float(ms_s),
            "px_layers_per_s": covered / (ms * 1e-3), "covered_px_layers": covered,
            "triangles_per_s": sum(m.n_tri for m in sc.layers) / (ms_r * 1e-3),
            "alg_bytes": int(alg), "alg_frac_of_peak": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        log(f"[bench] cfg{cid}: {ms:.3f} ms")
        del vis, ws, img, grads, tex, g1
    return out


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
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic("sh", names[dom])},
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        n = max(1, min(args.cpu_threads or host_threads(), nv))
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
                     "unit": "TFLOP/s", "frac": achieved / FP_PEAK_TFLOPS, "traffic": counter_traffic("ksdf", "ksdf_render"),
                     "flops_per_ray": ksdf_flops_per_ray(k, n, m, steps)},
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        from oracle import ksdf as K
        oopts = K.KsdfOpts(offsets=offs, beta=beta, occ_res=256, n_uniform=n, n_importance=m, march_steps=steps)
        occ_np = K.occupancy(grids, oopts)
        res_["cpu_baseline"] = ksdf_cpu_baseline(grids, oopts, occ_np, cams, 48000)
    print(json.dumps(res_), flush=True)


FIT_METRICS = {
    "fit": "shaded px·layers/s per texture-fitting iteration (k=7, 128 views at 800², RGB L2, Adam + clamp, "
           "graph replay); % HBM peak",
    "fit_l1q": "shaded px·layers/s per quantisation-aware fitting iteration (k=7, 128 views at 800², RGB L1, "
               "Adam on logits of 8-bit textures, graph replay); % HBM peak",
    "ngp": "shaded px·layers/s per neural-texture fitting iteration (k=7, 128 views at 800², hash grid + MLP "
           "baked at 1024², RGB L2, Adam, graph replay); % HBM peak",
}


def fit_cpu_baseline(sc, targets_np, loss, n_threads, n_views):
    """The oracle's fused-loss adjoint (forward recomputed inside) on a bounded sample of the views."""
    import concurrent.futures as cf

    import oracle as O
    O.build(force=False)
    vis = [O.raster_layers(sc.layers, sc.cameras[v]) for v in range(n_views)]

    def one(v):
        O.backward(sc.layers, sc.textures, sc.cameras[v], vis[v], target=targets_np[v], loss=loss)
        return int((vis[v] != np.uint64(0xFFFFFFFFFFFFFFFF)).sum())

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(n_threads) as ex:
        covered = sum(ex.map(one, range(n_views)))
    dt = time.perf_counter() - t0
    return {"value": covered / dt, "unit": "px*layers/s", "cores": n_threads, "kind": "oracle",
            "sample": f"{n_views} of the 128 views (full 800x800, k=7, visibility given), fused {loss.upper()} "
                      f"adjoint, {n_threads} threads, {dt:.1f} s wall"}


def ngp_cpu_baseline(sc, targets_np, fit, n_threads, n_views):
    """One iteration's parts on the oracle: one layer's bake + network backward at 1024^2 and the renderer's
    adjoint on a sample of views, scaled to all 7 layers and 128 views."""
    import concurrent.futures as cf

    import threadpoolctl

    import oracle as O
    from oracle import ngp as N
    O.build(force=False)
    import scenes as S
    cfg = N.NgpConfig(fit.cfg.resolutions, fit.cfg.log2_table)
    prm = S.ngp_params(5, 0, len(cfg.resolutions), cfg.log2_table, table_scale=1e-2).astype(np.float64)
    W = fit.sizes[0][0]
    with threadpoolctl.threadpool_limits(n_threads):
        t0 = time.perf_counter()
        tex = N.bake(prm, cfg, W, W)
        N.backward(prm, cfg, W, W, np.full((W, W, 4), 1e-3))
        t_net = time.perf_counter() - t0
    vis = [O.raster_layers(sc.layers, sc.cameras[v]) for v in range(n_views)]
    texs = [tex.astype(np.float32)] * sc.k

    def one(v):
        O.backward(sc.layers, texs, sc.cameras[v], vis[v], target=targets_np[v])
        return int((vis[v] != np.uint64(0xFFFFFFFFFFFFFFFF)).sum())

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(n_threads) as ex:
        covered = sum(ex.map(one, range(n_views)))
    t_ren = time.perf_counter() - t0
    t_iter = t_net * sc.k + t_ren * len(sc.cameras) / n_views
    covered_all = covered * len(sc.cameras) / n_views
    return {"value": covered_all / t_iter, "unit": "px*layers/s", "cores": n_threads, "kind": "oracle",
            "sample": f"1 of {sc.k} layers' bake + network backward at {W}^2 ({t_net:.1f} s) and {n_views} of "
                      f"{len(sc.cameras)} views' adjoint ({t_ren:.1f} s), {n_threads} threads, scaled to one "
                      f"iteration ({t_iter:.0f} s)"}


def run_fit(args):
    """Fitting iterations on fixed meshes (visibility rasterised once): graph-replayed, with a phase split
    from eager iterations."""
    import torch

    import paper_2409_02482_amd as P
    import scenes as S
    from paper_2409_02482_amd.fit import NeuralTextureFit, TextureFit, render_targets
    wl = args.workload
    log("[bench] building the config-5 scene")
    sc = S.make_config(5, n_views=128, resolution=(800, 800))
    targets = render_targets(sc.layers, sc.cameras, sc.textures_gt)
    iters = args.warmup + args.steps + 8
    loss = "l1" if wl == "fit_l1q" else "l2"
    if wl == "ngp":
        fit = NeuralTextureFit(sc.layers, sc.cameras, targets, tex_size=sc.textures[0].shape[1], max_iters=2 * iters)
    else:
        fit = TextureFit(sc.layers, sc.cameras, sc.textures, targets, mode="graph", max_iters=2 * iters, loss=loss,
                         quantize=(wl == "fit_l1q"))
    s = fit.stream
    k, views = fit.k, fit.views
    P_tot = views.total_pixels
    covered = int((fit.vis != -1).sum().item())

    if wl == "ngp":
        names = ["bake", "grad_zero", "shade_bwd", "ngp_backward", "adam"]

        def phases(ev):
            ev[0].record(s)
            P.ngp_bake(fit.params, fit.cfg, fit.sizes, tex=fit.tex, ws=fit.nws, stream=s)
            ev[1].record(s)
            with torch.cuda.stream(s):
                for g in fit.gtex:
                    g.zero_()
            ev[2].record(s)
            P.render_backward(fit.layers, fit.tex, views, fit.vis, fit.ws, grad_tex=fit.gtex, target=fit.targets,
                              loss_scale=1.0 / fit.n_scalars, sse=fit.sse, loss=fit.loss, stream=s)
            ev[3].record(s)
            P.ngp_backward(fit.params, fit.cfg, fit.sizes, fit.tex, fit.gtex, fit.nws, grad_params=fit.gp, stream=s)
            ev[4].record(s)
            P.adam_step(fit.params, fit.gp, fit.m, fit.v, fit.step, lr=fit.lr, lo=-1e30, hi=1e30, sse=fit.sse,
                        history=fit.history, stream=s)
            ev[5].record(s)
    else:
        names = ["shade_bwd", "adam"]

        def phases(ev):
            ev[0].record(s)
            P.render_backward(fit.layers, fit.tex, views, fit.vis, fit.ws, grad_tex=fit.grads, target=fit.targets,
                              loss_scale=fit.loss_scale, sse=fit.sse, loss=fit.loss, stream=s)
            ev[1].record(s)
            if fit.quantize:
                P.adam_step_squeezed(fit.params, fit.grads, fit.m, fit.v, fit.tex, fit.step, levels=fit.levels,
                                     lr=fit.lr, betas=fit.betas, eps=fit.eps, sse=fit.sse, history=fit.history,
                                     stream=s)
            else:
                P.adam_step(fit.params, fit.grads, fit.m, fit.v, fit.step, lr=fit.lr, betas=fit.betas, eps=fit.eps,
                            sse=fit.sse, history=fit.history, stream=s)
            ev[2].record(s)

    log("[bench] eager iterations (phase split)")
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(names) + 1)] for _ in range(args.warmup + 3)]
    for ev in evs:
        phases(ev)
    s.synchronize()
    ph = np.array([[ev[i].elapsed_time(ev[i + 1]) for i in range(len(names))] for ev in evs[args.warmup:]])
    ms_phase = ph.mean(0)
    log("[bench] graph replay")
    fit.capture()
    fit.run(max(args.warmup, 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_graph = fit.run(args.steps)
    torch.cuda.synchronize()
    ms_wall = (time.perf_counter() - t0) / args.steps * 1e3

    # algorithmic bytes per launch of the adjoint: keys, target, texels touched, gradient read-modify-write, mesh
    grads = fit.gtex if wl == "ngp" else fit.grads
    P.render_backward(fit.layers, fit.tex, views, fit.vis, fit.ws, grad_tex=grads, target=fit.targets,
                      loss_scale=1.0, sse=None, loss=fit.loss, stream=s)
    s.synchronize()
    U = [int((g != 0).any(dim=-1).sum().item()) for g in grads]
    G = sum(12 * m.n_vert + 8 * m.n_vert + 12 * m.n_tri for m in sc.layers)
    planes = sum(16 * int(g.shape[0]) * int(g.shape[1]) for g in grads)
    bm = {"shade_bwd": 8 * k * P_tot + 16 * P_tot + 16 * sum(U) + 2 * planes + G}
    n_par = sum(int(p.numel()) for p in fit.params)
    # Adam: parameter, gradient (read + reset), two moments, each read and written (+ texture write if squeezed)
    bm["adam"] = n_par * (4 * 8 + (4 if wl == "fit_l1q" else 0))
    dom = names[int(np.argmax(ms_phase))]
    if dom not in bm:
        dom = "shade_bwd"
    i_dom = names.index(dom)
    achieved = bm[dom] / (ms_phase[i_dom] * 1e-3) / 1e9
    h = fit.loss_history()
    res = {
        "metric": FIT_METRICS[wl], "value": covered / (ms_graph * 1e-3), "unit": "px*layers/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_graph, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"k={k} displaced shells, 128 ring views at 800x800, targets rendered from seeded "
                               f"ground-truth textures, {loss.upper()} loss"
                               + (", 8-bit quantised logits" if wl == "fit_l1q" else "")
                               + (", neural textures (8 levels 16..1024, 2^16 entries, MLP 64-64) baked at 1024^2"
                                  if wl == "ngp" else ", 1024^2 f32 RGBA textures"),
                   "views": len(sc.cameras), "k": k, "pixels": P_tot, "covered_px_layers": covered},
        "wall_ms_per_step": ms_wall,
        "phases_ms": {n: float(m) for n, m in zip(names, ms_phase)},
        "loss_first_last": [float(h[0]), float(h[-1])] if len(h) else None,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(wl, dom)},
    }
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        n = args.cpu_threads or host_threads()
        # seeded targets (the CPU timing takes no GPU output); 64 views keep the sample at seconds of CPU work
        tg = S.uniform_targets(5, sc.cameras[:64 if wl != "ngp" else 32])
        if wl == "ngp":
            res["cpu_baseline"] = ngp_cpu_baseline(sc, tg, fit, n, len(tg))
        else:
            res["cpu_baseline"] = fit_cpu_baseline(sc, tg, loss, n, len(tg))
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--views", type=int, default=64)
    ap.add_argument("--res", type=int, default=1024)
    ap.add_argument("--bin", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0, help="0: the host cores available (at most 16)")
    ap.add_argument("--no-small-configs", action="store_true", help="skip the configuration 1-3 measurements")
    ap.add_argument("--unfused", action="store_true", help="separate forward shading pass before the adjoint")
    ap.add_argument("--workload", default="metric", choices=["metric", "cfg4", "sh", "ksdf", "fit", "fit_l1q", "ngp"],
                    help="metric: k=7, 64 views at 1024^2; cfg4: k=9, 299,208 tris/layer, 64 mixed-size views; "
                         "sh: the metric scene rendered forward with baked 8-bit SH textures (degree 3, 2048^2 base); "
                         "ksdf: k-SDF volume rendering of the implicit stage (8 views at 512^2); "
                         "fit / fit_l1q / ngp: texture-fitting iterations on config 5 (L2; L1 on 8-bit logits; "
                         "neural textures)")
    ap.add_argument("--graph", action="store_true", help="replay the step from a captured HIP graph")
    ap.add_argument("--autotune", action="store_true", help="pick the raster bin size with vs_autotune")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="run one plain device copy of this many MiB first (HBM counter calibration)")
    ap.add_argument("--calibrate-gather", type=int, default=0, metavar="MIB",
                    help="run one gather of this many MiB in 64-byte rows first (second counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this benchmark measures one GPU only; --gpus must be 1 (views would shard across GPUs, "
              "with one all-reduce of the texture gradients per step)", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        calibration_copy(args.calibrate_copy)
    if args.calibrate_gather:
        calibration_gather(args.calibrate_gather)
    if args.workload == "sh":
        return run_sh(args)
    if args.workload == "ksdf":
        return run_ksdf(args)
    if args.workload in ("fit", "fit_l1q", "ngp"):
        return run_fit(args)

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
        "metric": METRIC if args.workload == "metric" else CFG4_METRIC,
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
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic(args.workload, dom_name),
                     "issue": issue_rate(args.workload, dom_name)},
    }
    if graph is not None:
        res["graph_ms_per_step"] = graph_ms
    log("[bench] copy peak")
    copy = measured_copy_peak()
    res["roofline"]["measured_copy_peak"] = copy
    res["roofline"]["frac_of_measured_copy"] = achieved / copy
    if args.workload == "metric" and not args.no_small_configs:
        res["configs"] = small_configs(P, S, torch)
    if not args.no_cpu_baseline and args.workload == "metric":
        log("[bench] cpu baseline (oracle)")
        n = args.cpu_threads or host_threads()
        res["cpu_baseline"] = cpu_baseline(scene, n)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()

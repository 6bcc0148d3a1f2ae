"""Texture fitting on fixed meshes: the training pattern the renderer serves.

Textures are optimised on fixed geometry (Sec. 4.3, "Texturing Meshes"), so
visibility is rasterised once and every iteration is

    fused shade + adjoint of the RGB L2 loss (writes dL/dtexture and the SSE)
    fused Adam step + projection to [0, 1] + gradient reset
    on-device bookkeeping (SSE history for the PSNR curve, step counter)

With quantize=True the parameters are logits and the rendered texture is
q(sigmoid(logit)) rounded to 8 bits (Sec. 4.3 "Squeezing and
Quantization"), the quantiser passed straight through in the gradient; with
loss="l1" the fused loss is the paper's L1 instead of L2.

Two launch strategies with identical arithmetic:
  "graph":    all views in one batched launch per kernel, the iteration
              captured once in a HIP graph and replayed;
  "per_view": one launch per view per iteration, eager.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import binding as R


def psnr_from_sse(sse: np.ndarray, n_scalars: int) -> np.ndarray:
    mse = np.asarray(sse, np.float64) / n_scalars
    return 10.0 * np.log10(1.0 / np.maximum(mse, 1e-30))


CHECKPOINT_VERSION = 1


def save_state(path: str, state: dict, meta: Optional[dict] = None) -> None:
    """Write named tensors or lists of tensors (copied to host memory) with torch.save."""
    out = {"version": CHECKPOINT_VERSION, "meta": dict(meta or {}), "tensors": {}}
    for name, val in state.items():
        if isinstance(val, (list, tuple)):
            out["tensors"][name] = [t.detach().to("cpu", copy=True) for t in val]
        else:
            out["tensors"][name] = val.detach().to("cpu", copy=True)
    tmp = path + ".tmp"
    torch.save(out, tmp)
    os.replace(tmp, path)


def load_state(path: str, into: dict, meta: Optional[dict] = None) -> None:
    """Copy a save_state file into existing tensors of the same names, shapes and dtypes, in place (so a
    captured graph that holds their addresses stays valid).  Nothing is written unless every tensor fits."""
    rec = torch.load(path, map_location="cpu", weights_only=True)
    if rec.get("version") != CHECKPOINT_VERSION:
        raise ValueError(f"{path}: checkpoint version {rec.get('version')} (expected {CHECKPOINT_VERSION})")
    if meta is not None:
        for key, val in meta.items():
            if rec["meta"].get(key) != val:
                raise ValueError(f"{path}: {key} = {rec['meta'].get(key)!r}, this run has {val!r}")
    saved = rec["tensors"]
    pairs = []
    for name, dst in into.items():
        if name not in saved:
            raise ValueError(f"{path}: no tensor {name!r}")
        src = saved[name]
        dl = list(dst) if isinstance(dst, (list, tuple)) else [dst]
        sl = list(src) if isinstance(src, (list, tuple)) else [src]
        if len(dl) != len(sl):
            raise ValueError(f"{path}: {name} has {len(sl)} tensors, expected {len(dl)}")
        for i, (d, t) in enumerate(zip(dl, sl)):
            if d.shape != t.shape or d.dtype != t.dtype:
                raise ValueError(f"{path}: {name}[{i}] is {tuple(t.shape)} {t.dtype}, expected "
                                 f"{tuple(d.shape)} {d.dtype}")
            pairs.append((d, t))
    for d, t in pairs:
        d.copy_(t)


class TextureFit:
    """Adam on RGBA f32 textures of k fixed shells seen from many views."""

    def __init__(self, meshes, cameras: Sequence, init_textures: Sequence[np.ndarray], targets: torch.Tensor,
                 mode: str = "graph", lr: float = 1e-2, betas=(0.9, 0.999), eps: float = 1e-8, bin: int = 0,
                 max_iters: int = 1024, device: str = "cuda", loss: str = "l2", quantize: bool = False,
                 levels: int = 255):
        if mode not in ("graph", "per_view"):
            raise ValueError(mode)
        if loss not in ("l2", "l1"):
            raise ValueError(loss)
        self.mode, self.lr, self.betas, self.eps = mode, lr, betas, eps
        self.loss, self.quantize, self.levels = loss, quantize, levels
        self.layers = R.Layers(meshes, device)
        self.views = R.Views(cameras, device)
        self.k = self.layers.k
        init = [torch.from_numpy(np.ascontiguousarray(t, np.float32)).to(device) for t in init_textures]
        if quantize:
            # logits of the initial texture (kept off 0 and 1 so they stay finite)
            lim = 0.5 / max(levels, 255)
            self.params = [torch.logit(t.clamp(lim, 1.0 - lim)) for t in init]
            self.tex = [torch.empty_like(t) for t in init]
            R.squeeze(self.params, self.tex, levels)
        else:
            self.params = init
            self.tex = self.params
        self.grads = [torch.zeros_like(p) for p in self.params]
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.step = torch.zeros(1, dtype=torch.int32, device=device)
        self.sse = torch.zeros(1, dtype=torch.float64, device=device)
        self.history = torch.zeros(max_iters, dtype=torch.float64, device=device)
        self.targets = targets
        self.n_scalars = 3 * self.views.total_pixels
        self.loss_scale = 1.0 / self.n_scalars
        self.stream = torch.cuda.Stream(device=device)
        self.graph: Optional[R.Graph] = None
        with torch.cuda.stream(self.stream):
            if mode == "graph":
                self.vis, self.ws = R.raster(self.layers, self.views, bin=bin, stream=self.stream)
            else:
                self.per_view = []
                for v, cam in enumerate(cameras):
                    vv = R.Views([cam], device)
                    vis, ws = R.raster(self.layers, vv, bin=bin, stream=self.stream)
                    tgt = self.views.image(targets, v).reshape(-1, 4)
                    self.per_view.append((vv, vis, ws, tgt))
        self.stream.synchronize()

    def _iteration(self):
        s = self.stream
        if self.mode == "graph":
            R.render_backward(self.layers, self.tex, self.views, self.vis, self.ws, grad_tex=self.grads,
                              target=self.targets, loss_scale=self.loss_scale, sse=self.sse, loss=self.loss, stream=s)
        else:
            for vv, vis, ws, tgt in self.per_view:
                R.render_backward(self.layers, self.tex, vv, vis, ws, grad_tex=self.grads, target=tgt,
                                  loss_scale=self.loss_scale, sse=self.sse, loss=self.loss, stream=s)
        if self.quantize:
            R.adam_step_squeezed(self.params, self.grads, self.m, self.v, self.tex, self.step, levels=self.levels,
                                 lr=self.lr, betas=self.betas, eps=self.eps, sse=self.sse, history=self.history,
                                 stream=s)
        else:
            R.adam_step(self.params, self.grads, self.m, self.v, self.step, lr=self.lr, betas=self.betas,
                        eps=self.eps, sse=self.sse, history=self.history, stream=s)

    def capture(self):
        if self.mode != "graph":
            raise RuntimeError("only the batched mode is captured")
        self.graph = R.Graph(self.stream)
        with self.graph:
            self._iteration()

    def run(self, iters: int) -> float:
        """Run iterations; returns milliseconds per iteration (stream time)."""
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        for _ in range(iters):
            if self.graph is not None:
                self.graph.replay()
            else:
                self._iteration()
        e1.record(self.stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / max(iters, 1)

    def loss_history(self) -> np.ndarray:
        """Per iteration, the unscaled loss sum over all RGB scalars (squared or absolute errors)."""
        self.stream.synchronize()
        n = int(self.step.item())
        return self.history[:min(n, self.history.numel())].cpu().numpy()

    def _state(self) -> dict:
        # the rendered texture of the quantised mode is a function of the logits: re-derived on load
        return {"params": self.params, "m": self.m, "v": self.v, "step": self.step, "history": self.history}

    def _meta(self) -> dict:
        return {"k": self.k, "loss": self.loss, "quantize": bool(self.quantize), "levels": int(self.levels),
                "lr": float(self.lr), "betas": [float(b) for b in self.betas], "eps": float(self.eps),
                "views": [list(hw) for hw in self.views.sizes]}

    def save(self, path: str) -> None:
        """Checkpoint the fit between iterations: parameters, Adam moments, step and loss history."""
        self.stream.synchronize()
        save_state(path, self._state(), self._meta())

    def load(self, path: str) -> None:
        """Resume from save(): the same tensors are overwritten in place, so a captured graph stays valid."""
        self.stream.synchronize()
        load_state(path, self._state(), self._meta())
        if self.quantize:
            R.squeeze(self.params, self.tex, self.levels, stream=self.stream)
        for g in self.grads:
            g.zero_()
        self.sse.zero_()
        torch.cuda.synchronize()

    def psnr(self) -> np.ndarray:
        if self.loss != "l2":
            raise ValueError("the per-iteration history holds absolute errors under the L1 loss")
        return psnr_from_sse(self.loss_history(), self.n_scalars)


class NeuralTextureFit:
    """Neural textures (hash grid + MLP, Sec. 4.3) fit through the renderer.

    Per iteration: bake the textures at their texel centres, the fused shade +
    adjoint (L2 or L1) gives dL/dtexture, the network backward carries it to the
    parameters, and Adam (unbounded) updates them; the same launches can be
    captured in a HIP graph."""

    def __init__(self, meshes, cameras: Sequence, targets: torch.Tensor, tex_size: int, levels: int = 8,
                 log2_table: int = 16, base_res: int = 16, lr: float = 1e-2, loss: str = "l2", config: int = 5,
                 max_iters: int = 1024, device: str = "cuda"):
        import scenes as S  # seeded initial parameters
        self.layers = R.Layers(meshes, device)
        self.views = R.Views(cameras, device)
        self.k = self.layers.k
        self.cfg = R.NgpConfig(S.ngp_resolutions(levels, base_res, tex_size), log2_table)
        self.sizes = [(tex_size, tex_size)] * self.k
        self.params = [torch.from_numpy(S.ngp_params(config, l, levels, log2_table, table_scale=1e-2)).to(device)
                       for l in range(self.k)]
        self.m = [torch.zeros_like(p) for p in self.params]
        self.v = [torch.zeros_like(p) for p in self.params]
        self.gp = [torch.zeros_like(p) for p in self.params]
        self.tex = [torch.empty(tex_size, tex_size, 4, device=device) for _ in range(self.k)]
        self.gtex = [torch.zeros_like(t) for t in self.tex]
        self.nws = R.ngp_workspace(self.cfg, self.sizes, device)
        self.step = torch.zeros(1, dtype=torch.int32, device=device)
        self.sse = torch.zeros(1, dtype=torch.float64, device=device)
        self.history = torch.zeros(max_iters, dtype=torch.float64, device=device)
        self.targets, self.lr, self.loss = targets, lr, loss
        self.n_scalars = 3 * self.views.total_pixels
        self.stream = torch.cuda.Stream(device=device)
        self.graph: Optional[R.Graph] = None
        with torch.cuda.stream(self.stream):
            self.vis, self.ws = R.raster(self.layers, self.views, stream=self.stream)
        self.stream.synchronize()

    def _iteration(self):
        s = self.stream
        R.ngp_bake(self.params, self.cfg, self.sizes, tex=self.tex, ws=self.nws, stream=s)
        with torch.cuda.stream(s):
            for g in self.gtex:
                g.zero_()
        R.render_backward(self.layers, self.tex, self.views, self.vis, self.ws, grad_tex=self.gtex,
                          target=self.targets, loss_scale=1.0 / self.n_scalars, sse=self.sse, loss=self.loss, stream=s)
        R.ngp_backward(self.params, self.cfg, self.sizes, self.tex, self.gtex, self.nws, grad_params=self.gp, stream=s)
        R.adam_step(self.params, self.gp, self.m, self.v, self.step, lr=self.lr, lo=-1e30, hi=1e30, sse=self.sse,
                    history=self.history, stream=s)

    def capture(self):
        self.graph = R.Graph(self.stream)
        with self.graph:
            self._iteration()

    def run(self, iters: int) -> float:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(self.stream)
        for _ in range(iters):
            if self.graph is not None:
                self.graph.replay()
            else:
                self._iteration()
        e1.record(self.stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / max(iters, 1)

    def loss_history(self) -> np.ndarray:
        self.stream.synchronize()
        n = int(self.step.item())
        return self.history[:min(n, self.history.numel())].cpu().numpy()


def render_targets(meshes, cameras, textures: Sequence[np.ndarray], device="cuda") -> torch.Tensor:
    """Target images [sum_v H_v W_v, 4] rendered by the GPU path from ground-truth textures."""
    layers = R.Layers(meshes, device)
    views = R.Views(cameras, device)
    vis, ws = R.raster(layers, views)
    tex = [torch.from_numpy(np.ascontiguousarray(t, np.float32)).to(device) for t in textures]
    out = R.render(layers, tex, views, vis, ws)
    torch.cuda.synchronize()
    del vis, ws
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="k=7 texture fitting: batched+graph vs per-view launches")
    ap.add_argument("--views", type=int, default=128)
    ap.add_argument("--res", type=int, default=800)
    ap.add_argument("--iters", type=int, default=200)
    ap.add_argument("--modes", default="graph,per_view")
    ap.add_argument("--loss", default="l2", choices=["l2", "l1"])
    ap.add_argument("--quantize", action="store_true", help="fit logits of 8-bit quantised textures")
    ap.add_argument("--neural", action="store_true",
                    help="fit neural textures (hash grid + MLP baked at 1024^2 texel centres) instead of texels")
    args = ap.parse_args(argv)
    import scenes as S  # seeded synthetic inputs
    sc = S.make_config(5, n_views=args.views, resolution=(args.res, args.res))
    targets = render_targets(sc.layers, sc.cameras, sc.textures_gt)
    if args.neural:
        res = {"config": f"k={sc.k} shells, {args.views} views at {args.res}x{args.res}, {args.iters} Adam iterations, "
                         f"{args.loss} loss, neural textures (8 levels 16..1024, 2^16 entries, MLP 64x64) baked at 1024^2"}
        for mode in args.modes.split(","):
            if mode not in ("graph", "eager"):
                continue
            fit = NeuralTextureFit(sc.layers, sc.cameras, targets, tex_size=sc.textures[0].shape[1],
                                   loss=args.loss, max_iters=args.iters + 8)
            if mode == "graph":
                fit.capture()
            first_ms = fit.run(1)
            ms = fit.run(args.iters - 1)
            h = fit.loss_history() / fit.n_scalars
            curve = psnr_from_sse(fit.loss_history(), fit.n_scalars) if args.loss == "l2" else h
            res[mode] = {"ms_per_iter": ms, "first_iter_ms": first_ms, "first": float(curve[0]), "last": float(curve[-1]),
                         "curve": [round(float(x), 6) for x in curve]}
            print(f"[fit] neural {mode}: {ms:.3f} ms/iter, {'PSNR' if args.loss == 'l2' else 'MAE'} "
                  f"{curve[0]:.4f} -> {curve[-1]:.4f}", file=sys.stderr, flush=True)
            del fit
            torch.cuda.empty_cache()
        print(json.dumps(res))
        return
    res = {"config": f"k={sc.k} shells, {args.views} views at {args.res}x{args.res}, {args.iters} Adam iterations, "
                     f"{args.loss} loss" + (", 8-bit quantised logits" if args.quantize else "")}
    for mode in args.modes.split(","):
        fit = TextureFit(sc.layers, sc.cameras, sc.textures, targets, mode=mode, max_iters=args.iters + 8,
                         loss=args.loss, quantize=args.quantize)
        if mode == "graph":
            fit.capture()
        # the first iteration carries one-time costs (code-object loading, the graph's first upload):
        # it is timed on its own, and ms_per_iter is the steady rate of the other iterations
        first_ms = fit.run(1)
        ms = fit.run(args.iters - 1)
        # L2: PSNR per iteration; L1: mean absolute error per RGB scalar per iteration
        name, unit = ("psnr", "dB") if args.loss == "l2" else ("mae", "")
        p = fit.psnr() if args.loss == "l2" else fit.loss_history() / fit.n_scalars
        res[mode] = {"ms_per_iter": ms, "first_iter_ms": first_ms, f"{name}_first": float(p[0]),
                     f"{name}_last": float(p[-1]), name: [round(float(x), 6) for x in p]}
        print(f"[fit] {mode}: {ms:.3f} ms/iter, {name.upper()} {p[0]:.4f} -> {p[-1]:.4f} {unit}", file=sys.stderr,
              flush=True)
        del fit
        torch.cuda.empty_cache()
    if "graph" in res and "per_view" in res:
        res["speedup_graph_vs_per_view"] = res["per_view"]["ms_per_iter"] / res["graph"]["ms_per_iter"]
        res[f"max_{name}_gap"] = float(np.max(np.abs(np.array(res["graph"][name]) - np.array(res["per_view"][name]))))
    print(json.dumps(res))


if __name__ == "__main__":
    main()

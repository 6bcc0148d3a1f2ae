"""PyTorch-facing binding of the gfx950 renderer.

Torch supplies device memory and the stream; every step of the render runs
in the HIP kernels behind the C ABI (include/vs.h).  The classes here only
marshal tensors into the C structs:

  Layers    k meshes on the device (layer 0 outermost)
  Views     batched cameras (host + device view tables)
  raster / render / render_backward   thin wrappers of the three entry points
  Renderer  owns the visibility buffer and workspace of a fixed scene and
            exposes a differentiable ``__call__(*textures) -> rgba``
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as C


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t: torch.Tensor, dtype, what: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return t


def _shape(t: torch.Tensor, shape, what: str) -> torch.Tensor:
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _arg(t: torch.Tensor, dtype, shape, what: str) -> torch.Tensor:
    """Shape first (a mismatch is reported even for a host tensor), then device, dtype and layout."""
    return _dev(_shape(t, shape, what), dtype, what)


def _count(seq, n: int, what: str):
    if len(seq) != n:
        raise ValueError(f"{what}: {len(seq)} given, {n} expected (one per layer)")
    return seq


def _check_vis(vis: torch.Tensor, layers: "Layers", views: "Views") -> torch.Tensor:
    if vis.numel() != layers.k * views.total_pixels:
        raise ValueError(f"vis has {vis.numel()} slots, k * total pixels = {layers.k * views.total_pixels}")
    return _dev(vis, torch.int64, "vis")


def _check_ws(ws: torch.Tensor) -> torch.Tensor:
    return _dev(ws, torch.uint8, "workspace")


class Layers:
    """k meshes on the device.  ``meshes``: objects with xyz [V,3], uv [V,2], tri [T,3] (numpy or torch)."""

    def __init__(self, meshes, device="cuda"):
        self.k = len(meshes)
        if not 1 <= self.k <= C.VS_MAX_LAYERS:
            raise ValueError(f"k = {self.k} outside 1..{C.VS_MAX_LAYERS}")
        self.tensors = []
        self.c = (C.VsMesh * self.k)()
        for l, m in enumerate(meshes):
            xyz = torch.as_tensor(np.asarray(m.xyz, np.float32)).to(device).contiguous()
            uv = torch.as_tensor(np.asarray(m.uv, np.float32)).to(device).contiguous()
            tri = torch.as_tensor(np.asarray(m.tri, np.int32)).to(device).contiguous()
            self.tensors.append((xyz, uv, tri))
            self.c[l] = C.VsMesh(xyz.data_ptr(), uv.data_ptr(), tri.data_ptr(), xyz.shape[0], tri.shape[0])
        self.n_tri = [int(t[2].shape[0]) for t in self.tensors]


def camera_struct(cam) -> C.VsCamera:
    c = C.VsCamera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = np.asarray(cam.R, np.float64).reshape(9)
    t = np.asarray(cam.t, np.float64).reshape(3)
    for i in range(9):
        c.R[i] = float(R[i])
    for i in range(3):
        c.t[i] = float(t[i])
    c.z_near = float(getattr(cam, "z_near", 0.01))
    return c


class Views:
    """Batched cameras: the host view table (vs_views_prepare) and its device copy."""

    def __init__(self, cameras: Sequence, device="cuda"):
        n = len(cameras)
        cams = (C.VsCamera * n)(*[camera_struct(c) for c in cameras])
        self.host = (C.VsView * (n + 1))()
        C.check(C.load().vs_views_prepare(ctypes.addressof(cams), n, ctypes.addressof(self.host)),
                "vs_views_prepare")
        raw = np.frombuffer(bytes(self.host), np.uint8).copy()
        self.dev = torch.from_numpy(raw).to(device)
        self.c = C.VsViews(ctypes.addressof(self.host), self.dev.data_ptr(), n)
        self.n = n
        self.sizes = [(int(c.height), int(c.width)) for c in cameras]
        self.pix_offset = [int(self.host[v].pix_offset) for v in range(n + 1)]
        self.total_pixels = self.pix_offset[n]

    def image(self, flat: torch.Tensor, v: int) -> torch.Tensor:
        """View v of a flat [sum_v H_v W_v, C] buffer as [H, W, C]."""
        h, w = self.sizes[v]
        return flat[self.pix_offset[v]:self.pix_offset[v + 1]].view(h, w, -1)

    def vis_planes(self, vis: torch.Tensor, k: int, v: int) -> torch.Tensor:
        """View v of a visibility buffer as [k, H, W] (int64 storage of the u64 keys)."""
        h, w = self.sizes[v]
        o = k * self.pix_offset[v]
        return vis[o:o + k * h * w].view(k, h, w)


def _check_textures(textures: Sequence[torch.Tensor], k: Optional[int] = None):
    """Count and shapes of the layer textures ([H, W, 4] each), before any device check."""
    if k is not None:
        _count(textures, k, "textures")
    for l, t in enumerate(textures):
        if t.dim() != 3 or t.shape[2] != 4:
            raise ValueError(f"texture {l} must be [H, W, 4], got {tuple(t.shape)}")


def textures_struct(textures: Sequence[torch.Tensor], k: Optional[int] = None):
    _check_textures(textures, k)
    arr = (C.VsTexture * len(textures))()
    for l, t in enumerate(textures):
        _dev(t, torch.float32, f"texture {l}")
        arr[l] = C.VsTexture(t.data_ptr(), t.shape[1], t.shape[0])
    return arr


def _raster_opts(bin=0, count_fragments=False, direct=False, list_capacity=0):
    flags = (C.VS_RASTER_COUNT_FRAGMENTS if count_fragments else 0) | (C.VS_RASTER_DIRECT if direct else 0)
    return C.VsRasterOpts(int(bin), flags, int(list_capacity))


def workspace_bytes(layers: Layers, views: Views, bin: int = 0, list_capacity: int = 0) -> int:
    opts = _raster_opts(bin, list_capacity=list_capacity)
    n = C.load().vs_raster_workspace_bytes(ctypes.addressof(layers.c), layers.k, ctypes.byref(views.c),
                                           ctypes.byref(opts))
    if n == 0:
        raise C.VsError(C.VS_ERR_ARG, "vs_raster_workspace_bytes", C.load().vs_last_error().decode() or
                        "invalid layers, views or options")
    return int(n)


def alloc_workspace(layers: Layers, views: Views, bin: int = 0, device="cuda", list_capacity: int = 0) -> torch.Tensor:
    return torch.empty(workspace_bytes(layers, views, bin, list_capacity), dtype=torch.uint8, device=device)


def raster(layers: Layers, views: Views, vis: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
           bin: int = 0, count_fragments: bool = False, direct: bool = False, list_capacity: int = 0, stream=None):
    """vs_raster_layers: returns (vis int64[sum_v k H_v W_v] holding u64 keys, workspace)."""
    dev = views.dev.device
    if vis is None:
        vis = torch.empty(layers.k * views.total_pixels, dtype=torch.int64, device=dev)
    if ws is None:
        ws = alloc_workspace(layers, views, bin, dev, list_capacity)
    _check_vis(vis, layers, views)
    _check_ws(ws)
    opts = _raster_opts(bin, count_fragments, direct, list_capacity)
    C.check(C.load().vs_raster_layers(ctypes.addressof(layers.c), layers.k, ctypes.byref(views.c), vis.data_ptr(),
                                      ws.data_ptr(), ws.numel(), ctypes.byref(opts), _stream(stream)),
            "vs_raster_layers")
    return vis, ws


def _shade_opts(eps_T=0.0, wrap=0, target=None, loss_scale=1.0, loss="l2", count_paths=False):
    return C.VsShadeOpts(float(eps_T), int(wrap), 0 if target is None else target.data_ptr(), float(loss_scale),
                         C.VS_LOSS[loss], C.VS_SHADE_COUNT_PATHS if count_paths else 0)


def render(layers: Layers, textures, views: Views, vis: torch.Tensor, ws: torch.Tensor,
           out: Optional[torch.Tensor] = None, eps_T: float = 0.0, wrap: int = 0, stream=None) -> torch.Tensor:
    """vs_render: [sum_v H_v W_v, 4] RGBA (A = 1 - transmittance)."""
    _check_textures(textures, layers.k)
    if out is not None:
        _shape(out, (views.total_pixels, 4), "out")
    _check_vis(vis, layers, views)
    _check_ws(ws)
    if out is None:
        out = torch.empty(views.total_pixels, 4, dtype=torch.float32, device=vis.device)
    _arg(out, torch.float32, (views.total_pixels, 4), "out")
    tex = textures_struct(textures, layers.k)
    opts = _shade_opts(eps_T, wrap)
    C.check(C.load().vs_render(ctypes.addressof(layers.c), ctypes.addressof(tex), layers.k, ctypes.byref(views.c),
                               vis.data_ptr(), ws.data_ptr(), ws.numel(), out.data_ptr(), ctypes.byref(opts),
                               _stream(stream)), "vs_render")
    return out


def render_noalloc(layers: Layers, textures, views: Views, vis: torch.Tensor, out: torch.Tensor, bin: int = 0,
                   eps_T: float = 0.0, wrap: int = 0, stream=None) -> torch.Tensor:
    """vs_render_noalloc: raster into ``vis`` and shade into ``out`` with the library's static workspace
    (no device allocation by the library; both buffers are the caller's)."""
    _check_textures(textures, layers.k)
    _shape(out, (views.total_pixels, 4), "out")
    _check_vis(vis, layers, views)
    _arg(out, torch.float32, (views.total_pixels, 4), "out")
    tex = textures_struct(textures, layers.k)
    ropts = _raster_opts(bin)
    sopts = _shade_opts(eps_T, wrap)
    C.check(C.load().vs_render_noalloc(ctypes.addressof(layers.c), ctypes.addressof(tex), layers.k,
                                       ctypes.byref(views.c), vis.data_ptr(), out.data_ptr(), ctypes.byref(ropts),
                                       ctypes.byref(sopts), _stream(stream)), "vs_render_noalloc")
    return out


def sh_texture_bytes(width: int, height: int, degree: int) -> int:
    """Bytes of one shell's packed SH levels 0..degree (level d: max(1, W >> d) x max(1, H >> d) texels,
    2d + 1 RGBA byte words each)."""
    return sum(max(1, int(width) >> d) * max(1, int(height) >> d) * (2 * d + 1) * 4 for d in range(int(degree) + 1))


def sh_textures_struct(sh_textures: Sequence, k: Optional[int] = None, degree: Optional[int] = None) -> ctypes.Array:
    """sh_textures[l] = (data, width, height): data a contiguous uint8 device tensor of packed levels."""
    if k is not None:
        _count(sh_textures, k, "SH textures")
    arr = (C.VsShTexture * len(sh_textures))()
    for l, (data, w, h) in enumerate(sh_textures):
        _dev(data, torch.uint8, f"SH texture {l}")
        if degree is not None and data.numel() < sh_texture_bytes(w, h, degree):
            raise ValueError(f"SH texture {l}: {data.numel()} bytes, degree {degree} at {w}x{h} needs "
                             f"{sh_texture_bytes(w, h, degree)}")
        arr[l] = C.VsShTexture(data.data_ptr(), int(w), int(h))
    return arr


def render_sh(layers: Layers, sh_textures, views: Views, vis: torch.Tensor, ws: torch.Tensor, degree: int = 3,
              vmin: float = -15.0, vmax: float = 15.0, view_alpha: bool = True, out: Optional[torch.Tensor] = None,
              eps_T: float = 0.0, wrap: int = 0, stream=None) -> torch.Tensor:
    """vs_render_sh: [sum_v H_v W_v, 4] RGBA from baked 8-bit SH textures (A = 1 - transmittance)."""
    _count(sh_textures, layers.k, "SH textures")
    for l, (data, w, h) in enumerate(sh_textures):
        if 0 <= int(degree) <= 3 and data.numel() < sh_texture_bytes(w, h, degree):
            raise ValueError(f"SH texture {l}: {data.numel()} bytes, degree {degree} at {w}x{h} needs "
                             f"{sh_texture_bytes(w, h, degree)}")
    if out is not None:
        _shape(out, (views.total_pixels, 4), "out")
    _check_vis(vis, layers, views)
    _check_ws(ws)
    if out is None:
        out = torch.empty(views.total_pixels, 4, dtype=torch.float32, device=vis.device)
    _arg(out, torch.float32, (views.total_pixels, 4), "out")
    if not 0 <= int(degree) <= 3:
        raise ValueError(f"SH degree {degree} outside 0..3")
    tex = sh_textures_struct(sh_textures, layers.k, degree)
    opts = C.VsShOpts(float(vmin), float(vmax), float(eps_T), int(wrap), int(degree), int(bool(view_alpha)))
    C.check(C.load().vs_render_sh(ctypes.addressof(layers.c), ctypes.addressof(tex), layers.k, ctypes.byref(views.c),
                                  vis.data_ptr(), ws.data_ptr(), ws.numel(), out.data_ptr(), ctypes.byref(opts),
                                  _stream(stream)), "vs_render_sh")
    return out


def render_backward(layers: Layers, textures, views: Views, vis: torch.Tensor, ws: torch.Tensor,
                    grad_rgba: Optional[torch.Tensor] = None, grad_tex: Optional[List[torch.Tensor]] = None,
                    target: Optional[torch.Tensor] = None, loss_scale: float = 1.0,
                    out: Optional[torch.Tensor] = None, sse: Optional[torch.Tensor] = None, wrap: int = 0,
                    loss: str = "l2", eps_T: float = 0.0, count_paths: bool = False,
                    stream=None) -> List[torch.Tensor]:
    """vs_render_backward: accumulates dL/dtexture into grad_tex (zeros if None) and returns it.
    With eps_T > 0 the layer walk stops where vs_render's does (the gradient of that image)."""
    # counts and shapes first, then devices and dtypes
    _check_textures(textures, layers.k)
    if grad_tex is not None:
        _count(grad_tex, layers.k, "grad_tex")
        for l, (g, t) in enumerate(zip(grad_tex, textures)):
            _shape(g, t.shape, f"grad_tex[{l}]")
    img = (views.total_pixels, 4)
    if grad_rgba is None and target is None:
        raise ValueError("render_backward needs grad_rgba or target")
    for name, t in (("grad_rgba", grad_rgba), ("target", target), ("out", out)):
        if t is not None:
            _shape(t, img, name)
    if sse is not None and sse.numel() < 1:
        raise ValueError("sse must hold one float64")
    _check_vis(vis, layers, views)
    _check_ws(ws)
    tex = textures_struct(textures, layers.k)
    if grad_tex is None:
        grad_tex = [torch.zeros_like(t) for t in textures]
    for l, (g, t) in enumerate(zip(grad_tex, textures)):
        _arg(g, torch.float32, t.shape, f"grad_tex[{l}]")
    for name, t in (("grad_rgba", grad_rgba), ("target", target), ("out", out)):
        if t is not None:
            _arg(t, torch.float32, img, name)
    if sse is not None:
        _dev(sse, torch.float64, "sse")
    gp = (ctypes.c_void_p * layers.k)(*[g.data_ptr() for g in grad_tex])
    opts = _shade_opts(eps_T, wrap, target, loss_scale, loss, count_paths)
    C.check(C.load().vs_render_backward(
        ctypes.addressof(layers.c), ctypes.addressof(tex), layers.k, ctypes.byref(views.c), vis.data_ptr(),
        ws.data_ptr(), ws.numel(), None if grad_rgba is None else grad_rgba.data_ptr(), ctypes.addressof(gp),
        None if out is None else out.data_ptr(), None if sse is None else sse.data_ptr(), ctypes.byref(opts),
        _stream(stream)), "vs_render_backward")
    return grad_tex


def read_status(ws: torch.Tensor, stream=None) -> dict:
    out = (ctypes.c_int64 * C.VS_STAT_COUNT)()
    C.check(C.load().vs_read_status(ws.data_ptr(), ws.numel(), ctypes.addressof(out), _stream(stream)),
            "vs_read_status")
    return {n: int(out[i]) for i, n in enumerate(C.STAT_NAMES)}


def autotune(layers: Layers, views: Views, vis: torch.Tensor, ws: torch.Tensor, cache_path: Optional[str] = None,
             count_fragments: bool = False, list_capacity: int = 0, stream=None) -> int:
    """vs_autotune: the fastest bin size for this problem (vis and ws are overwritten)."""
    opts = _raster_opts(0, count_fragments, False, list_capacity)
    C.check(C.load().vs_autotune(ctypes.addressof(layers.c), layers.k, ctypes.byref(views.c), vis.data_ptr(),
                                 ws.data_ptr(), ws.numel(), ctypes.byref(opts),
                                 None if cache_path is None else cache_path.encode(), _stream(stream)),
            "vs_autotune")
    return int(opts.bin)


def adam_step(params, grads, m, v, step: torch.Tensor, lr=1e-2, betas=(0.9, 0.999), eps=1e-8, lo=0.0, hi=1.0,
              sse: Optional[torch.Tensor] = None, history: Optional[torch.Tensor] = None, stream=None):
    """vs_adam_step: fused Adam + projection to [lo, hi] + gradient reset on k texture planes."""
    k = len(params)
    for name, arr in (("params", params), ("grads", grads), ("m", m), ("v", v)):
        _count(arr, k, name)
        for l, t in enumerate(arr):
            _arg(t, torch.float32, params[l].shape, f"{name}[{l}]")
    _dev(step, torch.int32, "step")
    if history is not None:
        _dev(history, torch.float64, "history")
    ptr = lambda arr: (ctypes.c_void_p * k)(*[t.data_ptr() for t in arr])  # noqa: E731
    counts = (ctypes.c_int64 * k)(*[t.numel() for t in params])
    opts = C.VsAdamOpts(lr, betas[0], betas[1], eps, lo, hi)
    hist_len = 0 if history is None else history.numel()
    keep = [ptr(params), ptr(grads), ptr(m), ptr(v)]
    C.check(C.load().vs_adam_step(ctypes.addressof(keep[0]), ctypes.addressof(keep[1]), ctypes.addressof(keep[2]),
                                  ctypes.addressof(keep[3]), ctypes.addressof(counts), k, ctypes.byref(opts),
                                  step.data_ptr(), None if sse is None else sse.data_ptr(),
                                  None if history is None else history.data_ptr(), hist_len, _stream(stream)),
            "vs_adam_step")


def squeeze(params, tex, levels: int = 255, stream=None):
    """vs_squeeze: tex = q(sigmoid(params)) (q: rounding to levels steps; 0 = none)."""
    k = len(params)
    for name, arr in (("params", params), ("tex", tex)):
        _count(arr, k, name)
        for l, t in enumerate(arr):
            _arg(t, torch.float32, params[l].shape, f"{name}[{l}]")
    keep = [(ctypes.c_void_p * k)(*[t.data_ptr() for t in a]) for a in (params, tex)]
    counts = (ctypes.c_int64 * k)(*[t.numel() for t in params])
    C.check(C.load().vs_squeeze(ctypes.addressof(keep[0]), ctypes.addressof(keep[1]), ctypes.addressof(counts), k,
                                int(levels), _stream(stream)), "vs_squeeze")


def adam_step_squeezed(params, grads, m, v, tex, step: torch.Tensor, levels: int = 255, lr=1e-2, betas=(0.9, 0.999),
                       eps=1e-8, sse: Optional[torch.Tensor] = None, history: Optional[torch.Tensor] = None,
                       stream=None):
    """vs_adam_step_squeezed: Adam on logits (straight-through quantiser), tex rewritten, gradient reset."""
    k = len(params)
    for name, arr in (("params", params), ("grads", grads), ("m", m), ("v", v), ("tex", tex)):
        _count(arr, k, name)
        for l, t in enumerate(arr):
            _arg(t, torch.float32, params[l].shape, f"{name}[{l}]")
    _dev(step, torch.int32, "step")
    if history is not None:
        _dev(history, torch.float64, "history")
    keep = [(ctypes.c_void_p * k)(*[t.data_ptr() for t in a]) for a in (params, grads, m, v, tex)]
    counts = (ctypes.c_int64 * k)(*[t.numel() for t in params])
    opts = C.VsAdamOpts(lr, betas[0], betas[1], eps, 0.0, 0.0)
    hist_len = 0 if history is None else history.numel()
    C.check(C.load().vs_adam_step_squeezed(*[ctypes.addressof(a) for a in keep], ctypes.addressof(counts), k,
                                           int(levels), ctypes.byref(opts), step.data_ptr(),
                                           None if sse is None else sse.data_ptr(),
                                           None if history is None else history.data_ptr(), hist_len,
                                           _stream(stream)), "vs_adam_step_squeezed")


class NgpConfig:
    """Neural texture shape: per-level grid resolutions and the hash-table size 2^log2_table."""

    def __init__(self, resolutions: Sequence[int], log2_table: int):
        if not 1 <= len(resolutions) <= 16:
            raise ValueError("1..16 levels")
        self.resolutions = [int(r) for r in resolutions]
        self.log2_table = int(log2_table)
        self.c = C.VsNgpConfig(len(self.resolutions), self.log2_table,
                               (ctypes.c_int32 * 16)(*(self.resolutions + [0] * (16 - len(self.resolutions)))))
        self.param_count = int(C.load().vs_ngp_param_count(ctypes.byref(self.c)))
        if self.param_count < 0:
            raise ValueError("invalid neural texture configuration: " + C.load().vs_last_error().decode())


def _sizes(textures_hw):
    k = len(textures_hw)
    return (ctypes.c_int32 * k)(*[int(w) for w, h in textures_hw]), (ctypes.c_int32 * k)(*[int(h) for w, h in textures_hw])


def ngp_bake(params, cfg: NgpConfig, sizes, tex=None, ws: Optional[torch.Tensor] = None, stream=None):
    """vs_ngp_bake: RGBA textures [H, W, 4] of the neural textures params[l] at sizes[l] = (W, H);
    with ws (ngp_workspace) the activations are kept for ngp_backward."""
    k = len(params)
    _count(sizes, k, "sizes")
    for l, p in enumerate(params):
        _shape(_dev(p, torch.float32, f"params[{l}]"), (cfg.param_count,), f"params[{l}]")
    if tex is None:
        tex = [torch.empty(h, w, 4, dtype=torch.float32, device=params[0].device) for w, h in sizes]
    _count(tex, k, "tex")
    for l, (t, (w, h)) in enumerate(zip(tex, sizes)):
        _arg(t, torch.float32, (h, w, 4), f"tex[{l}]")
    if ws is not None:
        _check_ws(ws)
    ws_, hs_ = _sizes(sizes)
    keep = [(ctypes.c_void_p * k)(*[t.data_ptr() for t in a]) for a in (params, tex)]
    C.check(C.load().vs_ngp_bake(ctypes.addressof(keep[0]), ctypes.byref(cfg.c), k, ctypes.addressof(ws_),
                                 ctypes.addressof(hs_), ctypes.addressof(keep[1]),
                                 None if ws is None else ws.data_ptr(), 0 if ws is None else ws.numel(),
                                 _stream(stream)), "vs_ngp_bake")
    return tex


def ngp_workspace(cfg: NgpConfig, sizes, device="cuda") -> torch.Tensor:
    ws_, hs_ = _sizes(sizes)
    n = int(C.load().vs_ngp_workspace_bytes(ctypes.byref(cfg.c), len(sizes), ctypes.addressof(ws_),
                                            ctypes.addressof(hs_)))
    return torch.empty(max(n, 256), dtype=torch.uint8, device=device)


def ngp_backward(params, cfg: NgpConfig, sizes, tex, grad_tex, ws: torch.Tensor, grad_params=None, stream=None):
    """vs_ngp_backward of the last ngp_bake given ws (with the same params and textures tex):
    accumulates dL/dparams (zeros if None) from dL/dtexture and returns it."""
    k = len(params)
    _count(sizes, k, "sizes")
    if grad_params is None:
        grad_params = [torch.zeros_like(p) for p in params]
    for name, arr in (("params", params), ("tex", tex), ("grad_tex", grad_tex), ("grad_params", grad_params)):
        _count(arr, k, name)
        for l, t in enumerate(arr):
            w, h = sizes[l]
            want = (cfg.param_count,) if name in ("params", "grad_params") else (h, w, 4)
            _arg(t, torch.float32, want, f"{name}[{l}]")
    _check_ws(ws)
    ws_, hs_ = _sizes(sizes)
    keep = [(ctypes.c_void_p * k)(*[t.data_ptr() for t in a]) for a in (params, tex, grad_tex, grad_params)]
    C.check(C.load().vs_ngp_backward(ctypes.addressof(keep[0]), ctypes.byref(cfg.c), k, ctypes.addressof(ws_),
                                     ctypes.addressof(hs_), ctypes.addressof(keep[1]), ctypes.addressof(keep[2]),
                                     ctypes.addressof(keep[3]), ws.data_ptr(), ws.numel(), _stream(stream)),
            "vs_ngp_backward")
    return grad_params


class KsdfField:
    """k-SDF fields on device: SDF grid f32 [(R+1)^3] and RGBA grid f32 [(Ra+1)^3, 4] over the cube [lo, hi]^3."""

    def __init__(self, sdf: torch.Tensor, sdf_res: int, rgba: torch.Tensor, rgba_res: int, lo: float, hi: float):
        self.sdf = _dev(sdf, torch.float32, "sdf")
        self.rgba = _dev(rgba, torch.float32, "rgba")
        if self.sdf.numel() != (sdf_res + 1) ** 3 or self.rgba.numel() != 4 * (rgba_res + 1) ** 3:
            raise ValueError("grid sizes do not match the resolutions")
        self.c = C.VsKsdfField(self.sdf.data_ptr(), self.rgba.data_ptr(), int(sdf_res), int(rgba_res), float(lo),
                               float(hi))


def ksdf_opts(offsets, beta: float, occ_threshold: float = 1e-4, occ_res: int = 256, n_uniform: int = 64,
              n_importance: int = 32, march_steps: int = 1024, pdf_floor: float = 1e-5) -> C.VsKsdfOpts:
    offs = [float(o) for o in offsets]
    if not 1 <= len(offs) <= 16:
        raise ValueError("1..16 surfaces")
    return C.VsKsdfOpts(len(offs), (ctypes.c_double * 16)(*(offs + [0.0] * (16 - len(offs)))), float(beta),
                        float(occ_threshold), int(occ_res), int(n_uniform), int(n_importance), int(march_steps),
                        float(pdf_floor))


def ksdf_occupancy(field: KsdfField, opts: C.VsKsdfOpts, occ: Optional[torch.Tensor] = None, stream=None):
    """vs_ksdf_occupancy: the occupancy bit grid (int32 words; bit i & 31 of word i >> 5)."""
    words = int(C.load().vs_ksdf_occupancy_words(opts.occ_res))
    if occ is None:
        occ = torch.empty(max(words, 1), dtype=torch.int32, device=field.sdf.device)
    _dev(occ, torch.int32, "occ")
    if occ.numel() < words:
        raise ValueError("occ too small")
    C.check(C.load().vs_ksdf_occupancy(ctypes.byref(field.c), ctypes.byref(opts), occ.data_ptr(), _stream(stream)),
            "vs_ksdf_occupancy")
    return occ


def ksdf_render(field: KsdfField, opts: C.VsKsdfOpts, occ: torch.Tensor, views: Views, out=None,
                layers: bool = False, samples: bool = False, stream=None):
    """vs_ksdf_render: RGBA [total pixels, 4]; optionally per-surface (C_j, A_j) [k, total, 4] and the final
    sample parameters [total, n_uniform + n_importance] (f64)."""
    total = views.total_pixels
    dev = field.sdf.device
    if out is None:
        out = torch.empty(total, 4, dtype=torch.float32, device=dev)
    _arg(out, torch.float32, (total, 4), "out")
    lay = torch.empty(opts.k, total, 4, dtype=torch.float32, device=dev) if layers else None
    smp = torch.empty(total, opts.n_uniform + opts.n_importance, dtype=torch.float64, device=dev) if samples else None
    _dev(occ, torch.int32, "occ")
    if occ.numel() < int(C.load().vs_ksdf_occupancy_words(opts.occ_res)):
        raise ValueError("occ too small for occ_res")
    C.check(C.load().vs_ksdf_render(ctypes.byref(field.c), ctypes.byref(opts), occ.data_ptr(), ctypes.byref(views.c),
                                    out.data_ptr(), None if lay is None else lay.data_ptr(),
                                    None if smp is None else smp.data_ptr(), _stream(stream)), "vs_ksdf_render")
    if layers or samples:
        return out, lay, smp
    return out


class Graph:
    """A HIP graph captured from calls into the library on one (non-default) stream."""

    def __init__(self, stream: torch.cuda.Stream):
        self.stream = stream
        self.handle = ctypes.c_void_p()

    def __enter__(self):
        C.check(C.load().vs_graph_begin(_stream(self.stream)), "vs_graph_begin")
        return self

    def __exit__(self, exc_type, exc, tb):
        h = ctypes.c_void_p()
        st = C.load().vs_graph_end(_stream(self.stream), ctypes.byref(h))
        if exc_type is None:
            C.check(st, "vs_graph_end")
        self.handle = h
        return False

    def replay(self):
        C.check(C.load().vs_graph_launch(self.handle, _stream(self.stream)), "vs_graph_launch")

    def __del__(self):
        try:
            if self.handle:
                C.load().vs_graph_destroy(self.handle)
        except Exception:
            pass


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, renderer, *textures):
        ctx.renderer = renderer
        ctx.save_for_backward(*textures)
        return render(renderer.layers, textures, renderer.views, renderer.vis, renderer.ws,
                      eps_T=renderer.eps_T, wrap=renderer.wrap)

    @staticmethod
    def backward(ctx, grad_out):
        r = ctx.renderer
        textures = ctx.saved_tensors
        grads = render_backward(r.layers, textures, r.views, r.vis, r.ws, grad_rgba=grad_out.contiguous(),
                                wrap=r.wrap, eps_T=r.eps_T)
        return (None, *grads)


class Renderer:
    """A fixed scene (meshes + cameras): rasterised once, then differentiable in the textures.

    Geometry and cameras receive no gradient: textures are fit on fixed meshes.
    """

    def __init__(self, meshes, cameras, device="cuda", bin: int = 0, eps_T: float = 0.0, wrap: int = 0):
        self.layers = meshes if isinstance(meshes, Layers) else Layers(meshes, device)
        self.views = cameras if isinstance(cameras, Views) else Views(cameras, device)
        self.eps_T, self.wrap, self.bin = eps_T, wrap, bin
        self.vis, self.ws = raster(self.layers, self.views, bin=bin)

    def rasterize(self):
        raster(self.layers, self.views, self.vis, self.ws, bin=self.bin)
        return self.vis

    def __call__(self, *textures: torch.Tensor) -> torch.Tensor:
        _count(textures, self.layers.k, "textures")
        return _RenderFn.apply(self, *textures)

    def status(self) -> dict:
        return read_status(self.ws)

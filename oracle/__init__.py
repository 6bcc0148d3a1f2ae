"""FP64 CPU oracle for the layered-mesh renderer -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it, and it shares no code
with them: it consumes the seeded inputs of ``scenes`` only.

The C++ source is ``oracle/vs_oracle.cpp``; this module is a ctypes wrapper
around it (argument marshalling only).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vs_oracle.cpp")
# VS_ORACLE_LIB names another build of the same source (the sanitizer test loads an instrumented one)
_LIB = os.environ.get("VS_ORACLE_LIB") or os.path.join(_HERE, "libvs_oracle.so")
EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)

CXXFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fno-finite-math-only",
            "-shared", "-fPIC", "-Wall", "-Werror"]


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (strict IEEE, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", *CXXFLAGS, _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _Cam(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("R", ctypes.c_double * 9), ("t", ctypes.c_double * 3), ("z_near", ctypes.c_double)]


class _Layer(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_void_p), ("uv", ctypes.c_void_p), ("tri", ctypes.c_void_p),
                ("n_vert", ctypes.c_int32), ("n_tri", ctypes.c_int32),
                ("tex", ctypes.c_void_p), ("tex_w", ctypes.c_int32), ("tex_h", ctypes.c_int32)]


class _ShLayer(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.vso_camera_bytes.restype = ctypes.c_int
        L.vso_layer_bytes.restype = ctypes.c_int
        L.vso_project.argtypes = [vp, i32, vp, vp, vp, vp, vp]
        L.vso_raster.argtypes = [vp, vp, ctypes.c_int, vp, vp]
        L.vso_coverage.argtypes = [vp, vp, vp, vp]
        L.vso_shade.argtypes = [i32, vp, vp, vp, ctypes.c_int, vp, vp, vp]
        L.vso_backward.argtypes = [i32, vp, vp, vp, ctypes.c_int, vp, vp, ctypes.c_int, vp]
        L.vso_fd.argtypes = [i32, vp, vp, vp, ctypes.c_int, vp, vp, ctypes.c_int, i32, vp, dbl, vp]
        L.vso_sh_basis.argtypes = [vp, vp]
        L.vso_sh_layer_bytes.restype = ctypes.c_int
        L.vso_shade_sh.argtypes = [i32, vp, vp, vp, vp, ctypes.c_int, dbl, dbl, ctypes.c_int, ctypes.c_int, vp]
        for f in ("vso_raster", "vso_coverage", "vso_shade", "vso_backward", "vso_fd", "vso_shade_sh"):
            getattr(L, f).restype = ctypes.c_int
        assert L.vso_camera_bytes() == ctypes.sizeof(_Cam), "camera layout mismatch"
        assert L.vso_layer_bytes() == ctypes.sizeof(_Layer), "layer layout mismatch"
        assert L.vso_sh_layer_bytes() == ctypes.sizeof(_ShLayer), "SH layer layout mismatch"
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _cam(c) -> _Cam:
    cc = _Cam()
    cc.width, cc.height = int(c.width), int(c.height)
    cc.fx, cc.fy, cc.cx, cc.cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
    R = np.asarray(c.R, np.float64).reshape(9)
    t = np.asarray(c.t, np.float64).reshape(3)
    for q in range(9):
        cc.R[q] = float(R[q])
    for q in range(3):
        cc.t[q] = float(t[q])
    cc.z_near = float(c.z_near)
    return cc


class _Layers:
    """Keeps contiguous copies alive while C holds raw pointers."""

    def __init__(self, meshes, textures=None):
        self.keep = []
        n = len(meshes)
        self.arr = (_Layer * n)()
        for l, m in enumerate(meshes):
            xyz = np.ascontiguousarray(m.xyz, np.float32)
            uv = np.ascontiguousarray(m.uv, np.float32)
            tri = np.ascontiguousarray(m.tri, np.int32)
            self.keep += [xyz, uv, tri]
            L = self.arr[l]
            L.xyz, L.uv, L.tri = xyz.ctypes.data, uv.ctypes.data, tri.ctypes.data
            L.n_vert, L.n_tri = xyz.shape[0], tri.shape[0]
            if textures is not None:
                tex = np.ascontiguousarray(textures[l], np.float32)
                self.keep.append(tex)
                L.tex = tex.ctypes.data
                L.tex_h, L.tex_w = tex.shape[0], tex.shape[1]

    def ptr(self, l: int = 0):
        return ctypes.cast(ctypes.byref(self.arr, l * ctypes.sizeof(_Layer)), ctypes.c_void_p)


def project(mesh, cam):
    """Step 1: (X, Y) in 1/256 px, w = 1/z, valid flag per vertex."""
    n = mesh.xyz.shape[0]
    X = np.empty(n, np.int64); Y = np.empty(n, np.int64); w = np.empty(n, np.float64); v = np.empty(n, np.uint8)
    xyz = np.ascontiguousarray(mesh.xyz, np.float32)
    cc = _cam(cam)
    lib().vso_project(_ptr(xyz), n, ctypes.byref(cc), _ptr(X), _ptr(Y), _ptr(w), _ptr(v))
    return X, Y, w, v.astype(bool)


def raster(mesh, cam, mode: str = "bbox"):
    """Visibility plane [H, W] u64 for one mesh and one view, plus cull stats."""
    L = _Layers([mesh])
    cc = _cam(cam)
    vis = np.empty((cam.height, cam.width), np.uint64)
    st = np.zeros(4, np.int64)
    lib().vso_raster(L.ptr(), ctypes.byref(cc), 0 if mode == "brute" else 1, _ptr(vis), _ptr(st))
    return vis, {"culled_invalid": int(st[0]), "culled_degenerate": int(st[1]), "bad_index": int(st[2]),
                 "fragments": int(st[3])}


def raster_layers(meshes, cam, mode: str = "bbox"):
    """[k, H, W] visibility planes of one view."""
    return np.stack([raster(m, cam, mode)[0] for m in meshes], 0)


def coverage(mesh, cam):
    L = _Layers([mesh])
    cc = _cam(cam)
    pos = np.empty((cam.height, cam.width), np.int32)
    neg = np.empty((cam.height, cam.width), np.int32)
    lib().vso_coverage(L.ptr(), ctypes.byref(cc), _ptr(pos), _ptr(neg))
    return pos, neg


def shade(meshes, textures, cam, vis, wrap: int = 0, debug: bool = False):
    """[H, W, 4] f64 RGBA of one view (A = 1 - T); with debug also barycentrics and UVs."""
    k = len(meshes)
    L = _Layers(meshes, textures)
    cc = _cam(cam)
    vis = np.ascontiguousarray(vis, np.uint64)
    out = np.empty((cam.height, cam.width, 4), np.float64)
    lam = np.empty((k, cam.height, cam.width, 3)) if debug else None
    uvo = np.empty((k, cam.height, cam.width, 2)) if debug else None
    err = lib().vso_shade(k, L.ptr(), ctypes.byref(cc), _ptr(vis), wrap, _ptr(out), _ptr(lam), _ptr(uvo))
    if err:
        raise RuntimeError("oracle: visibility key names an invalid triangle")
    return (out, lam, uvo) if debug else out


_LOSSES = {"l2": 0, "l1": 1}


def backward(meshes, textures, cam, vis, grad_out=None, target=None, wrap: int = 0, loss: str = "l2") -> List[np.ndarray]:
    """Analytic texture gradient (f64, one array per layer) of one view.

    With a target the loss is sum_p ||RGB_p - target_p||^2 (loss="l2") or sum_p |RGB_p - target_p|_1
    (loss="l1"); otherwise sum_p <grad_out_p, out_p>."""
    k = len(meshes)
    L = _Layers(meshes, textures)
    cc = _cam(cam)
    vis = np.ascontiguousarray(vis, np.uint64)
    grads = [np.zeros(np.asarray(t).shape, np.float64) for t in textures]
    gp = (ctypes.c_void_p * k)(*[g.ctypes.data for g in grads])
    go = None if grad_out is None else np.ascontiguousarray(grad_out, np.float64)
    tg = None if target is None else np.ascontiguousarray(target, np.float32)
    err = lib().vso_backward(k, L.ptr(), ctypes.byref(cc), _ptr(vis), wrap, _ptr(go), _ptr(tg), _LOSSES[loss], gp)
    if err:
        raise RuntimeError("oracle: visibility key names an invalid triangle")
    return grads


def finite_diff(meshes, textures, cam, vis, entries, h: float = 1e-3, grad_out=None, target=None,
                wrap: int = 0, loss: str = "l2") -> np.ndarray:
    """Central FD (FP64) of the loss w.r.t. texel scalars entries[n] = (layer, j, i, ch)."""
    k = len(meshes)
    L = _Layers(meshes, textures)
    cc = _cam(cam)
    vis = np.ascontiguousarray(vis, np.uint64)
    ent = np.ascontiguousarray(entries, np.int32).reshape(-1, 4)
    out = np.empty(ent.shape[0], np.float64)
    go = None if grad_out is None else np.ascontiguousarray(grad_out, np.float64)
    tg = None if target is None else np.ascontiguousarray(target, np.float32)
    err = lib().vso_fd(k, L.ptr(), ctypes.byref(cc), _ptr(vis), wrap, _ptr(go), _ptr(tg), _LOSSES[loss], ent.shape[0],
                       _ptr(ent), float(h), _ptr(out))
    if err:
        raise RuntimeError("oracle: visibility key names an invalid triangle")
    return out


def render(meshes, textures, cam, wrap: int = 0, mode: str = "bbox"):
    """Visibility [k, H, W] and image [H, W, 4] of one view."""
    vis = raster_layers(meshes, cam, mode)
    return vis, shade(meshes, textures, cam, vis, wrap)


# ----------------------------------------------------------------------------- baked SH appearance
def sh_basis(d) -> np.ndarray:
    """Real orthonormal spherical harmonics (degree <= 3, 16 values) of unit directions d [..., 3]."""
    d = np.ascontiguousarray(d, np.float64).reshape(-1, 3)
    out = np.empty((d.shape[0], 16), np.float64)
    for n in range(d.shape[0]):
        lib().vso_sh_basis(_ptr(d[n]), out[n].ctypes.data_as(ctypes.c_void_p))
    return out


def shade_sh(meshes, sh_textures, cam, vis, degree: int = 3, vmin: float = -15.0, vmax: float = 15.0,
             wrap: int = 0, view_alpha: bool = True):
    """[H, W, 4] f64 RGBA of one view under the baked SH appearance.

    sh_textures[l] has .data (uint8, packed levels), .width and .height (level 0)."""
    k = len(meshes)
    L = _Layers(meshes)
    keep = [np.ascontiguousarray(t.data, np.uint8) for t in sh_textures]
    S = (_ShLayer * k)(*[_ShLayer(a.ctypes.data, t.width, t.height) for a, t in zip(keep, sh_textures)])
    cc = _cam(cam)
    vis = np.ascontiguousarray(vis, np.uint64)
    out = np.empty((cam.height, cam.width, 4), np.float64)
    err = lib().vso_shade_sh(k, L.ptr(), S, ctypes.byref(cc), _ptr(vis), int(degree), float(vmin), float(vmax),
                             int(wrap), int(bool(view_alpha)), _ptr(out))
    if err:
        raise RuntimeError("oracle: visibility key names an invalid triangle" if err == 1 else "oracle: bad degree")
    return out


# ----------------------------------------------------------------------------- squeezing and quantisation
def squeeze_quantize(theta, levels: int = 255) -> np.ndarray:
    """Texture from logits (Sec. 4.3 "Squeezing and Quantization"): q(sigmoid(theta)),
    q(x) = round(levels x) / levels with ties to even, decided in FP64; levels = 0: no quantisation."""
    s = 1.0 / (1.0 + np.exp(-np.asarray(theta, np.float64)))
    if levels:
        s = np.rint(levels * s) / levels
    return s.astype(np.float32)

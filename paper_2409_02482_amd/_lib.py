"""ctypes view of the C ABI in include/vs.h (argument marshalling only).

Loading fails loudly if the HIP library has not been built: there is no CPU
fallback anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# VS_LIB names another build of the same sources (the sanitizer test loads one with instrumented host code)
LIB_PATH = os.environ.get("VS_LIB") or os.path.join(_HERE, "libvs.so")

c_vp, c_i32, c_i64, c_f32, c_f64, c_sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float,
                                          ctypes.c_double, ctypes.c_size_t)

VS_OK, VS_ERR_ARG, VS_ERR_SIZE, VS_ERR_WORKSPACE, VS_ERR_HIP, VS_ERR_UNSUPPORTED = range(6)
VS_MAX_LAYERS = 16
VS_EMPTY = 0xFFFFFFFFFFFFFFFF
VS_RASTER_COUNT_FRAGMENTS = 1
VS_RASTER_DIRECT = 2
STAT_NAMES = ["culled_invalid", "culled_degenerate", "bad_index", "fragments", "bad_key", "bin_overflow",
              "scatter_wave", "scatter_half", "scatter_quarter", "scatter_direct"]
VS_STAT_COUNT = 10
VS_SHADE_COUNT_PATHS = 1
VS_NOALLOC_SCRATCH_BYTES = 64 << 20


class VsMesh(ctypes.Structure):
    _fields_ = [("xyz", c_vp), ("uv", c_vp), ("tri", c_vp), ("n_vert", c_i32), ("n_tri", c_i32)]


class VsTexture(ctypes.Structure):
    _fields_ = [("rgba", c_vp), ("width", c_i32), ("height", c_i32)]


class VsCamera(ctypes.Structure):
    _fields_ = [("width", c_i32), ("height", c_i32), ("fx", c_f64), ("fy", c_f64), ("cx", c_f64), ("cy", c_f64),
                ("R", c_f64 * 9), ("t", c_f64 * 3), ("z_near", c_f64)]


class VsView(ctypes.Structure):
    _fields_ = [("cam", VsCamera), ("pix_offset", c_i64), ("tile_offset", c_i64 * 4)]


class VsViews(ctypes.Structure):
    _fields_ = [("host", c_vp), ("dev", c_vp), ("n_views", c_i32)]


class VsRasterOpts(ctypes.Structure):
    _fields_ = [("bin", c_i32), ("flags", c_i32), ("list_capacity", c_i64)]


class VsAdamOpts(ctypes.Structure):
    _fields_ = [("lr", c_f32), ("beta1", c_f32), ("beta2", c_f32), ("eps", c_f32), ("lo", c_f32), ("hi", c_f32)]


class VsShadeOpts(ctypes.Structure):
    _fields_ = [("eps_T", c_f32), ("wrap", c_i32), ("target", c_vp), ("loss_scale", c_f32), ("loss", c_i32),
                ("flags", c_i32)]


VS_LOSS = {"l2": 0, "l1": 1}


class VsShTexture(ctypes.Structure):
    _fields_ = [("data", c_vp), ("width", c_i32), ("height", c_i32)]


class VsShOpts(ctypes.Structure):
    _fields_ = [("vmin", c_f32), ("vmax", c_f32), ("eps_T", c_f32), ("wrap", c_i32), ("degree", c_i32),
                ("view_alpha", c_i32)]


class VsNgpConfig(ctypes.Structure):
    _fields_ = [("levels", c_i32), ("log2_table", c_i32), ("resolution", c_i32 * 16)]


class VsKsdfField(ctypes.Structure):
    _fields_ = [("sdf", c_vp), ("rgba", c_vp), ("sdf_res", c_i32), ("rgba_res", c_i32), ("lo", c_f64), ("hi", c_f64)]


class VsKsdfOpts(ctypes.Structure):
    _fields_ = [("k", c_i32), ("offsets", c_f64 * 16), ("beta", c_f64), ("occ_threshold", c_f64),
                ("occ_res", c_i32), ("n_uniform", c_i32), ("n_importance", c_i32), ("march_steps", c_i32),
                ("pdf_floor", c_f64)]


# name -> (restype, argtypes); every symbol declared in include/vs.h
SIGNATURES = {
    "vs_version": (ctypes.c_char_p, []),
    "vs_last_error": (ctypes.c_char_p, []),
    "vs_status_string": (ctypes.c_char_p, [c_i32]),
    "vs_views_prepare": (c_i32, [c_vp, c_i32, c_vp]),
    "vs_raster_workspace_bytes": (c_sz, [c_vp, c_i32, c_vp, c_vp]),
    "vs_raster_layers": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_sz, c_vp, c_vp]),
    "vs_render": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_sz, c_vp, c_vp, c_vp]),
    "vs_render_noalloc": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "vs_render_sh": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_sz, c_vp, c_vp, c_vp]),
    "vs_render_backward": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_sz, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "vs_read_status": (c_i32, [c_vp, c_sz, c_vp, c_vp]),
    "vs_autotune": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_sz, c_vp, ctypes.c_char_p, c_vp]),
    "vs_adam_step": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_i32, c_vp]),
    "vs_squeeze": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_i32, c_vp]),
    "vs_adam_step_squeezed": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp, c_i32,
                                      c_vp]),
    "vs_ngp_param_count": (ctypes.c_int64, [c_vp]),
    "vs_ngp_workspace_bytes": (c_sz, [c_vp, c_i32, c_vp, c_vp]),
    "vs_ngp_bake": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "vs_ngp_backward": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "vs_ksdf_occupancy_words": (ctypes.c_int64, [c_i32]),
    "vs_ksdf_occupancy": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "vs_ksdf_render": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "vs_graph_begin": (c_i32, [c_vp]),
    "vs_graph_end": (c_i32, [c_vp, c_vp]),
    "vs_graph_launch": (c_i32, [c_vp, c_vp]),
    "vs_graph_destroy": (c_i32, [c_vp]),
}

_lib = None


class VsError(RuntimeError):
    def __init__(self, status: int, what: str, msg: str):
        super().__init__(f"{what}: status {status}: {msg}")
        self.status = status


def load(path: str = LIB_PATH):
    """Load libvs.so (built by paper_2409_02482_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"HIP library {path} is not built; run `python -c 'import __graft_entry__ as g; "
                               f"g.build()'` (hipcc --offload-arch=gfx950)")
        L = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status: int, what: str):
    if status != VS_OK:
        msg = load().vs_last_error().decode(errors="replace")
        raise VsError(status, what, msg)

"""MI355X (gfx950) renderer for layered semi-transparent textured mesh shells.

Hot path of Volumetric Surfaces (arXiv 2409.02482): fixed-order, sorting-free
rendering of k nested UV-textured mesh shells and its texture adjoint, baked
SH appearance, quantisation-aware and neural-texture fitting, and the k-SDF
volume-rendering forward of the implicit stage, as hand-written HIP kernels
behind a C ABI (include/vs.h).
"""
from ._lib import LIB_PATH, VsError, load  # noqa: F401
from .binding import (Graph, KsdfField, Layers, NgpConfig, Renderer, Views, adam_step,  # noqa: F401
                     adam_step_squeezed, alloc_workspace, autotune, ksdf_occupancy, ksdf_opts, ksdf_render,
                     ngp_backward, ngp_bake, ngp_workspace, raster, read_status, render, render_backward,
                     render_noalloc, render_sh,
                     squeeze, workspace_bytes)

__all__ = ["Layers", "Views", "Renderer", "raster", "render", "render_backward", "render_noalloc", "render_sh", "read_status",
           "workspace_bytes", "alloc_workspace", "autotune", "adam_step", "adam_step_squeezed", "squeeze",
           "NgpConfig", "ngp_bake", "ngp_backward", "ngp_workspace", "KsdfField", "ksdf_opts", "ksdf_occupancy",
           "ksdf_render", "Graph",
           "load", "VsError", "LIB_PATH"]

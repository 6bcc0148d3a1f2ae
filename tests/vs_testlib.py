"""Shared helpers for the GPU parity tests: run the HIP path and the oracle on the same seeded inputs."""
from __future__ import annotations

import sys

import numpy as np

import scenes as S

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)

# tolerances: FP32 shading after FP64 texel coordinates, FP32 atomics for gradients
COLOUR_ATOL = 1e-5          # max-abs per channel vs the FP64 oracle
GRAD_RTOL = 1e-4            # ||g - g_ref||_inf / ||g_ref||_inf


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_render(scene, textures=None, bin=0, eps_T=0.0, wrap=0, count_fragments=False, direct=False,
               list_capacity=0):
    """Raster + render on the GPU. Returns (P, layers, views, vis, ws, rgba, textures_t)."""
    import torch
    import paper_2409_02482_amd as P
    layers = P.Layers(scene.layers)
    views = P.Views(scene.cameras)
    tex = [torch.from_numpy(np.ascontiguousarray(t)).cuda() for t in (textures or scene.textures)]
    vis, ws = P.raster(layers, views, bin=bin, count_fragments=count_fragments, direct=direct,
                       list_capacity=list_capacity)
    rgba = P.render(layers, tex, views, vis, ws, eps_T=eps_T, wrap=wrap)
    torch.cuda.synchronize()
    return P, layers, views, vis, ws, rgba, tex


def vis_numpy(views, vis, k, v):
    return views.vis_planes(vis, k, v).cpu().numpy().view(np.uint64)


def oracle_vis(scene, views, vis, v):
    """The oracle's own visibility of view v, asserted equal to the GPU's buffer first.

    The oracle's shading, adjoint and finite differences then run on the oracle's own rasterisation:
    no input of the oracle ever comes from the HIP path."""
    import oracle as O
    want = O.raster_layers(scene.layers, scene.cameras[v])
    assert_vis_equal(vis_numpy(views, vis, scene.k, v), want, f"view {v}")
    return want


def img_numpy(views, rgba, v):
    return views.image(rgba, v).cpu().numpy().astype(np.float64)


def assert_vis_equal(got, want, what=""):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        l, j, i = bad[0]
        raise AssertionError(f"{what}: {bad.shape[0]} visibility slots differ; first at layer {l} pixel "
                             f"({i},{j}): gpu {int(got[l, j, i]):#x} oracle {int(want[l, j, i]):#x}")


def assert_colour_close(got, want, what=""):
    err = np.abs(got - want).max()
    assert err <= COLOUR_ATOL, f"{what}: colour max-abs error {err:.3e} > {COLOUR_ATOL}"
    return err


def grad_rel_err(got, want):
    num = max(np.abs(g - w).max() for g, w in zip(got, want))
    den = max(np.abs(w).max() for w in want)
    return num / den


def pick_entries(rng, grads, n):
    """n (layer, j, i, ch) entries drawn among those with a non-zero reference gradient."""
    out = []
    k = len(grads)
    nz = [np.argwhere(np.abs(g) > 0) for g in grads]
    while len(out) < n:
        l = int(rng.integers(0, k))
        if nz[l].shape[0] == 0:
            continue
        j, i, ch = nz[l][rng.integers(0, nz[l].shape[0])]
        out.append((l, int(j), int(i), int(ch)))
    return np.array(out, np.int32)


def small_mixed_scene(k=3, n_lat=60, n_lon=120, sizes=((96, 80), (37, 53), (128, 128), (17, 300)), tex=64,
                      config=90):
    """A small scene with ragged view sizes (not multiples of any tile) for batched tests."""
    layers = S.displaced_shells(2, k, n_lat, n_lon)
    textures = [S.smooth_texture(config, l, tex, tex, opaque=(l == k - 1)) for l in range(k)]
    cams = S.ring_cameras(config, len(sizes), list(sizes))
    return S.Scene("small-mixed", layers, textures, cams)

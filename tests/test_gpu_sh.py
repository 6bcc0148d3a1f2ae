"""GPU parity of the baked spherical-harmonic appearance (vs_render_sh) against the FP64 oracle.

Bar: colour within 1e-5 max-abs per channel (visibility is the same bit-exact
buffer as for RGBA textures).  Cases: every SH degree, with and without the
grazing-angle alpha weight, repeat and clamp, ragged views, degenerate level
sizes (levels of one texel), the paper's 2048^2 mixed-resolution textures on
the full-size k = 7 scene, and the early-exit error bound.
"""
import numpy as np
import pytest

import oracle as O
import scenes as S
from vs_testlib import COLOUR_ATOL, assert_colour_close, img_numpy, oracle_vis, say, small_mixed_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    import paper_2409_02482_amd as P
    P.load()
    return torch


def _sh_render(scene, sh, degree=3, view_alpha=True, wrap=0, eps_T=0.0, vmin=-15.0, vmax=15.0):
    import torch
    import paper_2409_02482_amd as P
    layers, views = P.Layers(scene.layers), P.Views(scene.cameras)
    vis, ws = P.raster(layers, views)
    dev = [(torch.from_numpy(t.data).cuda(), t.width, t.height) for t in sh]
    out = P.render_sh(layers, dev, views, vis, ws, degree=degree, vmin=vmin, vmax=vmax, view_alpha=view_alpha,
                      eps_T=eps_T, wrap=wrap)
    torch.cuda.synchronize()
    st = P.read_status(ws)
    assert st["bad_key"] == 0 and st["culled_invalid"] == 0, st
    return views, vis, out


def _check(scene, sh, what, views_to_check=None, **kw):
    say(f"[gpu] sh {what}: {len(scene.cameras)} views k={scene.k}")
    views, vis, out = _sh_render(scene, sh, **kw)
    worst = 0.0
    for v in (views_to_check if views_to_check is not None else range(len(scene.cameras))):
        cam = scene.cameras[v]
        visn = oracle_vis(scene, views, vis, v)
        want = O.shade_sh(scene.layers, sh, cam, visn, degree=kw.get("degree", 3), vmin=kw.get("vmin", -15.0),
                          vmax=kw.get("vmax", 15.0), wrap=kw.get("wrap", 0), view_alpha=kw.get("view_alpha", True))
        worst = max(worst, assert_colour_close(img_numpy(views, out, v), want, f"sh {what} view {v}"))
    say(f"[gpu] sh {what}: colour err {worst:.2e}")
    return worst


def _sh_set(scene_k, sizes, degree=3, config=70):
    return [S.sh_texture(config, l, w, h, degree=degree, opaque=(l == scene_k - 1)) for l, (w, h) in enumerate(sizes)]


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
@pytest.mark.parametrize("view_alpha", [True, False], ids=["alpha_w", "no_alpha_w"])
def test_sh_degrees_ragged_views(torch_cuda, degree, view_alpha):
    sc = small_mixed_scene(k=3, config=71)
    sh = _sh_set(3, [(64, 48), (40, 72), (32, 32)], degree=degree)
    _check(sc, sh, f"deg{degree}", degree=degree, view_alpha=view_alpha)


def test_sh_clamp_and_range(torch_cuda):
    sc = small_mixed_scene(k=3, config=72)
    sh = _sh_set(3, [(48, 48), (64, 32), (16, 80)], config=72)
    _check(sc, sh, "clamp", wrap=1)
    _check(sc, sh, "range", vmin=-4.0, vmax=6.0)


def test_sh_degenerate_levels(torch_cuda):
    """Level sizes that collapse to one texel (and odd sizes that round down)."""
    sc = small_mixed_scene(k=3, sizes=((64, 64), (17, 23)), config=73)
    sh = _sh_set(3, [(1, 1), (3, 2), (5, 9)], config=73)
    _check(sc, sh, "degenerate")
    _check(sc, sh, "degenerate clamp", wrap=1)


def test_sh_full_size_k7(torch_cuda):
    """The k = 7 shells (101,760 triangles per layer) at 1024^2 with 2048^2 mixed-resolution textures."""
    sc = S.make_config(2)
    sh = _sh_set(sc.k, [(2048, 2048)] * sc.k, config=74)
    err = _check(sc, sh, "k7 full size")
    assert err <= COLOUR_ATOL


def test_sh_early_exit_within_bound(torch_cuda):
    import torch
    sc = small_mixed_scene(k=3, config=75)
    sh = _sh_set(3, [(32, 32)] * 3, config=75)
    eps = 2.0 ** -10
    _, _, exact = _sh_render(sc, sh)
    _, _, fast = _sh_render(sc, sh, eps_T=eps)
    # stopping once T < eps drops at most eps * max|c| <= eps of colour per channel
    assert float((exact - fast).abs().max()) <= eps + 1e-6


def test_sh_full_batch_bench_launch(torch_cuda):
    """The baked-SH workload at full size in its benchmarked launch: k = 7 shells, 64 ring views at 1024^2,
    degree 3 in 8 bits with 2048^2 mixed-resolution levels, one batched raster and one vs_render_sh over all
    views, two steps over the same buffers; every view against the oracle on host threads."""
    import concurrent.futures as cf
    import os

    import torch
    import paper_2409_02482_amd as P
    say("[gpu] sh full batch: building the k = 7 scene, 64 views at 1024^2")
    sc = S.make_config(6, n_views=64, resolution=(1024, 1024), with_targets=False)
    k = sc.k
    sh = [S.sh_texture(60, l, 2048, 2048, degree=3, opaque=(l == k - 1)) for l in range(k)]
    layers, views = P.Layers(sc.layers, "cuda"), P.Views(sc.cameras, "cuda")
    sh_dev = [(torch.from_numpy(t.data).cuda(), t.width, t.height) for t in sh]
    out = torch.empty(views.total_pixels, 4, dtype=torch.float32, device="cuda")
    vis = torch.empty(k * views.total_pixels, dtype=torch.int64, device="cuda")
    ws = P.alloc_workspace(layers, views, 0, "cuda")
    for step in range(2):
        P.raster(layers, views, vis, ws, bin=0)
        P.render_sh(layers, sh_dev, views, vis, ws, degree=3, out=out)
    torch.cuda.synchronize()
    st = P.read_status(ws)
    assert st["bad_key"] == 0 and st["culled_invalid"] == 0, st
    vis_h, out_h = vis.cpu(), out.cpu()
    del vis, out, ws
    torch.cuda.empty_cache()

    def one(v):
        cam = sc.cameras[v]
        vis_o = O.raster_layers(sc.layers, cam)
        if not np.array_equal(views.vis_planes(vis_h, k, v).numpy().view(np.uint64), vis_o):
            return v, None
        want = O.shade_sh(sc.layers, sh, cam, vis_o, degree=3)
        return v, float(np.abs(views.image(out_h, v).numpy().astype(np.float64) - want).max())

    with cf.ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as ex:
        res = list(ex.map(one, range(len(sc.cameras))))
    bad = [v for v, e in res if e is None]
    assert not bad, f"visibility differs in views {bad[:8]}"
    worst = max(e for _, e in res)
    say(f"[gpu] sh full batch: {len(res)} views, vis bit-exact, colour err {worst:.2e}")
    assert worst <= COLOUR_ATOL

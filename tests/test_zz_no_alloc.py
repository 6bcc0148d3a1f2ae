"""The no-allocation entry point (vs_render_noalloc) through the C ABI: two
calls in a row on one device, the second with a smaller input, each equal to
vs_raster_layers + vs_render on caller-allocated buffers (visibility bit for
bit; the colours come from the same kernels and must be identical)."""
import numpy as np
import pytest
import torch

import scenes as S

pytestmark = pytest.mark.gpu


def _reference(P, layers, tex, views):
    vis, ws = P.raster(layers, views)
    rgba = P.render(layers, tex, views, vis, ws)
    return vis, rgba


def _noalloc(P, layers, tex, views):
    vis = torch.full((layers.k * views.total_pixels,), 7, dtype=torch.int64, device="cuda")   # stale contents
    out = torch.full((views.total_pixels, 4), -1.0, dtype=torch.float32, device="cuda")
    P.render_noalloc(layers, tex, views, vis, out)
    return vis, out


def _case(P, cfg, res, tex_res, n_views):
    sc = S.make_config(cfg, resolution=res, tex_res=tex_res)
    cams = S.ring_cameras(3, n_views, [res] * n_views) if n_views > 1 else sc.cameras
    layers = P.Layers(sc.layers)
    views = P.Views(cams)
    tex = [torch.from_numpy(t).cuda() for t in sc.textures]
    return layers, tex, views


def test_noalloc_equals_raster_then_render_twice():
    import paper_2409_02482_amd as P
    torch.cuda.set_device(0)
    # first call: config 2 scene (k = 7, 101,760 triangles per layer) in two 512 x 384 views
    # second call: config 1 scene (k = 3, 1,280 triangles per layer), one 256 x 256 view
    cases = [(2, (512, 384), 256, 2), (1, (256, 256), 64, 1)]
    for cfg, res, tex_res, n_views in cases:
        layers, tex, views = _case(P, cfg, res, tex_res, n_views)
        print(f"[noalloc] config {cfg}, {n_views} view(s) of {res}, k = {layers.k}", flush=True)
        need = P.workspace_bytes(layers, views)
        assert need <= (64 << 20)
        vis_n, out_n = _noalloc(P, layers, tex, views)
        vis_r, out_r = _reference(P, layers, tex, views)
        torch.cuda.synchronize()
        assert torch.equal(vis_n, vis_r), "visibility differs from vs_raster_layers"
        covered = int((vis_r != -1).sum())
        assert covered > 0
        err = (out_n - out_r).abs().max().item()
        assert err == 0.0, f"colour differs from vs_render by {err}"


def test_noalloc_rejects_a_workspace_beyond_the_scratch():
    import paper_2409_02482_amd as P
    from paper_2409_02482_amd import _lib as C
    torch.cuda.set_device(0)
    layers, tex, views = _case(P, 2, (1024, 1024), 64, 8)
    assert P.workspace_bytes(layers, views) > C.VS_NOALLOC_SCRATCH_BYTES
    vis = torch.empty(layers.k * views.total_pixels, dtype=torch.int64, device="cuda")
    out = torch.empty(views.total_pixels, 4, dtype=torch.float32, device="cuda")
    with pytest.raises(C.VsError) as e:
        P.render_noalloc(layers, tex, views, vis, out)
    assert e.value.status == C.VS_ERR_WORKSPACE
    # the library still works afterwards
    layers, tex, views = _case(P, 1, (96, 80), 32, 1)
    vis_n, out_n = _noalloc(P, layers, tex, views)
    vis_r, out_r = _reference(P, layers, tex, views)
    torch.cuda.synchronize()
    assert torch.equal(vis_n, vis_r) and torch.equal(out_n, out_r)

"""GPU parity of the k = 9 configuration at full size: 299,208 triangles per
layer, 64 ring views of uneven size from 512 x 512 to 1920 x 1080, the bin
size picked by vs_autotune, then one batched raster and one fused shade + RGB
L2 adjoint launch over all views, two steps over the same buffers.

The step is also captured in a HIP graph and replayed twice; each replay
equals the eager step.  Every view is checked against the FP64 oracle, the
views spread over host threads: visibility bit-exact, the image written by the fused launch within
1e-5, the squared-error sum within 1e-5 relative, and the texture gradient
summed over all 64 views within 1e-4 normwise.
"""
import concurrent.futures as cf
import os
import threading

import numpy as np
import pytest

import oracle as O
import scenes as S
from vs_testlib import COLOUR_ATOL, EMPTY, GRAD_RTOL, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    import paper_2409_02482_amd as P
    P.load()
    return torch


def test_cfg4_step_full_batch(torch_cuda):
    torch = torch_cuda
    import paper_2409_02482_amd as P
    say("[gpu] cfg4 full batch: building the k = 9 scene, 64 mixed views")
    sc = S.make_config(4)
    assert len(sc.cameras) == 64 and sc.k == 9
    k, nv = sc.k, len(sc.cameras)
    layers = P.Layers(sc.layers, "cuda")
    views = P.Views(sc.cameras, "cuda")
    tex = [torch.from_numpy(t).cuda() for t in sc.textures]
    target = torch.from_numpy(np.concatenate([t.reshape(-1, 4) for t in sc.targets])).cuda()
    grads = [torch.zeros_like(t) for t in tex]
    out = torch.empty(views.total_pixels, 4, dtype=torch.float32, device="cuda")
    vis = torch.empty(k * views.total_pixels, dtype=torch.int64, device="cuda")
    ws = P.alloc_workspace(layers, views, 8, "cuda")   # the smallest bin needs the largest workspace
    bin_size = P.autotune(layers, views, vis, ws)
    say(f"[gpu] cfg4 full batch: autotuned bin {bin_size}")
    sse = torch.zeros(1, dtype=torch.float64, device="cuda")
    loss_scale = 1.0 / (views.total_pixels * 3)
    for step in range(2):
        say(f"[gpu] cfg4 full batch: step {step}")
        P.raster(layers, views, vis, ws, bin=bin_size)
        for g in grads:
            g.zero_()
        sse.zero_()
        P.render_backward(layers, tex, views, vis, ws, grad_tex=grads, target=target, loss_scale=loss_scale,
                          out=out, sse=sse)
        torch.cuda.synchronize()
    st = P.read_status(ws)
    assert st["culled_invalid"] == 0 and st["bad_index"] == 0 and st["bad_key"] == 0, st

    # The same step captured in a HIP graph (raster, gradient and SSE reset, fused shade + adjoint) and
    # replayed twice, with eager work and synchronisations between the replays: every replay must equal
    # the eager step, which is checked against the oracle below (visibility and image bit for bit, the
    # SSE and the gradient up to the order of their floating-point atomics).
    eager = (vis.clone(), out.clone(), [g.clone() for g in grads], sse.item())
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        P.raster(layers, views, vis, ws, bin=bin_size)
        for g in grads:
            g.zero_()
        sse.zero_()
        P.render_backward(layers, tex, views, vis, ws, grad_tex=grads, target=target, loss_scale=loss_scale,
                          out=out, sse=sse)
    for rep in range(2):
        vis.fill_(0)
        out.fill_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        gerr = max((a - b).abs().max().item() for a, b in zip(grads, eager[2])) / \
            max(b.abs().max().item() for b in eager[2])
        serr = abs(sse.item() - eager[3]) / eager[3]
        say(f"[gpu] cfg4 graph replay {rep}: vis {'equal' if torch.equal(vis, eager[0]) else 'DIFFERS'}, "
            f"image {'equal' if torch.equal(out, eager[1]) else 'DIFFERS'}, sse rel {serr:.1e}, grad rel {gerr:.1e}")
        assert torch.equal(vis, eager[0]) and torch.equal(out, eager[1])
        assert serr <= 1e-9 and gerr <= 1e-5
    del graph, eager
    vis_h = vis.cpu()
    out_h = out.cpu()
    got = [g.cpu().numpy().astype(np.float64) for g in grads]
    sse_got = sse.item()
    del vis, out, grads, ws
    torch.cuda.empty_cache()

    say("[gpu] cfg4 full batch: oracle over all views")
    O.build(force=False)
    lock = threading.Lock()
    want = [np.zeros(t.shape, np.float64) for t in sc.textures]
    totals = {"sse": 0.0, "covered": 0, "colour": 0.0}

    def one(v):
        cam = sc.cameras[v]
        vis_o = O.raster_layers(sc.layers, cam)
        vis_g = views.vis_planes(vis_h, k, v).numpy().view(np.uint64)
        if not np.array_equal(vis_g, vis_o):
            return f"view {v}: {int((vis_g != vis_o).sum())} visibility slots differ"
        img = O.shade(sc.layers, sc.textures, cam, vis_o)
        err = float(np.abs(views.image(out_h, v).numpy().astype(np.float64) - img).max())
        sse_v = float(((img[..., :3] - sc.targets[v][..., :3].astype(np.float64)) ** 2).sum())
        gv = O.backward(sc.layers, sc.textures, cam, vis_o, target=sc.targets[v])
        with lock:
            for a, b in zip(want, gv):
                a += b
            totals["sse"] += sse_v
            totals["covered"] += int((vis_o != EMPTY).sum())
            totals["colour"] = max(totals["colour"], err)
        return None

    n_threads = max(1, min(16, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(n_threads) as ex:
        problems = [p for p in ex.map(one, range(nv)) if p]
    assert not problems, problems[:4]
    want = [w * loss_scale for w in want]
    num = max(np.abs(g - w).max() for g, w in zip(got, want))
    den = max(np.abs(w).max() for w in want)
    say(f"[gpu] cfg4 full batch: {nv} views, {totals['covered']} covered slots, vis bit-exact, "
        f"colour err {totals['colour']:.2e}, sse rel err {abs(sse_got - totals['sse']) / totals['sse']:.2e}, "
        f"grad rel err {num / den:.2e}")
    assert totals["covered"] > 0.3 * k * views.total_pixels
    assert totals["colour"] <= COLOUR_ATOL
    assert abs(sse_got - totals["sse"]) <= 1e-5 * totals["sse"]
    assert num / den <= GRAD_RTOL

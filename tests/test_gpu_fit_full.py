"""GPU parity of the benchmarked fitting iteration at full size: configuration 5
(k = 7 shells, 1024^2 RGBA textures, 128 ring views at 800 x 800), visibility
rasterised once by TextureFit, then the fused shade + RGB L2 adjoint over all
128 views in one launch, as the bench's phase split runs it.

Targets are the oracle's images of the ground-truth textures; every view is
checked against the FP64 oracle on host threads: visibility bit-exact, the
squared-error sum within 1e-5 relative, and the texture gradient summed over
the 128 views within 1e-4 normwise.
"""
import concurrent.futures as cf
import os
import threading

import numpy as np
import pytest

import oracle as O
import scenes as S
from vs_testlib import GRAD_RTOL, say

pytestmark = pytest.mark.gpu


def _pool():
    return cf.ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1)))


def test_fit_iteration_full_size(torch_cuda_fit):
    torch = torch_cuda_fit
    import paper_2409_02482_amd as P
    from paper_2409_02482_amd.fit import TextureFit
    say("[gpu] fit full size: building configuration 5 (128 views at 800^2)")
    sc = S.make_config(5, n_views=128, resolution=(800, 800))
    O.build(force=False)
    vis_o = {}

    def target(v):
        cam = sc.cameras[v]
        vis_o[v] = O.raster_layers(sc.layers, cam)
        return O.shade(sc.layers, sc.textures_gt, cam, vis_o[v]).astype(np.float32)

    say("[gpu] fit full size: oracle targets")
    with _pool() as ex:
        tg = list(ex.map(target, range(len(sc.cameras))))
    targets = torch.from_numpy(np.concatenate([t.reshape(-1, 4) for t in tg])).cuda()
    fit = TextureFit(sc.layers, sc.cameras, sc.textures, targets, mode="graph", max_iters=4)
    s = fit.stream
    with torch.cuda.stream(s):
        for g in fit.grads:
            g.zero_()
        fit.sse.zero_()
    say("[gpu] fit full size: fused adjoint over 128 views")
    P.render_backward(fit.layers, fit.tex, fit.views, fit.vis, fit.ws, grad_tex=fit.grads, target=fit.targets,
                      loss_scale=fit.loss_scale, sse=fit.sse, loss=fit.loss, stream=s)
    s.synchronize()
    st = P.read_status(fit.ws)
    assert st["culled_invalid"] == 0 and st["bad_index"] == 0 and st["bad_key"] == 0, st
    vis_h = fit.vis.cpu()
    got = [g.cpu().numpy().astype(np.float64) for g in fit.grads]
    sse_got = fit.sse.item()
    k = fit.k

    lock = threading.Lock()
    want = [np.zeros(t.shape, np.float64) for t in sc.textures]
    acc = {"sse": 0.0}

    def one(v):
        cam = sc.cameras[v]
        if not np.array_equal(fit.views.vis_planes(vis_h, k, v).numpy().view(np.uint64), vis_o[v]):
            return v
        img = O.shade(sc.layers, sc.textures, cam, vis_o[v])
        sse_v = float(((img[..., :3] - tg[v][..., :3].astype(np.float64)) ** 2).sum())
        gv = O.backward(sc.layers, sc.textures, cam, vis_o[v], target=tg[v])
        with lock:
            for a, b in zip(want, gv):
                a += b
            acc["sse"] += sse_v
        return None

    say("[gpu] fit full size: oracle adjoint over 128 views")
    with _pool() as ex:
        bad = [v for v in ex.map(one, range(len(sc.cameras))) if v is not None]
    assert not bad, f"visibility differs in views {bad[:8]}"
    want = [w * fit.loss_scale for w in want]
    num = max(np.abs(g - w).max() for g, w in zip(got, want))
    den = max(np.abs(w).max() for w in want)
    say(f"[gpu] fit full size: vis bit-exact, sse rel err {abs(sse_got - acc['sse']) / acc['sse']:.2e}, "
        f"grad rel err {num / den:.2e}")
    assert abs(sse_got - acc["sse"]) <= 1e-5 * acc["sse"]
    assert num / den <= GRAD_RTOL


@pytest.fixture(scope="module")
def torch_cuda_fit():
    import torch
    assert torch.cuda.is_available()
    import paper_2409_02482_amd as P
    P.load()
    return torch

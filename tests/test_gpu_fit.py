"""GPU tests of the fitting pattern: fused Adam kernel, graph capture, batched vs per-view, autotune."""
import numpy as np
import pytest

import scenes as S
from vs_testlib import say, small_mixed_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    import paper_2409_02482_amd as P
    P.load()
    return torch


def test_adam_step_matches_reference(torch_cuda):
    """Fused Adam + clamp + gradient reset against the textbook update written in plain PyTorch (fp32)."""
    torch = torch_cuda
    import paper_2409_02482_amd as P
    g = torch.Generator(device="cpu").manual_seed(0)
    shapes = [(8, 12, 4), (5, 3, 4), (16, 16, 4)]
    params = [torch.rand(s, generator=g).cuda() for s in shapes]
    ref = [p.clone() for p in params]
    m = [torch.zeros_like(p) for p in params]
    v = [torch.zeros_like(p) for p in params]
    rm = [torch.zeros_like(p) for p in params]
    rv = [torch.zeros_like(p) for p in params]
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    sse = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist = torch.zeros(8, dtype=torch.float64, device="cuda")
    lr, b1, b2, eps = 0.05, 0.9, 0.999, 1e-8
    for t in range(1, 6):
        grads = [(torch.rand(s, generator=g) - 0.5).cuda() for s in shapes]
        rgrads = [x.clone() for x in grads]
        sse.fill_(float(t))
        P.adam_step(params, grads, m, v, step, lr=lr, betas=(b1, b2), eps=eps, sse=sse, history=hist)
        torch.cuda.synchronize()
        for i in range(len(shapes)):
            rm[i] = b1 * rm[i] + (1 - b1) * rgrads[i]
            rv[i] = b2 * rv[i] + (1 - b2) * rgrads[i] * rgrads[i]
            mh = rm[i] / (1 - b1 ** t)
            vh = rv[i] / (1 - b2 ** t)
            ref[i] = (ref[i] - lr * mh / (vh.sqrt() + eps)).clamp(0.0, 1.0)
            assert torch.allclose(params[i], ref[i], rtol=1e-5, atol=1e-6)
            assert torch.count_nonzero(grads[i]) == 0
        assert int(step.item()) == t
        assert sse.item() == 0.0
    assert hist[:5].cpu().tolist() == [1.0, 2.0, 3.0, 4.0, 5.0]


def _small_fit_scene():
    sc = small_mixed_scene(k=3, sizes=((96, 80), (64, 64), (80, 96), (72, 72)), tex=64, config=98)
    gt = [S.smooth_texture(99, l, 64, 64, opaque=(l == 2)) for l in range(3)]
    init = []
    for l in range(3):
        t = np.full((64, 64, 4), 0.5, np.float32)
        t[..., 3] = 1.0 if l == 2 else 0.5
        init.append(t)
    return sc, gt, init


def test_graph_replay_equals_eager_and_per_view(torch_cuda):
    torch = torch_cuda
    from paper_2409_02482_amd.fit import TextureFit, render_targets
    sc, gt, init = _small_fit_scene()
    targets = render_targets(sc.layers, sc.cameras, gt)
    say("[gpu] fit: eager batched")
    eager = TextureFit(sc.layers, sc.cameras, init, targets, mode="graph", max_iters=64)
    eager.run(20)
    say("[gpu] fit: graph batched")
    graph = TextureFit(sc.layers, sc.cameras, init, targets, mode="graph", max_iters=64)
    graph.capture()
    # replays with eager host-side work and synchronisations in between
    for _ in range(4):
        graph.run(5)
        torch.cuda.synchronize()
        _ = [p.sum().item() for p in graph.params]
    say("[gpu] fit: per-view eager")
    pv = TextureFit(sc.layers, sc.cameras, init, targets, mode="per_view", max_iters=64)
    pv.run(20)
    pe, pg, pp = eager.psnr(), graph.psnr(), pv.psnr()
    assert len(pe) == len(pg) == len(pp) == 20
    assert pe[-1] > pe[0] + 3.0, f"fitting did not improve: {pe[0]:.2f} -> {pe[-1]:.2f}"
    # identical arithmetic; only the order of floating-point atomics differs
    assert np.max(np.abs(pe - pg)) < 1e-3
    assert np.max(np.abs(pe - pp)) < 1e-3
    for a, b, c in zip(eager.params, graph.params, pv.params):
        assert torch.allclose(a, b, atol=1e-4) and torch.allclose(a, c, atol=1e-4)


def test_autotune_picks_a_bin_and_results_are_identical(torch_cuda, tmp_path):
    torch = torch_cuda
    import paper_2409_02482_amd as P
    sc = small_mixed_scene(k=3, sizes=((256, 192), (128, 128)), config=100)
    layers, views = P.Layers(sc.layers), P.Views(sc.cameras)
    ws = P.alloc_workspace(layers, views, bin=8)
    vis = torch.empty(layers.k * views.total_pixels, dtype=torch.int64, device="cuda")
    cache = str(tmp_path / "tune.txt")
    b = P.autotune(layers, views, vis, ws, cache_path=cache)
    assert b in (8, 16, 32, 64)
    ref = vis.clone()
    vis2, _ = P.raster(layers, views, ws=P.alloc_workspace(layers, views, bin=b), bin=b)
    assert torch.equal(vis2, ref)
    # cache hit returns the same answer without timing
    assert P.autotune(layers, views, vis, ws, cache_path=cache) == b
    assert open(cache).read().count("\n") == 1


@pytest.mark.parametrize("quantize", [False, True], ids=["texels", "quantised_logits"])
def test_checkpoint_resume_continues_the_curve(torch_cuda, tmp_path, quantize):
    """Save after 10 iterations; a fresh fit (graph-captured) that loads the file continues the run: its
    state after loading equals the saved one bit for bit, and its next 10 PSNR values and final texels equal
    those of the uninterrupted run (up to the order of floating-point atomics)."""
    torch = torch_cuda
    from paper_2409_02482_amd.fit import TextureFit, render_targets
    sc, gt, init = _small_fit_scene()
    targets = render_targets(sc.layers, sc.cameras, gt)
    loss = "l1" if quantize else "l2"
    a = TextureFit(sc.layers, sc.cameras, init, targets, mode="graph", max_iters=64, loss=loss, quantize=quantize)
    a.capture()
    a.run(10)
    path = str(tmp_path / "fit.pt")
    a.save(path)
    saved = [p.clone() for p in a.params] + [m.clone() for m in a.m] + [v.clone() for v in a.v]
    a.run(10)
    b = TextureFit(sc.layers, sc.cameras, init, targets, mode="graph", max_iters=64, loss=loss, quantize=quantize)
    b.capture()          # captured before loading: the load writes in place
    b.load(path)
    now = [p.clone() for p in b.params] + [m.clone() for m in b.m] + [v.clone() for v in b.v]
    assert all(torch.equal(x, y) for x, y in zip(saved, now))
    assert int(b.step.item()) == 10
    b.run(10)
    ha, hb = a.loss_history(), b.loss_history()
    assert len(ha) == len(hb) == 20
    assert np.array_equal(ha[:10], hb[:10])
    rel = np.abs(ha[10:] - hb[10:]) / ha[10:]
    say(f"[gpu] resume ({loss}{', quantised' if quantize else ''}): loss curve rel gap {rel.max():.2e}")
    assert rel.max() < 1e-4
    # parameters (the texels, or their logits); a quantised texel may land on the neighbouring 8-bit level
    for x, y in zip(a.params, b.params):
        assert torch.allclose(x, y, atol=1e-4)
    with pytest.raises(ValueError):
        TextureFit(sc.layers, sc.cameras, init, targets, mode="graph", max_iters=64,
                   loss="l2" if quantize else "l1").load(path)

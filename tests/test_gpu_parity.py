"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Bar: visibility bit-exact; colour within 1e-5 max-abs per channel; texture
gradients within 1e-4 (||g - g_ref||_inf / ||g_ref||_inf) of the oracle's
analytic adjoint and, on 64 sampled texels, of central finite differences.
"""
import numpy as np
import pytest

import oracle as O
import scenes as S
from vs_testlib import (EMPTY, GRAD_RTOL, assert_colour_close, assert_vis_equal, gpu_render, grad_rel_err,
                        img_numpy, oracle_vis, pick_entries, say, small_mixed_scene, vis_numpy)

pytestmark = pytest.mark.gpu


def torch_sync():
    import torch
    torch.cuda.synchronize()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    import paper_2409_02482_amd as P
    P.load()
    return torch


def _check_scene(scene, what, views_to_check=None, expect_clean=True, **kw):
    say(f"[gpu] {what}: raster+render {len(scene.cameras)} views k={scene.k}")
    P, layers, views, vis, ws, rgba, tex = gpu_render(scene, count_fragments=True, **kw)
    torch_sync()
    st = P.read_status(ws)
    if expect_clean:
        assert st["culled_invalid"] == 0 and st["bad_index"] == 0 and st["bad_key"] == 0, st
    frags = 0
    for v in (views_to_check if views_to_check is not None else range(len(scene.cameras))):
        cam = scene.cameras[v]
        say(f"[gpu] {what}: oracle view {v} {cam.width}x{cam.height}")
        want = np.stack([O.raster(m, cam)[0] for m in scene.layers])
        got = vis_numpy(views, vis, scene.k, v)
        assert_vis_equal(got, want, f"{what} view {v}")
        img = O.shade(scene.layers, scene.textures, cam, want, wrap=kw.get("wrap", 0))
        err = assert_colour_close(img_numpy(views, rgba, v), img, f"{what} view {v}")
        say(f"[gpu] {what}: view {v} vis bit-exact, colour err {err:.2e}")
    return st


def test_cfg1_vis_and_colour(torch_cuda):
    _check_scene(S.make_config(1), "cfg1")


def test_cfg1_fragment_count_matches_oracle(torch_cuda):
    sc = S.make_config(1)
    P, layers, views, vis, ws, rgba, tex = gpu_render(sc, count_fragments=True)
    st = P.read_status(ws)
    want = sum(O.raster(m, sc.cameras[0])[1]["fragments"] for m in sc.layers)
    assert st["fragments"] == want


def test_cfg2_vis_and_colour_full_size(torch_cuda):
    _check_scene(S.make_config(2), "cfg2")


def test_ragged_multiview_batch(torch_cuda):
    _check_scene(small_mixed_scene(), "ragged")


def test_clamp_wrap(torch_cuda):
    _check_scene(small_mixed_scene(k=2, sizes=((64, 48),), config=91), "clamp", wrap=1)


def test_projection_bit_exact(torch_cuda):
    """White-box: the projected vertices in the workspace equal the oracle's step 1 bit for bit."""
    sc = S.make_config(4, n_views=3, latlong=(40, 80), with_targets=False)
    P, layers, views, vis, ws, rgba, tex = gpu_render(sc)
    raw = ws.cpu().numpy()
    vpv = sum(m.n_vert for m in sc.layers)
    # layout: 256-byte status block, then the 16-pixel tile -> view table (int32, 256-aligned)
    n16 = int(views.host[views.n].tile_offset[1])
    off0 = 256 + (n16 * 4 + 255) // 256 * 256
    rec = np.frombuffer(raw[off0:off0 + 16 * vpv * len(sc.cameras)].tobytes(),
                        dtype=[("X", "<i4"), ("Y", "<i4"), ("w", "<f8")]).reshape(len(sc.cameras), vpv)
    for v, cam in enumerate(sc.cameras):
        off = 0
        for m in sc.layers:
            X, Y, w, valid = O.project(m, cam)
            r = rec[v, off:off + m.n_vert]
            assert valid.all()
            assert np.array_equal(r["X"], X) and np.array_equal(r["Y"], Y)
            assert np.array_equal(r["w"].view(np.uint64), w.view(np.uint64))
            off += m.n_vert


def test_determinism_and_batched_equals_single(torch_cuda):
    sc = small_mixed_scene()
    P, layers, views, vis, ws, rgba, tex = gpu_render(sc)
    vis_b = vis.clone()
    rgba_b = rgba.clone()
    vis2, _ = P.raster(layers, views, ws=ws)
    assert torch_cuda.equal(vis2, vis_b)
    for v, cam in enumerate(sc.cameras):
        one = S.Scene("one", sc.layers, sc.textures, [cam])
        _, _, views1, vis1, ws1, rgba1, _ = gpu_render(one)
        assert torch_cuda.equal(views1.vis_planes(vis1, sc.k, 0), views.vis_planes(vis_b, sc.k, v))
        assert torch_cuda.equal(views1.image(rgba1, 0), views.image(rgba_b, v))


def test_early_exit_within_tolerance(torch_cuda):
    sc = small_mixed_scene(k=5, config=92)
    _check_scene(sc, "eps", eps_T=2.0 ** -20)


def test_edge_cases_counted(torch_cuda):
    """Near-plane, NaN, guard-band and zero-area triangles are culled and counted; bad ids are counted."""
    xyz = np.array([
        [-0.5, -0.5, 1.0], [0.5, -0.5, 1.0], [0.0, 0.5, 1.0],
        [-0.5, 0.0, 1.0], [0.0, 0.0, 1.0], [0.5, 0.0, 1.0],
        [-0.5, -0.5, 0.005], [0.5, 0.5, 0.005],
        [np.nan, 0.0, 1.0],
        [5000.0, 0.0, 1.0],
    ], np.float32)
    tri = np.array([[0, 1, 2], [3, 4, 5], [0, 6, 7], [0, 1, 8], [0, 1, 9], [0, 0, 1], [0, 1, 99]], np.int32)
    mesh = S.Mesh(xyz, np.zeros((xyz.shape[0], 2), np.float32) + 0.5, tri)
    cam = S.Camera(32, 32, 16.0, 16.0, 16.0, 16.0, np.eye(3), np.zeros(3))
    sc = S.Scene("edge", [mesh], [S.constant_texture(4, 4, [1, 0.5, 0.25, 1])], [cam])
    st = _check_scene(sc, "edge", expect_clean=False)
    assert st["culled_degenerate"] == 2 and st["culled_invalid"] == 3 and st["bad_index"] == 1
    assert st["bad_key"] == 0


def test_tiny_views(torch_cuda):
    sc = small_mixed_scene(k=2, sizes=((1, 1), (2, 3), (15, 1), (1, 17)), config=93)
    _check_scene(sc, "tiny")


# ---------------------------------------------------------------------------- gradients
def _gpu_backward(P, layers, views, vis, ws, tex, grad_rgba=None, target=None, wrap=0):
    import torch
    grads = P.render_backward(layers, tex, views, vis, ws, grad_rgba=grad_rgba, target=target, wrap=wrap)
    torch.cuda.synchronize()
    return [g.cpu().numpy().astype(np.float64) for g in grads]


def test_cfg1_gradient_linear_loss(torch_cuda):
    torch = torch_cuda
    sc = S.make_config(1)
    cam = sc.cameras[0]
    P, layers, views, vis, ws, rgba, tex = gpu_render(sc)
    g = S.upstream_grad(1, cam)
    got = _gpu_backward(P, layers, views, vis, ws, tex, grad_rgba=torch.from_numpy(g.reshape(-1, 4)).cuda())
    visn = oracle_vis(sc, views, vis, 0)
    want = O.backward(sc.layers, sc.textures, cam, visn, grad_out=g.astype(np.float64))
    err = grad_rel_err(got, want)
    say(f"[gpu] cfg1 grad rel err {err:.2e}")
    assert err <= GRAD_RTOL
    ent = pick_entries(np.random.default_rng(7), want, 64)
    fd = O.finite_diff(sc.layers, sc.textures, cam, visn, ent, h=1e-3, grad_out=g.astype(np.float64))
    gg = np.array([got[l][j, i, c] for l, j, i, c in ent])
    assert np.all(np.abs(gg - fd) <= 1e-4 * np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max()))


def test_cfg3_gradient_l2_full_size(torch_cuda):
    """config 3: config 2 plus the RGB L2 loss against a seeded target; FD (h = 1e-3) on 64 texels."""
    torch = torch_cuda
    sc = S.make_config(3)
    cam = sc.cameras[0]
    say("[gpu] cfg3 forward")
    P, layers, views, vis, ws, rgba, tex = gpu_render(sc)
    tgt = torch.from_numpy(sc.targets[0].reshape(-1, 4)).cuda()
    sse = torch.zeros(1, dtype=torch.float64, device="cuda")
    out2 = torch.empty_like(rgba)
    say("[gpu] cfg3 backward (fused L2)")
    grads = P.render_backward(layers, tex, views, vis, ws, target=tgt, out=out2, sse=sse)
    torch.cuda.synchronize()
    got = [g.cpu().numpy().astype(np.float64) for g in grads]
    assert torch.allclose(out2, rgba, rtol=0, atol=1e-6), "fused backward's forward image differs from vs_render"
    visn = oracle_vis(sc, views, vis, 0)
    say("[gpu] cfg3 oracle backward")
    want = O.backward(sc.layers, sc.textures, cam, visn, target=sc.targets[0])
    err = grad_rel_err(got, want)
    say(f"[gpu] cfg3 grad rel err {err:.2e}")
    assert err <= GRAD_RTOL
    img = O.shade(sc.layers, sc.textures, cam, visn)
    sse_ref = ((img[..., :3] - sc.targets[0][..., :3].astype(np.float64)) ** 2).sum()
    assert abs(sse.item() - sse_ref) <= 1e-5 * sse_ref
    ent = pick_entries(np.random.default_rng(3), want, 64)
    fd = O.finite_diff(sc.layers, sc.textures, cam, visn, ent, h=1e-3, target=sc.targets[0])
    gg = np.array([got[l][j, i, c] for l, j, i, c in ent])
    bad = np.abs(gg - fd) > 1e-4 * np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max())
    assert not bad.any(), f"{bad.sum()} FD mismatches, worst {np.abs(gg - fd).max():.3e}"


def test_ragged_gradient_matches_oracle(torch_cuda):
    torch = torch_cuda
    sc = small_mixed_scene(config=94)
    P, layers, views, vis, ws, rgba, tex = gpu_render(sc)
    gs = [S.upstream_grad(94, c, v) for v, c in enumerate(sc.cameras)]
    flat = torch.from_numpy(np.concatenate([g.reshape(-1, 4) for g in gs])).cuda()
    got = _gpu_backward(P, layers, views, vis, ws, tex, grad_rgba=flat)
    want = [np.zeros(t.shape) for t in sc.textures]
    for v, cam in enumerate(sc.cameras):
        w = O.backward(sc.layers, sc.textures, cam, oracle_vis(sc, views, vis, v), grad_out=gs[v].astype(np.float64))
        want = [a + b for a, b in zip(want, w)]
    assert grad_rel_err(got, want) <= GRAD_RTOL


# texture sizes that exercise each scatter path of the adjoint: the LDS window (magnified
# texels), degenerate widths and heights (corners that coincide or wrap onto themselves), and
# the direct-atomic fallback (minified texels: a wavefront's footprint exceeds the window)
_TEX_CASES = {
    "window": ((64, 64), (48, 80), (64, 64)),
    "degenerate": ((1, 1), (3, 2), (1, 5)),
    "minified": ((1024, 1024), (2048, 256), (256, 2048)),
}


@pytest.mark.parametrize("wrap", [0, 1], ids=["repeat", "clamp"])
@pytest.mark.parametrize("case", sorted(_TEX_CASES))
def test_gradient_scatter_paths(torch_cuda, case, wrap):
    torch = torch_cuda
    base = small_mixed_scene(config=96, sizes=((96, 80), (37, 53), (64, 64)))
    textures = [S.uniform_texture(96, l, w, h, opaque=(l == base.k - 1)) for l, (w, h) in enumerate(_TEX_CASES[case])]
    sc = S.Scene(base.name, base.layers, textures, base.cameras)
    say(f"[gpu] scatter paths: {case} wrap={wrap}")
    P, layers, views, vis, ws, rgba, tex = gpu_render(sc, wrap=wrap)
    gs = [S.upstream_grad(96, c, v) for v, c in enumerate(sc.cameras)]
    flat = torch.from_numpy(np.concatenate([g.reshape(-1, 4) for g in gs])).cuda()
    got = _gpu_backward(P, layers, views, vis, ws, tex, grad_rgba=flat, wrap=wrap)
    want = [np.zeros(t.shape) for t in sc.textures]
    for v, cam in enumerate(sc.cameras):
        w = O.backward(sc.layers, sc.textures, cam, oracle_vis(sc, views, vis, v), grad_out=gs[v].astype(np.float64),
                       wrap=wrap)
        want = [a + b for a, b in zip(want, w)]
    err = grad_rel_err(got, want)
    say(f"[gpu] scatter paths: {case} wrap={wrap} grad rel err {err:.2e}")
    assert err <= GRAD_RTOL
    # per layer too, so that a small layer cannot hide behind a large one
    for l in range(sc.k):
        if np.abs(want[l]).max() == 0:
            assert np.abs(got[l]).max() == 0, f"layer {l}"
        else:
            assert grad_rel_err([got[l]], [want[l]]) <= GRAD_RTOL, f"layer {l}"


def test_autograd_function(torch_cuda):
    torch = torch_cuda
    import paper_2409_02482_amd as P
    sc = small_mixed_scene(config=95)
    r = P.Renderer(sc.layers, sc.cameras)
    tex = [torch.from_numpy(t).cuda().requires_grad_(True) for t in sc.textures]
    out = r(*tex)
    g = torch.from_numpy(np.random.default_rng(5).uniform(-1, 1, tuple(out.shape)).astype(np.float32)).cuda()
    (out * g).sum().backward()
    ref = P.render_backward(r.layers, [t.detach() for t in tex], r.views, r.vis, r.ws, grad_rgba=g)
    torch.cuda.synchronize()
    for a, b in zip(tex, ref):
        assert torch.isfinite(a.grad).all() and torch.isfinite(b).all()
        # two runs of the same float atomics in different orders: compare normwise
        err = (a.grad - b).abs().max().item() / max(b.abs().max().item(), 1e-30)
        say(f"[gpu] autograd vs direct: rel err {err:.2e}")
        assert err <= 1e-5


# ---------------------------------------------------------------------------- raster variants
@pytest.mark.parametrize("bin", [8, 16, 32, 64])
def test_every_bin_size_is_bit_exact(torch_cuda, bin):
    sc = small_mixed_scene(k=3, sizes=((200, 150), (37, 53), (129, 65)), config=96)
    _check_scene(sc, f"bin{bin}", bin=bin)


def _soup_layer(rng, n, x0, x1, y0, y1, radius, cam):
    """n random triangles (random winding) with vertices within `radius` px of centres in
    [x0, x1) x [y0, y1) px, at random depths in [1, 3], for a camera at the origin looking down +z."""
    c = np.stack([rng.uniform(x0, x1, n), rng.uniform(y0, y1, n)], 1)
    px = c[:, None, :] + rng.uniform(-radius, radius, (n, 3, 2))
    z = rng.uniform(1.0, 3.0, (n, 3))
    xyz = np.stack([(px[..., 0] - cam.cx) * z / cam.fx, (px[..., 1] - cam.cy) * z / cam.fy, z], -1)
    uv = rng.uniform(0.0, 1.0, (n * 3, 2))
    return S.Mesh(xyz.reshape(-1, 3).astype(np.float32), uv.astype(np.float32),
                  np.arange(n * 3, dtype=np.int32).reshape(n, 3))


@pytest.mark.parametrize("bin", [8, 64])
def test_crowded_bin_both_sides(torch_cuda, bin):
    """20,000 small triangles per layer of both windings inside one 64 x 56 bin (hundreds of
    wavefronts reserving places on the same two list sides), plus larger triangles across the
    bin edges (places in their other bins taken after the first-bin ones): bit-exact."""
    rng = np.random.default_rng(4242 + bin)
    cam = S.Camera(160, 120, 100.0, 100.0, 80.0, 60.0, np.eye(3), np.zeros(3))
    crowded = [_soup_layer(rng, 20000, 2, 62, 2, 54, 3.0, cam) for _ in range(2)]
    wide = _soup_layer(rng, 3000, 0, 160, 0, 120, 20.0, cam)
    layers = [S.Mesh(np.concatenate([m.xyz, wide.xyz]), np.concatenate([m.uv, wide.uv]),
                     np.concatenate([m.tri, wide.tri + m.xyz.shape[0]])) for m in crowded]
    tex = [S.uniform_texture(5, l, 16, 16, opaque=(l == 1)) for l in range(2)]
    sc = S.Scene("crowded", layers, tex, [cam])
    _check_scene(sc, f"crowded bin{bin}", bin=bin)


def test_direct_raster_equals_binned(torch_cuda):
    """Two independent GPU rasterisers (binned LDS tiles, direct global atomics) agree bit for bit."""
    sc = S.make_config(2, resolution=(512, 384))
    say("[gpu] direct vs binned")
    _, _, views, vis_b, _, _, _ = gpu_render(sc)
    _, _, _, vis_d, _, _, _ = gpu_render(sc, direct=True)
    assert torch_cuda.equal(vis_b, vis_d)


def test_list_overflow_falls_back_exactly(torch_cuda):
    """A triangle-list capacity far too small: overflowing bins rasterise from the full layer, still exact."""
    sc = small_mixed_scene(k=2, sizes=((96, 80), (64, 64)), config=97)
    st = _check_scene(sc, "overflow", list_capacity=200, expect_clean=True)
    assert st["bin_overflow"] > 0


@pytest.mark.parametrize("k", [1, 8, 10, 16])
def test_layer_counts_up_to_the_maximum(torch_cuda, k):
    """Layer counts that select each variant of the adjoint (ceilings 4, 8 and 16; 7 and 9 are covered by
    the configurations) up to the maximum of 16 layers, on ragged views: visibility bit-exact, colour, and
    the texture gradient of a linear loss."""
    torch = torch_cuda
    sc = small_mixed_scene(k=k, config=120 + k)
    _check_scene(sc, f"k={k}")
    P, layers, views, vis, ws, rgba, tex = gpu_render(sc)
    gs = [S.upstream_grad(120 + k, c, v) for v, c in enumerate(sc.cameras)]
    flat = torch.from_numpy(np.concatenate([g.reshape(-1, 4) for g in gs])).cuda()
    got = _gpu_backward(P, layers, views, vis, ws, tex, grad_rgba=flat)
    want = [np.zeros(t.shape) for t in sc.textures]
    for v, cam in enumerate(sc.cameras):
        w = O.backward(sc.layers, sc.textures, cam, oracle_vis(sc, views, vis, v), grad_out=gs[v].astype(np.float64))
        want = [a + b for a, b in zip(want, w)]
    err = grad_rel_err(got, want)
    say(f"[gpu] k={k}: grad rel err {err:.2e}")
    assert err <= GRAD_RTOL
    assert all(np.abs(w).max() > 0 for w in want[:1])


def test_scatter_retry_paths_are_taken_and_exact(torch_cuda):
    """Texture sizes swept on one 256^2 view of the displaced shells, from magnified to strongly minified texels,
    so that every scatter path of the adjoint occurs: the whole wavefront's LDS window, the half and quarter
    wavefront retries, and direct atomics (counted in the status block with VS_SHADE_COUNT_PATHS).  Every
    size's gradient is compared with the oracle's."""
    torch = torch_cuda
    base = small_mixed_scene(config=97, sizes=((256, 256),))
    cam = base.cameras[0]
    names = ["scatter_wave", "scatter_half", "scatter_quarter", "scatter_direct"]
    seen = np.zeros(4, np.int64)
    g = S.upstream_grad(97, cam)
    flat = torch.from_numpy(g.reshape(-1, 4)).cuda()
    for W in (64, 512, 1024, 2048):
        textures = [S.uniform_texture(97, l, W, W, opaque=(l == base.k - 1)) for l in range(base.k)]
        sc = S.Scene(base.name, base.layers, textures, base.cameras)
        P, layers, views, vis, ws, rgba, tex = gpu_render(sc)
        grads = P.render_backward(layers, tex, views, vis, ws, grad_rgba=flat, count_paths=True)
        st = P.read_status(ws)
        counts = np.array([st[n] for n in names])
        got = [t.cpu().numpy().astype(np.float64) for t in grads]
        want = O.backward(sc.layers, sc.textures, cam, oracle_vis(sc, views, vis, 0), grad_out=g.astype(np.float64))
        err = grad_rel_err(got, want)
        say(f"[gpu] scatter paths, {W}^2 textures: counts {dict(zip(names, counts.tolist()))}, grad rel err {err:.2e}")
        assert err <= GRAD_RTOL
        seen += counts
        del grads, got, want, tex
    assert (seen > 0).all(), f"scatter paths never taken: {[n for n, c in zip(names, seen) if c == 0]}"

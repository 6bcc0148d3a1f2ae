"""CPU checks of the C ABI: the library loads, exports every declared symbol,
struct layouts agree with the C compiler, and host-side validation rejects bad
arguments before anything is enqueued (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import scenes as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def C():
    from paper_2409_02482_amd import _lib
    _lib.load()
    return _lib


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "vs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vs_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol(C):
    lib = C.load()
    names = _declared_symbols()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), f"libvs.so does not export {n}"
        assert n in C.SIGNATURES, f"binding has no signature for {n}"
    out = subprocess.run(["nm", "-D", "--defined-only", C.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (vs_\w+)", out))
    assert set(names) <= exported


def test_struct_layouts_match_c(C, tmp_path):
    prog = tmp_path / "sz.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "vs.h"\nint main(void){'
                    'printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(vs_mesh),'
                    'sizeof(vs_texture), sizeof(vs_camera), sizeof(vs_view), sizeof(vs_views), sizeof(vs_raster_opts),'
                    'sizeof(vs_shade_opts), offsetof(vs_view, pix_offset), offsetof(vs_shade_opts, target),'
                    'offsetof(vs_raster_opts, list_capacity), sizeof(vs_sh_texture), sizeof(vs_sh_opts),'
                    'offsetof(vs_sh_opts, view_alpha)); printf("%zu %zu %zu %zu\\n", sizeof(vs_ngp_config),'
                    'sizeof(vs_ksdf_field), sizeof(vs_ksdf_opts), offsetof(vs_ksdf_opts, pdf_floor));'
                    'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = [ctypes.sizeof(C.VsMesh), ctypes.sizeof(C.VsTexture), ctypes.sizeof(C.VsCamera),
            ctypes.sizeof(C.VsView), ctypes.sizeof(C.VsViews), ctypes.sizeof(C.VsRasterOpts),
            ctypes.sizeof(C.VsShadeOpts), C.VsView.pix_offset.offset, C.VsShadeOpts.target.offset,
            C.VsRasterOpts.list_capacity.offset, ctypes.sizeof(C.VsShTexture), ctypes.sizeof(C.VsShOpts),
            C.VsShOpts.view_alpha.offset, ctypes.sizeof(C.VsNgpConfig), ctypes.sizeof(C.VsKsdfField),
            ctypes.sizeof(C.VsKsdfOpts), C.VsKsdfOpts.pdf_floor.offset]
    assert got == want


def _cams(sizes):
    from paper_2409_02482_amd.binding import camera_struct
    cams = S.ring_cameras(3, len(sizes), sizes)
    return (C_lib().VsCamera * len(cams))(*[camera_struct(c) for c in cams]), cams


def C_lib():
    from paper_2409_02482_amd import _lib
    return _lib


def test_views_prepare_offsets(C):
    sizes = [(512, 512), (640, 480), (37, 53), (1920, 1080), (1, 1)]
    arr, cams = _cams(sizes)
    out = (C.VsView * (len(sizes) + 1))()
    assert C.load().vs_views_prepare(ctypes.addressof(arr), len(sizes), ctypes.addressof(out)) == C.VS_OK
    pix, tiles = 0, [0, 0, 0, 0]
    for v, (w, h) in enumerate(sizes + [(0, 0)]):
        assert out[v].pix_offset == pix
        assert list(out[v].tile_offset) == tiles
        pix += w * h
        # tiles of the four slots: 8x8, 16x16, 32x32 and the 64 x 56 raster bins
        tiles = [t + (-(-w // sw)) * (-(-h // sh)) for t, sw, sh in zip(tiles, (8, 16, 32, 64), (8, 16, 32, 56))]
    assert out[0].cam.width == 512 and abs(out[3].cam.fy - cams[3].fy) == 0


def test_views_prepare_rejects_bad_camera(C):
    arr, _ = _cams([(64, 64), (64, 64)])
    out = (C.VsView * 3)()
    arr[1].width = 0
    assert C.load().vs_views_prepare(ctypes.addressof(arr), 2, ctypes.addressof(out)) == C.VS_ERR_SIZE
    arr[1].width = 64
    arr[1].z_near = 0.0
    assert C.load().vs_views_prepare(ctypes.addressof(arr), 2, ctypes.addressof(out)) == C.VS_ERR_ARG
    arr[1].z_near = 0.01
    arr[1].R[4] = float("nan")
    assert C.load().vs_views_prepare(ctypes.addressof(arr), 2, ctypes.addressof(out)) == C.VS_ERR_ARG
    assert b"rotation" in C.load().vs_last_error()


def _fake_call_args(C, k=2, n_views=1):
    """Host-side structs with non-null fake device pointers: only validation runs."""
    arr, _ = _cams([(64, 48)] * n_views)
    host = (C.VsView * (n_views + 1))()
    assert C.load().vs_views_prepare(ctypes.addressof(arr), n_views, ctypes.addressof(host)) == 0
    views = C.VsViews(ctypes.addressof(host), 0x1000, n_views)
    meshes = (C.VsMesh * k)(*[C.VsMesh(0x1000, 0x2000, 0x3000, 10, 5) for _ in range(k)])
    tex = (C.VsTexture * k)(*[C.VsTexture(0x4000, 8, 8) for _ in range(k)])
    return host, views, meshes, tex


def test_raster_validation_without_gpu(C):
    L = C.load()
    host, views, meshes, tex = _fake_call_args(C)
    need = L.vs_raster_workspace_bytes(ctypes.addressof(meshes), 2, ctypes.byref(views), None)
    assert need >= 256 + 2 * 0
    # k out of range
    assert L.vs_raster_layers(ctypes.addressof(meshes), 0, ctypes.byref(views), 0x5000, 0x100000, need, None,
                              None) == C.VS_ERR_SIZE
    assert L.vs_raster_layers(ctypes.addressof(meshes), 17, ctypes.byref(views), 0x5000, 0x100000, need, None,
                              None) == C.VS_ERR_SIZE
    # null vis
    assert L.vs_raster_layers(ctypes.addressof(meshes), 2, ctypes.byref(views), None, 0x100000, need, None,
                              None) == C.VS_ERR_ARG
    # workspace too small / misaligned / null
    assert L.vs_raster_layers(ctypes.addressof(meshes), 2, ctypes.byref(views), 0x5000, 0x100000, need - 1, None,
                              None) == C.VS_ERR_WORKSPACE
    assert L.vs_raster_layers(ctypes.addressof(meshes), 2, ctypes.byref(views), 0x5000, 0x100010, need, None,
                              None) == C.VS_ERR_WORKSPACE
    assert L.vs_raster_layers(ctypes.addressof(meshes), 2, ctypes.byref(views), 0x5000, None, need, None,
                              None) == C.VS_ERR_WORKSPACE
    # null mesh pointer
    meshes[1].tri = None
    assert L.vs_raster_layers(ctypes.addressof(meshes), 2, ctypes.byref(views), 0x5000, 0x100000, need, None,
                              None) == C.VS_ERR_ARG
    assert b"layer 1" in L.vs_last_error()
    # an empty layer (no triangles, or no vertices) is rejected, not rastered
    meshes[1].tri = 0x3000
    for field in ("n_tri", "n_vert"):
        setattr(meshes[0], field, 0)
        assert L.vs_raster_layers(ctypes.addressof(meshes), 2, ctypes.byref(views), 0x5000, 0x100000, need, None,
                                  None) == C.VS_ERR_SIZE
        assert b"layer 0: empty mesh" in L.vs_last_error()
        meshes[0].n_tri, meshes[0].n_vert = 5, 10
    # more than 2^28 vertices or triangles in a layer (the kernels address them with 32-bit byte offsets)
    for field in ("n_tri", "n_vert"):
        setattr(meshes[0], field, (1 << 28) + 1)
        assert L.vs_raster_layers(ctypes.addressof(meshes), 2, ctypes.byref(views), 0x5000, 0x100000, need, None,
                                  None) == C.VS_ERR_SIZE
        assert b"more than 268435456 vertices or triangles" in L.vs_last_error()
        meshes[0].n_tri, meshes[0].n_vert = 5, 10
    # a tampered view table
    host[1].pix_offset += 1
    assert L.vs_raster_layers(ctypes.addressof(meshes), 2, ctypes.byref(views), 0x5000, 0x100000, need, None,
                              None) == C.VS_ERR_ARG


def test_render_validation_without_gpu(C):
    L = C.load()
    host, views, meshes, tex = _fake_call_args(C)
    need = L.vs_raster_workspace_bytes(ctypes.addressof(meshes), 2, ctypes.byref(views), None)
    bad = C.VsShadeOpts(0.0, 7, None, 1.0, 0)
    assert L.vs_render(ctypes.addressof(meshes), ctypes.addressof(tex), 2, ctypes.byref(views), 0x5000, 0x100000,
                       need, 0x6000, ctypes.byref(bad), None) == C.VS_ERR_UNSUPPORTED
    neg = C.VsShadeOpts(-1.0, 0, None, 1.0, 0)
    assert L.vs_render(ctypes.addressof(meshes), ctypes.addressof(tex), 2, ctypes.byref(views), 0x5000, 0x100000,
                       need, 0x6000, ctypes.byref(neg), None) == C.VS_ERR_ARG
    tex[0].width = 20000
    assert L.vs_render(ctypes.addressof(meshes), ctypes.addressof(tex), 2, ctypes.byref(views), 0x5000, 0x100000,
                       need, 0x6000, None, None) == C.VS_ERR_SIZE
    tex[0].width = 8
    gp = (ctypes.c_void_p * 2)(0x7000, None)
    assert L.vs_render_backward(ctypes.addressof(meshes), ctypes.addressof(tex), 2, ctypes.byref(views), 0x5000,
                                0x100000, need, 0x6000, ctypes.addressof(gp), None, None, None, None) == C.VS_ERR_ARG
    gp = (ctypes.c_void_p * 2)(0x7000, 0x8000)
    # an unknown shading flag
    odd = C.VsShadeOpts(0.0, 0, None, 1.0, 0, 6)
    assert L.vs_render_backward(ctypes.addressof(meshes), ctypes.addressof(tex), 2, ctypes.byref(views), 0x5000,
                                0x100000, need, 0x6000, ctypes.addressof(gp), None, None, ctypes.byref(odd),
                                None) == C.VS_ERR_UNSUPPORTED
    # neither grad_rgba nor a target
    assert L.vs_render_backward(ctypes.addressof(meshes), ctypes.addressof(tex), 2, ctypes.byref(views), 0x5000,
                                0x100000, need, None, ctypes.addressof(gp), None, None, None, None) == C.VS_ERR_ARG


def test_render_noalloc_validation_without_gpu(C):
    """vs_render_noalloc rejects, before any HIP call, arguments either of its two steps would reject and a
    problem whose workspace exceeds the static scratch."""
    L = C.load()
    host, views, meshes, tex = _fake_call_args(C)
    call = lambda ro=None, so=None, vis=0x5000, out=0x6000, k=2: L.vs_render_noalloc(  # noqa: E731
        ctypes.addressof(meshes), ctypes.addressof(tex), k, ctypes.byref(views), vis, out,
        None if ro is None else ctypes.byref(ro), None if so is None else ctypes.byref(so), None)
    assert call(k=0) == C.VS_ERR_SIZE
    assert call(vis=None) == C.VS_ERR_ARG
    assert call(out=None) == C.VS_ERR_ARG
    assert call(ro=C.VsRasterOpts(12, 0, 0)) == C.VS_ERR_UNSUPPORTED
    assert call(ro=C.VsRasterOpts(0, 0, -1)) == C.VS_ERR_SIZE
    assert call(so=C.VsShadeOpts(0.0, 3, None, 1.0, 0)) == C.VS_ERR_UNSUPPORTED
    assert call(so=C.VsShadeOpts(1.5, 0, None, 1.0, 0)) == C.VS_ERR_ARG
    tex[1].width = 0
    assert call() == C.VS_ERR_SIZE
    tex[1].width = 8
    # a list capacity that alone needs more than the scratch
    big = C.VsRasterOpts(0, 0, C.VS_NOALLOC_SCRATCH_BYTES // 4)
    assert call(ro=big) == C.VS_ERR_WORKSPACE
    assert b"static scratch" in L.vs_last_error()
    # the same limit from the problem size: 5M triangles per layer need more than 64 MiB
    for m in meshes:
        m.n_tri, m.n_vert = 5_000_000, 2_600_000
    assert call() == C.VS_ERR_WORKSPACE


def test_render_sh_validation_without_gpu(C):
    L = C.load()
    host, views, meshes, _ = _fake_call_args(C)
    need = L.vs_raster_workspace_bytes(ctypes.addressof(meshes), 2, ctypes.byref(views), None)
    tex = (C.VsShTexture * 2)(*[C.VsShTexture(0x4000, 16, 8) for _ in range(2)])

    def call(opts, t=tex):
        return L.vs_render_sh(ctypes.addressof(meshes), ctypes.addressof(t), 2, ctypes.byref(views), 0x5000,
                              0x100000, need, 0x6000, None if opts is None else ctypes.byref(opts), None)

    assert call(None) == C.VS_ERR_ARG
    assert call(C.VsShOpts(-15.0, 15.0, 0.0, 0, 4, 1)) == C.VS_ERR_UNSUPPORTED      # degree 4
    assert call(C.VsShOpts(-15.0, 15.0, 0.0, 2, 3, 1)) == C.VS_ERR_UNSUPPORTED      # wrap 2
    assert call(C.VsShOpts(15.0, -15.0, 0.0, 0, 3, 1)) == C.VS_ERR_ARG              # vmin >= vmax
    assert call(C.VsShOpts(-15.0, 15.0, 0.0, 0, 3, 2)) == C.VS_ERR_ARG              # view_alpha 2
    tex[1].data = 0x4002
    assert call(C.VsShOpts(-15.0, 15.0, 0.0, 0, 3, 1)) == C.VS_ERR_ARG              # misaligned bytes
    tex[1].data = 0x4000
    tex[0].height = 0
    assert call(C.VsShOpts(-15.0, 15.0, 0.0, 0, 3, 1)) == C.VS_ERR_SIZE
    assert b"SH texture 0" in L.vs_last_error()


def test_ngp_host_calls(C):
    """Parameter count and workspace size are host-only; bad configurations are refused without a GPU."""
    from oracle import ngp as N
    L = C.load()
    res = [4, 8, 18, 40]
    cfg = C.VsNgpConfig(4, 8, (ctypes.c_int32 * 16)(*(res + [0] * 12)))
    assert L.vs_ngp_param_count(ctypes.byref(cfg)) == N.param_count(N.NgpConfig(res, 8))
    w = (ctypes.c_int32 * 2)(40, 33)
    h = (ctypes.c_int32 * 2)(24, 47)
    # 256 staging rows per 16 x 16 tile: (3*2 + 3*3) tiles; 2L + 64*4 + 4 floats per row, 256-byte rounded
    nbytes = L.vs_ngp_workspace_bytes(ctypes.byref(cfg), 2, ctypes.addressof(w), ctypes.addressof(h))
    rows = (3 * 2 + 3 * 3) * 256
    assert nbytes >= rows * (8 + 4 * 64 + 4) * 4
    bad = C.VsNgpConfig(0, 8, (ctypes.c_int32 * 16)())
    assert L.vs_ngp_param_count(ctypes.byref(bad)) == -1
    bad = C.VsNgpConfig(2, 30, (ctypes.c_int32 * 16)(4, 8))
    assert L.vs_ngp_param_count(ctypes.byref(bad)) == -1
    p = (ctypes.c_void_p * 2)(0x10000, 0x20000)
    t = (ctypes.c_void_p * 2)(0x30000, None)
    assert L.vs_ngp_bake(ctypes.addressof(p), ctypes.byref(cfg), 2, ctypes.addressof(w), ctypes.addressof(h),
                         ctypes.addressof(t), None, 0, None) == C.VS_ERR_ARG
    w[0] = 0
    assert L.vs_ngp_bake(ctypes.addressof(p), ctypes.byref(cfg), 2, ctypes.addressof(w), ctypes.addressof(h),
                         ctypes.addressof(t), None, 0, None) == C.VS_ERR_SIZE


def test_ksdf_host_validation(C):
    """Occupancy word counts and option checks of the k-SDF calls, refused on the host without a GPU."""
    L = C.load()
    assert L.vs_ksdf_occupancy_words(256) == 256 ** 3 // 32
    assert L.vs_ksdf_occupancy_words(5) == (125 + 31) // 32
    assert L.vs_ksdf_occupancy_words(0) == 0 and L.vs_ksdf_occupancy_words(2000) == 0
    field = C.VsKsdfField(0x10000, 0x20000, 64, 32, -1.25, 1.25)

    def opts(**kw):
        a = dict(k=3, offsets=[0.0, 0.01, 0.02], beta=1000.0, occ_threshold=1e-4, occ_res=64, n_uniform=64,
                 n_importance=32, march_steps=1024, pdf_floor=1e-5)
        a.update(kw)
        offs = list(a["offsets"]) + [0.0] * (16 - len(a["offsets"]))
        return C.VsKsdfOpts(a["k"], (ctypes.c_double * 16)(*offs), a["beta"], a["occ_threshold"], a["occ_res"],
                            a["n_uniform"], a["n_importance"], a["march_steps"], a["pdf_floor"])

    def occ(o, f=field, out=0x30000):
        return L.vs_ksdf_occupancy(ctypes.byref(f), ctypes.byref(o), out, None)

    assert occ(opts(), out=None) == C.VS_ERR_ARG
    assert occ(opts(k=0)) == C.VS_ERR_ARG
    assert occ(opts(offsets=[0.0, 0.02, 0.01])) == C.VS_ERR_ARG         # offsets must not decrease
    assert occ(opts(beta=0.0)) == C.VS_ERR_ARG
    assert occ(opts(occ_res=0)) == C.VS_ERR_SIZE
    assert occ(opts(n_importance=31)) == C.VS_ERR_ARG
    assert occ(opts(n_uniform=100, n_importance=32)) == C.VS_ERR_ARG    # more than 128 samples
    assert occ(opts(march_steps=1000)) == C.VS_ERR_ARG
    assert occ(opts(pdf_floor=0.0)) == C.VS_ERR_ARG
    assert occ(opts(), f=C.VsKsdfField(0x10000, 0x20008, 64, 32, -1.25, 1.25)) == C.VS_ERR_ARG   # misaligned rgba
    assert occ(opts(), f=C.VsKsdfField(0x10000, 0x20000, 64, 32, 1.0, -1.0)) == C.VS_ERR_ARG
    assert occ(opts(), f=C.VsKsdfField(0x10000, 0x20000, 2048, 32, -1.0, 1.0)) == C.VS_ERR_SIZE
    host, views, _, _ = _fake_call_args(C)
    assert L.vs_ksdf_render(ctypes.byref(field), ctypes.byref(opts()), 0x30000, ctypes.byref(views), None, None,
                            None, None) == C.VS_ERR_ARG
    assert L.vs_ksdf_render(ctypes.byref(field), ctypes.byref(opts()), 0x30000, ctypes.byref(views), 0x40008, None,
                            None, None) == C.VS_ERR_ARG


def test_status_strings(C):
    L = C.load()
    assert L.vs_status_string(0) == b"VS_OK"
    assert L.vs_status_string(3) == b"VS_ERR_WORKSPACE"
    assert L.vs_version().startswith(b"volsurf")


# ---------------------------------------------------------------------------- binding argument checks
class _NoCalls:
    """Stands in for the library: any entry point reached means a check came too late."""

    def __getattr__(self, name):
        raise AssertionError(f"the library was called ({name}) before the arguments were checked")


@pytest.fixture()
def host_scene(C, monkeypatch):
    """A k = 3 scene whose layers and views live in host memory, and a library that must not be called."""
    import torch

    from paper_2409_02482_amd import binding as B
    sc = S.make_config(1, resolution=(24, 16), tex_res=8, with_targets=False)
    layers = B.Layers(sc.layers, device="cpu")
    views = B.Views(sc.cameras, device="cpu")
    monkeypatch.setattr(B.C, "load", lambda: _NoCalls())
    tex = [torch.zeros(8, 8, 4) for _ in range(3)]
    vis = torch.zeros(3 * views.total_pixels, dtype=torch.int64)
    ws = torch.zeros(1024, dtype=torch.uint8)
    return B, layers, views, tex, vis, ws


def test_binding_rejects_wrong_counts_and_shapes(host_scene):
    import torch
    B, layers, views, tex, vis, ws = host_scene
    P = views.total_pixels
    img = torch.zeros(P, 4)
    bad = [
        ("textures", lambda: B.render(layers, tex[:2], views, vis, ws)),
        ("texture shape", lambda: B.render(layers, tex[:2] + [torch.zeros(8, 8, 3)], views, vis, ws)),
        ("vis", lambda: B.render(layers, tex, views, vis[:-1], ws)),
        ("out", lambda: B.render(layers, tex, views, vis, ws, out=torch.zeros(P - 1, 4))),
        ("bwd textures", lambda: B.render_backward(layers, tex[:1], views, vis, ws, grad_rgba=img)),
        ("grad_tex count", lambda: B.render_backward(layers, tex, views, vis, ws, grad_rgba=img,
                                                     grad_tex=[torch.zeros(8, 8, 4)] * 2)),
        ("grad_tex shape", lambda: B.render_backward(layers, tex, views, vis, ws, grad_rgba=img,
                                                     grad_tex=[torch.zeros(8, 8, 4)] * 2 + [torch.zeros(4, 8, 4)])),
        ("grad_rgba", lambda: B.render_backward(layers, tex, views, vis, ws, grad_rgba=torch.zeros(P, 3))),
        ("target", lambda: B.render_backward(layers, tex, views, vis, ws, target=torch.zeros(P + 1, 4))),
        ("bwd out", lambda: B.render_backward(layers, tex, views, vis, ws, grad_rgba=img, out=torch.zeros(2, 4))),
        ("no upstream", lambda: B.render_backward(layers, tex, views, vis, ws)),
        ("bwd vis", lambda: B.render_backward(layers, tex, views, vis[:5], ws, grad_rgba=img)),
        ("raster vis", lambda: B.raster(layers, views, vis=vis[:-3], ws=ws)),
        ("sh count", lambda: B.render_sh(layers, [(torch.zeros(8 * 8 * 64, dtype=torch.uint8), 8, 8)] * 2,
                                         views, vis, ws)),
        ("sh bytes", lambda: B.render_sh(layers, [(torch.zeros(100, dtype=torch.uint8), 8, 8)] * 3,
                                         views, vis, ws)),
        ("adam count", lambda: B.adam_step(tex, tex, tex[:2], tex, torch.zeros(1, dtype=torch.int32))),
        ("adam shape", lambda: B.adam_step(tex, tex, tex[:2] + [torch.zeros(4, 4, 4)], tex,
                                           torch.zeros(1, dtype=torch.int32))),
        ("squeeze", lambda: B.squeeze(tex, tex[:1])),
    ]
    for what, call in bad:
        with pytest.raises(ValueError):
            call()

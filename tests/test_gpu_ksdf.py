"""GPU parity of k-SDF volume rendering (vs_ksdf_occupancy / vs_ksdf_render) against the FP64 oracle.

Bar: occupancy bits identical (decided in FP64 on both sides); colours and
per-surface (C_j, A_j) within 1e-5 max-abs; rays without samples identical;
uniform sample positions bit-exact where no importance round moves them; with
importance rounds, every final sample within one inter-sample gap of the
oracle's (the GPU's interval weights are FP32, which shifts the CDF by about
1e-6 relative: a sample drawn where the pdf is only its floor moves by up to
one gap, and carries no weight, which the colour bar confirms).
Cases: ragged views, a distant camera whose corner rays miss the cube,
k = 1 / 2 / 3 / 7 / 16 (the maximum), offsets inside and outside the main surface (up to
77 / beta), no importance sampling, two-slot sample counts, 64 and
2048 march steps, odd occupancy resolutions (a partial last bit word), and the
full-size grids and views of the bench on 4,800 sampled rays per view (half
of them in the silhouette band).  A ray with a march midpoint within 1e-9
voxel of an interior voxel face (the oracle flags it from its own
coordinates) is left out and counted: which voxel holds such a midpoint
depends on the last bits of its coordinate, so its result is not unique.
"""
import math

import numpy as np
import pytest

import scenes as S
from oracle import ksdf as K
from vs_testlib import say

pytestmark = pytest.mark.gpu

BETA = math.exp(7.0)
TOL = 1e-5


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    import paper_2409_02482_amd as P
    P.load()
    return torch


def _setup(torch, grids, k, occ_res, offsets=None, **kw):
    import paper_2409_02482_amd as P
    field = P.KsdfField(torch.from_numpy(grids.sdf).cuda(), grids.sdf_res,
                        torch.from_numpy(grids.rgba.reshape(-1, 4)).cuda(), grids.rgba_res, grids.lo, grids.hi)
    offs = S.ksdf_offsets(k, BETA) if offsets is None else offsets
    opts = P.ksdf_opts(offs, BETA, occ_res=occ_res, **kw)
    oopts = K.KsdfOpts(offsets=offs, beta=BETA, occ_res=occ_res,
                       **{a: b for a, b in kw.items() if a in ("n_uniform", "n_importance", "march_steps")})
    return P, field, opts, oopts


def _occ_bits(torch, occ, Ro):
    w = occ.cpu().numpy().view(np.uint32)
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint32)[None]) & 1).reshape(-1)
    return bits[:Ro ** 3].reshape(Ro, Ro, Ro).astype(np.uint8)


@pytest.mark.parametrize("occ_res", [40, 37])
def test_ksdf_occupancy_bit_exact(torch_cuda, occ_res):
    torch = torch_cuda
    g = S.ksdf_grids(61, 48, 24)
    P, field, opts, oopts = _setup(torch, g, 3, occ_res)
    occ = P.ksdf_occupancy(field, opts)
    torch.cuda.synchronize()
    got = _occ_bits(torch, occ, occ_res)
    want = K.occupancy(g, oopts)
    say(f"[gpu] ksdf occupancy Ro={occ_res}: {int(want.sum())} occupied, {int((got != want).sum())} differ")
    assert 0 < want.sum() < want.size
    assert np.array_equal(got, want)


CASES = {
    "k3": dict(k=3, kw=dict(n_uniform=64, n_importance=32, march_steps=512)),
    "k7": dict(k=7, kw=dict(n_uniform=64, n_importance=32, march_steps=1024)),
    "k1_no_importance": dict(k=1, kw=dict(n_uniform=32, n_importance=0, march_steps=64)),
    "two_slots": dict(k=2, kw=dict(n_uniform=100, n_importance=28, march_steps=2048)),
    # the maximum number of surfaces
    "k16_max": dict(k=16, kw=dict(n_uniform=64, n_importance=32, march_steps=512)),
    # offsets beyond 60 / beta: one exponential per surface instead of a shared factor
    "wide_offsets": dict(k=3, kw=dict(n_uniform=64, n_importance=32, march_steps=512),
                         offsets=[-0.02, 0.03, 0.07]),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_ksdf_render_matches_oracle(torch_cuda, case):
    torch = torch_cuda
    import paper_2409_02482_amd as P
    c = CASES[case]
    g = S.ksdf_grids(62, 48, 24)
    P, field, opts, oopts = _setup(torch, g, c["k"], 40, offsets=c.get("offsets"), **c["kw"])
    cams = S.ring_cameras(63, 2, [(40, 32), (37, 29)])
    cams.append(S.make_camera(23, 19, [0.5, 0.4, 4.5]))          # corner rays miss the cube
    views = P.Views(cams)
    occ_np = K.occupancy(g, oopts)
    occ = P.ksdf_occupancy(field, opts)
    rgba, lay, smp = P.ksdf_render(field, opts, occ, views, layers=True, samples=True)
    torch.cuda.synchronize()
    assert np.array_equal(_occ_bits(torch, occ, 40), occ_np)
    rgba, lay, smp = rgba.cpu().numpy(), lay.cpu().numpy(), smp.cpu().numpy()
    off = 0
    for v, cam in enumerate(cams):
        want = K.render(g, oopts, occ_np, cam)
        n = cam.width * cam.height
        sl = slice(off, off + n)
        empty_w = want["samples"][:, 0] < 0
        empty_g = smp[sl, 0] < 0
        o, d = K.camera_rays(cam)
        # rays with a march midpoint on a voxel face have no unique result: left out, and counted
        keep = ~K.march_on_face(o, d, oopts.occ_res, g.lo, g.hi, oopts.march_steps)
        t_in, t_out, _ = K.box_interval(o, d, g.lo, g.hi)
        span = np.where(empty_w, 1.0, t_out - t_in)
        dt = np.abs(smp[sl] - want["samples"])
        terr = (dt / span[:, None])[~empty_w & keep].max() if (~empty_w & keep).any() else 0.0
        gap = np.diff(want["samples"], axis=1).max(1)
        err = np.abs(rgba[sl] - want["rgba"])[keep].max()
        lerr = np.abs(lay[:, sl] - want["layers"])[:, keep].max()
        say(f"[gpu] ksdf {case} view {v}: colour err {err:.2e}, layer err {lerr:.2e}, "
            f"sample err {terr:.2e} (x interval), empty rays {int(empty_w.sum())}/{n}, "
            f"face rays left out {int((~keep).sum())}")
        assert (~keep).sum() <= max(1, n // 100)
        assert np.array_equal(empty_g[keep], empty_w[keep])
        assert (smp[sl][empty_w & keep] == -1.0).all() and (rgba[sl][empty_w & keep] == 0.0).all()
        assert err <= TOL and lerr <= TOL
        assert (dt.max(1) <= np.maximum(gap, 0.0))[~empty_w & keep].all()
        if oopts.n_importance == 0:
            assert np.array_equal(smp[sl][keep], want["samples"][keep])
        off += n
    # the distant view has rays that miss the cube and rays that meet no occupied voxel
    assert empty_w.sum() > 0


def test_ksdf_full_size_sampled_rays(torch_cuda):
    """The benchmarked workload (256^3 SDF, 128^3 RGBA, 256^3 occupancy, k = 7, the same 8 ring views at
    512^2) on sampled rays of every view: colours from the benchmarked call (image only, two calls over the
    same buffers), per-surface values from a second call that also writes them."""
    torch = torch_cuda
    import paper_2409_02482_amd as P
    g = S.ksdf_grids(5, 256, 128)
    P, field, opts, oopts = _setup(torch, g, 7, 256)
    cams = S.ring_cameras(5, 8, [(512, 512)] * 8)
    views = P.Views(cams)
    occ = P.ksdf_occupancy(field, opts)
    img = torch.empty(views.total_pixels, 4, dtype=torch.float32, device="cuda")
    for _ in range(2):
        P.ksdf_render(field, opts, occ, views, out=img)
    rgba, lay, smp = P.ksdf_render(field, opts, occ, views, layers=True, samples=True)
    torch.cuda.synchronize()
    assert torch.equal(img, rgba)
    rng = np.random.default_rng(64)
    vox = rng.integers(0, 256 ** 3, 200000)
    got_occ = _occ_bits(torch, occ, 256).reshape(-1)
    assert np.array_equal(got_occ[vox], K.occupancy_at(g, oopts, vox).astype(np.uint8))
    occ_np = K.occupancy(g, oopts)
    assert np.array_equal(got_occ, occ_np.reshape(-1))
    rgba, lay = rgba.cpu().numpy(), lay.cpu().numpy()
    off = 0
    for v, cam in enumerate(cams):
        o, d = K.camera_rays(cam)
        n = cam.width * cam.height
        # 2,400 rays drawn uniformly over the view and 2,400 from the silhouette band of the main surface
        # (rays passing the centre at a distance between 0.9 and 1.1, where the surfaces are grazed)
        miss = np.linalg.norm(np.cross(o, d), axis=1)
        band = np.flatnonzero((miss > 0.9) & (miss < 1.1))
        pick = np.unique(np.concatenate([rng.choice(n, 2400, replace=False), rng.choice(band, 2400, replace=False)]))
        face = K.march_on_face(o[pick], d[pick], oopts.occ_res, g.lo, g.hi, oopts.march_steps)
        pick = pick[~face]
        want = K.render_rays(g, oopts, occ_np, o[pick], d[pick])
        err = np.abs(rgba[off + pick] - want["rgba"]).max()
        lerr = np.abs(lay[:, off + pick] - want["layers"]).max()
        hit = (want["rgba"][:, 3] > 0).sum()
        say(f"[gpu] ksdf full size view {v}: colour err {err:.2e}, layer err {lerr:.2e} on {len(pick)} rays "
            f"({hit} covered, {int(face.sum())} face rays left out)")
        assert err <= TOL and lerr <= TOL and hit > 1000 and len(pick) >= 4000
        assert face.sum() <= len(face) // 100
        off += n

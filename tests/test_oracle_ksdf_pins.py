"""Pins of the k-SDF volume-rendering oracle (Sec. 4.1-4.2, Sec. 4.4), CPU only.

  V1  trilinear field lookups reproduce affine fields exactly at arbitrary
      points (layout [z][y][x], weights and base vertex), clamped outside
  V2  occupancy is conservative: brute force over points inside every voxel of
      an affine SDF (reproduced exactly by the grid) finds no point with density
      above the threshold in a voxel left empty; several surfaces give the union
      of their single-surface grids; a peak density beta/4 below the threshold
      leaves the grid empty
  V3  pixel rays: unit length, the principal-point ray is the camera's forward
      axis from the eye; slab intervals in closed form and against a dense walk
  V4  uniform sampling: with every voxel occupied the samples are the midpoints
      t_in + (i + 1/2)(t_out - t_in)/n; with one occupied slab all samples lie
      in occupied march steps, equally spaced in occupied length
  V5  NeuS weights: along a monotonically decreasing SDF the transmittance
      telescopes, T_i = Phi_i / Phi_0 and sum_i w_i = 1 - Phi_{N-1} / Phi_0
  V6  importance sampling: linear inversion of the piecewise-constant pdf
      equals np.interp on the CDF; zero weights give the uniform-pdf quantiles;
      merging keeps the samples sorted and their SDF values attached
  V7  normals of an affine SDF are its unit gradient, and on a generic grid the
      gradient equals central differences inside cells; blending constant
      appearance over planes facing the camera gives the closed-form
      composite sum_j xi a alpha_w (1 - a alpha_w)^j
  V8  rays that miss the cube or meet no occupied voxel render zero
  V9  appearance is taken at the start of each interval: a left Riemann-Stieltjes
      sum of a monotone field lies on the known side of the continuous value
"""
import math

import numpy as np
import pytest

import scenes as S
from oracle import ksdf as K

BETA = math.exp(7.0)


def _grids(sdf_coef, res=16, rgba=None, rgba_res=8, lo=-1.0, hi=1.0):
    sdf = S.affine_grid(res, lo, hi, sdf_coef)
    if rgba is None:
        rgba = np.tile(np.float32([0.2, 0.5, 0.8, 0.6]), ((rgba_res + 1) ** 3, 1))
    return S.KsdfGrids(sdf, res, rgba, rgba_res, lo, hi)


def test_v1_trilinear_reproduces_affine():
    coef = (0.3, -0.7, 0.25, 1.1)
    g = S.affine_grid(12, -1.5, 2.0, coef).astype(np.float64)
    rng = np.random.default_rng(1)
    p = rng.uniform(-1.5, 2.0, (500, 3))
    got = K.trilinear(g.reshape(-1, 1), 12, -1.5, 2.0, p)[:, 0]
    want = coef[0] + p @ np.asarray(coef[1:])
    np.testing.assert_allclose(got, want, atol=2e-6)        # the grid holds f32 vertex values
    # outside the cube the lookup clamps to the boundary
    q = np.array([[3.0, 0.0, 0.0], [0.0, -4.0, 0.5], [0.1, 0.2, 9.0]])
    got = K.trilinear(g.reshape(-1, 1), 12, -1.5, 2.0, q)[:, 0]
    want = coef[0] + np.clip(q, -1.5, 2.0) @ np.asarray(coef[1:])
    np.testing.assert_allclose(got, want, atol=2e-6)
    # a 4-channel grid: each channel its own affine field
    coefs = [(0.1, 1, 0, 0), (0.2, 0, 1, 0), (0.3, 0, 0, 1), (0.4, 1, 1, 1)]
    g4 = np.stack([S.affine_grid(6, -1, 1, c) for c in coefs], -1)
    p = rng.uniform(-1, 1, (50, 3))
    got = K.trilinear(g4, 6, -1, 1, p)
    for ch, c in enumerate(coefs):
        np.testing.assert_allclose(got[:, ch], c[0] + p @ np.asarray(c[1:], float), atol=2e-6)


def test_v2_occupancy_conservative_union_and_empty():
    n = np.array([0.48, -0.6, 0.64])                        # unit normal
    g = _grids((0.05, *n), res=16)
    opts = K.KsdfOpts(offsets=[0.0], beta=60.0, occ_res=12, occ_threshold=1e-2)
    occ = K.occupancy(g, opts)
    assert 0 < occ.sum() < occ.size
    # brute force: points inside each voxel (corners, centre, random); density above the threshold -> occupied
    Ro, ho = 12, 2.0 / 12
    rng = np.random.default_rng(2)
    offs = np.concatenate([np.array([[a, b, c] for a in (0, 1) for b in (0, 1) for c in (0, 1)], float),
                           [[0.5, 0.5, 0.5]], rng.uniform(0, 1, (24, 3))])
    idx = np.stack(np.meshgrid(np.arange(Ro), np.arange(Ro), np.arange(Ro), indexing="ij"), -1).reshape(-1, 3)
    pts = -1.0 + (idx[:, None, ::-1] + offs[None]) * ho          # [voxel, point, xyz]
    dens = K.logistic_density(0.05 + pts @ n, 60.0)
    must = (dens > 1e-2).any(1).reshape(Ro, Ro, Ro)
    assert not (must & (occ == 0)).any()
    # several surfaces: the union of their single-surface grids
    offsets = [0.0, 0.2, 0.45]
    occ3 = K.occupancy(g, K.KsdfOpts(offsets=offsets, beta=60.0, occ_res=12, occ_threshold=1e-2))
    union = np.zeros_like(occ3)
    for o in offsets:
        union |= K.occupancy(g, K.KsdfOpts(offsets=[o], beta=60.0, occ_res=12, occ_threshold=1e-2))
    assert np.array_equal(occ3, union) and occ3.sum() > occ.sum()
    # peak density beta/4 at or below the threshold: nothing is occupied
    assert K.occupancy(g, K.KsdfOpts(offsets=[0.0], beta=4e-2, occ_res=12, occ_threshold=1e-2)).sum() == 0


def test_v3_rays_and_slabs():
    cam = S.make_camera(33, 21, [0.4, -0.7, 2.5])
    o, v = K.camera_rays(cam)
    np.testing.assert_allclose(np.linalg.norm(v, axis=1), 1.0, atol=1e-15)
    np.testing.assert_allclose(o[0], [0.4, -0.7, 2.5], atol=1e-14)
    # the ray through the principal point (W/2, H/2) is the forward axis: use an even-sized camera
    cam2 = S.make_camera(32, 20, [0.4, -0.7, 2.5])
    o2, v2 = K.camera_rays(cam2)
    fwd = -np.array([0.4, -0.7, 2.5]) / np.linalg.norm([0.4, -0.7, 2.5])
    centre = v2.reshape(20, 32, 3)[9:11, 15:17].mean((0, 1))
    np.testing.assert_allclose(centre / np.linalg.norm(centre), fwd, atol=1e-12)
    # slabs: a ray along -z from z = 3 through (0.2, -0.3) meets [-1, 1]^3 on [2, 4]
    t_in, t_out, hit = K.box_interval(np.array([[0.2, -0.3, 3.0], [2.0, 0.0, 3.0]]),
                                      np.array([[0.0, 0.0, -1.0], [0.0, 0.0, -1.0]]), -1.0, 1.0)
    assert hit.tolist() == [True, False]
    assert (t_in[0], t_out[0]) == (2.0, 4.0)
    # oblique rays: the interval is where a dense walk along the ray is inside the cube
    rng = np.random.default_rng(3)
    o = rng.uniform(-3.0, 3.0, (20, 3)) + np.array([0.0, 0.0, 4.0])
    v = rng.normal(size=(20, 3)) - np.array([0.0, 0.0, 2.0])
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    t_in, t_out, hit = K.box_interval(o, v, -1.0, 1.0)
    ts = np.linspace(0.0, 12.0, 240001)
    for r in range(20):
        inside = (np.abs(o[r][None] + ts[:, None] * v[r][None]) <= 1.0).all(1)
        assert hit[r] == inside.any()
        if inside.any():
            assert abs(ts[inside][0] - t_in[r]) <= 1e-4 and abs(ts[inside][-1] - t_out[r]) <= 1e-4
    # a diagonal ray from outside a corner
    d = np.array([[-1.0, -1.0, -1.0]]) / math.sqrt(3.0)
    t_in, t_out, hit = K.box_interval(np.array([[2.0, 2.0, 2.0]]), d, -1.0, 1.0)
    np.testing.assert_allclose([t_in[0], t_out[0]], [math.sqrt(3.0), 3 * math.sqrt(3.0)], rtol=1e-15)


def test_v4_uniform_samples():
    o = np.array([[0.1, 0.2, 3.0], [-0.3, 0.1, 3.0]])
    v = np.array([[0.0, 0.0, -1.0], [0.05, -0.02, -1.0]])
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    t_in, t_out, hit = K.box_interval(o, v, -1.0, 1.0)
    full = np.ones((8, 8, 8), np.uint8)
    st = K.march_occupied(o, v, t_in, t_out, full, -1.0, 1.0, 256)
    assert st.all()
    t = K.uniform_samples(t_in, t_out, st, 64)
    want = t_in[:, None] + (np.arange(64) + 0.5)[None] * ((t_out - t_in) / 64)[:, None]
    np.testing.assert_allclose(t, want, rtol=1e-14)
    # one occupied slab of voxels z in [0, 0.75) (254 steps put a slab face inside a step, past its midpoint)
    slab = np.zeros((8, 8, 8), np.uint8)
    slab[4:7] = 1
    st = K.march_occupied(o, v, t_in, t_out, slab, -1.0, 1.0, 254)
    t = K.uniform_samples(t_in, t_out, st, 64)
    z = o[:, None, 2] + t * v[:, None, 2]
    D = (t_out - t_in) / 254
    assert (z > -D[:, None]).all() and (z < 0.75 + D[:, None]).all()
    # the occupied steps are exactly those whose midpoint lies in the slab
    tm = t_in[:, None] + (np.arange(254)[None] + 0.5) * D[:, None]
    zm = o[:, None, 2] + tm * v[:, None, 2]
    assert np.array_equal(st, (zm >= 0.0) & (zm < 0.75))
    gaps = np.diff(t, axis=1)
    np.testing.assert_allclose(gaps, gaps[:, :1] * np.ones_like(gaps), rtol=1e-9)


def test_v5_neus_weights_telescope():
    rng = np.random.default_rng(5)
    d = np.sort(rng.uniform(-0.05, 0.05, (4, 40)), axis=1)[:, ::-1].copy()     # decreasing along each ray
    for off in (0.0, 0.01):
        w = K.neus_weights(d, off, 300.0)
        phi = K.logistic_cdf(d + off, 300.0)
        np.testing.assert_allclose(w.sum(1), 1.0 - phi[:, -1] / phi[:, 0], rtol=1e-12)
        T = np.cumsum(np.concatenate([np.zeros((4, 1)), w], 1), 1)[:, :-1]    # weight mass before interval i
        np.testing.assert_allclose(1.0 - T, phi[:, :-1] / phi[:, :1], rtol=1e-10, atol=1e-15)
    # increasing SDF (ray leaving the surface): no weight
    assert K.neus_weights(d[:, ::-1].copy(), 0.0, 300.0).sum() == 0.0


def test_v6_importance_sampling():
    rng = np.random.default_rng(6)
    t = np.sort(rng.uniform(1.0, 2.0, (3, 20)), axis=1)
    d = np.sort(rng.uniform(-0.05, 0.05, (3, 20)), axis=1)[:, ::-1].copy()
    offsets = [0.0, 0.012]
    tn = K.importance_round(t, d, offsets, 200.0, 16, 1e-5)
    W = sum(K.neus_weights(d, o, 200.0) for o in offsets)
    u = (np.arange(16) + 0.5) / 16
    for r in range(3):
        pdf = (W[r] + 1e-5) / (W[r] + 1e-5).sum()
        cdf = np.concatenate([[0.0], np.cumsum(pdf)])
        np.testing.assert_allclose(tn[r], np.interp(u, cdf, t[r]), rtol=1e-13)
    assert (np.diff(tn, axis=1) >= 0).all()
    # zero weights (far outside every surface): quantiles of the uniform pdf over the N-1 intervals
    far = np.full((3, 20), 5.0)
    tn = K.importance_round(t, far, offsets, 200.0, 16, 1e-5)
    x = u * 19
    i = np.floor(x).astype(int)
    want = t[:, i] + (x - i) * (t[:, i + 1] - t[:, i])
    np.testing.assert_allclose(tn, want, rtol=1e-12)
    # merging keeps order and carries the SDF values
    tt, dd = K.merge_sorted(t, d, tn, -tn)
    assert (np.diff(tt, axis=1) >= 0).all()
    for r in range(3):
        lookup = dict(zip(t[r], d[r]))
        lookup.update(zip(tn[r], -tn[r]))
        assert all(lookup[a] == b for a, b in zip(tt[r], dd[r]))


def test_v7_normals_and_blend_closed_form():
    n = np.array([0.6, 0.0, -0.8])
    g = _grids((0.1, *n), res=8)
    p = np.random.default_rng(7).uniform(-0.8, 0.8, (40, 3))
    np.testing.assert_allclose(K.sdf_normals(g, p), np.tile(n, (40, 1)), atol=1e-6)
    # a generic grid: the gradient equals central differences of the lookup away from cell faces
    gg = S.ksdf_grids(7, 12, 4)
    rng = np.random.default_rng(8)
    inv = 12 / (gg.hi - gg.lo)
    q = rng.uniform(gg.lo + 0.1, gg.hi - 0.1, (400, 3))
    frac = (q - gg.lo) * inv % 1.0
    q = q[((frac > 0.01) & (frac < 0.99)).all(1)]
    fd = np.stack([(K.sdf_at(gg, q + h) - K.sdf_at(gg, q - h)) / 2e-5 for h in np.eye(3) * 1e-5], 1)
    np.testing.assert_allclose(K.sdf_gradient(gg, q), fd, rtol=1e-6, atol=1e-8)
    # planes z = 0 - o_j facing a camera on +z; constant appearance (xi, a); densities peaked enough for
    # each surface's weights to sum to 1 over the samples
    xi, a = np.array([0.2, 0.5, 0.8]), 0.6
    g = _grids((0.0, 0.0, 0.0, 1.0), res=16, lo=-1.0, hi=1.0)
    offsets = [0.0, 0.05, 0.1]
    opts = K.KsdfOpts(offsets=offsets, beta=2000.0, occ_res=32, n_uniform=64, n_importance=32, march_steps=512)
    occ = K.occupancy(g, opts)
    o = np.array([[0.05, -0.1, 2.0], [0.3, 0.2, 2.0]])
    v = np.array([[0.0, 0.0, -1.0], [0.0, 0.0, -1.0]])
    out = K.render_rays(g, opts, occ, o, v)
    aw = 2.0 / (1.0 + math.exp(-10.0)) - 1.0
    A = a * aw
    want_rgb = sum(xi * A * (1 - A) ** j for j in range(3))
    np.testing.assert_allclose(out["rgba"][:, :3], np.tile(want_rgb, (2, 1)), atol=1e-9)
    np.testing.assert_allclose(out["rgba"][:, 3], 1 - (1 - A) ** 3, atol=1e-9)
    np.testing.assert_allclose(out["layers"][:, :, 3], A, atol=1e-9)


def test_v8_empty_rays():
    g = _grids((0.0, 0.0, 0.0, 1.0), res=8)
    opts = K.KsdfOpts(offsets=[0.0], beta=500.0, occ_res=8, n_uniform=16, n_importance=8, march_steps=128)
    occ = K.occupancy(g, opts)
    o = np.array([[3.0, 3.0, 3.0], [0.5, 0.5, 3.0]])
    v = np.array([[0.0, 0.0, -1.0], [0.0, 0.0, -1.0]])
    out = K.render_rays(g, opts, np.zeros_like(occ), o, v)
    assert (out["rgba"] == 0).all() and (out["samples"] == -1).all()
    out = K.render_rays(g, opts, occ, o, v)
    assert (out["rgba"][0] == 0).all() and out["rgba"][1, 3] > 0.5


def test_v9_appearance_at_section_starts():
    """A single plane crossed along -z with appearance decreasing along the ray: each interval takes the
    appearance at its start, so the quadrature lies above the continuous value xi(t_surface) (a logistic
    crossing centred on the surface) by less than the largest sample gap times the slope."""
    g = _grids((0.0, 0.0, 0.0, 1.0), res=16, lo=-1.0, hi=1.0)
    rgba = S.affine_grid(8, -1.0, 1.0, (0.5, 0.0, 0.0, 0.3))                  # xi = 0.5 + 0.3 z
    g.rgba = np.stack([rgba, rgba, rgba, np.ones_like(rgba)], -1)
    opts = K.KsdfOpts(offsets=[0.0], beta=150.0, occ_res=32, n_uniform=32, n_importance=16, march_steps=512,
                      occ_threshold=1e-3)
    occ = K.occupancy(g, opts)
    o = np.array([[0.05, -0.1, 2.0]])
    v = np.array([[0.0, 0.0, -1.0]])
    out = K.render_rays(g, opts, occ, o, v)
    C, t = out["layers"][0, 0, 0], out["samples"][0]
    wsum = out["layers"][0, 0, 3] / (2.0 / (1.0 + math.exp(-10.0)) - 1.0)
    cont = 0.5 * wsum                                                         # xi(z = 0) = 0.5, times sum w
    gap = np.diff(t)[np.abs(o[0, 2] - t[:-1]) < 0.1].max()
    assert cont < C < cont + 0.3 * gap

"""Pins of the oracle's baked spherical-harmonic appearance (Sec. 4.3, Sec. 4.2), CPU only.

  S1  the SH basis against SciPy's complex spherical harmonics, turned into the
      real form (this pins every constant and sign convention)
  S2  orthonormality of the basis by exact quadrature on the sphere
  S3  a camera-facing quad with one coefficient image affine in the texel
      indices at its own level resolution and every other coefficient constant:
      closed form sigmoid(sum_i sh_i Y_i(v)) per pixel, with and without the
      grazing-angle alpha weight, for every level
  S4  coefficients above the requested degree are never read
  S5  two layers: the closed-form fixed-order blend of two constant SH shells
"""
import numpy as np
import pytest
from scipy.special import sph_harm_y

import scenes as S

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


def _real_sh_scipy(d):
    """Real orthonormal SH (index l^2 + l + m), built from SciPy's complex ones (Condon-Shortley phase)."""
    d = np.asarray(d, np.float64)
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    theta = np.arccos(np.clip(z, -1.0, 1.0))        # polar
    phi = np.arctan2(y, x)                          # azimuth
    out = np.empty((d.shape[0], 16))
    for l in range(4):
        for m in range(-l, l + 1):
            c = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                val = np.sqrt(2.0) * (-1.0) ** m * c.real
            elif m < 0:
                val = np.sqrt(2.0) * (-1.0) ** m * c.imag
            else:
                val = c.real
            out[:, l * l + l + m] = val
    return out


def _unit(rng, n):
    d = rng.normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_s1_basis_matches_scipy(oracle_lib):
    O = oracle_lib
    d = _unit(np.random.default_rng(1), 64)
    d = np.vstack([d, np.eye(3), -np.eye(3)])
    np.testing.assert_allclose(O.sh_basis(d), _real_sh_scipy(d), atol=1e-13)


def test_s2_orthonormal_by_quadrature(oracle_lib):
    """Gauss-Legendre in cos(theta) x uniform azimuth integrates products of degree <= 6 exactly."""
    O = oracle_lib
    ct, wt = np.polynomial.legendre.leggauss(8)
    phis = 2 * np.pi * np.arange(16) / 16
    st = np.sqrt(1 - ct ** 2)
    d = np.array([[s * np.cos(p), s * np.sin(p), c] for c, s in zip(ct, st) for p in phis])
    w = np.array([wc * 2 * np.pi / 16 for wc in wt for _ in phis])
    Y = O.sh_basis(d)
    gram = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(16), atol=1e-12)


def _facing_quad(x0, x1, y0, y1, z):
    xyz = np.array([[x0, y0, z], [x1, y0, z], [x1, y1, z], [x0, y1, z]], np.float32)
    uv = np.array([[0, 0], [1, 0], [1, 1], [0, 1]], np.float32)
    tri = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    return S.Mesh(xyz, uv, tri)


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _decode(q, vmin, vmax):
    return vmin + (vmax - vmin) * np.asarray(q, np.float64) / 255.0


def _const_levels(rng, W0, H0, degree):
    """Per level: a constant byte per (coefficient, channel), broadcast over the texels."""
    levels, consts = [], []
    for l in range(degree + 1):
        w, h = S.sh_level_dims(W0, H0, l)
        c = rng.integers(100, 156, (2 * l + 1, 4)).astype(np.uint8)
        consts.append(c)
        levels.append(np.broadcast_to(c, (h, w, 2 * l + 1, 4)).copy())
    return levels, consts


@pytest.mark.parametrize("view_alpha", [False, True])
@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_s3_affine_coefficient_closed_form(oracle_lib, level, view_alpha):
    O = oracle_lib
    W = H = 96
    cam = S.Camera(W, H, 60.0, 55.0, 47.0, 49.0, np.eye(3), np.zeros(3))
    mesh = _facing_quad(-0.7, 0.72, -0.75, 0.68, 1.0)
    W0, H0, deg, vmin, vmax = 32, 16, 3, -15.0, 15.0
    rng = np.random.default_rng(10 + level)
    levels, consts = _const_levels(rng, W0, H0, deg)
    # coefficient m* of degree `level` is affine in the texel indices of its own level, in every channel
    mstar = level  # the middle-ish coefficient of the degree (m index within 0..2l)
    wl, hl = S.sh_level_dims(W0, H0, level)
    ii, jj = np.meshgrid(np.arange(wl), np.arange(hl))
    # a + b i + c j per channel, slopes doubled per level so that the range stays inside [0, 255]
    aff = [(a, b << level, c << level) for a, b, c in [(40, 3, 4), (200, -3, -3), (90, 3, -2), (150, -2, 3)]]
    for ch, (a, b, c) in enumerate(aff):
        vals = a + b * ii + c * jj
        assert vals.min() >= 0 and vals.max() <= 255
        levels[level][:, :, mstar, ch] = vals.astype(np.uint8)
    tex = S.sh_pack(levels, W0, H0)
    vis = O.raster_layers([mesh], cam)
    img = O.shade_sh([mesh], [tex], cam, vis, degree=deg, vmin=vmin, vmax=vmax, wrap=0, view_alpha=view_alpha)
    # closed form: the quad is fronto-parallel, so UV is affine in screen space between its snapped corners
    X, Y, _, _ = O.project(mesh, cam)
    xs0, xs1, ys0, ys1 = X[0] / 256, X[1] / 256, Y[0] / 256, Y[2] / 256
    j, i = np.mgrid[0:H, 0:W].astype(np.float64)
    u = (i + 0.5 - xs0) / (xs1 - xs0)
    v = (j + 0.5 - ys0) / (ys1 - ys0)
    dc = np.stack([(i + 0.5 - cam.cx) / cam.fx, (j + 0.5 - cam.cy) / cam.fy, np.ones_like(i)], -1)
    d = dc / np.linalg.norm(dc, axis=-1, keepdims=True)
    Yb = _real_sh_scipy(d.reshape(-1, 3)).reshape(H, W, 16)
    x_l, y_l = u * wl - 0.5, v * hl - 0.5
    raw = np.zeros((H, W, 4))
    for l in range(deg + 1):
        for m in range(2 * l + 1):
            for ch in range(4):
                if l == level and m == mstar:
                    a, b, c = aff[ch]
                    sh = _decode(a + b * x_l + c * y_l, vmin, vmax)   # bilinear reproduces the affine map
                else:
                    sh = _decode(consts[l][m, ch], vmin, vmax)
                raw[..., ch] += sh * Yb[..., l * l + m]
    rgba = _sigmoid(raw)
    if view_alpha:
        rgba[..., 3] *= 2 * _sigmoid(10 * np.abs(d[..., 2])) - 1       # face normal is +-z
    want = np.empty_like(rgba)
    want[..., :3] = rgba[..., :3] * rgba[..., 3:4]
    want[..., 3] = rgba[..., 3]
    hit = vis[0] != EMPTY
    sel = hit & (x_l >= 0) & (x_l <= wl - 1) & (y_l >= 0) & (y_l <= hl - 1)
    assert sel.sum() > 0.25 * W * H
    np.testing.assert_allclose(img[sel], want[sel], atol=1e-12)
    assert np.all(img[~hit] == 0.0)


def test_s4_higher_degrees_are_not_read(oracle_lib):
    O = oracle_lib
    cam = S.Camera(48, 40, 40.0, 40.0, 24.0, 20.0, np.eye(3), np.zeros(3))
    mesh = _facing_quad(-0.5, 0.5, -0.45, 0.5, 1.0)
    vis = O.raster_layers([mesh], cam)
    t = S.sh_texture(3, 0, 16, 16, degree=3)
    for deg in range(3):
        low = S.sh_pack(S.sh_unpack(t)[:deg + 1], 16, 16)
        garbled = S.sh_unpack(t)
        for l in range(deg + 1, 4):
            garbled[l] = np.full_like(garbled[l], 255)
        a = O.shade_sh([mesh], [low], cam, vis, degree=deg)
        b = O.shade_sh([mesh], [S.sh_pack(garbled, 16, 16)], cam, vis, degree=deg)
        assert np.array_equal(a, b)
    full = O.shade_sh([mesh], [t], cam, vis, degree=3)
    assert not np.array_equal(full, O.shade_sh([mesh], [t], cam, vis, degree=2))


def test_s5_two_constant_layers_blend(oracle_lib):
    O = oracle_lib
    cam = S.Camera(40, 40, 30.0, 30.0, 20.0, 20.0, np.eye(3), np.zeros(3))
    outer = _facing_quad(-0.6, 0.6, -0.6, 0.6, 1.0)
    inner = _facing_quad(-0.4, 0.5, -0.5, 0.4, 1.5)
    rng = np.random.default_rng(5)
    texs, consts = [], []
    for _ in range(2):
        lv, c = _const_levels(rng, 8, 8, 1)
        texs.append(S.sh_pack(lv, 8, 8))
        consts.append(c)
    vis = O.raster_layers([outer, inner], cam)
    img = O.shade_sh([outer, inner], texs, cam, vis, degree=1, view_alpha=False)
    j, i = np.mgrid[0:40, 0:40].astype(np.float64)
    dc = np.stack([(i + 0.5 - 20) / 30, (j + 0.5 - 20) / 30, np.ones_like(i)], -1)
    d = dc / np.linalg.norm(dc, axis=-1, keepdims=True)
    Yb = _real_sh_scipy(d.reshape(-1, 3)).reshape(40, 40, 16)

    def layer_rgba(c):
        raw = np.zeros((40, 40, 4))
        for l in range(2):
            for m in range(2 * l + 1):
                raw += _decode(c[l][m], -15, 15)[None, None, :] * Yb[..., l * l + m, None]
        return _sigmoid(raw)

    r0, r1 = layer_rgba(consts[0]), layer_rgba(consts[1])
    h0, h1 = vis[0] != EMPTY, vis[1] != EMPTY
    a0 = np.where(h0, r0[..., 3], 0.0)
    a1 = np.where(h1, r1[..., 3], 0.0)
    C = a0[..., None] * r0[..., :3] + (1 - a0)[..., None] * a1[..., None] * r1[..., :3]
    A = 1 - (1 - a0) * (1 - a1)
    assert (h0 & h1).sum() > 100 and not (h1 & ~h0).any()
    np.testing.assert_allclose(img[..., :3], C, atol=1e-12)
    np.testing.assert_allclose(img[..., 3], A, atol=1e-12)

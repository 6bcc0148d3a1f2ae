"""Pins of the oracle's L1 loss adjoint and of squeezing + quantisation (Sec. 4.3), CPU only.

  Q1  L1 adjoint against central finite differences: the loss is piecewise
      linear in one texel scalar, so with a step below every residual's distance
      to its kink the difference quotient is exact up to rounding
  Q2  L1 adjoint = the (P6-pinned) linear-loss adjoint with the upstream
      gradient sign(RGB - target), alpha 0
  Q3  squeeze + quantise: values on the grid k / levels, monotone in the logit,
      the tie at sigmoid(0) = 1/2 (127.5 -> 128, ties to even), saturation,
      levels = 0 leaves the sigmoid unquantised, and a brute-force nearest-grid
      search agrees everywhere off ties
"""
import numpy as np
import pytest

import scenes as S
from test_oracle_pins import _pick_entries, _small_shells


def _setup(scene):
    if scene == "cfg1":
        sc = S.make_config(1, resolution=(128, 128), tex_res=64)
        return sc.layers, sc.textures, sc.cameras[0]
    meshes = _small_shells(k=4)
    tex = [S.smooth_texture(81, l, 48, 32, opaque=(l == 3)) for l in range(4)]
    return meshes, tex, S.ring_cameras(81, 1, [(120, 96)])[0]


@pytest.mark.parametrize("scene", ["cfg1", "shells"])
def test_q1_l1_adjoint_equals_central_fd(oracle_lib, scene):
    O = oracle_lib
    meshes, tex, cam = _setup(scene)
    vis = O.raster_layers(meshes, cam)
    tgt = S.uniform_targets(81, [cam])[0]
    img = O.shade(meshes, tex, cam, vis)
    resid = np.abs(img[..., :3] - tgt[..., :3].astype(np.float64))
    h = 1e-7
    # a texel scalar moves a pixel's colour by at most h (bilinear weight <= 1, alpha and T <= 1
    # for colour channels; an alpha texel moves C by at most h * max|c - S| <= h): keep the kinks away
    assert resid.min() > 10 * h
    grads = O.backward(meshes, tex, cam, vis, target=tgt, loss="l1")
    rng = np.random.default_rng(82)
    ent = np.concatenate([_pick_entries(rng, grads, 48), _pick_entries(rng, grads, 16, nonzero=False)])
    fd = O.finite_diff(meshes, tex, cam, vis, ent, h=h, target=tgt, loss="l1")
    an = np.array([grads[l][j, i, ch] for l, j, i, ch in ent])
    scale = np.abs(an).max()
    np.testing.assert_allclose(an, fd, rtol=1e-6, atol=1e-7 * scale)
    assert np.count_nonzero(an) >= 48


def test_q2_l1_adjoint_is_linear_adjoint_with_sign_upstream(oracle_lib):
    O = oracle_lib
    meshes, tex, cam = _setup("shells")
    vis = O.raster_layers(meshes, cam)
    tgt = S.uniform_targets(83, [cam])[0]
    img = O.shade(meshes, tex, cam, vis)
    g = np.zeros(img.shape)
    g[..., :3] = np.sign(img[..., :3] - tgt[..., :3].astype(np.float64))
    a = O.backward(meshes, tex, cam, vis, target=tgt, loss="l1")
    b = O.backward(meshes, tex, cam, vis, grad_out=g)
    for x, y in zip(a, b):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-12)
    # and L1 is not L2 (the loss switch is honoured)
    c = O.backward(meshes, tex, cam, vis, target=tgt, loss="l2")
    assert max(np.abs(x - y).max() for x, y in zip(a, c)) > 1e-3


def test_q3_squeeze_quantize(oracle_lib):
    O = oracle_lib
    theta = np.linspace(-12.0, 12.0, 20001)
    q = O.squeeze_quantize(theta, 255).astype(np.float64)
    codes = q * 255.0
    np.testing.assert_allclose(codes, np.round(codes), atol=1e-4)          # on the grid (f32 storage)
    assert np.all(np.diff(q) >= 0.0)                                         # monotone
    assert O.squeeze_quantize(np.array([0.0]), 255)[0] == np.float32(128 / 255)   # 127.5 -> 128
    assert O.squeeze_quantize(np.array([-40.0]), 255)[0] == 0.0
    assert O.squeeze_quantize(np.array([40.0]), 255)[0] == 1.0
    s = 1.0 / (1.0 + np.exp(-theta))
    np.testing.assert_allclose(O.squeeze_quantize(theta, 0), s.astype(np.float32), rtol=0, atol=0)
    # brute force: the nearest of the 256 grid values, away from ties
    grid = np.arange(256) / 255.0
    near = grid[np.argmin(np.abs(s[:, None] - grid[None, :]), axis=1)]
    off_tie = np.abs(s * 255.0 - np.floor(s * 255.0) - 0.5) > 1e-9
    np.testing.assert_array_equal(q[off_tie], near[off_tie].astype(np.float32))

"""Hand-derived worked example for the oracle (tests/golden/tiny_triangle.json)."""
import json
import os

import numpy as np

import scenes as S

HERE = os.path.dirname(os.path.abspath(__file__))


def _load():
    fx = json.load(open(os.path.join(HERE, "golden", "tiny_triangle.json")))
    c = fx["camera"]
    cam = S.Camera(c["width"], c["height"], c["fx"], c["fy"], c["cx"], c["cy"],
                   np.array(c["R"], float).reshape(3, 3), np.array(c["t"], float), c["z_near"])
    mesh = S.Mesh(np.array(fx["xyz"], np.float32), np.array(fx["uv"], np.float32), np.array(fx["tri"], np.int32))
    return fx, cam, mesh


def test_golden_coverage_and_key(oracle_lib):
    fx, cam, mesh = _load()
    vis, st = oracle_lib.raster(mesh, cam)
    cov = (vis != oracle_lib.EMPTY).astype(int)
    assert cov.tolist() == fx["covered"]
    key = np.uint64(int(fx["depth_key_hex"], 16))
    assert np.all(vis[cov == 1] == key)


def test_golden_colour(oracle_lib):
    fx, cam, mesh = _load()
    tex = np.array(fx["texture_2x2_rgba"], np.float32)
    vis, img = oracle_lib.render([mesh], [tex], cam)
    i, j = fx["pixel"]
    np.testing.assert_allclose(img[j, i], fx["colour_single_layer"], atol=1e-15)
    front = S.constant_texture(2, 2, fx["two_layers"]["front_rgba"])
    vis2, img2 = oracle_lib.render([mesh, mesh], [front, tex], cam)
    np.testing.assert_allclose(img2[j, i], fx["two_layers"]["colour"], atol=1e-15)

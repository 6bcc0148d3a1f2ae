"""Pins of the neural-texture oracle (hash-grid encoding + MLP at texel centres, Sec. 4.3), CPU only.

  N1  vertex indexing: dense levels are a bijection of the (N+1)^2 vertices onto
      0..(N+1)^2-1 in row-major order; hashed levels reduce the spatial hash
      (x * 1 XOR y * 2654435761) mod 2^32 to the table, checked on hand-worked
      values and against Python's unbounded integers
  N2  bilinear interpolation: dense-level tables holding an affine function of
      the vertex coordinates reproduce it exactly at every texel centre; a
      constant hashed table gives the constant
  N3  the MLP: weights that pass features through give the closed form
      sigmoid of a ReLU of an affine map
  N4  the analytic backward against central finite differences on parameters of
      every kind (tables of dense and hashed levels, weights, biases); the
      network is piecewise linear up to the sigmoid, so away from ReLU kinks
      the difference quotient is exact up to rounding
"""
import numpy as np
import pytest

import scenes as S
from oracle import ngp as N


def _cfg(levels=4, base=4, finest=40, log2_table=8):
    return N.NgpConfig(S.ngp_resolutions(levels, base, finest), log2_table)


def test_n1_vertex_indexing():
    # dense: N = 5 -> 36 vertices <= 64
    x, y = np.meshgrid(np.arange(6), np.arange(6))
    q = N.vertex_index(x.reshape(-1), y.reshape(-1), 5, 64)
    assert sorted(q.tolist()) == list(range(36)) and q[7] == 1 * 6 + 1
    # hashed: N = 20 -> 441 vertices > 256
    T = 256
    assert N.vertex_index(np.array([3]), np.array([0]), 20, T)[0] == 3
    assert N.vertex_index(np.array([0]), np.array([1]), 20, T)[0] == 2654435761 % 256      # 177
    assert N.vertex_index(np.array([5]), np.array([1]), 20, T)[0] == (5 ^ 2654435761) % 256
    rng = np.random.default_rng(1)
    xs, ys = rng.integers(0, 5000, 200), rng.integers(0, 5000, 200)
    want = [((int(a) ^ ((int(b) * 2654435761) % 2 ** 32)) % 2 ** 32) % T for a, b in zip(xs, ys)]
    assert N.vertex_index(xs, ys, 4999, T).tolist() == want


def test_n2_bilinear_reproduces_affine_tables():
    cfg = _cfg(levels=3, base=4, finest=7, log2_table=8)       # resolutions 4, 5, 7: all dense
    assert all((n + 1) ** 2 <= cfg.table for n in cfg.resolutions)
    tables = np.zeros((cfg.levels, cfg.table, 2))
    coef = [(0.3, 0.05, -0.02), (-0.1, 0.01, 0.04), (0.2, -0.03, 0.03)]
    for l, n in enumerate(cfg.resolutions):
        for y in range(n + 1):
            for x in range(n + 1):
                a, b, c = coef[l]
                tables[l, y * (n + 1) + x] = [a + b * x + c * y, 2 * a - c * x + b * y]
    u, v = N.texel_centres(13, 9)
    e = N.encode(tables, cfg, u, v)
    for l, n in enumerate(cfg.resolutions):
        a, b, c = coef[l]
        np.testing.assert_allclose(e[:, 2 * l], a + b * u * n + c * v * n, atol=1e-14)
        np.testing.assert_allclose(e[:, 2 * l + 1], 2 * a - c * u * n + b * v * n, atol=1e-14)
    # a hashed level with a constant table gives the constant
    cfg2 = N.NgpConfig([30], 6)
    t2 = np.full((1, 64, 2), [0.25, -0.5])
    np.testing.assert_allclose(N.encode(t2, cfg2, u, v), np.tile([0.25, -0.5], (u.size, 1)), atol=1e-15)


def test_n3_mlp_closed_form():
    cfg = N.NgpConfig([3], 4)
    lay = N.param_layout(cfg)
    p = np.zeros(N.param_count(cfg))

    def put(name, arr):
        o, s = lay[name]
        p[o:o + int(np.prod(s))] = np.asarray(arr, np.float64).reshape(-1)

    tables = np.zeros((1, 16, 2))
    tables[0, :, 0] = 0.7
    tables[0, :, 1] = -0.4
    put("tables", tables)
    W1 = np.zeros((64, 2)); W1[0, 0] = 2.0; W1[1, 1] = 3.0; W1[2, 0] = -1.0
    put("W1", W1); put("b1", np.r_[0.1, 2.0, 0.0, np.zeros(61)])
    W2 = np.eye(64); put("W2", W2); put("b2", np.zeros(64))
    W3 = np.zeros((4, 64)); W3[0, 0] = 1.0; W3[1, 1] = 1.0; W3[2, 2] = 5.0; W3[3, 0] = -1.0; W3[3, 1] = 0.5
    put("W3", W3); put("b3", [0.0, 0.0, 0.3, 0.2])
    h = [max(2 * 0.7 + 0.1, 0), max(3 * -0.4 + 2.0, 0), max(-0.7, 0)]
    o = np.array([h[0], h[1], 5 * h[2] + 0.3, -h[0] + 0.5 * h[1] + 0.2])
    tex = N.bake(p, cfg, 5, 4)
    np.testing.assert_allclose(tex, np.broadcast_to(1 / (1 + np.exp(-o)), (4, 5, 4)), atol=1e-15)


def test_n4_backward_equals_central_fd():
    cfg = _cfg(levels=4, base=4, finest=40, log2_table=8)    # levels 4, 8, 18, 40: the last two hashed
    assert any((n + 1) ** 2 > cfg.table for n in cfg.resolutions)
    p = S.ngp_params(5, 0, cfg.levels, cfg.log2_table).astype(np.float64)
    W, H = 24, 20
    g = np.random.default_rng(6).uniform(-1, 1, (H, W, 4))
    grad = N.backward(p, cfg, W, H, g)
    lay = N.param_layout(cfg)
    rng = np.random.default_rng(7)
    picks = []
    for name in ("tables", "W1", "b1", "W2", "b2", "W3", "b3"):
        o, s = lay[name]
        n = int(np.prod(s))
        cand = np.arange(o, o + n)
        if name == "tables":
            cand = cand[np.abs(grad[o:o + n]) > 0]
        picks += list(rng.choice(cand, size=min(8, cand.size), replace=False))
    h = 1e-6

    def loss(q):
        return float((N.bake(q, cfg, W, H) * g).sum())

    fd = []
    for i in picks:
        qp, qm = p.copy(), p.copy()
        qp[i] += h
        qm[i] -= h
        fd.append((loss(qp) - loss(qm)) / (2 * h))
    fd = np.array(fd)
    an = grad[picks]
    np.testing.assert_allclose(an, fd, rtol=1e-5, atol=1e-7 * np.abs(fd).max())
    assert np.count_nonzero(an) >= len(picks) - 4

"""Neural texture oracle (FP64, NumPy) -- TEST INFRASTRUCTURE ONLY.

A neural texture (Sec. 4.3 "Texturing Meshes") is a 2-D multiresolution hash
grid followed by a small MLP; it is grounded to a target resolution by
evaluating it at the texel centres only (Sec. 4.3, Fig. 5), which gives an
ordinary RGBA texture that the renderer samples bilinearly.

Definitions (our reading where the paper gives no numbers):
  * level l of L has resolution N_l (given); its vertices are the integer
    points 0..N_l of x = u N_l, y = v N_l;
  * a level with (N_l + 1)^2 <= T vertices is stored densely,
    index = y (N_l + 1) + x; otherwise index = (x * 1 XOR y * 2654435761) mod 2^32,
    masked to T - 1 (T a power of two; the spatial hash of Instant-NGP);
  * each vertex holds F = 2 features; the level's feature at (u, v) is the
    bilinear interpolation of its 4 surrounding vertices; the encoding is the
    concatenation over levels (level-major);
  * MLP: z1 = W1 e + b1, h1 = relu(z1) (64); z2 = W2 h1 + b2, h2 = relu(z2) (64);
    o = W3 h2 + b3 (4); texel RGBA = sigmoid(o);
  * texel (i, j) is evaluated at its centre ((i + 1/2)/W, (j + 1/2)/H).

Parameters of one layer are one flat float array:
  tables [L][T][F] | W1 [64][L F] | b1 [64] | W2 [64][64] | b2 [64] | W3 [4][64] | b3 [4].
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List

import numpy as np

HIDDEN = 64
OUT = 4
FEATURES = 2
PRIME_Y = 2654435761


@dataclass
class NgpConfig:
    resolutions: List[int]   # N_l per level
    log2_table: int          # T = 2^log2_table entries per level

    @property
    def levels(self) -> int:
        return len(self.resolutions)

    @property
    def table(self) -> int:
        return 1 << self.log2_table


def param_layout(cfg: NgpConfig) -> Dict[str, tuple]:
    """name -> (offset, shape) in the flat parameter array."""
    L, T, F = cfg.levels, cfg.table, FEATURES
    shapes = [("tables", (L, T, F)), ("W1", (HIDDEN, L * F)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)),
              ("b2", (HIDDEN,)), ("W3", (OUT, HIDDEN)), ("b3", (OUT,))]
    out, off = {}, 0
    for name, shape in shapes:
        out[name] = (off, shape)
        off += int(np.prod(shape))
    out["total"] = (off, ())
    return out


def param_count(cfg: NgpConfig) -> int:
    return param_layout(cfg)["total"][0]


def unpack(params: np.ndarray, cfg: NgpConfig) -> Dict[str, np.ndarray]:
    lay = param_layout(cfg)
    p = np.asarray(params, np.float64)
    return {k: p[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in lay.items() if k != "total"}


def vertex_index(x: np.ndarray, y: np.ndarray, N: int, T: int) -> np.ndarray:
    x = np.asarray(x, np.uint64)
    y = np.asarray(y, np.uint64)
    if (N + 1) ** 2 <= T:
        return (y * np.uint64(N + 1) + x).astype(np.int64)
    h = (x ^ ((y * np.uint64(PRIME_Y)) & np.uint64(0xFFFFFFFF))) & np.uint64(0xFFFFFFFF)
    return (h & np.uint64(T - 1)).astype(np.int64)


def texel_centres(W: int, H: int):
    j, i = np.mgrid[0:H, 0:W]
    return ((i + 0.5) / W).reshape(-1), ((j + 0.5) / H).reshape(-1)


def encode(tables: np.ndarray, cfg: NgpConfig, u: np.ndarray, v: np.ndarray, with_corners: bool = False):
    """[n, L F] encoding; optionally the per-level corner indices [L][4][n] and weights [L][4][n]."""
    n = u.shape[0]
    e = np.zeros((n, cfg.levels * FEATURES))
    corners = []
    for l, N in enumerate(cfg.resolutions):
        x, y = u * N, v * N
        x0, y0 = np.floor(x), np.floor(y)
        fx, fy = x - x0, y - y0
        xi, yi = x0.astype(np.int64), y0.astype(np.int64)
        idx, wts = [], []
        for dy in (0, 1):
            for dx in (0, 1):
                w = (fx if dx else 1 - fx) * (fy if dy else 1 - fy)
                q = vertex_index(xi + dx, yi + dy, N, cfg.table)
                e[:, l * FEATURES:(l + 1) * FEATURES] += w[:, None] * tables[l][q]
                idx.append(q)
                wts.append(w)
        corners.append((idx, wts))
    return (e, corners) if with_corners else e


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def forward(params: np.ndarray, cfg: NgpConfig, u: np.ndarray, v: np.ndarray):
    P = unpack(params, cfg)
    e, corners = encode(P["tables"], cfg, u, v, with_corners=True)
    z1 = e @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    o = h2 @ P["W3"].T + P["b3"]
    return dict(e=e, corners=corners, z1=z1, h1=h1, z2=z2, h2=h2, o=o, t=_sigmoid(o))


def bake(params: np.ndarray, cfg: NgpConfig, W: int, H: int) -> np.ndarray:
    """The RGBA texture [H, W, 4] the neural texture stands for (evaluated at texel centres)."""
    u, v = texel_centres(W, H)
    return forward(params, cfg, u, v)["t"].reshape(H, W, OUT)


def backward(params: np.ndarray, cfg: NgpConfig, W: int, H: int, dtex: np.ndarray) -> np.ndarray:
    """dL/dparams (flat, FP64) given dL/dtexture [H, W, 4] of the baked texture."""
    P = unpack(params, cfg)
    u, v = texel_centres(W, H)
    f = forward(params, cfg, u, v)
    g = np.asarray(dtex, np.float64).reshape(-1, OUT)
    do = g * f["t"] * (1.0 - f["t"])
    dW3 = do.T @ f["h2"]
    db3 = do.sum(0)
    dz2 = (do @ P["W3"]) * (f["z2"] > 0)
    dW2 = dz2.T @ f["h1"]
    db2 = dz2.sum(0)
    dz1 = (dz2 @ P["W2"]) * (f["z1"] > 0)
    dW1 = dz1.T @ f["e"]
    db1 = dz1.sum(0)
    de = dz1 @ P["W1"]
    dtab = np.zeros_like(P["tables"])
    for l, (idx, wts) in enumerate(f["corners"]):
        for q, w in zip(idx, wts):
            for c in range(FEATURES):
                np.add.at(dtab[l, :, c], q, w * de[:, l * FEATURES + c])
    out = np.zeros(param_count(cfg))
    lay = param_layout(cfg)
    for name, arr in (("tables", dtab), ("W1", dW1), ("b1", db1), ("W2", dW2), ("b2", db2), ("W3", dW3),
                      ("b3", db3)):
        o, s = lay[name]
        out[o:o + int(np.prod(s))] = arr.reshape(-1)
    return out

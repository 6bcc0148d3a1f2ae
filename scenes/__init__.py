"""Seeded synthetic inputs for the layered-mesh renderer.

This module only *builds inputs*: nested closed triangle-mesh shells with
per-vertex UVs, RGBA UV textures, pinhole cameras and loss targets.  It holds
none of the renderer's arithmetic (no projection, snapping, rasterisation,
texture filtering or compositing), so both the CPU oracle and the HIP path can
consume its output without sharing any of the method's code.

The scenes stand in for the baked shells of the paper (a main surface plus k-1
support shells that never intersect, traversed outermost to innermost,
Sec. 4.1 "Support Surfaces as Shells"; baked meshes with UV atlases and
resolution-grounded textures, Sec. 4.3).  The paper's datasets and trained
assets are not used: smooth, nested, closed, star-shaped shells of about 1e5
triangles per layer with 1024^2 textures have the same structure.

Conventions (shared by every consumer):
  * layer 0 is the OUTERMOST shell;
  * a mesh is (xyz f32 [V,3], uv f32 [V,2], tri i32 [T,3]), triangles wound
    counter-clockwise seen from outside (outward normals);
  * a texture is f32 [H,W,4] straight RGBA, row j holds v in [j/H,(j+1)/H);
  * a camera is world->camera (R, t) in OpenCV axes (x right, y down,
    z forward) with pinhole intrinsics fx, fy, cx, cy in pixels; pixel (i, j)
    has its centre at (i + 0.5, j + 0.5).

Seeds: every random draw uses ``np.random.default_rng([config, purpose, index])``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# purposes for the seed sequence [config, purpose, index]
P_GEOMETRY = 1
P_TEXTURE = 2
P_CAMERA = 3
P_TARGET = 4
P_GT_TEXTURE = 5
P_UPSTREAM = 6
P_PICK = 7
P_SH = 8
P_NGP = 9
P_KSDF = 10

Z_NEAR = 0.01


# --------------------------------------------------------------------------
# data containers
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Mesh:
    xyz: np.ndarray   # f32 [V,3]
    uv: np.ndarray    # f32 [V,2]
    tri: np.ndarray   # i32 [T,3]

    @property
    def n_vert(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tri(self) -> int:
        return int(self.tri.shape[0])


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray      # f64 [3,3] world->camera rotation, rows (right, down, forward)
    t: np.ndarray      # f64 [3]
    z_near: float = Z_NEAR

    @property
    def n_pix(self) -> int:
        return self.width * self.height


@dataclasses.dataclass
class Scene:
    name: str
    layers: List[Mesh]
    textures: List[np.ndarray]          # f32 [H,W,4] each
    cameras: List[Camera]
    targets: Optional[List[np.ndarray]] = None   # f32 [H,W,4] per view (A unused)
    description: str = ""

    @property
    def k(self) -> int:
        return len(self.layers)


# --------------------------------------------------------------------------
# cameras
# --------------------------------------------------------------------------
def look_at(eye: Sequence[float], target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)) -> Tuple[np.ndarray, np.ndarray]:
    """World->camera (R, t) for an OpenCV camera at ``eye`` looking at ``target``.

    Rows of R are the camera axes in world coordinates: right, down, forward.
    """
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f = f / np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r = r / np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f], 0)
    t = -R @ eye
    return R, t


def pinhole(width: int, height: int, fov_y_deg: float = 40.0) -> Tuple[float, float, float, float]:
    """Square-pixel intrinsics from a vertical field of view; principal point at the centre."""
    fy = (height / 2.0) / math.tan(math.radians(fov_y_deg) / 2.0)
    return fy, fy, width / 2.0, height / 2.0


def make_camera(width: int, height: int, eye, fov_y_deg: float = 40.0, target=(0.0, 0.0, 0.0)) -> Camera:
    R, t = look_at(eye, target)
    fx, fy, cx, cy = pinhole(width, height, fov_y_deg)
    return Camera(width, height, fx, fy, cx, cy, R, t)


def ring_cameras(config: int, n: int, resolutions: Sequence[Tuple[int, int]], distance: float = 3.0,
                 fov_y_deg: float = 40.0, elev_deg: float = 15.0) -> List[Camera]:
    """``n`` cameras on a jittered ring around the origin.

    Azimuth 2*pi*v/n + U(+-pi/n), elevation U[-elev, elev], looking at the
    origin.  ``resolutions`` has one (W, H) per view.
    """
    rng = np.random.default_rng([config, P_CAMERA, 0])
    az = 2 * np.pi * np.arange(n) / n + rng.uniform(-np.pi / n, np.pi / n, n)
    el = np.radians(rng.uniform(-elev_deg, elev_deg, n))
    cams = []
    for v in range(n):
        eye = distance * np.array([np.cos(el[v]) * np.sin(az[v]), np.sin(el[v]), np.cos(el[v]) * np.cos(az[v])])
        w, h = resolutions[v]
        cams.append(make_camera(w, h, eye, fov_y_deg))
    return cams


MIXED_RESOLUTIONS = [(512, 512), (640, 480), (800, 800), (1024, 768), (1024, 1024),
                     (1280, 720), (1600, 900), (1920, 1080)]


def mixed_resolutions(config: int, n: int) -> List[Tuple[int, int]]:
    """n/8 views of each of the eight mixed resolutions, in seeded shuffled order."""
    per = n // len(MIXED_RESOLUTIONS)
    res = [r for r in MIXED_RESOLUTIONS for _ in range(per)]
    res += MIXED_RESOLUTIONS[: n - len(res)]
    rng = np.random.default_rng([config, P_CAMERA, 1])
    order = rng.permutation(len(res))
    return [res[i] for i in order]


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
def _orient_outward(pos: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """Flip triangles whose normal points towards the origin (star-shaped surfaces)."""
    a, b, c = pos[tri[:, 0]], pos[tri[:, 1]], pos[tri[:, 2]]
    n = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", n, (a + b + c)) < 0
    tri = tri.copy()
    tri[flip, 1], tri[flip, 2] = tri[flip, 2].copy(), tri[flip, 1].copy()
    return tri


def icosphere(subdiv: int) -> Tuple[np.ndarray, np.ndarray]:
    """Unit icosphere: 10*4^s+2 vertices, 20*4^s faces (outward)."""
    p = (1 + 5 ** 0.5) / 2
    v = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0), (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
         (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4), (11, 10, 2),
         (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9), (4, 9, 5),
         (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(x, np.float64) / np.linalg.norm(x) for x in v]
    faces = list(f)
    for _ in range(subdiv):
        cache = {}

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    pos = np.array(verts)
    tri = _orient_outward(pos, np.array(faces, np.int64))
    return pos, tri


def _sphere_uv(d: np.ndarray) -> np.ndarray:
    """Spherical UV, polar axis +y: u = lon/(2 pi) + 1/2 with lon = atan2(x, z), v = polar angle / pi."""
    lon = np.arctan2(d[:, 0], d[:, 2])
    u = lon / (2 * np.pi) + 0.5
    v = np.arccos(np.clip(d[:, 1], -1.0, 1.0)) / np.pi
    return np.stack([u, v], 1)


def spherical_uv_mesh(dirs: np.ndarray, tri: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Give a unit-sphere mesh per-vertex spherical UVs.

    Corners of seam-crossing triangles get u+1 (so u in [0, 1.5)), on
    duplicated vertices; a pole vertex is duplicated per triangle with u set to
    the mean of the other two corners.  Returns (dirs', uv, tri').
    """
    uv = _sphere_uv(dirs)
    pole = np.abs(np.abs(dirs[:, 1]) - 1.0) < 1e-12
    out_dirs = list(dirs)
    out_uv = [tuple(x) for x in uv]
    dup = {}
    new_tri = tri.copy()
    for t in range(tri.shape[0]):
        idx = list(tri[t])
        us = [uv[i, 0] for i in idx]
        np_idx = [i for i in idx if not pole[i]]
        nu = [uv[i, 0] for i in np_idx]
        shift = (max(nu) - min(nu)) > 0.5 if nu else False
        corner_u = []
        for i in idx:
            u = uv[i, 0]
            if shift and not pole[i] and u < 0.5:
                u = u + 1.0
            corner_u.append(u)
        for c, i in enumerate(idx):
            if pole[i]:
                others = [corner_u[q] for q in range(3) if not pole[idx[q]]]
                u = float(np.mean(others))
                key = (i, round(u, 12))
            else:
                u = corner_u[c]
                if u == uv[i, 0]:
                    continue
                key = (i, round(u, 12))
            if key not in dup:
                out_dirs.append(dirs[i])
                out_uv.append((u, uv[i, 1]))
                dup[key] = len(out_dirs) - 1
            new_tri[t, c] = dup[key]
    return np.array(out_dirs), np.array(out_uv), new_tri


def latlong_mesh(n_lat: int, n_lon: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Unit-sphere lat-long grid, polar axis +y.

    (n_lat-1) rings of (n_lon+1) vertices (seam column duplicated, u = j/n_lon)
    plus two pole vertices (u = 0.5); quads split in two; each pole cap is a fan.
    Vertices: (n_lat-1)*(n_lon+1)+2.  Triangles: 2*n_lon*(n_lat-1).
    """
    rings = n_lat - 1
    th = np.pi * np.arange(1, n_lat) / n_lat
    u = np.arange(n_lon + 1) / n_lon
    lon = 2 * np.pi * (u - 0.5)
    TH, LON = np.meshgrid(th, lon, indexing="ij")
    d = np.stack([np.sin(TH) * np.sin(LON), np.cos(TH), np.sin(TH) * np.cos(LON)], -1).reshape(-1, 3)
    uv = np.stack(np.broadcast_arrays(u[None, :], (th / np.pi)[:, None]), -1).reshape(-1, 2)
    north = rings * (n_lon + 1)
    south = north + 1
    d = np.concatenate([d, [[0.0, 1.0, 0.0], [0.0, -1.0, 0.0]]], 0)
    uv = np.concatenate([uv, [[0.5, 0.0], [0.5, 1.0]]], 0)
    vid = np.arange(rings * (n_lon + 1)).reshape(rings, n_lon + 1)
    tris = []
    a = vid[:-1, :-1]; b = vid[:-1, 1:]; c = vid[1:, :-1]; e = vid[1:, 1:]
    tris.append(np.stack([a, c, b], -1).reshape(-1, 3))
    tris.append(np.stack([b, c, e], -1).reshape(-1, 3))
    j = np.arange(n_lon)
    tris.append(np.stack([np.full(n_lon, north), vid[0, j + 1], vid[0, j]], -1))
    tris.append(np.stack([np.full(n_lon, south), vid[-1, j], vid[-1, j + 1]], -1))
    tri = np.concatenate(tris, 0).astype(np.int64)
    tri = _orient_outward(d, tri)
    return d, uv, tri


def sine_field(config: int, n_terms: int = 8):
    """Seeded smooth field s(x) = (1/n) sum_m sin(w_m <n_m, x> + phi_m), |s| <= 1."""
    rng = np.random.default_rng([config, P_GEOMETRY, 0])
    nm = rng.normal(size=(n_terms, 3))
    nm /= np.linalg.norm(nm, axis=1, keepdims=True)
    om = rng.uniform(2.0, 6.0, n_terms)
    ph = rng.uniform(0.0, 2 * np.pi, n_terms)

    def s(x: np.ndarray) -> np.ndarray:
        return np.sin((x @ nm.T) * om + ph).mean(axis=1)

    return s


def displaced_shells(config: int, k: int, n_lat: int, n_lon: int, amp: float = 0.05,
                     offset: float = 0.06) -> List[Mesh]:
    """k nested level sets R_o(x) = 1 + o + amp*s(x) of a displaced sphere SDF.

    Offsets o = linspace(-offset, +offset, k); layer 0 has o = +offset (outermost).
    The displacement is shared by all shells, so shells are nested and never touch.
    """
    d, uv, tri = latlong_mesh(n_lat, n_lon)
    s = sine_field(config)(d)
    offs = np.linspace(-offset, offset, k)[::-1]
    out = []
    for o in offs:
        pos = d * (1.0 + o + amp * s)[:, None]
        out.append(Mesh(pos.astype(np.float32), uv.astype(np.float32), tri.astype(np.int32)))
    return out


def icosphere_shells(radii: Sequence[float], subdiv: int = 3) -> List[Mesh]:
    dirs, tri = icosphere(subdiv)
    dirs, uv, tri = spherical_uv_mesh(dirs, tri)
    return [Mesh((dirs * r).astype(np.float32), uv.astype(np.float32), tri.astype(np.int32)) for r in radii]


# --------------------------------------------------------------------------
# textures and targets
# --------------------------------------------------------------------------
def uniform_texture(config: int, layer: int, w: int, h: int, opaque: bool, purpose: int = P_TEXTURE) -> np.ndarray:
    """RGB i.i.d. U[0,1], alpha i.i.d. U[0.1,0.9] (alpha = 1 if opaque)."""
    rng = np.random.default_rng([config, purpose, layer])
    t = np.empty((h, w, 4), np.float32)
    t[..., :3] = rng.uniform(0.0, 1.0, (h, w, 3))
    t[..., 3] = 1.0 if opaque else rng.uniform(0.1, 0.9, (h, w))
    return t


def smooth_texture(config: int, layer: int, w: int, h: int, opaque: bool, purpose: int = P_TEXTURE) -> np.ndarray:
    """Per channel 0.5 + 0.5*(1/6) sum_m sin(2 pi (a_m u + b_m v) + phi_m), a_m, b_m in [1,8] integers.

    Integer a_m keeps the texture periodic in u.  Alpha is mapped to [0.1, 0.9]
    (alpha = 1 if opaque).  Sampled at texel centres ((i+.5)/W, (j+.5)/H).
    """
    rng = np.random.default_rng([config, purpose, layer])
    u = (np.arange(w) + 0.5) / w
    v = (np.arange(h) + 0.5) / h
    t = np.empty((h, w, 4), np.float32)
    for ch in range(4):
        a = rng.integers(1, 9, 6)
        b = rng.integers(1, 9, 6)
        ph = rng.uniform(0, 2 * np.pi, 6)
        acc = np.zeros((h, w))
        for m in range(6):
            acc += np.sin(2 * np.pi * (a[m] * u[None, :] + b[m] * v[:, None]) + ph[m])
        val = 0.5 + 0.5 * acc / 6.0
        if ch == 3:
            val = 1.0 if opaque else 0.1 + 0.8 * val
        t[..., ch] = val
    return t


def constant_texture(w: int, h: int, rgba: Sequence[float]) -> np.ndarray:
    t = np.empty((h, w, 4), np.float32)
    t[...] = np.asarray(rgba, np.float32)
    return t


@dataclasses.dataclass
class ShTexture:
    """A shell's baked spherical-harmonic texture: 8-bit coefficients, packed by level.

    Degree l (0..degree) is stored at level l of max(1, width >> l) x max(1, height >> l)
    texels, levels one after another, each texel-major [H_l][W_l][2l+1][4] (the 2l+1
    coefficients of a texel adjacent, each as R, G, B, A bytes)."""
    data: np.ndarray      # uint8 [total bytes]
    width: int            # level-0 size
    height: int
    degree: int


def sh_level_dims(width: int, height: int, level: int) -> Tuple[int, int]:
    return max(1, width >> level), max(1, height >> level)


def sh_pack(levels: Sequence[np.ndarray], width: int, height: int) -> ShTexture:
    """Pack per-level arrays [H_l][W_l][2l+1][4] (uint8) into an ShTexture."""
    for l, a in enumerate(levels):
        w, h = sh_level_dims(width, height, l)
        assert a.shape == (h, w, 2 * l + 1, 4) and a.dtype == np.uint8, (l, a.shape)
    data = np.concatenate([np.ascontiguousarray(a).reshape(-1) for a in levels])
    return ShTexture(data, width, height, len(levels) - 1)


def sh_unpack(t: ShTexture) -> List[np.ndarray]:
    out, off = [], 0
    for l in range(t.degree + 1):
        w, h = sh_level_dims(t.width, t.height, l)
        n = h * w * (2 * l + 1) * 4
        out.append(t.data[off:off + n].reshape(h, w, 2 * l + 1, 4))
        off += n
    return out


def sh_texture(config: int, layer: int, width: int, height: int, degree: int = 3, opaque: bool = False) -> ShTexture:
    """Seeded 8-bit SH coefficients, i.i.d. per texel (the hardest case for filtering).

    With the decoding range [-15, 15]: degree-0 RGB bytes in [68, 187] (the DC term alone
    gives colours sigmoid([-2, 2])), degree-0 alpha bytes in [105, 187] (255 if opaque), and
    every higher-degree byte in [115, 140] (coefficients within +-1.5)."""
    rng = np.random.default_rng([config, P_SH, layer])
    levels = []
    for l in range(degree + 1):
        w, h = sh_level_dims(width, height, l)
        if l == 0:
            a = np.empty((h, w, 1, 4), np.uint8)
            a[..., :3] = rng.integers(68, 188, (h, w, 1, 3), dtype=np.uint8)
            a[..., 3] = 255 if opaque else rng.integers(105, 188, (h, w, 1), dtype=np.uint8)
        else:
            a = rng.integers(115, 141, (h, w, 2 * l + 1, 4), dtype=np.uint8)
        levels.append(a)
    return sh_pack(levels, width, height)


def ngp_resolutions(levels: int, base: int, finest: int) -> List[int]:
    """Geometric level resolutions floor(base * b^l), b = (finest / base)^(1 / (levels - 1))."""
    if levels == 1:
        return [base]
    b = np.exp((np.log(finest) - np.log(base)) / (levels - 1))
    return [int(np.floor(base * b ** l + 1e-9)) for l in range(levels)]


def ngp_params(config: int, layer: int, levels: int, log2_table: int, hidden: int = 64, out: int = 4,
               features: int = 2, table_scale: float = 1.0) -> np.ndarray:
    """Seeded flat f32 parameters of one neural texture: tables U(-s, s), weights N(0, 1/fan_in), biases 0.1 N(0, 1).

    Layout: tables [L][T][F] | W1 [hidden][L F] | b1 | W2 [hidden][hidden] | b2 | W3 [out][hidden] | b3."""
    rng = np.random.default_rng([config, P_NGP, layer])
    T = 1 << log2_table
    parts = [rng.uniform(-table_scale, table_scale, levels * T * features),
             rng.normal(0.0, 1.0 / np.sqrt(levels * features), hidden * levels * features),
             0.1 * rng.normal(size=hidden),
             rng.normal(0.0, 1.0 / np.sqrt(hidden), hidden * hidden), 0.1 * rng.normal(size=hidden),
             rng.normal(0.0, 1.0 / np.sqrt(hidden), out * hidden), 0.1 * rng.normal(size=out)]
    return np.concatenate(parts).astype(np.float32)


@dataclasses.dataclass
class KsdfGrids:
    """Fields of a k-SDF on the cube [lo, hi]^3 given at grid vertices ([z][y][x] order).

    ``sdf`` f32 [(R+1)^3] is the main signed distance (positive outside);
    ``rgba`` f32 [(Ra+1)^3, 4] is straight RGB plus the transparency field.
    """
    sdf: np.ndarray
    sdf_res: int
    rgba: np.ndarray
    rgba_res: int
    lo: float
    hi: float


def _grid_points(res: int, lo: float, hi: float) -> np.ndarray:
    ax = lo + (hi - lo) * np.arange(res + 1) / res
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    return np.stack([x.reshape(-1), y.reshape(-1), z.reshape(-1)], -1)


def ksdf_grids(config: int, sdf_res: int, rgba_res: int, lo: float = -1.25, hi: float = 1.25,
               amp: float = 0.05) -> KsdfGrids:
    """The displaced sphere |x| - (1 + amp s(x/|x|)) of the shell scenes as a vertex grid, and a smooth RGBA field.

    Appearance per channel: 0.5 + 0.5 (1/6) sum_m sin(<f_m, x> + phi_m) with
    |f_m| in [2, 8]; the transparency channel is mapped to [0.1, 0.9].
    """
    p = _grid_points(sdf_res, lo, hi)
    r = np.linalg.norm(p, axis=1)
    dirs = np.where(r[:, None] > 0, p / np.maximum(r, 1e-300)[:, None], np.array([0.0, 1.0, 0.0]))
    sdf = (r - (1.0 + amp * sine_field(config)(dirs))).astype(np.float32)
    q = _grid_points(rgba_res, lo, hi)
    rng = np.random.default_rng([config, P_KSDF, 0])
    rgba = np.empty((q.shape[0], 4), np.float32)
    for ch in range(4):
        f = rng.normal(size=(6, 3))
        f *= (rng.uniform(2.0, 8.0, 6) / np.linalg.norm(f, axis=1))[:, None]
        ph = rng.uniform(0.0, 2 * np.pi, 6)
        val = 0.5 + 0.5 * np.sin(q @ f.T + ph).mean(axis=1)
        rgba[:, ch] = 0.1 + 0.8 * val if ch == 3 else val
    return KsdfGrids(sdf, sdf_res, rgba, rgba_res, lo, hi)


def affine_grid(res: int, lo: float, hi: float, coef: Sequence[float]) -> np.ndarray:
    """f32 [(res+1)^3] vertex values of a + b x + c y + d z (grid values of an affine field)."""
    p = _grid_points(res, lo, hi)
    return (coef[0] + p @ np.asarray(coef[1:4], np.float64)).astype(np.float32)


def ksdf_offsets(k: int, beta: float) -> List[float]:
    """Support shells inside the main surface at multiples of the logistic standard deviation pi / (sqrt(3) beta)."""
    step = math.pi / (math.sqrt(3.0) * beta)
    return [j * step for j in range(k)]


def uniform_targets(config: int, cams: Sequence[Camera]) -> List[np.ndarray]:
    """Per-view target images, RGB i.i.d. U[0,1], A = 0 (unused by the RGB L2 loss)."""
    out = []
    for v, c in enumerate(cams):
        rng = np.random.default_rng([config, P_TARGET, v])
        t = np.zeros((c.height, c.width, 4), np.float32)
        t[..., :3] = rng.random((c.height, c.width, 3), dtype=np.float32)
        out.append(t)
    return out


# --------------------------------------------------------------------------
# the benchmark configurations
# --------------------------------------------------------------------------
CONFIG_NAMES = {
    1: "k3-icosphere-256",
    2: "k7-displaced-1024",
    3: "k7-displaced-1024-fwdbwd",
    4: "k9-300k-64views-mixed",
    5: "k7-fit-128views-800",
    6: "k7-1024-64views-fwdbwd",
}


def make_config(i: int, *, n_views: Optional[int] = None, resolution: Optional[Tuple[int, int]] = None,
                latlong: Optional[Tuple[int, int]] = None, tex_res: Optional[int] = None,
                with_targets: bool = True) -> Scene:
    """Build configuration ``i``.

    1: k=3 icosphere shells (subdiv 3, radii 1.0/0.9/0.8), 256^2 view at distance 3,
       fov 40, 256^2 i.i.d. textures, innermost alpha 1.
    2: k=7 displaced shells (offsets -0.06..0.06, amplitude 0.05, lat-long 160x320,
       101,760 triangles per layer), 1024^2 single view, 1024^2 smooth textures.
    3: config 2 plus i.i.d. targets for an RGB L2 loss.
    4: k=9 displaced shells, lat-long 274x548 (299,208 triangles per layer), 64 ring
       views of mixed resolution 512^2..1920x1080, targets.
    5: config-2 shells seen from 128 ring views at 800^2; textures initialised to
       RGB 0.5, alpha 0.5 (innermost 1); the ground-truth textures are returned as
       ``textures_gt`` attribute (config-2 recipe, different seed).
    6: config-2 shells seen from 64 ring views at 1024^2, with targets.
    Optional overrides shrink a configuration for tests (views, resolution,
    mesh density, texture size).
    """
    name = CONFIG_NAMES[i]
    if i == 1:
        layers = icosphere_shells([1.0, 0.9, 0.8], subdiv=3)
        tr = tex_res or 256
        tex = [uniform_texture(1, l, tr, tr, opaque=(l == 2)) for l in range(3)]
        w, h = resolution or (256, 256)
        cams = [make_camera(w, h, (0.0, 0.0, 3.0))]
        return Scene(name, layers, tex, cams, None, "k=3 icosphere shells, forward")
    if i in (2, 3, 5, 6):
        k = 7
        nl, nL = latlong or (160, 320)
        layers = displaced_shells(2, k, nl, nL)
        tr = tex_res or 1024
        if i == 5:
            tex = []
            for l in range(k):
                t = np.empty((tr, tr, 4), np.float32)
                t[..., :3] = 0.5
                t[..., 3] = 1.0 if l == k - 1 else 0.5
                tex.append(t)
        else:
            tex = [smooth_texture(2, l, tr, tr, opaque=(l == k - 1)) for l in range(k)]
        if i in (2, 3):
            w, h = resolution or (1024, 1024)
            cams = [make_camera(w, h, (0.0, 0.0, 3.0))]
        elif i == 5:
            n = n_views or 128
            cams = ring_cameras(5, n, [resolution or (800, 800)] * n)
        else:
            n = n_views or 64
            cams = ring_cameras(6, n, [resolution or (1024, 1024)] * n)
        targets = uniform_targets(i, cams) if (with_targets and i in (3, 6)) else None
        sc = Scene(name, layers, tex, cams, targets, "k=7 displaced shells")
        if i == 5:
            sc.textures_gt = [smooth_texture(5, l, tr, tr, opaque=(l == k - 1), purpose=P_GT_TEXTURE)
                              for l in range(k)]
        return sc
    if i == 4:
        k = 9
        nl, nL = latlong or (274, 548)
        layers = displaced_shells(2, k, nl, nL)
        tr = tex_res or 1024
        tex = [smooth_texture(4, l, tr, tr, opaque=(l == k - 1)) for l in range(k)]
        n = n_views or 64
        res = [resolution] * n if resolution else mixed_resolutions(4, n)
        cams = ring_cameras(4, n, res)
        targets = uniform_targets(4, cams) if with_targets else None
        return Scene(name, layers, tex, cams, targets, "k=9 displaced shells, mixed views")
    raise ValueError(f"unknown config {i}")


def upstream_grad(config: int, cam: Camera, view: int = 0) -> np.ndarray:
    """A seeded upstream gradient dL/d(RGBA) in [-1,1] for linear-loss adjoint tests."""
    rng = np.random.default_rng([config, P_UPSTREAM, view])
    return rng.uniform(-1.0, 1.0, (cam.height, cam.width, 4)).astype(np.float32)

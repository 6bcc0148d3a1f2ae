"""k-SDF volume-rendering oracle (FP64, NumPy) -- TEST INFRASTRUCTURE ONLY.

The implicit stage of the method (Sec. 4.1-4.2, Sec. 4.4 "Occupancy Grid" and
"Importance Sampling", supplement "Points sampling") renders k nested surfaces
given as signed distance fields by NeuS-style quadrature along each pixel ray
and blends the per-surface results in a fixed order.  The trained fields
(networks) are not available, so the fields are inputs given on dense grids
and sampled trilinearly; every step after the field lookups follows the paper.

Definitions (our reading where the paper gives no formula):
  * fields on the cube [lo, hi]^3: the main SDF d on (R+1)^3 vertices and a
    straight RGBA appearance field (RGB = xi, A = the transparency field) on
    (Ra+1)^3 vertices, both stored [z][y][x]; a grid of resolution R has
    cell coordinate c = (p - lo) * (R / (hi - lo)) clamped to [0, R], base
    vertex min(floor(c), R - 1), weights c - base;
  * surfaces d_j = d + o_j with constant offsets o_0 <= o_1 <= ..., j = 0 the
    outermost (positive offsets lie inside, Sec. 4.1);
  * logistic density phi_b(x) = b e^{-bx} / (1 + e^{-bx})^2 (Eq. 2) and its
    CDF Phi_b(x) = 1 / (1 + e^{-bx});
  * occupancy (Sec. 4.4): voxel (resolution Ro) with centre c is occupied
    iff for some j, phi_b(max(|d_j(c)| - diag/2, 0)) > tau, diag = sqrt(3) h_o
    (every point of the voxel is within diag/2 of its centre);
  * pixel rays: origin -R^T t, direction R^T ((i+.5-cx)/fx, (j+.5-cy)/fy, 1)
    normalised; the ray's parameter interval is its slab intersection with the
    cube, clipped to t >= 0;
  * occupied space along a ray is resolved by S equal march steps over that
    interval: step s covers [t_in + s D, t_in + (s+1) D], D = (t_out - t_in)/S,
    and is occupied iff the voxel holding its midpoint p = o + t_m v is
    (voxel coordinate (p - lo) Ro/(hi - lo), as for the fields); the n uniform
    samples sit at occupied-length positions rho_i = (i + 1/2) M / n (M
    occupied steps): sample i lies in the floor(rho_i)-th occupied step at
    fraction rho_i - floor(rho_i);
  * NeuS weights of surface j over sorted samples t_0..t_{N-1} (interval i
    between samples i and i+1): a_i = max((Phi_i - Phi_{i+1}) / Phi_i, 0)
    with Phi_i = Phi_b(d_j(x_i)) (0 where Phi_i = 0), T_i = prod_{l<i} (1 - a_l),
    w_i = T_i a_i;
  * importance sampling, two rounds with b/2 then b: W_i = sum_j w_{ij},
    pdf_i = (W_i + eps) / sum_l (W_l + eps), cdf c_0 = 0, c_{i+1} = c_i + pdf_i;
    m/2 new samples at u_q = (q + 1/2) / (m/2) by linear inversion inside the
    interval i with c_i <= u_q < c_{i+1}; merged into the sorted list
    (existing samples first on ties);
  * per surface C_j = sum_i w_ij xi(x_i), A_j = sum_i w_ij alpha_w(x_i) A(x_i),
    alpha_w = 2 sigmoid(10 |v . n|) - 1 (Sec. 4.2) with n the normalised
    gradient of d (supplement: normals are normalised SDF gradients; the
    paper takes its network's gradient by finite differences, a grid field's
    gradient is exact: the derivative of the trilinear interpolant inside
    the cell that holds the point);
  * blend (Sec. 4.2, exclusive product as for the meshes): RGB = sum_j C_j A_j
    prod_{l<j} (1 - A_l), alpha = 1 - prod_j (1 - A_j).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Sequence

import numpy as np


@dataclasses.dataclass
class KsdfField:
    sdf: np.ndarray        # [(R+1)^3] main SDF at grid vertices, [z][y][x]
    sdf_res: int           # R
    rgba: np.ndarray       # [(Ra+1)^3, 4] straight RGBA at grid vertices
    rgba_res: int          # Ra
    lo: float
    hi: float


@dataclasses.dataclass
class KsdfOpts:
    offsets: Sequence[float]        # o_j, non-decreasing, j = 0 outermost
    beta: float = math.exp(7.0)
    occ_threshold: float = 1e-4
    occ_res: int = 256
    n_uniform: int = 64
    n_importance: int = 32          # m, added in two rounds of m/2
    march_steps: int = 1024
    pdf_floor: float = 1e-5

    @property
    def k(self) -> int:
        return len(self.offsets)


# --------------------------------------------------------------------------
# fields
# --------------------------------------------------------------------------
def trilinear(grid: np.ndarray, res: int, lo: float, hi: float, p: np.ndarray) -> np.ndarray:
    """Trilinear interpolation of vertex values ``grid`` [(res+1)^3, C] at points p [n, 3] -> [n, C]."""
    g = np.asarray(grid, np.float64).reshape((res + 1) ** 3, -1)
    inv = res / (hi - lo)
    c = np.clip((np.asarray(p, np.float64) - lo) * inv, 0.0, float(res))
    b = np.minimum(np.floor(c), res - 1).astype(np.int64)
    f = c - b
    out = np.zeros((c.shape[0], g.shape[1]))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = ((f[:, 0] if dx else 1 - f[:, 0]) * (f[:, 1] if dy else 1 - f[:, 1])
                     * (f[:, 2] if dz else 1 - f[:, 2]))
                idx = ((b[:, 2] + dz) * (res + 1) + (b[:, 1] + dy)) * (res + 1) + (b[:, 0] + dx)
                out += w[:, None] * g[idx]
    return out


def sdf_at(field: KsdfField, p: np.ndarray) -> np.ndarray:
    return trilinear(field.sdf.reshape(-1, 1), field.sdf_res, field.lo, field.hi, p)[:, 0]


def rgba_at(field: KsdfField, p: np.ndarray) -> np.ndarray:
    return trilinear(field.rgba.reshape(-1, 4), field.rgba_res, field.lo, field.hi, p)


def logistic_density(x: np.ndarray, beta: float) -> np.ndarray:
    """phi_beta(x) = beta e^{-beta x} / (1 + e^{-beta x})^2 (Eq. 2), written for |x| to avoid overflow."""
    e = np.exp(-beta * np.abs(x))
    return beta * e / ((1.0 + e) * (1.0 + e))


def logistic_cdf(x: np.ndarray, beta: float) -> np.ndarray:
    return 1.0 / (1.0 + np.exp(-beta * x))


# --------------------------------------------------------------------------
# occupancy grid (Sec. 4.4)
# --------------------------------------------------------------------------
def occupancy_at(field: KsdfField, opts: KsdfOpts, vox: np.ndarray) -> np.ndarray:
    """Occupancy (bool) of the voxels with linear indices ``vox`` ((z Ro + y) Ro + x)."""
    Ro = opts.occ_res
    ho = (field.hi - field.lo) / Ro
    vox = np.asarray(vox, np.int64)
    x, y, z = vox % Ro, (vox // Ro) % Ro, vox // (Ro * Ro)
    centres = np.stack([field.lo + (x + 0.5) * ho, field.lo + (y + 0.5) * ho, field.lo + (z + 0.5) * ho], -1)
    dc = sdf_at(field, centres)
    half_diag = math.sqrt(3.0) * ho / 2.0
    occ = np.zeros(dc.shape, bool)
    with np.errstate(over="ignore"):
        for o in opts.offsets:
            delta = np.maximum(np.abs(dc + o) - half_diag, 0.0)
            occ |= logistic_density(delta, opts.beta) > opts.occ_threshold
    return occ


def occupancy(field: KsdfField, opts: KsdfOpts, chunk: int = 1 << 21) -> np.ndarray:
    """uint8 [Ro, Ro, Ro] ([z][y][x]); 1 where some surface may have density above the threshold."""
    Ro = opts.occ_res
    n = Ro ** 3
    out = np.empty(n, np.uint8)
    for a in range(0, n, chunk):
        out[a:a + chunk] = occupancy_at(field, opts, np.arange(a, min(a + chunk, n)))
    return out.reshape(Ro, Ro, Ro)


# --------------------------------------------------------------------------
# rays
# --------------------------------------------------------------------------
def camera_rays(cam) -> tuple:
    """Origins [P, 3] and unit directions [P, 3] of the pixel-centre rays of a pinhole camera (row-major pixels).

    Written out term by term (no BLAS) so that every ray is a fixed sequence of
    IEEE operations.
    """
    R = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    origin = np.array([-((R[0, q] * t[0] + R[1, q] * t[1]) + R[2, q] * t[2]) for q in range(3)])
    j, i = np.mgrid[0:cam.height, 0:cam.width]
    xc = ((i.reshape(-1) + 0.5) - cam.cx) / cam.fx
    yc = ((j.reshape(-1) + 0.5) - cam.cy) / cam.fy
    d = np.stack([(R[0, q] * xc + R[1, q] * yc) + R[2, q] for q in range(3)], -1)   # R^T (xc, yc, 1)
    n = np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
    d = d / n[:, None]
    return np.broadcast_to(origin, d.shape).copy(), d


def box_interval(o: np.ndarray, v: np.ndarray, lo: float, hi: float):
    """Slab intersection [t_in, t_out] of rays with the cube, clipped to t >= 0; hit mask."""
    t_in = np.zeros(o.shape[0])
    t_out = np.full(o.shape[0], np.inf)
    hit = np.ones(o.shape[0], bool)
    with np.errstate(divide="ignore", invalid="ignore"):
        for a in range(3):
            nz = v[:, a] != 0.0
            t1 = (lo - o[:, a]) / v[:, a]
            t2 = (hi - o[:, a]) / v[:, a]
            t_in = np.where(nz, np.maximum(t_in, np.minimum(t1, t2)), t_in)
            t_out = np.where(nz, np.minimum(t_out, np.maximum(t1, t2)), t_out)
            hit &= nz | ((o[:, a] >= lo) & (o[:, a] <= hi))
    hit &= t_out > t_in
    return t_in, t_out, hit


def march_midpoint_coords(o, v, t_in, t_out, Ro: int, lo: float, hi: float, steps: int) -> np.ndarray:
    """[n_rays, S, 3] voxel coordinates (before the floor) of the march-step midpoints.

    Step s spans [t_in + s D, t_in + (s+1) D] with D = (t_out - t_in)/S; its
    midpoint is the point p = o + t_m v, whose voxel coordinate is the grid's
    cell coordinate (p - lo) Ro/(hi - lo), the reading used for every grid.
    """
    D = (t_out - t_in) / steps
    tm = t_in[:, None] + (np.arange(steps)[None, :] + 0.5) * D[:, None]
    p = o[:, None, :] + tm[..., None] * v[:, None, :]
    return (p - lo) * (Ro / (hi - lo))


def march_occupied(o, v, t_in, t_out, occ: np.ndarray, lo: float, hi: float, steps: int) -> np.ndarray:
    """bool [n_rays, S]: march step s of each ray is occupied (the voxel holding its midpoint is)."""
    Ro = occ.shape[0]
    c = march_midpoint_coords(o, v, t_in, t_out, Ro, lo, hi, steps)
    vox = np.clip(np.floor(c), 0, Ro - 1).astype(np.int64)
    return occ[vox[..., 2], vox[..., 1], vox[..., 0]].astype(bool)


def march_on_face(o, v, occ_res: int, lo: float, hi: float, steps: int, tol: float = 1e-9) -> np.ndarray:
    """bool [n_rays]: some march midpoint of the ray lies within ``tol`` (in voxel units) of an interior
    voxel face.  There the voxel it falls in is decided by the last bits of its coordinate, which any other
    correct evaluation order may round the other way; the result of such a ray is not unique."""
    t_in, t_out, hit = box_interval(o, v, lo, hi)
    out = np.zeros(o.shape[0], bool)
    rows = np.flatnonzero(hit)
    for a in range(0, rows.size, 2048):
        r = rows[a:a + 2048]
        c = march_midpoint_coords(o[r], v[r], t_in[r], t_out[r], occ_res, lo, hi, steps)
        near = np.abs(c - np.rint(c)) <= tol
        interior = (np.rint(c) >= 1) & (np.rint(c) <= occ_res - 1)
        out[r] = (near & interior).any(axis=(1, 2))
    return out


def uniform_samples(t_in, t_out, occ_steps: np.ndarray, n: int):
    """[n_rays, n] sample parameters uniform in occupied length; rows with no occupied step are NaN."""
    S = occ_steps.shape[1]
    D = (t_out - t_in) / S
    out = np.full((occ_steps.shape[0], n), np.nan)
    for r in range(occ_steps.shape[0]):
        idx = np.flatnonzero(occ_steps[r])
        M = idx.size
        if M == 0:
            continue
        rho = ((np.arange(n) + 0.5) * M) / n
        q = np.floor(rho)
        out[r] = t_in[r] + (idx[q.astype(np.int64)] + (rho - q)) * D[r]
    return out


# --------------------------------------------------------------------------
# NeuS weights and importance sampling
# --------------------------------------------------------------------------
def neus_weights(d: np.ndarray, offset: float, beta: float) -> np.ndarray:
    """[rays, N-1] interval weights of the surface d + offset for samples [rays, N] sorted along each ray."""
    with np.errstate(over="ignore"):
        phi = logistic_cdf(d + offset, beta)
    num = phi[:, :-1] - phi[:, 1:]
    den = phi[:, :-1]
    a = np.where(den > 0.0, np.maximum(np.divide(num, den, out=np.zeros_like(num), where=den > 0.0), 0.0), 0.0)
    T = np.cumprod(np.concatenate([np.ones((a.shape[0], 1)), 1.0 - a[:, :-1]], 1), axis=1)
    return T * a


def importance_round(t: np.ndarray, d: np.ndarray, offsets, beta: float, m_round: int, eps: float):
    """New sample parameters [rays, m_round] by inverting the normalised sum of the k surfaces' weights."""
    W = sum(neus_weights(d, o, beta) for o in offsets)
    pdf = (W + eps) / (W + eps).sum(1, keepdims=True)
    cdf = np.concatenate([np.zeros((W.shape[0], 1)), np.cumsum(pdf, 1)], 1)     # [rays, N]
    u = (np.arange(m_round) + 0.5) / m_round
    N = t.shape[1]
    out = np.empty((t.shape[0], m_round))
    for r in range(t.shape[0]):
        i = np.clip(np.searchsorted(cdf[r], u, side="right") - 1, 0, N - 2)
        c0, c1 = cdf[r][i], cdf[r][i + 1]
        out[r] = t[r][i] + (u - c0) / (c1 - c0) * (t[r][i + 1] - t[r][i])
    return out


def merge_sorted(t: np.ndarray, d: np.ndarray, tn: np.ndarray, dn: np.ndarray):
    """Stable merge of existing (first on ties) and new samples, carrying their SDF values."""
    tt = np.concatenate([t, tn], 1)
    dd = np.concatenate([d, dn], 1)
    order = np.argsort(tt, axis=1, kind="stable")
    return np.take_along_axis(tt, order, 1), np.take_along_axis(dd, order, 1)


def sdf_gradient(field: KsdfField, p: np.ndarray) -> np.ndarray:
    """[n, 3] gradient of the trilinear SDF inside the cell holding each point (the cell of ``trilinear``)."""
    res, lo, hi = field.sdf_res, field.lo, field.hi
    g = np.asarray(field.sdf, np.float64).reshape(-1)
    inv = res / (hi - lo)
    c = np.clip((np.asarray(p, np.float64) - lo) * inv, 0.0, float(res))
    b = np.minimum(np.floor(c), res - 1).astype(np.int64)
    f = c - b
    out = np.zeros((c.shape[0], 3))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                idx = ((b[:, 2] + dz) * (res + 1) + (b[:, 1] + dy)) * (res + 1) + (b[:, 0] + dx)
                wx = f[:, 0] if dx else 1 - f[:, 0]
                wy = f[:, 1] if dy else 1 - f[:, 1]
                wz = f[:, 2] if dz else 1 - f[:, 2]
                sx, sy, sz = (1 if dx else -1), (1 if dy else -1), (1 if dz else -1)
                out[:, 0] += sx * wy * wz * g[idx]
                out[:, 1] += sy * wx * wz * g[idx]
                out[:, 2] += sz * wx * wy * g[idx]
    return out * inv


def sdf_normals(field: KsdfField, p: np.ndarray) -> np.ndarray:
    grad = sdf_gradient(field, p)
    n = np.linalg.norm(grad, axis=1, keepdims=True)
    return np.divide(grad, n, out=np.zeros_like(grad), where=n > 0.0)


# --------------------------------------------------------------------------
# whole forward
# --------------------------------------------------------------------------
def render_rays(field: KsdfField, opts: KsdfOpts, occ: np.ndarray, o: np.ndarray, v: np.ndarray) -> Dict[str, np.ndarray]:
    """Forward of the k-SDF renderer for rays (o, v): RGBA [n, 4], per-surface (C_j, A_j) [k, n, 4], samples [n, N]."""
    nr = o.shape[0]
    n, m = opts.n_uniform, opts.n_importance
    N = n + m
    rgba = np.zeros((nr, 4))
    layers = np.zeros((opts.k, nr, 4))
    samples = np.full((nr, N), -1.0)
    t_in, t_out, hit = box_interval(o, v, field.lo, field.hi)
    rows = np.flatnonzero(hit)
    if rows.size:
        st = march_occupied(o[rows], v[rows], t_in[rows], t_out[rows], occ, field.lo, field.hi, opts.march_steps)
        t = uniform_samples(t_in[rows], t_out[rows], st, n)
        ok = ~np.isnan(t[:, 0])
        rows, t = rows[ok], t[ok]
    if rows.size:
        ro, rv = o[rows], v[rows]

        def sdf_along(tt):
            p = ro[:, None, :] + tt[..., None] * rv[:, None, :]
            return sdf_at(field, p.reshape(-1, 3)).reshape(tt.shape)

        d = sdf_along(t)
        for beta_r in (opts.beta / 2.0, opts.beta):
            tn = importance_round(t, d, opts.offsets, beta_r, m // 2, opts.pdf_floor)
            t, d = merge_sorted(t, d, tn, sdf_along(tn))
        p = (ro[:, None, :] + t[:, :-1, None] * rv[:, None, :]).reshape(-1, 3)
        app = rgba_at(field, p).reshape(rows.size, N - 1, 4)
        nrm = sdf_normals(field, p).reshape(rows.size, N - 1, 3)
        vdotn = np.abs((nrm * rv[:, None, :]).sum(-1))
        alpha_w = 2.0 / (1.0 + np.exp(-10.0 * vdotn)) - 1.0
        Tacc = np.ones(rows.size)
        col = np.zeros((rows.size, 3))
        for j, off in enumerate(opts.offsets):
            w = neus_weights(d, off, opts.beta)
            C = (w[..., None] * app[..., :3]).sum(1)
            A = (w * alpha_w * app[..., 3]).sum(1)
            layers[j, rows, :3] = C
            layers[j, rows, 3] = A
            col += (Tacc * A)[:, None] * C
            Tacc = Tacc * (1.0 - A)
        rgba[rows, :3] = col
        rgba[rows, 3] = 1.0 - Tacc
        samples[rows] = t
    return dict(rgba=rgba, layers=layers, samples=samples)


def render(field: KsdfField, opts: KsdfOpts, occ: np.ndarray, cam) -> Dict[str, np.ndarray]:
    o, v = camera_rays(cam)
    return render_rays(field, opts, occ, o, v)

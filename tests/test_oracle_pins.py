"""Pins of the FP64 CPU oracle against facts that do not come from the oracle itself.

Each test ties one part of the oracle to geometry, closed forms or
independent constructions, so that a dropped term, a wrong sign, a swapped
index or a transposed operand anywhere in it fails at least one of them:

  P1  watertightness of the fill rule (planar lattice tilings, closed meshes)
  P2  coverage and depth against analytic ray-sphere intersection
  P3  fixed-order blending against its closed form (Sec. 4.2, Eq. 6, product over j < i)
  P4  perspective-correct UV against ray-plane (Moller-Trumbore) intersection
  P5  bilinear filtering at texel centres (Fig. 5) against an affine texture's closed form
  P6  analytic adjoint against central finite differences (exact: the image is affine in
      every single texel scalar)
  P7  brute force == bounding-box rasterisation
  P8  edge cases: ties, degenerate triangles, near-plane / guard-band / NaN culls, UV wrap
  P9  vertex snapping against an independent NumPy evaluation
"""
import numpy as np
import pytest

import scenes as S

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


def _ortho_cam(w, h):
    """Camera with R = I, t = 0, fx = fy = 1, cx = cy = 0: a vertex (x, y, 1) lands at pixel position (x, y)."""
    return S.Camera(w, h, 1.0, 1.0, 0.0, 0.0, np.eye(3), np.zeros(3))


def _small_shells(k=3, n_lat=40, n_lon=80, amp=0.05):
    d, uv, tri = S.latlong_mesh(n_lat, n_lon)
    s = S.sine_field(2)(d)
    out = []
    for o in np.linspace(-0.06, 0.06, k)[::-1]:
        pos = d * (1.0 + o + amp * s)[:, None]
        out.append(S.Mesh(pos.astype(np.float32), uv.astype(np.float32), tri.astype(np.int32)))
    return out


def _key_tri(vis):
    return (vis & np.uint64(0xFFFFFFFF)).astype(np.int64)


def _key_depth(vis):
    return (vis >> np.uint64(32)).astype(np.uint32).view(np.float32)


# ----------------------------------------------------------------------------- P1
def _lattice_tiling(rng, nx, ny, spacing, origin, flip_frac=0.3):
    """Planar grid tiling with vertices on the half-pixel lattice; random diagonals and windings."""
    pts = []
    for iy in range(ny + 1):
        for ix in range(nx + 1):
            x, y = origin[0] + spacing * ix, origin[1] + spacing * iy
            if 0 < ix < nx and 0 < iy < ny:
                x += rng.choice([-0.5, 0.0, 0.5])
                y += rng.choice([-0.5, 0.0, 0.5])
            pts.append((x, y, 1.0))
    vid = np.arange((nx + 1) * (ny + 1)).reshape(ny + 1, nx + 1)
    tris = []
    for iy in range(ny):
        for ix in range(nx):
            a, b, c, d = vid[iy, ix], vid[iy, ix + 1], vid[iy + 1, ix], vid[iy + 1, ix + 1]
            if rng.random() < 0.5:
                tt = [(a, b, d), (a, d, c)]
            else:
                tt = [(a, b, c), (b, d, c)]
            for t in tt:
                tris.append(t[::-1] if rng.random() < flip_frac else t)
    xyz = np.array(pts, np.float32)
    return S.Mesh(xyz, np.zeros((len(pts), 2), np.float32), np.array(tris, np.int32))


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("origin", [(1.0, 1.0), (0.5, 0.5), (1.5, 2.0)])
def test_p1_lattice_tiling_covers_every_centre_once(oracle_lib, seed, origin):
    O = oracle_lib
    rng = np.random.default_rng([101, seed])
    nx, ny, sp = 12, 9, 2.0
    mesh = _lattice_tiling(rng, nx, ny, sp, origin)
    W, H = 32, 24
    pos, neg = O.coverage(mesh, _ortho_cam(W, H))
    cov = pos + neg
    x0, y0 = origin
    x1, y1 = x0 + sp * nx, y0 + sp * ny
    cx = np.arange(W)[None, :] + 0.5
    cy = np.arange(H)[:, None] + 0.5
    strictly_in = (cx > x0) & (cx < x1) & (cy > y0) & (cy < y1)
    outside = (cx < x0) | (cx > x1) | (cy < y0) | (cy > y1)
    assert np.all(cov[strictly_in] == 1), "gap or overlap inside a tiling"
    assert np.all(cov[outside] == 0)
    # Rectangle boundary: the left and top edges are owned, the right and bottom ones are not.
    left = (cx == x0) & (cy > y0) & (cy < y1)
    top = (cy == y0) & (cx > x0) & (cx < x1)
    right = (cx == x1) & (cy > y0) & (cy < y1)
    bottom = (cy == y1) & (cx > x0) & (cx < x1)
    assert np.all(cov[left & np.ones_like(cov, bool)] == 1)
    assert np.all(cov[top & np.ones_like(cov, bool)] == 1)
    assert np.all(cov[right & np.ones_like(cov, bool)] == 0)
    assert np.all(cov[bottom & np.ones_like(cov, bool)] == 0)


def test_p1_fan_around_a_pixel_centre(oracle_lib):
    """n triangles meeting at a vertex that sits exactly on a pixel centre: exactly one covers it."""
    O = oracle_lib
    for n in (3, 4, 5, 6, 8, 12):
        ang = np.arange(n) * 2 * np.pi / n + 0.1
        c = (8.5, 8.5)
        ring = [(np.round((c[0] + 6 * np.cos(a)) * 2) / 2, np.round((c[1] + 6 * np.sin(a)) * 2) / 2, 1.0) for a in ang]
        xyz = np.array([(c[0], c[1], 1.0)] + ring, np.float32)
        tri = np.array([(0, 1 + q, 1 + (q + 1) % n) for q in range(n)], np.int32)
        mesh = S.Mesh(xyz, np.zeros((n + 1, 2), np.float32), tri)
        pos, neg = O.coverage(mesh, _ortho_cam(17, 17))
        assert pos[8, 8] + neg[8, 8] == 1


def _closed_cases():
    cases = []
    ico = S.icosphere_shells([1.0, 0.9], subdiv=3)
    cams = [S.make_camera(256, 256, (0, 0, 3.0))] + S.ring_cameras(11, 4, [(200, 160)] * 4)
    for c in cams:
        cases.append(("ico", ico[0], c, True))
    sh = _small_shells(k=2)
    for c in S.ring_cameras(12, 4, [(160, 128)] * 4):
        cases.append(("shell", sh[0], c, False))
    return cases


@pytest.mark.parametrize("case", range(9))
def test_p1_closed_mesh_signed_coverage_is_zero(oracle_lib, case):
    O = oracle_lib
    name, mesh, cam, convex = _closed_cases()[case]
    pos, neg = O.coverage(mesh, cam)
    assert np.array_equal(pos, neg), f"{name}: signed coverage non-zero at {np.argwhere(pos != neg)[:5]}"
    assert pos.sum() > 1000
    if convex:
        assert pos.max() == 1 and neg.max() == 1


# ----------------------------------------------------------------------------- P2
def _ray_sphere_entry(cam, ii, jj, center, rho):
    """Camera-space z of the first hit of the ray through screen point (ii, jj) with a sphere; NaN on a miss."""
    dx = (ii - cam.cx) / cam.fx
    dy = (jj - cam.cy) / cam.fy
    d2 = dx * dx + dy * dy + 1.0
    dc = dx * center[0] + dy * center[1] + center[2]
    disc = dc * dc - d2 * (center @ center - rho * rho)
    z = (dc - np.sqrt(np.where(disc >= 0, disc, np.nan))) / d2
    return z


def _inradius(mesh):
    p = mesh.xyz.astype(np.float64)
    a, b, c = p[mesh.tri[:, 0]], p[mesh.tri[:, 1]], p[mesh.tri[:, 2]]
    n = np.cross(b - a, c - a)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    return np.abs(np.einsum("ij,ij->i", n, a)).min()


@pytest.mark.parametrize("which", ["ico1", "ico08", "latlong"])
def test_p2_coverage_and_depth_match_analytic_spheres(oracle_lib, which):
    O = oracle_lib
    if which.startswith("ico"):
        r = 1.0 if which == "ico1" else 0.8
        mesh = S.icosphere_shells([r], subdiv=3)[0]
        cams = [S.make_camera(256, 256, (0, 0, 3.0))] + S.ring_cameras(21, 2, [(192, 144)] * 2)
    else:
        mesh = _small_shells(k=1, n_lat=60, n_lon=120, amp=0.0)[0]
        cams = [S.make_camera(256, 256, (0, 0, 3.0))] + S.ring_cameras(22, 2, [(192, 144)] * 2)
    r_out = np.linalg.norm(mesh.xyz.astype(np.float64), axis=1).max() * (1 + 1e-5)
    r_in = _inradius(mesh) * (1 - 1e-5)
    m = 1.0 / 128.0
    for cam in cams:
        vis, st = O.raster(mesh, cam)
        assert st["culled_invalid"] == 0 and st["culled_degenerate"] == 0
        j, i = np.mgrid[0:cam.height, 0:cam.width].astype(np.float64)
        center = np.asarray(cam.t, np.float64)
        zo, zi = [], []
        for ox in (-m, m):
            for oy in (-m, m):
                zo.append(_ray_sphere_entry(cam, i + 0.5 + ox, j + 0.5 + oy, center, r_out))
                zi.append(_ray_sphere_entry(cam, i + 0.5 + ox, j + 0.5 + oy, center, r_in))
        zo, zi = np.stack(zo), np.stack(zi)
        miss_all = np.all(np.isnan(zo), 0)
        hit_in_all = np.all(~np.isnan(zi), 0)
        assert np.all(vis[miss_all] == EMPTY)
        assert np.all(vis[hit_in_all] != EMPTY)
        z = _key_depth(vis).astype(np.float64)
        sel = hit_in_all
        lo = np.nanmin(zo[:, sel], 0) * (1 - 1e-6)
        hi = np.nanmax(zi[:, sel], 0) * (1 + 1e-6)
        assert np.all(z[sel] >= lo) and np.all(z[sel] <= hi)
        assert sel.sum() > 0.2 * cam.width * cam.height


# ----------------------------------------------------------------------------- P3
def _blend_closed_form(hit_mask, cols, alphas):
    """C = sum over hit layers l of c_l a_l prod_{hit j < l} (1 - a_j); A = 1 - prod (1 - a_l)."""
    k = len(cols)
    C = np.zeros(hit_mask.shape[1:] + (3,))
    T = np.ones(hit_mask.shape[1:])
    for l in range(k):
        h = hit_mask[l]
        C[h] += (T[h] * alphas[l])[:, None] * np.asarray(cols[l])[None, :]
        T[h] *= (1 - alphas[l])
    return C, 1 - T


@pytest.mark.parametrize("scene", ["ico", "shells"])
def test_p3_constant_layers_match_blend_closed_form(oracle_lib, scene):
    O = oracle_lib
    rng = np.random.default_rng(31)
    if scene == "ico":
        meshes = S.icosphere_shells([1.0, 0.9, 0.8])
        cam = S.make_camera(128, 128, (0, 0, 3.0))
    else:
        meshes = _small_shells(k=5)
        cam = S.ring_cameras(32, 1, [(160, 120)])[0]
    k = len(meshes)
    cols = [rng.uniform(0, 1, 3) for _ in range(k)]
    alphas = [float(a) for a in rng.uniform(0.1, 0.9, k)]
    tex = [S.constant_texture(8, 8, list(cols[l]) + [alphas[l]]) for l in range(k)]
    cols = [t[0, 0, :3].astype(np.float64) for t in tex]
    alphas = [float(t[0, 0, 3]) for t in tex]
    vis, img = O.render(meshes, tex, cam)
    hit = vis != EMPTY
    C, A = _blend_closed_form(hit, cols, alphas)
    np.testing.assert_allclose(img[..., :3], C, rtol=0, atol=1e-12)
    np.testing.assert_allclose(img[..., 3], A, rtol=0, atol=1e-12)
    # nested shells: a pixel that hits an inner shell hits every shell around it
    for l in range(k - 1):
        assert np.all(hit[l][hit[l + 1]])


def test_p3_identical_layers_geometric_series(oracle_lib):
    """n hit layers of one colour c and alpha a: C = c (1 - (1-a)^n), A = 1 - (1-a)^n."""
    O = oracle_lib
    meshes = S.icosphere_shells([1.0, 0.95, 0.9, 0.85, 0.8])
    cam = S.make_camera(96, 96, (0, 0, 3.0))
    c, a = np.array([0.25, 0.5, 0.75]), 0.375
    tex = [S.constant_texture(4, 4, list(c) + [a]) for _ in meshes]
    vis, img = O.render(meshes, tex, cam)
    n = (vis != EMPTY).sum(0)
    A = 1 - (1 - a) ** n
    np.testing.assert_allclose(img[..., 3], A, atol=1e-14)
    np.testing.assert_allclose(img[..., :3], A[..., None] * c, atol=1e-14)
    assert (n == 5).sum() > 100


def test_p3_order_is_outermost_first(oracle_lib):
    """Two layers, front red alpha 1/2 over opaque blue: (1/2, 0, 1/2); swapping the layer order gives blue."""
    O = oracle_lib
    meshes = S.icosphere_shells([1.0, 0.9])
    cam = S.make_camera(64, 64, (0, 0, 3.0))
    red = S.constant_texture(4, 4, [1, 0, 0, 0.5])
    blue = S.constant_texture(4, 4, [0, 0, 1, 1])
    vis, img = O.render(meshes, [red, blue], cam)
    both = (vis != EMPTY).all(0)
    np.testing.assert_allclose(img[both], np.broadcast_to([0.5, 0, 0.5, 1.0], img[both].shape), atol=1e-15)
    vis2, img2 = O.render(meshes[::-1], [blue, red], cam)
    np.testing.assert_allclose(img2[both], np.broadcast_to([0, 0, 1, 1.0], img2[both].shape), atol=1e-15)


# ----------------------------------------------------------------------------- P4
def _unproject_snapped(O, mesh, cam):
    X, Y, w, valid = O.project(mesh, cam)
    zc = 1.0 / w
    xs, ys = X / 256.0, Y / 256.0
    return np.stack([(xs - cam.cx) / cam.fx * zc, (ys - cam.cy) / cam.fy * zc, zc], 1)


def _moller_trumbore(orig, d, a, b, c):
    """Ray-triangle intersection (vectorised over rays / triangles): returns (t, u, v)."""
    e1, e2 = b - a, c - a
    p = np.cross(d, e2)
    det = np.einsum("...i,...i->...", e1, p)
    inv = 1.0 / det
    s = orig - a
    u = np.einsum("...i,...i->...", s, p) * inv
    q = np.cross(s, e1)
    v = np.einsum("...i,...i->...", d, q) * inv
    t = np.einsum("...i,...i->...", e2, q) * inv
    return t, u, v


@pytest.mark.parametrize("scene", ["ico", "shell"])
def test_p4_uv_matches_ray_plane_intersection(oracle_lib, scene):
    O = oracle_lib
    if scene == "ico":
        mesh = S.icosphere_shells([1.0])[0]
        cam = S.make_camera(128, 128, (0, 0, 3.0))
    else:
        mesh = _small_shells(k=1)[0]
        cam = S.ring_cameras(41, 1, [(160, 120)])[0]
    tex = [S.smooth_texture(41, 0, 64, 64, opaque=True)]
    vis = O.raster_layers([mesh], cam)
    img, lam, uvo = O.shade([mesh], tex, cam, vis, debug=True)
    P = _unproject_snapped(O, mesh, cam)
    hit = vis[0] != EMPTY
    jj, ii = np.nonzero(hit)
    t = _key_tri(vis[0])[hit]
    tri = mesh.tri[t]
    a, b, c = P[tri[:, 0]], P[tri[:, 1]], P[tri[:, 2]]
    d = np.stack([(ii + 0.5 - cam.cx) / cam.fx, (jj + 0.5 - cam.cy) / cam.fy, np.ones_like(ii, float)], 1)
    tt, u, v = _moller_trumbore(np.zeros(3), d, a, b, c)
    la, lb, lc = 1 - u - v, u, v
    assert np.all(la > -1e-9) and np.all(lb > -1e-9) and np.all(lc > -1e-9)
    uvv = mesh.uv.astype(np.float64)
    uv_mt = la[:, None] * uvv[tri[:, 0]] + lb[:, None] * uvv[tri[:, 1]] + lc[:, None] * uvv[tri[:, 2]]
    np.testing.assert_allclose(uvo[0][hit], uv_mt, atol=1e-9)
    # the hit depth is the ray's intersection depth
    np.testing.assert_allclose(_key_depth(vis[0])[hit], tt, rtol=2e-7)
    # the oracle's barycentrics are a partition of unity
    np.testing.assert_allclose(lam[0][hit].sum(-1), 1.0, atol=1e-12)


def test_p4_nearest_triangle_matches_brute_ray_cast(oracle_lib):
    """On sampled pixels, the visible triangle is the ray-cast nearest one (ties only near edges)."""
    O = oracle_lib
    mesh = _small_shells(k=1)[0]
    cam = S.ring_cameras(42, 1, [(160, 120)])[0]
    vis = O.raster_layers([mesh], cam)[0]
    P = _unproject_snapped(O, mesh, cam)
    a, b, c = P[mesh.tri[:, 0]], P[mesh.tri[:, 1]], P[mesh.tri[:, 2]]
    rng = np.random.default_rng(42)
    jj = rng.integers(0, cam.height, 400)
    ii = rng.integers(0, cam.width, 400)
    mism = 0
    for j, i in zip(jj, ii):
        d = np.array([(i + 0.5 - cam.cx) / cam.fx, (j + 0.5 - cam.cy) / cam.fy, 1.0])
        t, u, v = _moller_trumbore(np.zeros(3), d[None, :], a, b, c)
        ok = (u >= 0) & (v >= 0) & (u + v <= 1) & (t > 0)
        if not ok.any():
            assert vis[j, i] == EMPTY
            continue
        best = np.argmin(np.where(ok, t, np.inf))
        got = int(vis[j, i] & np.uint64(0xFFFFFFFF))
        if got != best:
            mism += 1
            # allowed only when the ray passes within a hair of the best triangle's boundary
            assert min(u[best], v[best], 1 - u[best] - v[best]) < 1e-3
    assert mism <= 4


# ----------------------------------------------------------------------------- P5
def _facing_quad(x0, x1, y0, y1, z, cam, uv_box=((0, 0), (1, 1))):
    (u0, v0), (u1, v1) = uv_box
    xyz = np.array([[x0, y0, z], [x1, y0, z], [x1, y1, z], [x0, y1, z]], np.float32)
    uv = np.array([[u0, v0], [u1, v0], [u1, v1], [u0, v1]], np.float32)
    tri = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    return S.Mesh(xyz, uv, tri)


@pytest.mark.parametrize("wrap", [0, 1])
def test_p5_affine_texture_closed_form(oracle_lib, wrap):
    """Texel (i, j) = a + b i + c j on a camera-facing quad with UV [0,1]^2.

    With texel centres at (i + 1/2)/W, bilinear filtering reproduces an affine
    function of x = uW - 1/2 exactly: colour = a + b x + c y (away from the
    border, where repeat wraps to the other side and clamp holds the edge texel).
    """
    O = oracle_lib
    W = H = 160
    cam = S.Camera(W, H, 100.0, 100.0, 80.0, 80.0, np.eye(3), np.zeros(3))
    mesh = _facing_quad(-0.7, 0.6, -0.65, 0.7, 1.0, cam)
    Wt, Ht = 32, 16
    ii, jj = np.meshgrid(np.arange(Wt), np.arange(Ht))
    coef = [(0.125, 1 / 64, 1 / 32), (0.5, -1 / 128, 1 / 64), (0.25, 1 / 256, -1 / 64)]
    tex = np.ones((Ht, Wt, 4), np.float32)
    for ch, (a, b, c) in enumerate(coef):
        tex[..., ch] = a + b * ii + c * jj
    vis, img = O.render([mesh], [tex], cam, wrap=wrap)
    X, Y, w, _ = O.project(mesh, cam)
    # fronto-parallel quad: UV is affine in screen space between the snapped corners
    xs0, xs1, ys0, ys1 = X[0] / 256, X[1] / 256, Y[0] / 256, Y[2] / 256
    j, i = np.mgrid[0:H, 0:W].astype(np.float64)
    u = (i + 0.5 - xs0) / (xs1 - xs0)
    v = (j + 0.5 - ys0) / (ys1 - ys0)
    x = u * Wt - 0.5
    y = v * Ht - 0.5
    hit = vis[0] != EMPTY
    assert hit.sum() > 0.5 * W * H
    for ch, (a, b, c) in enumerate(coef):
        if wrap == 1:
            want = a + b * np.clip(x, 0, Wt - 1) + c * np.clip(y, 0, Ht - 1)
            sel = hit
        else:
            want = a + b * x + c * y
            sel = hit & (x >= 0) & (x <= Wt - 1) & (y >= 0) & (y <= Ht - 1)
        np.testing.assert_allclose(img[..., ch][sel], want[sel], atol=1e-12)
    if wrap == 0:
        # across the repeat seam the two neighbours are the last and the first column
        a, b, c = coef[0]
        sel = hit & (x > Wt - 1) & (y >= 0) & (y <= Ht - 1)
        fx = x - (Wt - 1)
        want = (1 - fx) * (a + b * (Wt - 1) + c * y) + fx * (a + c * y)
        np.testing.assert_allclose(img[..., 0][sel], want[sel], atol=1e-12)
        assert sel.sum() > 10


# ----------------------------------------------------------------------------- P6
def _pick_entries(rng, grads, n, nonzero=True):
    out = []
    k = len(grads)
    while len(out) < n:
        l = int(rng.integers(0, k))
        g = grads[l]
        idx = np.argwhere(np.abs(g) > 0) if nonzero else None
        if nonzero:
            if idx.shape[0] == 0:
                continue
            j, i, ch = idx[rng.integers(0, idx.shape[0])]
        else:
            j, i, ch = rng.integers(0, g.shape[0]), rng.integers(0, g.shape[1]), rng.integers(0, 4)
        out.append((l, int(j), int(i), int(ch)))
    return np.array(out, np.int32)


@pytest.mark.parametrize("loss", ["linear", "l2"])
@pytest.mark.parametrize("scene", ["cfg1", "shells"])
def test_p6_adjoint_equals_central_fd(oracle_lib, loss, scene):
    O = oracle_lib
    if scene == "cfg1":
        sc = S.make_config(1, resolution=(128, 128), tex_res=64)
        meshes, tex, cam = sc.layers, sc.textures, sc.cameras[0]
    else:
        meshes = _small_shells(k=4)
        tex = [S.smooth_texture(61, l, 48, 32, opaque=(l == 3)) for l in range(4)]
        cam = S.ring_cameras(61, 1, [(120, 96)])[0]
    vis = O.raster_layers(meshes, cam)
    g = S.upstream_grad(61, cam).astype(np.float64) if loss == "linear" else None
    tgt = S.uniform_targets(61, [cam])[0] if loss == "l2" else None
    grads = O.backward(meshes, tex, cam, vis, grad_out=g, target=tgt)
    rng = np.random.default_rng(62)
    ent = np.concatenate([_pick_entries(rng, grads, 48), _pick_entries(rng, grads, 16, nonzero=False)])
    fd = O.finite_diff(meshes, tex, cam, vis, ent, h=1e-3, grad_out=g, target=tgt)
    an = np.array([grads[l][j, i, ch] for l, j, i, ch in ent])
    scale = np.abs(an).max()
    np.testing.assert_allclose(an, fd, rtol=1e-9, atol=1e-11 * scale)
    assert np.count_nonzero(an) >= 48
    # the step size does not matter: the loss is at most quadratic in one texel scalar
    fd2 = O.finite_diff(meshes, tex, cam, vis, ent[:8], h=0.25, grad_out=g, target=tgt)
    np.testing.assert_allclose(fd2, an[:8], rtol=1e-9, atol=1e-11 * scale)


def test_p6_opaque_innermost_layer_adjoint(oracle_lib):
    """alpha = 1 on the innermost shell (transmittance reaches 0): adjoint still exact."""
    O = oracle_lib
    meshes = S.icosphere_shells([1.0, 0.9])
    cam = S.make_camera(96, 96, (0, 0, 3.0))
    tex = [S.uniform_texture(63, 0, 16, 16, False), S.uniform_texture(63, 1, 16, 16, True)]
    vis = O.raster_layers(meshes, cam)
    g = S.upstream_grad(63, cam).astype(np.float64)
    grads = O.backward(meshes, tex, cam, vis, grad_out=g)
    rng = np.random.default_rng(63)
    ent = _pick_entries(rng, grads, 40)
    fd = O.finite_diff(meshes, tex, cam, vis, ent, grad_out=g)
    an = np.array([grads[l][j, i, ch] for l, j, i, ch in ent])
    np.testing.assert_allclose(an, fd, rtol=1e-9, atol=1e-12)


# ----------------------------------------------------------------------------- P7
@pytest.mark.parametrize("case", ["cfg1", "shells"])
def test_p7_brute_equals_bbox(oracle_lib, case):
    O = oracle_lib
    if case == "cfg1":
        sc = S.make_config(1, resolution=(160, 160))
        meshes, cam = sc.layers, sc.cameras[0]
    else:
        meshes = _small_shells(k=2, n_lat=20, n_lon=40)
        cam = S.ring_cameras(71, 1, [(96, 80)])[0]
    for m in meshes:
        a, sa = O.raster(m, cam, "bbox")
        b, sb = O.raster(m, cam, "brute")
        assert np.array_equal(a, b)
        assert sa == sb


# ----------------------------------------------------------------------------- P8
def test_p8_duplicate_triangle_smaller_id_wins(oracle_lib):
    O = oracle_lib
    mesh = S.icosphere_shells([1.0])[0]
    cam = S.make_camera(96, 96, (0, 0, 3.0))
    base, _ = O.raster(mesh, cam)
    nt = mesh.n_tri
    # put a copy of every triangle in front: the originals keep every pixel
    dup = S.Mesh(mesh.xyz, mesh.uv, np.concatenate([mesh.tri, mesh.tri], 0))
    v2, _ = O.raster(dup, cam)
    assert np.array_equal(v2, base)
    # copies first: the copies (now the smaller ids) win with identical depths
    dup2 = S.Mesh(mesh.xyz, mesh.uv, np.concatenate([mesh.tri[::-1], mesh.tri], 0))
    v3, _ = O.raster(dup2, cam)
    hit = base != EMPTY
    assert np.array_equal(_key_depth(v3)[hit], _key_depth(base)[hit])
    assert np.all(_key_tri(v3)[hit] < nt)
    assert np.array_equal(nt - 1 - _key_tri(v3)[hit], _key_tri(base)[hit])


def test_p8_degenerate_and_culled_triangles(oracle_lib):
    O = oracle_lib
    W = H = 32
    cam = S.Camera(W, H, 16.0, 16.0, 16.0, 16.0, np.eye(3), np.zeros(3))
    xyz = np.array([
        [-0.5, -0.5, 1.0], [0.5, -0.5, 1.0], [0.0, 0.5, 1.0],      # 0-2 a good triangle
        [-0.5, 0.0, 1.0], [0.0, 0.0, 1.0], [0.5, 0.0, 1.0],        # 3-5 collinear
        [-0.5, -0.5, 0.005], [0.5, 0.5, 0.005],                    # 6-7 in front of the near plane
        [np.nan, 0.0, 1.0],                                        # 8 NaN
        [5000.0, 0.0, 1.0],                                        # 9 beyond the +-2^16 px guard band
    ], np.float32)
    tri = np.array([[0, 1, 2], [3, 4, 5], [0, 6, 7], [0, 1, 8], [0, 1, 9], [0, 0, 1]], np.int32)
    mesh = S.Mesh(xyz, np.zeros((xyz.shape[0], 2), np.float32), tri)
    vis, st = O.raster(mesh, cam)
    assert st["culled_degenerate"] == 2 and st["culled_invalid"] == 3
    ids = np.unique(_key_tri(vis[vis != EMPTY]))
    assert list(ids) == [0]
    bad = S.Mesh(xyz, mesh.uv, np.array([[0, 1, 99]], np.int32))
    _, st2 = O.raster(bad, cam)
    assert st2["bad_index"] == 1


def test_p8_repeat_wrap_is_periodic_in_u(oracle_lib):
    """Under repeat, shifting every UV by +1 (exact in f32 here) leaves the image unchanged."""
    O = oracle_lib
    W = H = 64
    cam = S.Camera(W, H, 40.0, 40.0, 32.0, 32.0, np.eye(3), np.zeros(3))
    m0 = _facing_quad(-0.7, 0.7, -0.7, 0.7, 1.0, cam, uv_box=((0.75, 0.125), (1.25, 0.875)))
    m1 = S.Mesh(m0.xyz, (m0.uv + np.array([1.0, 0.0], np.float32)).astype(np.float32), m0.tri)
    m2 = S.Mesh(m0.xyz, (m0.uv - np.array([1.0, 0.0], np.float32)).astype(np.float32), m0.tri)
    tex = [S.uniform_texture(81, 0, 16, 16, opaque=True)]
    _, i0 = O.render([m0], tex, cam)
    _, i1 = O.render([m1], tex, cam)
    _, i2 = O.render([m2], tex, cam)
    np.testing.assert_allclose(i1, i0, atol=1e-12)
    np.testing.assert_allclose(i2, i0, atol=1e-12)
    # and clamp differs from repeat across the seam
    _, ic = O.render([m0], tex, cam, wrap=1)
    assert np.abs(ic - i0).max() > 1e-3


def test_p8_depth_tie_across_coplanar_triangles(oracle_lib):
    """Two coplanar overlapping triangles: the smaller id wins wherever both cover with equal depth."""
    O = oracle_lib
    cam = S.Camera(32, 32, 16.0, 16.0, 16.0, 16.0, np.eye(3), np.zeros(3))
    xyz = np.array([[-0.8, -0.8, 1.0], [0.8, -0.8, 1.0], [-0.8, 0.8, 1.0], [0.8, 0.8, 1.0]], np.float32)
    mesh = S.Mesh(xyz, np.zeros((4, 2), np.float32), np.array([[0, 1, 2], [0, 3, 2]], np.int32))
    vis, _ = O.raster(mesh, cam)
    ids = _key_tri(vis[vis != EMPTY])
    pos0, _ = O.coverage(S.Mesh(xyz, mesh.uv, mesh.tri[:1]), cam)
    pos1, neg1 = O.coverage(S.Mesh(xyz, mesh.uv, mesh.tri[1:]), cam)
    both = (pos0 > 0) & ((pos1 + neg1) > 0)
    assert both.sum() > 50
    assert np.all(_key_tri(vis)[both] == 0)
    assert set(np.unique(ids)) == {0, 1}


# ----------------------------------------------------------------------------- P9
def test_p9_snapping_matches_numpy(oracle_lib):
    O = oracle_lib
    sc = S.make_config(4, n_views=3, latlong=(60, 120), with_targets=False)
    for cam in sc.cameras:
        for mesh in sc.layers[:2]:
            X, Y, w, valid = O.project(mesh, cam)
            p = mesh.xyz.astype(np.float64)
            R, t = cam.R, cam.t
            xc = ((R[0, 0] * p[:, 0] + R[0, 1] * p[:, 1]) + R[0, 2] * p[:, 2]) + t[0]
            yc = ((R[1, 0] * p[:, 0] + R[1, 1] * p[:, 1]) + R[1, 2] * p[:, 2]) + t[1]
            zc = ((R[2, 0] * p[:, 0] + R[2, 1] * p[:, 1]) + R[2, 2] * p[:, 2]) + t[2]
            xs = cam.fx * (xc / zc) + cam.cx
            ys = cam.fy * (yc / zc) + cam.cy
            assert valid.all()
            assert np.array_equal(X, np.rint(xs * 256.0).astype(np.int64))
            assert np.array_equal(Y, np.rint(ys * 256.0).astype(np.int64))
            assert np.array_equal(w, 1.0 / zc)

// Plain, slow, single-threaded FP64 CPU oracle for the layered-mesh renderer.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file; only the tests, the smoke check and the CPU-baseline leg of
// the benchmark do.  It shares no code, header or constant with the HIP path.
//
// What it computes (Volumetric Surfaces, arXiv 2409.02482):
//   * each of the k baked meshes is rasterised on its own, keeping only the
//     first intersection of the pixel ray with that surface (Fig. 2c; the
//     sampling locations are found by rasterisation, Abstract/Sec. 1);
//   * the hit point's UV is interpolated and the layer's RGBA texture is read
//     bilinearly from the four surrounding texel centres, as an OpenGL texture
//     fetch does (Fig. 5 and Sec. 4.3 "Texturing Meshes");
//   * the k layers are alpha-blended in a fixed order, outermost first, with no
//     sorting (Sec. 4.2, Eq. 6; Sec. 1 "rasterization in a fixed order, from
//     outermost to innermost"; Sec. 4.3 "Baking Textures");
//   * the texture gradient of a loss on the blended image (textures are fit on
//     fixed meshes, Sec. 4.3 "Texturing Meshes").
// Readings where the paper is silent (fixed-point snapping, fill rule, depth
// quantity, camera axes, wrap mode, the product index of Eq. 6) are stated at
// each function.  Build: g++ -O2 -ffp-contract=off -fno-fast-math -shared -fPIC.
//
// Parity pins: see tests/test_oracle_pins.py (watertightness, analytic
// spheres, ray-plane barycentrics, affine textures, closed-form blending,
// exact finite differences, brute == bbox, edge cases) and
// tests/test_oracle_sh_pins.py (the baked SH appearance).

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>

namespace {

const uint64_t kEmpty = ~0ull;

struct Cam {
  int32_t width, height;
  double fx, fy, cx, cy;
  double R[9];
  double t[3];
  double z_near;
};

struct Layer {
  const float* xyz;      // [V][3]
  const float* uv;       // [V][2]
  const int32_t* tri;    // [T][3]
  int32_t n_vert, n_tri;
  const float* tex;      // [H][W][4] straight RGBA
  int32_t tex_w, tex_h;
};

// ---------------------------------------------------------------- step 1
// Vertex setup.  OpenCV pinhole camera (x right, y down, z forward), pixel
// centres at half-integers.  Screen positions are snapped to 1/256 pixel with
// round-half-even; a vertex at or in front of the near plane, non-finite, or
// beyond +-2^16 pixels invalidates its triangles (no clipping).  All FP64,
// evaluated left to right without fused multiply-add.
struct Vtx { int64_t X, Y; double w; bool valid; };

Vtx project(const float* p, const Cam& c) {
  Vtx v{0, 0, 0.0, false};
  const double px = p[0], py = p[1], pz = p[2];
  const double xc = ((c.R[0] * px + c.R[1] * py) + c.R[2] * pz) + c.t[0];
  const double yc = ((c.R[3] * px + c.R[4] * py) + c.R[5] * pz) + c.t[1];
  const double zc = ((c.R[6] * px + c.R[7] * py) + c.R[8] * pz) + c.t[2];
  if (!(std::isfinite(xc) && std::isfinite(yc) && std::isfinite(zc))) return v;
  if (!(zc > c.z_near)) return v;
  const double xs = c.fx * (xc / zc) + c.cx;
  const double ys = c.fy * (yc / zc) + c.cy;
  if (!(std::fabs(xs) < 65536.0 && std::fabs(ys) < 65536.0)) return v;
  v.X = (int64_t)std::nearbyint(xs * 256.0);
  v.Y = (int64_t)std::nearbyint(ys * 256.0);
  v.w = 1.0 / zc;
  v.valid = true;
  return v;
}

// ---------------------------------------------------------------- step 2
// Triangle setup.  Twice the signed screen area (y down).  Zero area: no
// coverage.  Negative area: corners b and c swap (with their attributes) so
// that every edge function is non-negative inside.
struct Tri {
  int32_t vid[3];        // corner vertex ids after orientation normalisation
  int64_t X[3], Y[3];
  double w[3];
  int64_t area2;         // > 0
  int orig_sign;         // sign of the area before normalisation
  bool tl[3];            // edge e0 = b->c, e1 = c->a, e2 = a->b owns its boundary
};

enum { kTriOk = 0, kTriInvalid = 1, kTriDegenerate = 2, kTriBadIndex = 3 };

// Top-left ownership of the directed edge P->Q in y-down screen space:
// an edge going up, or a horizontal edge going right.
bool top_left(int64_t px, int64_t py, int64_t qx, int64_t qy) {
  const int64_t dy = qy - py, dx = qx - px;
  return dy < 0 || (dy == 0 && dx > 0);
}

int setup_triangle(const Layer& L, const std::vector<Vtx>& vt, int32_t t, Tri& T) {
  int32_t id[3] = {L.tri[3 * t], L.tri[3 * t + 1], L.tri[3 * t + 2]};
  for (int q = 0; q < 3; ++q)
    if (id[q] < 0 || id[q] >= L.n_vert) return kTriBadIndex;
  for (int q = 0; q < 3; ++q)
    if (!vt[id[q]].valid) return kTriInvalid;
  const Vtx& a = vt[id[0]];
  const Vtx& b = vt[id[1]];
  const Vtx& c = vt[id[2]];
  int64_t area2 = (b.X - a.X) * (c.Y - a.Y) - (b.Y - a.Y) * (c.X - a.X);
  if (area2 == 0) return kTriDegenerate;
  T.orig_sign = area2 > 0 ? 1 : -1;
  if (area2 < 0) { std::swap(id[1], id[2]); area2 = -area2; }
  for (int q = 0; q < 3; ++q) {
    T.vid[q] = id[q];
    T.X[q] = vt[id[q]].X;
    T.Y[q] = vt[id[q]].Y;
    T.w[q] = vt[id[q]].w;
  }
  T.area2 = area2;
  T.tl[0] = top_left(T.X[1], T.Y[1], T.X[2], T.Y[2]);
  T.tl[1] = top_left(T.X[2], T.Y[2], T.X[0], T.Y[0]);
  T.tl[2] = top_left(T.X[0], T.Y[0], T.X[1], T.Y[1]);
  return kTriOk;
}

// Edge functions at the centre of pixel (i, j), in 1/256-pixel units:
// E0 = cross(c-b, P-b) (weight of corner a), E1 = cross(a-c, P-c), E2 = cross(b-a, P-a).
void edge_values(const Tri& T, int64_t i, int64_t j, int64_t E[3]) {
  const int64_t px = 256 * i + 128, py = 256 * j + 128;
  E[0] = (T.X[2] - T.X[1]) * (py - T.Y[1]) - (T.Y[2] - T.Y[1]) * (px - T.X[1]);
  E[1] = (T.X[0] - T.X[2]) * (py - T.Y[2]) - (T.Y[0] - T.Y[2]) * (px - T.X[2]);
  E[2] = (T.X[1] - T.X[0]) * (py - T.Y[0]) - (T.Y[1] - T.Y[0]) * (px - T.X[0]);
}

bool inside(const Tri& T, const int64_t E[3]) {
  for (int e = 0; e < 3; ++e) {
    if (E[e] > 0) continue;
    if (E[e] == 0 && T.tl[e]) continue;
    return false;
  }
  return true;
}

// Perspective-correct camera-space depth at the sample: 1/z interpolates
// linearly in screen space, so z = area2 / (E0 wa + E1 wb + E2 wc).  Rounded to
// float; the visibility key orders by that float, then by triangle id.
uint64_t depth_key(const Tri& T, const int64_t E[3], int32_t t) {
  const double s = ((double)E[0] * T.w[0] + (double)E[1] * T.w[1]) + (double)E[2] * T.w[2];
  const double z = (double)T.area2 / s;
  const float zf = (float)z;
  uint32_t bits;
  std::memcpy(&bits, &zf, 4);
  return ((uint64_t)bits << 32) | (uint32_t)t;
}

int64_t floor_div(int64_t a, int64_t b) {  // b > 0
  int64_t q = a / b;
  if ((a % b != 0) && (a < 0)) --q;
  return q;
}

void project_all(const Layer& L, const Cam& c, std::vector<Vtx>& vt) {
  vt.resize(L.n_vert);
  for (int32_t v = 0; v < L.n_vert; ++v) vt[v] = project(L.xyz + 3 * v, c);
}

// Pixel-centre range [lo, hi] covered by the triangle's fixed-point bbox, clipped to the view.
void bbox_pixels(const Tri& T, const Cam& c, int64_t& i0, int64_t& i1, int64_t& j0, int64_t& j1) {
  const int64_t mnx = std::min(T.X[0], std::min(T.X[1], T.X[2]));
  const int64_t mxx = std::max(T.X[0], std::max(T.X[1], T.X[2]));
  const int64_t mny = std::min(T.Y[0], std::min(T.Y[1], T.Y[2]));
  const int64_t mxy = std::max(T.Y[0], std::max(T.Y[1], T.Y[2]));
  i0 = -floor_div(-(mnx - 128), 256);  // ceil
  i1 = floor_div(mxx - 128, 256);
  j0 = -floor_div(-(mny - 128), 256);
  j1 = floor_div(mxy - 128, 256);
  i0 = std::max<int64_t>(i0, 0);
  j0 = std::max<int64_t>(j0, 0);
  i1 = std::min<int64_t>(i1, c.width - 1);
  j1 = std::min<int64_t>(j1, c.height - 1);
}

// ---------------------------------------------------------------- step 4 helpers
// Texel value with an optional FP64 perturbation of one scalar (for finite differences).
struct Perturb { int32_t layer, j, i, ch; double delta; };

double texel(const Layer& L, int32_t layer, int64_t j, int64_t i, int ch, const Perturb* pt) {
  double val = (double)L.tex[((size_t)j * L.tex_w + (size_t)i) * 4 + ch];
  if (pt && pt->layer == layer && pt->j == j && pt->i == i && pt->ch == ch) val += pt->delta;
  return val;
}

int64_t wrap_index(int64_t i, int64_t n, int wrap) {
  if (wrap == 1) return std::min<int64_t>(std::max<int64_t>(i, 0), n - 1);  // clamp to edge
  int64_t m = i % n;                                                      // repeat
  return m < 0 ? m + n : m;
}

// Bilinear footprint of a UV point: texel centres at ((i+1/2)/W, (j+1/2)/H)
// (Fig. 5), so the sample sits at x = u W - 1/2, y = v H - 1/2 in texel-centre
// coordinates.  Row j of the texture holds v in [j/H, (j+1)/H).
struct Footprint { int64_t i[2], j[2]; double fx, fy; };

Footprint footprint(double u, double v, int32_t W, int32_t H, int wrap) {
  const double x = u * W - 0.5, y = v * H - 0.5;
  const double xf = std::floor(x), yf = std::floor(y);
  Footprint f;
  f.fx = x - xf;
  f.fy = y - yf;
  const int64_t ix = (int64_t)xf, iy = (int64_t)yf;
  f.i[0] = wrap_index(ix, W, wrap);
  f.i[1] = wrap_index(ix + 1, W, wrap);
  f.j[0] = wrap_index(iy, H, wrap);
  f.j[1] = wrap_index(iy + 1, H, wrap);
  return f;
}

// Weight of corner (dj, di) of a footprint.
double corner_weight(const Footprint& f, int dj, int di) {
  const double wx = di ? f.fx : 1.0 - f.fx;
  const double wy = dj ? f.fy : 1.0 - f.fy;
  return wx * wy;
}

struct Hit {
  bool hit;
  double lam[3];     // perspective-correct barycentrics of the normalised corners
  double u, v;
  Footprint f;
  double rgba[4];
};

// Shade one (pixel, layer) slot: rebuild the triangle from the key, compute
// perspective-correct barycentrics lambda_q = E_q w_q / s, interpolate UV and
// fetch the texture bilinearly.
// The UV part of shade_slot: barycentrics and interpolated UV of the slot.
bool slot_uv(const Layer& L, const std::vector<Vtx>& vt, uint64_t key, int64_t i, int64_t j, Hit& h, int* err) {
  h.hit = false;
  if (key == kEmpty) return false;
  const int32_t t = (int32_t)(key & 0xffffffffu);
  Tri T;
  if (t < 0 || t >= L.n_tri || setup_triangle(L, vt, t, T) != kTriOk) { *err = 1; return false; }
  int64_t E[3];
  edge_values(T, i, j, E);
  const double s = ((double)E[0] * T.w[0] + (double)E[1] * T.w[1]) + (double)E[2] * T.w[2];
  h.hit = true;
  h.u = 0.0;
  h.v = 0.0;
  for (int q = 0; q < 3; ++q) {
    h.lam[q] = (double)E[q] * T.w[q] / s;
    h.u += h.lam[q] * (double)L.uv[2 * T.vid[q]];
    h.v += h.lam[q] * (double)L.uv[2 * T.vid[q] + 1];
  }
  return true;
}

Hit shade_slot(const Layer& L, int32_t layer, const std::vector<Vtx>& vt, uint64_t key, int64_t i, int64_t j,
               int wrap, const Perturb* pt, int* err) {
  Hit h;
  if (!slot_uv(L, vt, key, i, j, h, err)) return h;
  h.f = footprint(h.u, h.v, L.tex_w, L.tex_h, wrap);
  for (int ch = 0; ch < 4; ++ch) {
    double acc = 0.0;
    for (int dj = 0; dj < 2; ++dj)
      for (int di = 0; di < 2; ++di)
        acc += corner_weight(h.f, dj, di) * texel(L, layer, h.f.j[dj], h.f.i[di], ch, pt);
    h.rgba[ch] = acc;
  }
  return h;
}

// Fixed-order front-to-back blend of one pixel (Eq. 6 with the product over
// the layers in front, j < i): C = sum_l c_l a_l prod_{j<l} (1 - a_j), over the
// layers the pixel ray hits; A = 1 - prod_l (1 - a_l).  Background is black.
void blend_pixel(int k, const Hit* hits, double out[4]) {
  double C[3] = {0, 0, 0}, T = 1.0;
  for (int l = 0; l < k; ++l) {
    if (!hits[l].hit) continue;
    const double a = hits[l].rgba[3];
    for (int ch = 0; ch < 3; ++ch) C[ch] += T * a * hits[l].rgba[ch];
    T *= (1.0 - a);
  }
  out[0] = C[0];
  out[1] = C[1];
  out[2] = C[2];
  out[3] = 1.0 - T;
}

Cam to_cam(const void* p) { Cam c; std::memcpy(&c, p, sizeof(Cam)); return c; }

// ---------------------------------------------------------------- baked SH appearance
// The paper's baked representation (Sec. 4.3): per shell, spherical-harmonic
// coefficients of RGBA up to degree 3, (deg+1)^2 per channel, stored as 8-bit
// values that decode linearly to [vmin, vmax] ("Squeezing and Quantization",
// [-15, 15] in the paper).  Degree l is stored at the base resolution halved
// l times ("Mixed Resolutions": base colour at the highest resolution, the top
// degree at the lowest).  Each coefficient is read bilinearly from the four
// surrounding texel centres of its own level, each texel decoded first (the
// texel-centre predictions are interpolated, Sec. 4.3 and Fig. 5); the
// coefficients are then decoded with the view direction into RGBA.
// Readings where the paper is silent:
//   * the SH basis is the real, orthonormal one, index l^2 + l + m, with no
//     Condon-Shortley phase in the real form (Y_1^{-1}, Y_1^0, Y_1^1 are
//     proportional to y, z, x);
//   * the decoded sum passes through a sigmoid to give RGBA in (0, 1) (the
//     representation's values are unbounded before squeezing, and alpha must
//     lie in [0, 1], Sec. 4.1);
//   * v is the unit world-space direction of the pixel-centre ray, from the
//     camera through the pixel; n is the hit triangle's unit world-space face
//     normal; the grazing-angle weight 2 sigmoid(10 |v.n|) - 1 of Sec. 4.2
//     ("Transparency Attenuation") multiplies alpha when enabled;
//   * level l has max(1, W >> l) x max(1, H >> l) texels; bytes are stored
//     level after level, texel-major, the 2l+1 coefficients of a texel
//     adjacent, each as R, G, B, A.
struct ShLayer { const uint8_t* data; int32_t width, height; };

void sh_basis(const double d[3], double Y[16]) {
  const double x = d[0], y = d[1], z = d[2];
  const double pi = 3.14159265358979323846;
  Y[0] = 0.5 * std::sqrt(1.0 / pi);
  const double c1 = std::sqrt(3.0 / (4.0 * pi));
  Y[1] = c1 * y;
  Y[2] = c1 * z;
  Y[3] = c1 * x;
  const double c2a = 0.5 * std::sqrt(15.0 / pi), c2b = 0.25 * std::sqrt(5.0 / pi), c2c = 0.25 * std::sqrt(15.0 / pi);
  Y[4] = c2a * x * y;
  Y[5] = c2a * y * z;
  Y[6] = c2b * (3.0 * z * z - 1.0);
  Y[7] = c2a * x * z;
  Y[8] = c2c * (x * x - y * y);
  const double c3a = 0.25 * std::sqrt(35.0 / (2.0 * pi)), c3b = 0.5 * std::sqrt(105.0 / pi);
  const double c3c = 0.25 * std::sqrt(21.0 / (2.0 * pi)), c3d = 0.25 * std::sqrt(7.0 / pi);
  const double c3e = 0.25 * std::sqrt(105.0 / pi);
  Y[9] = c3a * y * (3.0 * x * x - y * y);
  Y[10] = c3b * x * y * z;
  Y[11] = c3c * y * (5.0 * z * z - 1.0);
  Y[12] = c3d * z * (5.0 * z * z - 3.0);
  Y[13] = c3c * x * (5.0 * z * z - 1.0);
  Y[14] = c3e * z * (x * x - y * y);
  Y[15] = c3a * x * (x * x - 3.0 * y * y);
}

int64_t level_dim(int32_t n, int l) { return std::max<int64_t>(1, (int64_t)n >> l); }

size_t level_offset(const ShLayer& S, int l) {
  size_t off = 0;
  for (int m = 0; m < l; ++m) off += (size_t)level_dim(S.width, m) * level_dim(S.height, m) * (2 * m + 1) * 4;
  return off;
}

// Unit world-space direction of the ray through the centre of pixel (i, j).
void pixel_ray(const Cam& c, int64_t i, int64_t j, double d[3]) {
  const double xc = ((double)i + 0.5 - c.cx) / c.fx, yc = ((double)j + 0.5 - c.cy) / c.fy, zc = 1.0;
  for (int q = 0; q < 3; ++q) d[q] = (c.R[q] * xc + c.R[3 + q] * yc) + c.R[6 + q] * zc;  // R^T (xc, yc, zc)
  const double n = std::sqrt((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]);
  for (int q = 0; q < 3; ++q) d[q] /= n;
}

// Unit face normal of triangle t from its world-space corners (zero if degenerate).
void face_normal(const Layer& L, int32_t t, double n[3]) {
  const int32_t* id = L.tri + 3 * (size_t)t;
  double p[3][3];
  for (int q = 0; q < 3; ++q)
    for (int e = 0; e < 3; ++e) p[q][e] = (double)L.xyz[3 * (size_t)id[q] + e];
  const double e1[3] = {p[1][0] - p[0][0], p[1][1] - p[0][1], p[1][2] - p[0][2]};
  const double e2[3] = {p[2][0] - p[0][0], p[2][1] - p[0][1], p[2][2] - p[0][2]};
  n[0] = e1[1] * e2[2] - e1[2] * e2[1];
  n[1] = e1[2] * e2[0] - e1[0] * e2[2];
  n[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double len = std::sqrt((n[0] * n[0] + n[1] * n[1]) + n[2] * n[2]);
  for (int q = 0; q < 3; ++q) n[q] = len > 0.0 ? n[q] / len : 0.0;
}

double sigmoid(double x) { return 1.0 / (1.0 + std::exp(-x)); }

// RGBA of one hit slot under the baked SH appearance.
void sh_rgba(const Layer& L, const ShLayer& S, const Hit& h, int32_t t, const double d[3], int degree, double vmin,
             double vmax, int wrap, int view_alpha, double rgba[4]) {
  double Y[16];
  sh_basis(d, Y);
  double raw[4] = {0, 0, 0, 0};
  for (int l = 0; l <= degree; ++l) {
    const int64_t Wl = level_dim(S.width, l), Hl = level_dim(S.height, l);
    const Footprint f = footprint(h.u, h.v, (int32_t)Wl, (int32_t)Hl, wrap);
    const uint8_t* base = S.data + level_offset(S, l);
    for (int m = 0; m < 2 * l + 1; ++m)
      for (int ch = 0; ch < 4; ++ch) {
        double sh = 0.0;
        for (int dj = 0; dj < 2; ++dj)
          for (int di = 0; di < 2; ++di) {
            const size_t texel = (size_t)f.j[dj] * Wl + (size_t)f.i[di];
            const double q = (double)base[(texel * (2 * l + 1) + m) * 4 + ch];
            sh += corner_weight(f, dj, di) * (vmin + (vmax - vmin) * q / 255.0);
          }
        raw[ch] += sh * Y[l * l + m];
      }
  }
  for (int ch = 0; ch < 4; ++ch) rgba[ch] = sigmoid(raw[ch]);
  if (view_alpha) {
    double n[3];
    face_normal(L, t, n);
    const double vn = std::fabs((d[0] * n[0] + d[1] * n[1]) + d[2] * n[2]);
    rgba[3] *= 2.0 * sigmoid(10.0 * vn) - 1.0;
  }
}

}  // namespace

extern "C" {

// Camera record as laid out by the Python wrapper (must match struct Cam).
int vso_camera_bytes() { return (int)sizeof(Cam); }
int vso_layer_bytes() { return (int)sizeof(Layer); }

// Step 1 on its own: snapped X, Y (1/256 px), w = 1/z and validity per vertex.
void vso_project(const float* xyz, int32_t n_vert, const void* cam, int64_t* X, int64_t* Y, double* w,
                 uint8_t* valid) {
  const Cam c = to_cam(cam);
  for (int32_t v = 0; v < n_vert; ++v) {
    Vtx p = project(xyz + 3 * v, c);
    X[v] = p.X;
    Y[v] = p.Y;
    w[v] = p.w;
    valid[v] = p.valid ? 1 : 0;
  }
}

// Steps 1-3 for one mesh and one view: visibility plane [H][W] of keys
// (float(z) bits << 32 | triangle id), EMPTY = 2^64 - 1 where nothing covers.
// mode 0 = brute force (every triangle at every pixel centre), mode 1 = the same
// test restricted to each triangle's fixed-point bounding box.
// stats[0] invalid-vertex culls, [1] degenerate culls, [2] bad indices,
// [3] covering (triangle, pixel) pairs.
int vso_raster(const void* layer, const void* cam, int mode, uint64_t* vis, int64_t* stats) {
  const Layer& L = *(const Layer*)layer;
  const Cam c = to_cam(cam);
  std::vector<Vtx> vt;
  project_all(L, c, vt);
  const size_t P = (size_t)c.width * c.height;
  for (size_t p = 0; p < P; ++p) vis[p] = kEmpty;
  int64_t st[4] = {0, 0, 0, 0};
  for (int32_t t = 0; t < L.n_tri; ++t) {
    Tri T;
    const int r = setup_triangle(L, vt, t, T);
    if (r == kTriInvalid) { ++st[0]; continue; }
    if (r == kTriDegenerate) { ++st[1]; continue; }
    if (r == kTriBadIndex) { ++st[2]; continue; }
    int64_t i0 = 0, i1 = c.width - 1, j0 = 0, j1 = c.height - 1;
    if (mode == 1) bbox_pixels(T, c, i0, i1, j0, j1);
    for (int64_t j = j0; j <= j1; ++j)
      for (int64_t i = i0; i <= i1; ++i) {
        int64_t E[3];
        edge_values(T, i, j, E);
        if (!inside(T, E)) continue;
        ++st[3];
        const uint64_t key = depth_key(T, E, t);
        uint64_t& slot = vis[(size_t)j * c.width + i];
        if (key < slot) slot = key;
      }
  }
  if (stats) for (int q = 0; q < 4; ++q) stats[q] = st[q];
  return 0;
}

// Coverage counts per pixel, split by the sign of each triangle's screen area
// before normalisation (a watertightness probe; uses the same inside test).
int vso_coverage(const void* layer, const void* cam, int32_t* pos, int32_t* neg) {
  const Layer& L = *(const Layer*)layer;
  const Cam c = to_cam(cam);
  std::vector<Vtx> vt;
  project_all(L, c, vt);
  const size_t P = (size_t)c.width * c.height;
  for (size_t p = 0; p < P; ++p) { pos[p] = 0; neg[p] = 0; }
  for (int32_t t = 0; t < L.n_tri; ++t) {
    Tri T;
    if (setup_triangle(L, vt, t, T) != kTriOk) continue;
    int64_t i0, i1, j0, j1;
    bbox_pixels(T, c, i0, i1, j0, j1);
    for (int64_t j = j0; j <= j1; ++j)
      for (int64_t i = i0; i <= i1; ++i) {
        int64_t E[3];
        edge_values(T, i, j, E);
        if (!inside(T, E)) continue;
        if (T.orig_sign > 0) ++pos[(size_t)j * c.width + i];
        else ++neg[(size_t)j * c.width + i];
      }
  }
  return 0;
}

// Step 4: shade one view.  vis holds k planes [k][H][W]; out is [H][W][4]
// (RGB, A = 1 - final transmittance).  Optional debug outputs (may be null):
// lam [k][H][W][3] barycentrics, uvo [k][H][W][2] interpolated UV (NaN where
// the layer is not hit).  wrap: 0 = repeat, 1 = clamp to edge.
int vso_shade(int32_t k, const void* layers, const void* cam, const uint64_t* vis, int wrap, double* out,
              double* lam, double* uvo) {
  const Layer* L = (const Layer*)layers;
  const Cam c = to_cam(cam);
  std::vector<std::vector<Vtx>> vt(k);
  for (int l = 0; l < k; ++l) project_all(L[l], c, vt[l]);
  const size_t P = (size_t)c.width * c.height;
  std::vector<Hit> hits(k);
  int err = 0;
  for (int64_t j = 0; j < c.height; ++j)
    for (int64_t i = 0; i < c.width; ++i) {
      const size_t p = (size_t)j * c.width + i;
      for (int l = 0; l < k; ++l) {
        hits[l] = shade_slot(L[l], l, vt[l], vis[(size_t)l * P + p], i, j, wrap, nullptr, &err);
        if (lam) for (int q = 0; q < 3; ++q) lam[((size_t)l * P + p) * 3 + q] = hits[l].hit ? hits[l].lam[q] : NAN;
        if (uvo) {
          uvo[((size_t)l * P + p) * 2 + 0] = hits[l].hit ? hits[l].u : NAN;
          uvo[((size_t)l * P + p) * 2 + 1] = hits[l].hit ? hits[l].v : NAN;
        }
      }
      blend_pixel(k, hits.data(), out + 4 * p);
    }
  return err;
}

// Step 5: adjoint of the blend and of the bilinear fetch for one view.
// grad_out [H][W][4] is dL/d(RGB, A); if target is non-null the loss is the
// RGB L2 loss sum_p ||RGB_p - target_p||^2 and grad_out is ignored.
// grad_tex[l] ([Ht][Wt][4] each) is ACCUMULATED.
//   dL/dc_l = g_rgb a_l T_l
//   dL/da_l = T_l <g_rgb, c_l - S_l> + g_A T_l prod_{m>l} (1 - a_m)
// with S_l the colour blended behind layer l; both follow from differentiating
// the blend above.  Each corner texel q receives its bilinear weight times these.
int vso_backward(int32_t k, const void* layers, const void* cam, const uint64_t* vis, int wrap,
                 const double* grad_out, const float* target, int loss, double* const* grad_tex) {
  const Layer* L = (const Layer*)layers;
  const Cam c = to_cam(cam);
  std::vector<std::vector<Vtx>> vt(k);
  for (int l = 0; l < k; ++l) project_all(L[l], c, vt[l]);
  const size_t P = (size_t)c.width * c.height;
  std::vector<Hit> hits(k);
  std::vector<double> T(k);
  int err = 0;
  for (int64_t j = 0; j < c.height; ++j)
    for (int64_t i = 0; i < c.width; ++i) {
      const size_t p = (size_t)j * c.width + i;
      double tr = 1.0, C[3] = {0, 0, 0};
      for (int l = 0; l < k; ++l) {
        hits[l] = shade_slot(L[l], l, vt[l], vis[(size_t)l * P + p], i, j, wrap, nullptr, &err);
        T[l] = tr;
        if (!hits[l].hit) continue;
        const double a = hits[l].rgba[3];
        for (int ch = 0; ch < 3; ++ch) C[ch] += tr * a * hits[l].rgba[ch];
        tr *= (1.0 - a);
      }
      double g[4];
      if (target) {
        // L2: d/dC (C - t)^2 = 2 (C - t);  L1 (Sec. 4.3): d/dC |C - t| = sign(C - t), 0 at a tie
        for (int ch = 0; ch < 3; ++ch) {
          const double d = C[ch] - (double)target[4 * p + ch];
          g[ch] = loss == 1 ? (double)((d > 0.0) - (d < 0.0)) : 2.0 * d;
        }
        g[3] = 0.0;
      } else {
        for (int ch = 0; ch < 4; ++ch) g[ch] = grad_out[4 * p + ch];
      }
      double S[3] = {0, 0, 0}, Pm = 1.0;
      for (int l = k - 1; l >= 0; --l) {
        if (!hits[l].hit) continue;
        const Hit& h = hits[l];
        const double a = h.rgba[3];
        double dc[3], da = 0.0;
        for (int ch = 0; ch < 3; ++ch) {
          dc[ch] = g[ch] * a * T[l];
          da += g[ch] * (h.rgba[ch] - S[ch]);
        }
        da = T[l] * da + g[3] * T[l] * Pm;
        for (int ch = 0; ch < 3; ++ch) S[ch] = a * h.rgba[ch] + (1.0 - a) * S[ch];
        Pm *= (1.0 - a);
        double* G = grad_tex[l];
        for (int dj = 0; dj < 2; ++dj)
          for (int di = 0; di < 2; ++di) {
            const double wq = corner_weight(h.f, dj, di);
            double* cell = G + ((size_t)h.f.j[dj] * L[l].tex_w + (size_t)h.f.i[di]) * 4;
            for (int ch = 0; ch < 3; ++ch) cell[ch] += wq * dc[ch];
            cell[3] += wq * da;
          }
      }
    }
  return err;
}

// Central finite differences of the loss with respect to single texel scalars,
// straight from the forward model (no adjoint involved).  entries [n][4] =
// (layer, row j, column i, channel).  Loss: if target is non-null, the RGB L2
// loss (loss = 0) or L1 loss (loss = 1); otherwise sum_p <g_p, out_p> with
// g = grad_out.  Only pixels whose
// footprint on that layer contains the texel can change, so only they are
// re-evaluated: out[e] = (L(+h) - L(-h)) / (2h).
int vso_fd(int32_t k, const void* layers, const void* cam, const uint64_t* vis, int wrap, const double* grad_out,
           const float* target, int loss_kind, int32_t n_entries, const int32_t* entries, double h, double* out) {
  const Layer* L = (const Layer*)layers;
  const Cam c = to_cam(cam);
  std::vector<std::vector<Vtx>> vt(k);
  for (int l = 0; l < k; ++l) project_all(L[l], c, vt[l]);
  const size_t P = (size_t)c.width * c.height;
  int err = 0;
  // footprint of every (layer, pixel)
  std::vector<Footprint> fp((size_t)k * P);
  std::vector<uint8_t> hit((size_t)k * P, 0);
  for (int64_t j = 0; j < c.height; ++j)
    for (int64_t i = 0; i < c.width; ++i)
      for (int l = 0; l < k; ++l) {
        const size_t p = (size_t)j * c.width + i;
        Hit hh = shade_slot(L[l], l, vt[l], vis[(size_t)l * P + p], i, j, wrap, nullptr, &err);
        if (hh.hit) { fp[(size_t)l * P + p] = hh.f; hit[(size_t)l * P + p] = 1; }
      }
  std::vector<Hit> hits(k);
  for (int32_t e = 0; e < n_entries; ++e) {
    const int32_t el = entries[4 * e], ej = entries[4 * e + 1], ei = entries[4 * e + 2], ec = entries[4 * e + 3];
    double acc = 0.0;
    for (size_t p = 0; p < P; ++p) {
      if (!hit[(size_t)el * P + p]) continue;
      const Footprint& f = fp[(size_t)el * P + p];
      if (!((f.i[0] == ei || f.i[1] == ei) && (f.j[0] == ej || f.j[1] == ej))) continue;
      const int64_t i = (int64_t)(p % c.width), j = (int64_t)(p / c.width);
      double loss[2];
      for (int sgn = 0; sgn < 2; ++sgn) {
        Perturb pt{el, ej, ei, ec, sgn == 0 ? h : -h};
        for (int l = 0; l < k; ++l)
          hits[l] = shade_slot(L[l], l, vt[l], vis[(size_t)l * P + p], i, j, wrap, &pt, &err);
        double o[4];
        blend_pixel(k, hits.data(), o);
        double lv = 0.0;
        if (target) {
          for (int ch = 0; ch < 3; ++ch) {
            const double d = o[ch] - (double)target[4 * p + ch];
            lv += loss_kind == 1 ? std::fabs(d) : d * d;
          }
        } else {
          for (int ch = 0; ch < 4; ++ch) lv += grad_out[4 * p + ch] * o[ch];
        }
        loss[sgn] = lv;
      }
      acc += loss[0] - loss[1];
    }
    out[e] = acc / (2.0 * h);
  }
  return err;
}

// Real spherical harmonics (degree <= 3) of a unit direction, for the pins.
void vso_sh_basis(const double* d, double* Y) { sh_basis(d, Y); }

int vso_sh_layer_bytes() { return (int)sizeof(ShLayer); }

// Baked SH appearance, forward: [H][W][4] f64 RGBA of one view (RGB over
// black, A = 1 - T), the layers blended as in vso_shade.
int vso_shade_sh(int32_t k, const void* layers, const void* sh_layers, const void* cam, const uint64_t* vis,
                 int degree, double vmin, double vmax, int wrap, int view_alpha, double* out) {
  const Layer* L = (const Layer*)layers;
  const ShLayer* S = (const ShLayer*)sh_layers;
  const Cam c = to_cam(cam);
  if (degree < 0 || degree > 3) return 2;
  std::vector<std::vector<Vtx>> vt(k);
  for (int l = 0; l < k; ++l) project_all(L[l], c, vt[l]);
  const size_t P = (size_t)c.width * c.height;
  std::vector<Hit> hits(k);
  int err = 0;
  for (int64_t j = 0; j < c.height; ++j)
    for (int64_t i = 0; i < c.width; ++i) {
      const size_t p = (size_t)j * c.width + i;
      double d[3];
      pixel_ray(c, i, j, d);
      for (int l = 0; l < k; ++l) {
        const uint64_t key = vis[(size_t)l * P + p];
        if (slot_uv(L[l], vt[l], key, i, j, hits[l], &err))
          sh_rgba(L[l], S[l], hits[l], (int32_t)(key & 0xffffffffu), d, degree, vmin, vmax, wrap, view_alpha,
                  hits[l].rgba);
      }
      blend_pixel(k, hits.data(), out + 4 * p);
    }
  return err;
}

}  // extern "C"

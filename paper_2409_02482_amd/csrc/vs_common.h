// Device-side data layout and exact arithmetic shared by the gfx950 kernels.
//
// The visibility computation is specified in integer arithmetic plus a fixed
// FP64 recipe so that it is reproducible bit for bit; this file holds that
// recipe.  It is compiled with -ffp-contract=off: no multiply-add may fuse
// in the projection and depth expressions below.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vs.h"

namespace vs {

constexpr int kMaxLayers = VS_MAX_LAYERS;
constexpr uint64_t kEmpty = VS_EMPTY;
constexpr int32_t kInvalidX = INT32_MIN;
constexpr int kWrapClamp = 1;   // vs_shade_opts::wrap value for clamp-to-edge (0 = repeat)

// Per-layer mesh table, passed by value as a kernel argument.
struct LayerTable {
  const float* xyz[kMaxLayers];
  const float* uv[kMaxLayers];
  const int32_t* tri[kMaxLayers];
  int32_t n_vert[kMaxLayers];
  int32_t n_tri[kMaxLayers];
  int64_t vert_off[kMaxLayers + 1];  // prefix of n_vert: layer l's vertices in one view's projected block
  int64_t tri_off[kMaxLayers + 1];   // prefix of n_tri
  int64_t tri_pad[kMaxLayers + 1];   // prefix of n_tri rounded up to 64: one layer per wavefront in per-triangle launches
  int32_t k;
};

// Per-layer texture table (and gradient planes), passed by value.
struct TexTable {
  const float4* tex[kMaxLayers];
  float* grad[kMaxLayers];
  int32_t w[kMaxLayers];
  int32_t h[kMaxLayers];
  double inv_w[kMaxLayers];
  double inv_h[kMaxLayers];
};

// Projected vertex: snapped screen position in 1/256 px and w = 1/z.
// X == kInvalidX marks a vertex that invalidates its triangles.
struct alignas(16) ProjVert {
  int32_t X, Y;
  double w;
};

// Workspace layout (offsets in bytes from the 256-aligned workspace base).
struct WsLayout {
  size_t status;     // VS_STAT_COUNT u64 counters
  size_t tile_view;  // int32 [16-pixel tiles of all views]: owning view (shading)
  size_t bin_view;   // int32 [raster bin tiles of all views]: owning view
  size_t proj;       // ProjVert [n_views][sum n_vert]
  size_t count;      // u32 [n_bins] entries per bin (before the scan: only those of triangles
                     //   for which the bin is not the first; the scan adds the reservations)
  size_t offset;     // u64 [n_bins] exclusive prefix of count
  size_t cursor;     // u32 [2 n_bins] per bin and side (front from the head, others from the
                     //   tail): first-bin places reserved by the count, then the scatter's
  size_t spans;      // SpanRec [n_views][sum n_tri]: box, depth bound and first-bin place of every triangle
  size_t partial;    // u64 [ceil(n_bins / 1024)] scan block totals
  size_t list;       // int32 [capacity] triangle ids of all bins
  int64_t n_tiles16, n_tiles_bin, n_bins, n_partial;
  uint64_t capacity;
  int bin, slot;
  size_t total;
};

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ------------------------------------------------------------------ step 1
// Camera transform, projection and snapping to 1/256 px (round half to even),
// w = 1/z.  FP64, left to right, unfused.
__device__ inline ProjVert project_vertex(const float* p, const vs_camera& c) {
  ProjVert o;
  o.X = kInvalidX;
  o.Y = kInvalidX;
  o.w = 0.0;
  const double px = p[0], py = p[1], pz = p[2];
  const double xc = ((c.R[0] * px + c.R[1] * py) + c.R[2] * pz) + c.t[0];
  const double yc = ((c.R[3] * px + c.R[4] * py) + c.R[5] * pz) + c.t[1];
  const double zc = ((c.R[6] * px + c.R[7] * py) + c.R[8] * pz) + c.t[2];
  if (!(__builtin_isfinite(xc) && __builtin_isfinite(yc) && __builtin_isfinite(zc))) return o;
  if (!(zc > c.z_near)) return o;
  const double xs = c.fx * (xc / zc) + c.cx;
  const double ys = c.fy * (yc / zc) + c.cy;
  if (!(__builtin_fabs(xs) < 65536.0 && __builtin_fabs(ys) < 65536.0)) return o;
  o.X = (int32_t)__builtin_rint(xs * 256.0);
  o.Y = (int32_t)__builtin_rint(ys * 256.0);
  o.w = 1.0 / zc;
  return o;
}

// ------------------------------------------------------------------ step 2
// Triangle after orientation normalisation.  Screen coordinates are integers
// below 2^25 in magnitude, so every edge-function value (< 2^51) is exact in
// FP64; the kernels evaluate edge functions in doubles.
struct TriSetup {
  double X[3], Y[3];
  double w[3];
  int32_t vid[3];
  double area2;      // > 0
  double th[3];      // inside iff E_e >= th_e: 0 for an owned (top/left) edge, 1 otherwise
  int orig_sign;     // sign of the screen area before normalisation
};

enum { kTriOk = 0, kTriInvalid = 1, kTriDegenerate = 2, kTriBadIndex = 3 };

// Top-left ownership of directed edge P->Q, y down: going up, or horizontal going right.
__device__ inline bool top_left(double px, double py, double qx, double qy) {
  const double dy = qy - py, dx = qx - px;
  return dy < 0.0 || (dy == 0.0 && dx > 0.0);
}

// The raw loads of one triangle's set-up: its three vertex ids (one 12-byte
// load) and its three projected vertices (three 16-byte loads, all in flight
// together).  An out-of-range id reads vertex 0 instead and marks the triangle
// bad.  Split from the arithmetic so that a thread can have the loads of
// several triangles in flight before it uses any of them.
struct TriLoad {
  int32_t id[3];
  int4 a, b, c;
  bool bad;
};

// Element e of a per-layer array, addressed as a 32-bit byte offset from the
// (uniform) array base: a layer holds at most VS_MAX_LAYER_ELEMS (2^28)
// vertices and triangles, so 16-byte vertex records and 12-byte triangles stay
// below 2^32 bytes, and the loads need no per-lane 64-bit address arithmetic.
template <typename T>
__device__ inline T elem_at(const void* base, uint32_t e) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (size_t)(e * (uint32_t)sizeof(T)));
}

// The three vertex ids of triangle t of a layer.
__device__ inline int3 load_ids(const int32_t* tri, uint32_t t) { return elem_at<int3>(tri, t); }

// OFF32: the vertices are addressed as 32-bit byte offsets from pv (a scalar base
// register, no per-lane 64-bit address arithmetic), else with 64-bit pointer
// arithmetic.  The raster kernel takes the former (1-3 % faster); the bin count
// kernel, which keeps two triangles' records live, the latter (with 32-bit
// offsets it needed 66 instead of 50 registers and ran slower).
template <bool OFF32 = false>
__device__ inline void load_vertices(int3 ids, int32_t n_vert, const ProjVert* pv, TriLoad& r) {
  r.id[0] = ids.x; r.id[1] = ids.y; r.id[2] = ids.z;
  r.bad = (uint32_t)ids.x >= (uint32_t)n_vert || (uint32_t)ids.y >= (uint32_t)n_vert ||
          (uint32_t)ids.z >= (uint32_t)n_vert;
  if (OFF32) {
    r.a = elem_at<int4>(pv, r.bad ? 0u : (uint32_t)ids.x);
    r.b = elem_at<int4>(pv, r.bad ? 0u : (uint32_t)ids.y);
    r.c = elem_at<int4>(pv, r.bad ? 0u : (uint32_t)ids.z);
  } else {
    r.a = *reinterpret_cast<const int4*>(pv + (r.bad ? 0 : ids.x));
    r.b = *reinterpret_cast<const int4*>(pv + (r.bad ? 0 : ids.y));
    r.c = *reinterpret_cast<const int4*>(pv + (r.bad ? 0 : ids.z));
  }
}

__device__ inline ProjVert proj_of(int4 r) {
  ProjVert o;
  o.X = r.x;
  o.Y = r.y;
  o.w = __hiloint2double(r.w, r.z);
  return o;
}

// Orientation normalisation and edge ownership of a loaded triangle.
// Branch-free until the status is chosen.
__device__ inline int setup_loaded(const TriLoad& q, TriSetup& T) {
  ProjVert a = proj_of(q.a), b = proj_of(q.b), c = proj_of(q.c);
  int32_t id[3] = {q.id[0], q.id[1], q.id[2]};
  const bool invalid = a.X == kInvalidX || b.X == kInvalidX || c.X == kInvalidX;
  double area2 = ((double)b.X - (double)a.X) * ((double)c.Y - (double)a.Y) -
                 ((double)b.Y - (double)a.Y) * ((double)c.X - (double)a.X);
  const bool neg = area2 < 0.0;
  T.orig_sign = neg ? -1 : 1;
  if (neg) {   // selects, not a branch around loads: the vertices are already in registers
    const ProjVert t = b; b = c; c = t;
    const int32_t ti = id[1]; id[1] = id[2]; id[2] = ti;
    area2 = -area2;
  }
  T.X[0] = a.X; T.Y[0] = a.Y; T.w[0] = a.w;
  T.X[1] = b.X; T.Y[1] = b.Y; T.w[1] = b.w;
  T.X[2] = c.X; T.Y[2] = c.Y; T.w[2] = c.w;
  T.vid[0] = id[0]; T.vid[1] = id[1]; T.vid[2] = id[2];
  T.area2 = area2;
  T.th[0] = top_left(T.X[1], T.Y[1], T.X[2], T.Y[2]) ? 0.0 : 1.0;
  T.th[1] = top_left(T.X[2], T.Y[2], T.X[0], T.Y[0]) ? 0.0 : 1.0;
  T.th[2] = top_left(T.X[0], T.Y[0], T.X[1], T.Y[1]) ? 0.0 : 1.0;
  return q.bad ? kTriBadIndex : invalid ? kTriInvalid : area2 == 0.0 ? kTriDegenerate : kTriOk;
}

// Triangle t of a layer (tri: its triangles); pv the projected vertices of
// the layer in this view.
template <bool OFF32 = false>
__device__ inline int setup_triangle(const int32_t* tri, uint32_t t, int32_t n_vert, const ProjVert* pv, TriSetup& T) {
  TriLoad q;
  load_vertices<OFF32>(load_ids(tri, t), n_vert, pv, q);
  return setup_loaded(q, T);
}

// Edge functions at sample point (px, py) (1/256 px units):
// E0 = cross(c-b, P-b), E1 = cross(a-c, P-c), E2 = cross(b-a, P-a).
__device__ inline void edge_values(const TriSetup& T, double px, double py, double E[3]) {
  E[0] = (T.X[2] - T.X[1]) * (py - T.Y[1]) - (T.Y[2] - T.Y[1]) * (px - T.X[1]);
  E[1] = (T.X[0] - T.X[2]) * (py - T.Y[2]) - (T.Y[0] - T.Y[2]) * (px - T.X[2]);
  E[2] = (T.X[1] - T.X[0]) * (py - T.Y[0]) - (T.Y[1] - T.Y[0]) * (px - T.X[0]);
}

// float(a / s), the quotient rounded to double first, for the operands of a
// depth key: a = area2 >= 1 and s = E0 wa + E1 wb + E2 wc >= area2 min(w),
// both normal and far inside the double range (w = 1/z of float-range depths),
// as is their quotient.  The steps are those of the IEEE FP64 division that
// hipcc emits (reciprocal estimate, two Newton steps, quotient, one residual
// step), without its operand scaling (v_div_scale: taken only for denormal or
// extreme operands) and its special-value fix-up (v_div_fixup: only for zero,
// infinite or NaN operands and results); the residual step is the plain FMA
// that v_div_fmas is when nothing was scaled.  For these operands the result is
// therefore the correctly rounded quotient, in 9 instead of 12 instructions
// (bin raster 4.95 -> 4.80 ms on the metric scene).  A guarded one-step form
// (the IEEE division only near a float rounding midpoint) took 5.06 ms.
__device__ inline float quotient_f32(double a, double s) {
  double r = __builtin_amdgcn_rcp(s);
  r = fma(r, fma(-s, r, 1.0), r);
  r = fma(r, fma(-s, r, 1.0), r);
  const double q0 = a * r;
  return (float)fma(fma(-s, q0, a), r, q0);
}

// Visibility key: bits of float(z) in the high word, triangle id in the low
// word; z = area2 / (E0 wa + E1 wb + E2 wc), the perspective-correct depth.
__device__ inline uint64_t depth_key(const TriSetup& T, double E0, double E1, double E2, uint32_t t) {
  const double s = (E0 * T.w[0] + E1 * T.w[1]) + E2 * T.w[2];
  const float zf = quotient_f32(T.area2, s);
  return ((uint64_t)__float_as_uint(zf) << 32) | (uint64_t)t;
}

// A key no smaller than any key this triangle can produce, for skipping the
// exact depth of fragments that cannot win.  Inside the triangle the edge
// values are non-negative and sum to area2, so 1/z <= max w, i.e.
// z >= 1 / max w; the computed z (three products, two sums, one quotient,
// each correctly rounded) is at least (1/max w)(1 - 5e-16).  The bound below
// sits 1e-12 under that and is rounded down to float, so
// float(z) >= lower and hence depth_key(...) >= the returned key.
__device__ inline uint64_t depth_lower_key(const TriSetup& T, uint32_t t) {
  const double maxw = fmax(T.w[0], fmax(T.w[1], T.w[2]));
  const double zlo = (1.0 / maxw) * (1.0 - 1e-12);
  const float lo = __double2float_rd(zlo);
  return ((uint64_t)__float_as_uint(lo) << 32) | (uint64_t)t;
}

// Binary search of the view that owns flat index g in a prefix array read
// with stride (records of vs_view).  Returns v with off(v) <= g < off(v+1).
__device__ inline int find_view_tile(const vs_view* views, int n_views, int64_t g, int slot) {
  int lo = 0, hi = n_views;  // invariant: off(lo) <= g < off(hi)
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (views[mid].tile_offset[slot] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

}  // namespace vs

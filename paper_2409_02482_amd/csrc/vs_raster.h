// Visibility kernels (steps 1-3): vertex projection and per-layer
// rasterisation into 64-bit (depth, triangle id) keys.
#pragma once

#include "vs_common.h"

namespace vs {

// Fill n u64 words with a value (grid-stride).
__global__ void __launch_bounds__(256) k_fill_u64(uint64_t* __restrict__ p, int64_t n, uint64_t val) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = val;
}

// Step 1 for every (view, layer, vertex).  grid.x covers the vertices of all
// layers of one view (vert_off prefix), grid.y = view.
__global__ void __launch_bounds__(256) k_project(const vs_view* __restrict__ views, LayerTable L,
                                                 ProjVert* __restrict__ proj, int64_t vpv) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (g >= vpv) return;
  int l = 0;
  while (l + 1 < L.k && L.vert_off[l + 1] <= g) ++l;
  const int64_t i = g - L.vert_off[l];
  proj[(int64_t)v * vpv + g] = project_vertex(L.xyz[l] + 3 * i, views[v].cam);
}

// Steps 2-3, direct form: one thread per (view, layer, triangle); the thread
// walks its triangle's fixed-point bounding box and takes a 64-bit atomic
// minimum into the layer's visibility plane (which must hold EMPTY before).
// grid.x covers the triangles of all layers (tri_off prefix), grid.y = view.
__global__ void __launch_bounds__(256) k_raster_direct(const vs_view* __restrict__ views, LayerTable L,
                                                       const ProjVert* __restrict__ proj, int64_t vpv,
                                                       unsigned long long* __restrict__ vis,
                                                       unsigned long long* __restrict__ status, int count_frags) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  const int k = L.k;
  if (g >= L.tri_off[k]) return;
  int l = 0;
  while (l + 1 < k && L.tri_off[l + 1] <= g) ++l;
  const int32_t t = (int32_t)(g - L.tri_off[l]);
  const vs_view& V = views[v];
  const int W = V.cam.width, H = V.cam.height;
  const ProjVert* P = proj + (int64_t)v * vpv + L.vert_off[l];
  TriSetup T;
  const int r = setup_triangle(L.tri[l] + 3 * (int64_t)t, L.n_vert[l], P, T);
  if (r != kTriOk) {
    const int slot = r == kTriInvalid ? VS_STAT_CULLED_INVALID
                   : r == kTriDegenerate ? VS_STAT_CULLED_DEGENERATE : VS_STAT_BAD_INDEX;
    atomicAdd(status + slot, 1ull);
    return;
  }
  const double mnx = fmin(T.X[0], fmin(T.X[1], T.X[2])), mxx = fmax(T.X[0], fmax(T.X[1], T.X[2]));
  const double mny = fmin(T.Y[0], fmin(T.Y[1], T.Y[2])), mxy = fmax(T.Y[0], fmax(T.Y[1], T.Y[2]));
  // pixel centres 256 i + 128 inside [mnx, mxx]
  const int i0 = max((int)ceil((mnx - 128.0) * (1.0 / 256.0)), 0);
  const int i1 = min((int)floor((mxx - 128.0) * (1.0 / 256.0)), W - 1);
  const int j0 = max((int)ceil((mny - 128.0) * (1.0 / 256.0)), 0);
  const int j1 = min((int)floor((mxy - 128.0) * (1.0 / 256.0)), H - 1);
  if (i0 > i1 || j0 > j1) return;
  unsigned long long* plane = vis + (int64_t)k * V.pix_offset + (int64_t)l * W * H;
  // d E / d(pixel step in x) and in y
  const double dx0 = -(T.Y[2] - T.Y[1]) * 256.0, dy0 = (T.X[2] - T.X[1]) * 256.0;
  const double dx1 = -(T.Y[0] - T.Y[2]) * 256.0, dy1 = (T.X[0] - T.X[2]) * 256.0;
  const double dx2 = -(T.Y[1] - T.Y[0]) * 256.0, dy2 = (T.X[1] - T.X[0]) * 256.0;
  double Er[3];
  edge_values(T, 256.0 * i0 + 128.0, 256.0 * j0 + 128.0, Er);
  unsigned long long frags = 0;
  for (int j = j0; j <= j1; ++j) {
    double E0 = Er[0], E1 = Er[1], E2 = Er[2];
    for (int i = i0; i <= i1; ++i) {
      if (E0 >= T.th[0] && E1 >= T.th[1] && E2 >= T.th[2]) {
        atomicMin(plane + (int64_t)j * W + i, (unsigned long long)depth_key(T, E0, E1, E2, (uint32_t)t));
        ++frags;
      }
      E0 += dx0; E1 += dx1; E2 += dx2;
    }
    Er[0] += dy0; Er[1] += dy1; Er[2] += dy2;
  }
  if (count_frags && frags) atomicAdd(status + VS_STAT_FRAGMENTS, frags);
}

}  // namespace vs

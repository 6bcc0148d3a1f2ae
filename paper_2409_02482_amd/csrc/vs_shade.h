// Shading kernels (steps 4-5): perspective-correct UV, bilinear texture
// fetch, fixed-order front-to-back blending, and the texture adjoint.
//
// Barycentrics, UVs and texel coordinates are computed in FP64 (an FP32 texel
// coordinate near 1024 has an ulp of 6e-5 texel); the fractional offsets,
// the bilinear blend and the compositing run in FP32.
#pragma once

#include "vs_common.h"

namespace vs {

constexpr int kShadeTile = 16;      // 16 x 16 pixel tiles, one 256-thread block each
constexpr int kShadeTileSlot = 1;   // vs_view::tile_offset slot of 16-pixel tiles

struct Foot {
  int32_t i0, i1, j0, j1;  // wrapped texel indices of the 2x2 footprint
  float fx, fy;            // offsets from texel centre (i0, j0)
};

__device__ inline int32_t wrap_texel(int64_t i, int32_t n, int wrap) {
  if (wrap == kWrapClamp) return (int32_t)(i < 0 ? 0 : (i >= n ? n - 1 : i));
  int64_t m = i % n;
  return (int32_t)(m < 0 ? m + n : m);
}

// Bilinear footprint: texel centres at (i + 1/2)/W, so the sample sits at
// x = u W - 1/2 in texel-centre coordinates.
__device__ inline Foot footprint(double u, double v, int32_t W, int32_t H, int wrap) {
  double x = u * (double)W - 0.5, y = v * (double)H - 0.5;
  x = fmin(fmax(x, -1.0e9), 1.0e9);
  y = fmin(fmax(y, -1.0e9), 1.0e9);
  const double xf = floor(x), yf = floor(y);
  Foot f;
  f.fx = (float)(x - xf);
  f.fy = (float)(y - yf);
  const int64_t ix = (int64_t)xf, iy = (int64_t)yf;
  f.i0 = wrap_texel(ix, W, wrap);
  f.i1 = wrap_texel(ix + 1, W, wrap);
  f.j0 = wrap_texel(iy, H, wrap);
  f.j1 = wrap_texel(iy + 1, H, wrap);
  return f;
}

__device__ inline float4 bilinear(const float4* __restrict__ tex, int32_t W, const Foot& f) {
#pragma clang fp contract(fast)
  const float4 t00 = tex[(int64_t)f.j0 * W + f.i0];
  const float4 t01 = tex[(int64_t)f.j0 * W + f.i1];
  const float4 t10 = tex[(int64_t)f.j1 * W + f.i0];
  const float4 t11 = tex[(int64_t)f.j1 * W + f.i1];
  const float w00 = (1.0f - f.fx) * (1.0f - f.fy), w01 = f.fx * (1.0f - f.fy);
  const float w10 = (1.0f - f.fx) * f.fy, w11 = f.fx * f.fy;
  float4 r;
  r.x = w00 * t00.x + w01 * t01.x + w10 * t10.x + w11 * t11.x;
  r.y = w00 * t00.y + w01 * t01.y + w10 * t10.y + w11 * t11.y;
  r.z = w00 * t00.z + w01 * t01.z + w10 * t10.z + w11 * t11.z;
  r.w = w00 * t00.w + w01 * t01.w + w10 * t10.w + w11 * t11.w;
  return r;
}

// Rebuild the triangle named by a key and compute the UV footprint at pixel
// (x, y).  Returns false (and counts a bad key) if the key names no valid triangle.
__device__ inline bool slot_footprint(const LayerTable& L, int l, const ProjVert* P, uint64_t key, int x, int y,
                                      int32_t W, int32_t H, int wrap, Foot& f,
                                      unsigned long long* status) {
  const uint32_t t = (uint32_t)(key & 0xffffffffu);
  TriSetup T;
  if (t >= (uint32_t)L.n_tri[l] || setup_triangle(L.tri[l] + 3 * (int64_t)t, L.n_vert[l], P, T) != kTriOk) {
    atomicAdd(status + VS_STAT_BAD_KEY, 1ull);
    return false;
  }
  double E[3];
  edge_values(T, 256.0 * x + 128.0, 256.0 * y + 128.0, E);
  const double s = (E[0] * T.w[0] + E[1] * T.w[1]) + E[2] * T.w[2];
  const double inv = 1.0 / s;
  const double la = E[0] * T.w[0] * inv, lb = E[1] * T.w[1] * inv, lc = E[2] * T.w[2] * inv;
  const float2* uv = reinterpret_cast<const float2*>(L.uv[l]);
  const float2 ua = uv[T.vid[0]], ub = uv[T.vid[1]], uc = uv[T.vid[2]];
  const double u = (la * (double)ua.x + lb * (double)ub.x) + lc * (double)uc.x;
  const double v = (la * (double)ua.y + lb * (double)ub.y) + lc * (double)uc.y;
  f = footprint(u, v, W, H, wrap);
  return true;
}

struct TileCoord {
  int v, x, y;
  bool valid;
};

__device__ inline TileCoord shade_tile_coord(const vs_view* __restrict__ views, int n_views) {
  TileCoord c;
  const int64_t g = blockIdx.x;
  c.v = find_view_tile(views, n_views, g, kShadeTileSlot);
  const vs_view& V = views[c.v];
  const int64_t local = g - V.tile_offset[kShadeTileSlot];
  const int tiles_x = (V.cam.width + kShadeTile - 1) / kShadeTile;
  const int tx = (int)(local % tiles_x), ty = (int)(local / tiles_x);
  c.x = tx * kShadeTile + (threadIdx.x % kShadeTile);
  c.y = ty * kShadeTile + (threadIdx.x / kShadeTile);
  c.valid = c.x < V.cam.width && c.y < V.cam.height;
  return c;
}

// Forward: one thread per pixel, 16x16 tiles, layers front to back.
__global__ void __launch_bounds__(256) k_shade_fwd(const vs_view* __restrict__ views, int n_views, LayerTable L,
                                                   TexTable X, const ProjVert* __restrict__ proj, int64_t vpv,
                                                   const uint64_t* __restrict__ vis, float4* __restrict__ out,
                                                   float eps_T, int wrap, unsigned long long* __restrict__ status) {
#pragma clang fp contract(fast)
  const TileCoord c = shade_tile_coord(views, n_views);
  const vs_view& V = views[c.v];
  const int W = V.cam.width, H = V.cam.height;
  const int64_t P = (int64_t)W * H;
  const int k = L.k;
  const int64_t pix = (int64_t)c.y * W + c.x;
  const uint64_t* vrow = vis + (int64_t)k * V.pix_offset + pix;
  float Cr = 0.f, Cg = 0.f, Cb = 0.f, T = c.valid ? 1.0f : 0.0f;
  for (int l = 0; l < k; ++l) {
    const uint64_t key = c.valid ? vrow[(int64_t)l * P] : kEmpty;
    if (key != kEmpty) {
      Foot f;
      if (slot_footprint(L, l, proj + (int64_t)c.v * vpv + L.vert_off[l], key, c.x, c.y, X.w[l], X.h[l], wrap, f,
                         status)) {
        const float4 s = bilinear(X.tex[l], X.w[l], f);
        const float ta = T * s.w;
        Cr += ta * s.x; Cg += ta * s.y; Cb += ta * s.z;
        T *= (1.0f - s.w);
      }
    }
    if (eps_T > 0.f && __all(T < eps_T)) break;
  }
  if (c.valid) out[V.pix_offset + pix] = make_float4(Cr, Cg, Cb, 1.0f - T);
}

// Backward: recompute the layers front to back (keeping c, a, T and the
// footprint of each hit layer), form dL/d(RGB, A), then walk back to front:
//   dL/dc_l = g_rgb a_l T_l,  dL/da_l = T_l <g_rgb, c_l - S_l> + g_A T_l prod_{m>l}(1 - a_m),
// S_l the colour blended behind layer l.  Division-free (a = 1 is fine).
// Each of the 4 corner texels receives its bilinear weight times these.
template <int KMAX>
__global__ void __launch_bounds__(256) k_shade_bwd(const vs_view* __restrict__ views, int n_views, LayerTable L,
                                                   TexTable X, const ProjVert* __restrict__ proj, int64_t vpv,
                                                   const uint64_t* __restrict__ vis,
                                                   const float4* __restrict__ grad_out,
                                                   const float4* __restrict__ target, float loss_scale,
                                                   float4* __restrict__ out, double* __restrict__ sse, int wrap,
                                                   unsigned long long* __restrict__ status) {
#pragma clang fp contract(fast)
  const TileCoord c = shade_tile_coord(views, n_views);
  const vs_view& V = views[c.v];
  const int W = V.cam.width, H = V.cam.height;
  const int64_t P = (int64_t)W * H;
  const int k = L.k;
  const int64_t pix = (int64_t)c.y * W + c.x;
  const uint64_t* vrow = vis + (int64_t)k * V.pix_offset + pix;
  float cr[KMAX], cg[KMAX], cb[KMAX], ca[KMAX], Tl[KMAX];
  Foot fp[KMAX];
  bool hit[KMAX];
  float Cr = 0.f, Cg = 0.f, Cb = 0.f, T = 1.0f;
#pragma unroll
  for (int l = 0; l < KMAX; ++l) {
    hit[l] = false;
    if (l < k && c.valid) {
      const uint64_t key = vrow[(int64_t)l * P];
      if (key != kEmpty &&
          slot_footprint(L, l, proj + (int64_t)c.v * vpv + L.vert_off[l], key, c.x, c.y, X.w[l], X.h[l], wrap,
                         fp[l], status)) {
        const float4 s = bilinear(X.tex[l], X.w[l], fp[l]);
        hit[l] = true;
        cr[l] = s.x; cg[l] = s.y; cb[l] = s.z; ca[l] = s.w; Tl[l] = T;
        const float ta = T * s.w;
        Cr += ta * s.x; Cg += ta * s.y; Cb += ta * s.z;
        T *= (1.0f - s.w);
      }
    }
  }
  float gr = 0.f, gg = 0.f, gb = 0.f, gA = 0.f;
  double my_sse = 0.0;
  if (c.valid) {
    const int64_t gp = V.pix_offset + pix;
    if (target) {
      const float4 tg = target[gp];
      const float dr = Cr - tg.x, dg = Cg - tg.y, db = Cb - tg.z;
      gr = 2.0f * loss_scale * dr; gg = 2.0f * loss_scale * dg; gb = 2.0f * loss_scale * db;
      my_sse = (double)dr * dr + (double)dg * dg + (double)db * db;
    } else {
      const float4 go = grad_out[gp];
      gr = go.x; gg = go.y; gb = go.z; gA = go.w;
    }
    if (out) out[gp] = make_float4(Cr, Cg, Cb, 1.0f - T);
  }
  float Sr = 0.f, Sg = 0.f, Sb = 0.f, Pm = 1.0f;
#pragma unroll
  for (int l = KMAX - 1; l >= 0; --l) {
    if (!hit[l]) continue;
    const float a = ca[l], Tv = Tl[l];
    const float dcr = gr * a * Tv, dcg = gg * a * Tv, dcb = gb * a * Tv;
    const float da = Tv * (gr * (cr[l] - Sr) + gg * (cg[l] - Sg) + gb * (cb[l] - Sb)) + gA * Tv * Pm;
    Sr = a * cr[l] + (1.0f - a) * Sr;
    Sg = a * cg[l] + (1.0f - a) * Sg;
    Sb = a * cb[l] + (1.0f - a) * Sb;
    Pm *= (1.0f - a);
    const Foot& f = fp[l];
    const float w00 = (1.0f - f.fx) * (1.0f - f.fy), w01 = f.fx * (1.0f - f.fy);
    const float w10 = (1.0f - f.fx) * f.fy, w11 = f.fx * f.fy;
    float* G = X.grad[l];
    const int32_t Wt = X.w[l];
    const int64_t q[4] = {((int64_t)f.j0 * Wt + f.i0) * 4, ((int64_t)f.j0 * Wt + f.i1) * 4,
                          ((int64_t)f.j1 * Wt + f.i0) * 4, ((int64_t)f.j1 * Wt + f.i1) * 4};
    const float wq[4] = {w00, w01, w10, w11};
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      unsafeAtomicAdd(G + q[n] + 0, wq[n] * dcr);
      unsafeAtomicAdd(G + q[n] + 1, wq[n] * dcg);
      unsafeAtomicAdd(G + q[n] + 2, wq[n] * dcb);
      unsafeAtomicAdd(G + q[n] + 3, wq[n] * da);
    }
  }
  if (sse) {
    // block reduction of the squared error, one atomic per block
    __shared__ double red[256];
    red[threadIdx.x] = my_sse;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) unsafeAtomicAdd(sse, red[0]);
  }
}

}  // namespace vs

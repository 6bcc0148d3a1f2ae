// Shading kernels (steps 4-5): perspective-correct UV, bilinear texture
// fetch, fixed-order front-to-back blending, and the texture adjoint.
//
// Barycentrics, UVs and texel coordinates are computed in FP64 (an FP32 texel
// coordinate near 1024 has an ulp of 6e-5 texel); the fractional offsets,
// the bilinear blend and the compositing run in FP32.
//
// Work decomposition: one 256-thread block per 16 x 16 pixel tile of one
// view, one thread per pixel, layers walked front to back.  Tiles of all
// views are numbered consecutively; the block -> tile mapping gives each XCD
// (blocks are dealt round-robin to the 8 XCDs) a contiguous run of tiles so
// that neighbouring tiles, which read neighbouring texels, share an L2.
#pragma once

#include "vs_common.h"

namespace vs {

constexpr int kShadeTile = 16;      // 16 x 16 pixel tiles, one 256-thread block each
constexpr int kShadeTileSlot = 1;   // vs_view::tile_offset slot of 16-pixel tiles
constexpr int kNumXcd = 8;

struct Foot {
  int32_t i0, i1, j0, j1;  // wrapped texel indices of the 2x2 footprint
  float fx, fy;            // offsets from texel centre (i0, j0)
};

// Split a texel-centre coordinate into the two neighbouring texel indices and
// the offset from the first, wrapping (repeat) or clamping to [0, n-1].
__device__ inline void split_coord(double x, int32_t n, double inv_n, int wrap, int32_t& i0, int32_t& i1,
                                   float& fr) {
  x = fmin(fmax(x, -1.0e9), 1.0e9);  // also maps NaN to a finite value
  if (wrap == kWrapClamp) {
    x = fmin(fmax(x, 0.0), (double)(n - 1));
    const double f = floor(x);
    i0 = (int32_t)f;
    fr = (float)(x - f);
    i1 = i0 + 1 < n ? i0 + 1 : n - 1;
    return;
  }
  const double f = floor(x);
  fr = (float)(x - f);
  double m = f - (double)n * floor(f * inv_n);  // f mod n, exact for |f| < 2^52
  int32_t i = (int32_t)m;
  if (i < 0) i += n;
  if (i >= n) i -= n;
  i0 = i;
  i1 = i + 1 == n ? 0 : i + 1;
}

// The second texel index of a footprint from the first (as split_coord pairs them).
__device__ inline int32_t next_index(int32_t i0, int32_t n, int wrap) {
  return wrap == kWrapClamp ? (i0 + 1 < n ? i0 + 1 : n - 1) : (i0 + 1 == n ? 0 : i0 + 1);
}

// Texel idx of a texture and float idx of a gradient plane, addressed as 32-bit
// byte offsets from the (uniform) plane base, so that the loads and atomics use
// a scalar base register and no per-lane 64-bit address arithmetic: a texture
// has at most 16384^2 texels, whose 16-byte texels and 4-byte gradient floats
// both stay below 2^32 bytes.
__device__ inline float4 texel_at(const float4* __restrict__ tex, uint32_t idx) {
  return *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(tex) + (size_t)(idx << 4));
}

__device__ inline void grad_add(float* G, uint32_t fidx, float val) {
  unsafeAtomicAdd(reinterpret_cast<float*>(reinterpret_cast<char*>(G) + (size_t)(fidx << 2)), val);
}

__device__ inline float4 bilinear(const float4* __restrict__ tex, int32_t W, const Foot& f) {
#pragma clang fp contract(fast)
  const uint32_t w = (uint32_t)W, r0 = (uint32_t)f.j0 * w, r1 = (uint32_t)f.j1 * w;
  const float4 t00 = texel_at(tex, r0 + (uint32_t)f.i0);
  const float4 t01 = texel_at(tex, r0 + (uint32_t)f.i1);
  const float4 t10 = texel_at(tex, r1 + (uint32_t)f.i0);
  const float4 t11 = texel_at(tex, r1 + (uint32_t)f.i1);
  const float gx = 1.0f - f.fx, gy = 1.0f - f.fy;
  const float w00 = gx * gy, w01 = f.fx * gy, w10 = gx * f.fy, w11 = f.fx * f.fy;
  float4 r;
  r.x = w00 * t00.x + w01 * t01.x + w10 * t10.x + w11 * t11.x;
  r.y = w00 * t00.y + w01 * t01.y + w10 * t10.y + w11 * t11.y;
  r.z = w00 * t00.z + w01 * t01.z + w10 * t10.z + w11 * t11.z;
  r.w = w00 * t00.w + w01 * t01.w + w10 * t10.w + w11 * t11.w;
  return r;
}

struct Tri3 { int32_t a, b, c; };

// Rebuild the triangle a key names and interpolate its UV at the pixel centre
// (px, py) (1/256 px units).  Barycentrics are perspective-correct:
// lambda_q = E_q w_q / sum_r E_r w_r, which does not depend on the winding,
// so no orientation normalisation is needed here.  Returns false (and counts
// a bad key) if the key names no valid triangle.
__device__ inline bool slot_uv(const int32_t* __restrict__ tri, int32_t n_tri, int32_t n_vert,
                               const ProjVert* __restrict__ P, const float2* __restrict__ uv, uint64_t key,
                               double px, double py, double& u, double& v, unsigned long long* status) {
#pragma clang fp contract(fast)
  const uint32_t t = (uint32_t)(key & 0xffffffffu);
  if (t >= (uint32_t)n_tri) {
    atomicAdd(status + VS_STAT_BAD_KEY, 1ull);
    return false;
  }
  const Tri3 id = elem_at<Tri3>(tri, t);
  if ((uint32_t)id.a >= (uint32_t)n_vert || (uint32_t)id.b >= (uint32_t)n_vert ||
      (uint32_t)id.c >= (uint32_t)n_vert) {
    atomicAdd(status + VS_STAT_BAD_KEY, 1ull);
    return false;
  }
  const ProjVert a = elem_at<ProjVert>(P, (uint32_t)id.a), b = elem_at<ProjVert>(P, (uint32_t)id.b),
                 c = elem_at<ProjVert>(P, (uint32_t)id.c);
  const float2 ua = elem_at<float2>(uv, (uint32_t)id.a), ub = elem_at<float2>(uv, (uint32_t)id.b),
               uc = elem_at<float2>(uv, (uint32_t)id.c);
  const double ax = a.X, ay = a.Y, bx = b.X, by = b.Y, cx = c.X, cy = c.Y;
  const double E0 = (cx - bx) * (py - by) - (cy - by) * (px - bx);
  const double E1 = (ax - cx) * (py - cy) - (ay - cy) * (px - cx);
  const double E2 = (bx - ax) * (py - ay) - (by - ay) * (px - ax);
  const double q0 = E0 * a.w, q1 = E1 * b.w, q2 = E2 * c.w;
  const double s = q0 + q1 + q2;
  // 1/s: hardware reciprocal refined by two Newton steps (relative error ~1e-16)
  double r = __builtin_amdgcn_rcp(s);
  r = r * (2.0 - s * r);
  r = r * (2.0 - s * r);
  const double la = q0 * r, lb = q1 * r, lc = q2 * r;
  u = la * (double)ua.x + lb * (double)ub.x + lc * (double)uc.x;
  v = la * (double)ua.y + lb * (double)ub.y + lc * (double)uc.y;
  return true;
}

// The slot's bilinear footprint in a W x H texture.
__device__ inline bool slot_footprint(const int32_t* __restrict__ tri, int32_t n_tri, int32_t n_vert,
                                      const ProjVert* __restrict__ P, const float2* __restrict__ uv, uint64_t key,
                                      double px, double py, int32_t W, int32_t H, double invW, double invH, int wrap,
                                      Foot& f, unsigned long long* status) {
  double u, v;
  if (!slot_uv(tri, n_tri, n_vert, P, uv, key, px, py, u, v, status)) return false;
  split_coord(u * (double)W - 0.5, W, invW, wrap, f.i0, f.i1, f.fx);
  split_coord(v * (double)H - 0.5, H, invH, wrap, f.j0, f.j1, f.fy);
  return true;
}

struct TileCoord {
  int v, x, y;
  bool valid;
  bool live;   // false for padding blocks of the XCD remap
};

// Block -> (view, tile) with an XCD-contiguous remap; tile_view[g] is the view of tile g.
// A tile whose table entry is out of range (a workspace not filled by
// vs_raster_layers for these views) is skipped rather than trusted.
__device__ inline TileCoord shade_tile_coord(const vs_view* __restrict__ views, int n_views,
                                             const int32_t* __restrict__ tile_view, int64_t n_tiles) {
  TileCoord c;
  const int64_t chunk = (n_tiles + kNumXcd - 1) / kNumXcd;
  const int64_t b = blockIdx.x;
  const int64_t g = (b % kNumXcd) * chunk + b / kNumXcd;
  c.v = 0; c.x = c.y = 0; c.valid = false;
  c.live = g < n_tiles;
  if (!c.live) return c;
  c.v = tile_view[g];
  if ((unsigned)c.v >= (unsigned)n_views) { c.v = 0; c.live = false; return c; }
  const vs_view& V = views[c.v];
  const int64_t local = g - V.tile_offset[kShadeTileSlot];
  const int tiles_x = (V.cam.width + kShadeTile - 1) / kShadeTile;
  const int64_t ty = local / tiles_x, tx = local - ty * tiles_x;
  if (local < 0 || ty * kShadeTile >= V.cam.height) { c.live = false; return c; }
  // lane bits: 0 = dx, 1 = dy, 2..4 = 2-pixel column, 5 = 2-pixel row; wave w covers rows 4w..4w+3.
  // Every wave still reads whole 16-pixel row segments, and each DPP quad is a 2 x 2 pixel block.
  const int t = threadIdx.x, lane = t & 63;
  c.x = (int)tx * kShadeTile + ((lane >> 2) & 7) * 2 + (lane & 1);
  c.y = (int)ty * kShadeTile + (t >> 6) * 4 + ((lane >> 5) & 1) * 2 + ((lane >> 1) & 1);
  c.valid = c.x < V.cam.width && c.y < V.cam.height;
  return c;
}

__host__ __device__ inline int64_t shade_grid_blocks(int64_t n_tiles) {
  return (n_tiles + kNumXcd - 1) / kNumXcd * kNumXcd;
}

// tile_view[g] = view owning 16-pixel tile g.
__global__ void __launch_bounds__(256) k_tile_view(const vs_view* __restrict__ views, int n_views,
                                                   int32_t* __restrict__ tile_view, int64_t n_tiles) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_tiles) return;
  tile_view[g] = find_view_tile(views, n_views, g, kShadeTileSlot);
}

// Forward: one thread per pixel, layers front to back.
__global__ void __launch_bounds__(256) k_shade_fwd(const vs_view* __restrict__ views, int n_views,
                                                   const int32_t* __restrict__ tile_view,
                                                   int64_t n_tiles, LayerTable L, TexTable X,
                                                   const ProjVert* __restrict__ proj, int64_t vpv,
                                                   const uint64_t* __restrict__ vis, float4* __restrict__ out,
                                                   float eps_T, int wrap, unsigned long long* __restrict__ status) {
#pragma clang fp contract(fast)
  const TileCoord c = shade_tile_coord(views, n_views, tile_view, n_tiles);
  if (!c.live) return;
  const vs_view& V = views[c.v];
  const int W = V.cam.width, H = V.cam.height;
  const int64_t P = (int64_t)W * H;
  const int k = L.k;
  const int64_t pix = (int64_t)c.y * W + c.x;
  const uint64_t* vrow = vis + (int64_t)k * V.pix_offset + pix;
  const ProjVert* pview = proj + (int64_t)c.v * vpv;
  const double px = 256.0 * c.x + 128.0, py = 256.0 * c.y + 128.0;
  float Cr = 0.f, Cg = 0.f, Cb = 0.f, T = c.valid ? 1.0f : 0.0f;
  // keys of the first layers are requested together (several loads in flight)
  constexpr int kPre = 4;
  uint64_t pre[kPre];
#pragma unroll
  for (int l = 0; l < kPre; ++l) pre[l] = (l < k && c.valid) ? vrow[l * P] : kEmpty;
  for (int l = 0; l < k; ++l) {
    uint64_t key;
    if (l < kPre) {
      key = pre[0];
#pragma unroll
      for (int q = 1; q < kPre; ++q) key = (l == q) ? pre[q] : key;
    } else {
      key = c.valid ? vrow[l * P] : kEmpty;
    }
    if (key != kEmpty) {
      Foot f;
      const int32_t Wt = X.w[l], Ht = X.h[l];
      if (slot_footprint(L.tri[l], L.n_tri[l], L.n_vert[l], pview + L.vert_off[l],
                         reinterpret_cast<const float2*>(L.uv[l]), key, px, py, Wt, Ht, X.inv_w[l], X.inv_h[l],
                         wrap, f, status)) {
        const float4 s = bilinear(X.tex[l], Wt, f);
        const float ta = T * s.w;
        Cr += ta * s.x; Cg += ta * s.y; Cb += ta * s.z;
        T *= (1.0f - s.w);
      }
    }
    if (eps_T > 0.f && __all(T < eps_T)) break;
  }
  if (c.valid) out[V.pix_offset + pix] = make_float4(Cr, Cg, Cb, 1.0f - T);
}

// Wavefront min / max without the LDS pipe: inclusive row scans with DPP
// row shifts (row_shr:n moves lane i - n into lane i; lanes with no source
// keep the identity), so lane 15 of each 16-lane row holds the row's result.
// Call with every lane active.
// Then row_bcast:15 (rows 1 and 3 take lane 15 / 47) and row_bcast:31 (rows 2 and 3
// take lane 31) carry the row results to lane 63.
__device__ inline int32_t wave_min(int32_t v) {
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x111, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x112, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x114, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x118, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x142, 0xa, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT32_MAX, v, 0x143, 0xc, 0xf, false));
  return __builtin_amdgcn_readlane(v, 63);
}

__device__ inline int32_t wave_max(int32_t v) {
  v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x111, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x112, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x114, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x118, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x142, 0xa, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(INT32_MIN, v, 0x143, 0xc, 0xf, false));
  return __builtin_amdgcn_readlane(v, 63);
}

// Orders this wavefront's LDS accesses (a wave's LDS instructions execute in order).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Relative texel offset of index i from reference r in [-n/2, n/2) (repeat) or plain difference (clamp).
__device__ inline int32_t rel_index(int32_t i, int32_t r, int32_t n, int wrap) {
  int32_t d = i - r;
  if (wrap == kWrapClamp) return d;
  if (d >= (n >> 1)) d -= n;
  else if (d < -(n >> 1)) d += n;
  return d;
}

__device__ inline int32_t abs_index(int32_t r, int32_t d, int32_t n, int wrap) {
  int32_t i = r + d;
  if (wrap == kWrapClamp) return i;
  if (i >= n) i -= n;
  else if (i < 0) i += n;
  return i;
}

// Texels in each wavefront's LDS gradient window, and blocks per CU, by the
// largest layer count of the instantiation: up to 9 layers the kernel is held
// to 80 registers, so six blocks of 320-texel windows (25 KiB each) share a CU
// (9 layers spill 4 registers there and still run 2.3 % faster than at five
// blocks of 384-texel windows: 7.76 against 7.94 ms on the k = 9 scene); the
// 16-layer instantiation runs two blocks.
template <int KMAX> struct BwdShape {
  static constexpr int win = KMAX <= 9 ? 320 : 384;
  static constexpr int blocks = KMAX <= 9 ? 6 : 2;
};
constexpr bool kMergeX2 = true;   // third butterfly step (x +- 2) before the window

// Value of v in lane (lane ^ 1), (lane ^ 2) or (lane ^ 4), with DPP (no LDS):
// quad_perm [1,0,3,2], quad_perm [2,3,0,1], and row_shl:4 / row_shr:4 picked by lane bit 2.
__device__ inline int32_t lane_xor1(int32_t v) { return __builtin_amdgcn_mov_dpp(v, 0xb1, 0xf, 0xf, false); }
__device__ inline int32_t lane_xor2(int32_t v) { return __builtin_amdgcn_mov_dpp(v, 0x4e, 0xf, 0xf, false); }
__device__ inline int32_t lane_xor4(int32_t v, bool bit2) {
  const int32_t up = __builtin_amdgcn_mov_dpp(v, 0x104, 0xf, 0xf, false);    // row_shl:4 -> lane + 4
  const int32_t down = __builtin_amdgcn_mov_dpp(v, 0x114, 0xf, 0xf, false);  // row_shr:4 -> lane - 4
  return bit2 ? down : up;
}

// v + (v of lane (lane ^ 2^STEP)) for the lower lane of a pair: xor 1 and xor 2 are quad
// permutations; for xor 4 the lower lane (bit 2 clear) reads lane + 4 (row_shl:4).  The
// caller runs this with exactly the lanes of merging pairs active, so every source lane
// a lower lane reads is active; what an upper lane computes is discarded.
template <int STEP>
__device__ inline float add_upper(float v) {
  constexpr int ctrl = STEP == 0 ? 0xb1 : STEP == 1 ? 0x4e : 0x104;
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xf, 0xf, false));
}

// One butterfly step of merging contributions by base texel: lanes (lane, lane ^ 2^step)
// holding the same key combine their 16 values in the lower lane; the upper lane drops out.
// Runs with only the merging lanes active, so the lane exchange folds into the adds
// (16 v_add_f32_dpp per step).
template <int STEP>
__device__ inline void merge_by_key(int32_t& key, float (&v)[16], int lane) {
  const bool bit = (lane >> STEP) & 1;
  const int32_t other = STEP == 0 ? lane_xor1(key) : STEP == 1 ? lane_xor2(key) : lane_xor4(key, bit);
  const bool same = key >= 0 && other == key;
  if (same) {
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = add_upper<STEP>(v[q]);
  }
  if (same && bit) key = -1;
}

// Backward: recompute the layers front to back (keeping T in front of each hit layer and
// its bilinear footprint), form dL/d(RGB, A), then walk back to front:
//   dL/dc_l = g_rgb a_l T_l,  dL/da_l = T_l <g_rgb, c_l - S_l> + g_A T_l prod_{m>l}(1 - a_m),
// S_l the colour blended behind layer l.  Division-free (a = 1 is fine).
// Each of the 4 corner texels receives its bilinear weight times these.
//
// Scatter, per wavefront (16 x 4 pixels) and layer: neighbouring pixels
// mostly share their base texel (a texel spans several pixels when
// magnified), so the lanes of each 4 x 2 pixel group that share a base
// texel first sum their 16 contributions in registers (DPP butterfly steps:
// x +- 1, y +- 1, x +- 2).  The survivors add into an LDS texel window
// (wrap-aware, relative to the first surviving lane's base texel) with plain
// read-modify-writes, one lane per base texel and round (an owner word per
// cell elects it); the window is then flushed with global float atomics whose
// lanes cover consecutive floats, and zeroed by the same pass, so it starts
// every use empty.  A window covers the base texels' bounding box plus one
// column and one row: the second corner of a footprint is always the next
// cell (wrapping happens when the window is mapped back to texels; a corner
// that coincides with the base texel at a clamped edge was folded onto it and
// adds zero).  A footprint larger than the window is retried per half
// wavefront, then per quarter; a quarter that still does not fit uses direct
// global atomics.
// Window size against occupancy (k = 7, 64 views): 384 texels at five blocks per
// CU took 7.86 ms at 1024^2 and 5.42 ms at 800^2; 320 texels at six blocks 7.32 and
// 5.26 ms; 256 texels at six blocks 7.66 and 5.64 ms (more footprints overflow to the
// half and quarter retries); 272 texels at seven blocks (72 registers, 7 spilled) 7.29
// and 5.44 ms; 240 texels at eight (64 registers, 13 spilled) 7.41 and 5.70 ms.  Four
// blocks per CU measured 10 % slower than five.
template <int KMAX>
__global__ void __launch_bounds__(256, BwdShape<KMAX>::blocks) k_shade_bwd(const vs_view* __restrict__ views, int n_views,
                                                   const int32_t* __restrict__ tile_view, int64_t n_tiles,
                                                   LayerTable L, TexTable X, const ProjVert* __restrict__ proj,
                                                   int64_t vpv, const uint64_t* __restrict__ vis,
                                                   const float4* __restrict__ grad_out,
                                                   const float4* __restrict__ target, float loss_scale,
                                                   int loss,
                                                   float4* __restrict__ out, double* __restrict__ sse, int wrap,
                                                   float eps_T, unsigned long long* __restrict__ status,
                                                   int count_paths) {
#pragma clang fp contract(fast)
  constexpr int kWaveWin = BwdShape<KMAX>::win;
  __shared__ __align__(16) float win_all[4][kWaveWin * 5];   // per wave: RGBA sums, then the owner words
  __shared__ double sred[4];
  const TileCoord c = shade_tile_coord(views, n_views, tile_view, n_tiles);
  if (!c.live) return;  // uniform per block
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  float* win = win_all[tid >> 6];
  float4* wg = reinterpret_cast<float4*>(win);                     // [cell] RGBA sums
  int32_t* owner = reinterpret_cast<int32_t*>(win + kWaveWin * 4);  // [cell]
  // the window is zero before its first use; every flush leaves it zero again
  for (int e = lane; e < kWaveWin; e += 64) wg[e] = make_float4(0.f, 0.f, 0.f, 0.f);
  const vs_view& V = views[c.v];
  const int W = V.cam.width, H = V.cam.height;
  const int64_t P = (int64_t)W * H;
  const int k = L.k;
  const int64_t pix = (int64_t)c.y * W + c.x;
  const uint64_t* vrow = vis + (int64_t)k * V.pix_offset + pix;
  const ProjVert* pview = proj + (int64_t)c.v * vpv;
  const double px = 256.0 * c.x + 128.0, py = 256.0 * c.y + 128.0;
  // every layer's key is requested before any is used (k loads in flight)
  uint64_t keys[KMAX];
#pragma unroll
  for (int l = 0; l < KMAX; ++l) keys[l] = (l < k && c.valid) ? vrow[l * P] : kEmpty;
  // Kept per hit layer for the backward walk: T in front of it and the footprint; the
  // sample itself is re-read there (four texels, still cache resident), which keeps the
  // register count, and so the number of resident wavefronts, up: keeping the samples
  // instead costs either spills (at five blocks per CU) or a block per CU.
  float Tl[KMAX], fxs[KMAX], fys[KMAX];
  int32_t ij[KMAX];   // packed (j0 << 16 | i0); i1, j1 follow from them
  uint32_t hitmask = 0;
  // T starts at 0 on padding lanes, as in k_shade_fwd, so that both kernels take the same early exit
  float Cr = 0.f, Cg = 0.f, Cb = 0.f, T = c.valid ? 1.0f : 0.0f;
  bool walk = true;
#pragma unroll
  for (int l = 0; l < KMAX; ++l) {
    Foot f;
    if (walk && keys[l] != kEmpty &&
        slot_footprint(L.tri[l], L.n_tri[l], L.n_vert[l], pview + L.vert_off[l],
                       reinterpret_cast<const float2*>(L.uv[l]), keys[l], px, py, X.w[l], X.h[l], X.inv_w[l],
                       X.inv_h[l], wrap, f, status)) {
      const float4 s = bilinear(X.tex[l], X.w[l], f);
      hitmask |= 1u << l;
      Tl[l] = T;
      fxs[l] = f.fx; fys[l] = f.fy;
      ij[l] = (f.j0 << 16) | f.i0;
      const float ta = T * s.w;
      Cr += ta * s.x; Cg += ta * s.y; Cb += ta * s.z;
      T *= (1.0f - s.w);
    }
    // the forward kernel's early exit: the layers behind it are neither blended nor differentiated
    if (l < k && eps_T > 0.f && __all(T < eps_T)) walk = false;
  }
  float gr = 0.f, gg = 0.f, gb = 0.f, gA = 0.f;
  double my_sse = 0.0;
  if (c.valid) {
    const int64_t gp = V.pix_offset + pix;
    if (target) {
      const float4 tg = target[gp];
      const float dr = Cr - tg.x, dg = Cg - tg.y, db = Cb - tg.z;
      if (loss == VS_LOSS_L1) {
        // d|x|/dx = sign(x), 0 at a tie
        auto sgn = [](float x) { return (float)((x > 0.0f) - (x < 0.0f)); };
        gr = loss_scale * sgn(dr); gg = loss_scale * sgn(dg); gb = loss_scale * sgn(db);
        my_sse = (double)fabsf(dr) + (double)fabsf(dg) + (double)fabsf(db);
      } else {
        const float s2 = 2.0f * loss_scale;
        gr = s2 * dr; gg = s2 * dg; gb = s2 * db;
        my_sse = (double)dr * dr + (double)dg * dg + (double)db * db;
      }
    } else {
      const float4 go = grad_out[gp];
      gr = go.x; gg = go.y; gb = go.z; gA = go.w;
    }
    if (out) out[gp] = make_float4(Cr, Cg, Cb, 1.0f - T);
  }
  float Sr = 0.f, Sg = 0.f, Sb = 0.f, Pm = 1.0f;
  uint32_t n_path[4] = {0u, 0u, 0u, 0u};   // wavefront-uniform: window per wave / half / quarter, direct
#pragma unroll
  for (int l = KMAX - 1; l >= 0; --l) {
    if (l >= k) continue;  // uniform
    const bool hit = (hitmask >> l) & 1u;
    if (!__any(hit)) continue;  // uniform per wavefront
    const int32_t Wt = X.w[l], Ht = X.h[l];
    float v[16];
    int32_t key = -1, i0 = 0, j0 = 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = 0.0f;
    if (hit) {
      i0 = ij[l] & 0xffff; j0 = ij[l] >> 16;
      Foot f;
      f.i0 = i0; f.j0 = j0; f.i1 = next_index(i0, Wt, wrap); f.j1 = next_index(j0, Ht, wrap);
      f.fx = fxs[l]; f.fy = fys[l];
      const float4 smp = bilinear(X.tex[l], Wt, f);   // the same sample as the forward walk
      const float a = smp.w, Tv = Tl[l];
      const float aT = a * Tv;
      float d[4];
      d[0] = gr * aT; d[1] = gg * aT; d[2] = gb * aT;
      d[3] = Tv * (gr * (smp.x - Sr) + gg * (smp.y - Sg) + gb * (smp.z - Sb)) + gA * Tv * Pm;
      Sr = a * smp.x + (1.0f - a) * Sr;
      Sg = a * smp.y + (1.0f - a) * Sg;
      Sb = a * smp.z + (1.0f - a) * Sb;
      Pm *= (1.0f - a);
      const float fx = fxs[l], fy = fys[l], gx = 1.0f - fx, gy = 1.0f - fy;
      const float wq[4] = {gx * gy, fx * gy, gx * fy, fx * fy};
#pragma unroll
      for (int n = 0; n < 4; ++n) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) v[n * 4 + ch] = wq[n] * d[ch];
      }
      key = j0 * Wt + i0;
    }
    // Clamped at the last column or row (or a texture one texel wide or high), corners
    // coincide: fold them onto the base texel's row or column, so that the corner
    // after it receives zero.  Uniform test: never taken for repeat-wrapped textures
    // wider and higher than one texel.
    if (wrap == kWrapClamp || Wt == 1 || Ht == 1) {
      if (hit && next_index(i0, Wt, wrap) == i0) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) { v[ch] += v[4 + ch]; v[4 + ch] = 0.f; v[8 + ch] += v[12 + ch]; v[12 + ch] = 0.f; }
      }
      if (hit && next_index(j0, Ht, wrap) == j0) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) { v[ch] += v[8 + ch]; v[8 + ch] = 0.f; v[4 + ch] += v[12 + ch]; v[12 + ch] = 0.f; }
      }
    }
    merge_by_key<0>(key, v, lane);
    merge_by_key<1>(key, v, lane);
    if (kMergeX2) merge_by_key<2>(key, v, lane);
    const bool live_all = key >= 0;
    bool direct = false;   // a quarter wavefront whose footprint did not fit: direct atomics below
    float* G = X.grad[l];
    // A footprint larger than the window is retried per half wavefront (lanes
    // 0-31, then 32-63), a half that does not fit per quarter (16 lanes: an
    // 8 x 2 pixel block); a quarter that still does not fit uses direct atomics.
    for (int pass = 0, npass = 1; pass < npass; ++pass) {   // uniform control flow
      const bool live = live_all && (npass == 1 || (lane >> (npass == 2 ? 5 : 4)) == pass);
      const uint64_t live_bits = __ballot(live);
      if (live_bits == 0) continue;
      // window relative to the base texel of the first surviving lane, wrap-aware
      const int first = __builtin_ctzll(live_bits);
      const int32_t ri = __builtin_amdgcn_readlane(i0, first), rj = __builtin_amdgcn_readlane(j0, first);
      const int32_t di = live ? rel_index(i0, ri, Wt, wrap) : 0;
      const int32_t dj = live ? rel_index(j0, rj, Ht, wrap) : 0;
      const int32_t dmin_i = wave_min(live ? di : INT32_MAX);
      const int32_t dmax_i = wave_max(live ? di : INT32_MIN) + 1;
      const int32_t dmin_j = wave_min(live ? dj : INT32_MAX);
      const int32_t dmax_j = wave_max(live ? dj : INT32_MIN) + 1;
      const int32_t ww = dmax_i - dmin_i + 1, wh = dmax_j - dmin_j + 1;
      if (ww * wh <= kWaveWin) {
        ++n_path[npass == 1 ? 0 : npass == 2 ? 1 : 2];
        const int32_t c00 = (dj - dmin_j) * ww + (di - dmin_i);
        const int32_t cells[4] = {c00, c00 + 1, c00 + ww, c00 + ww + 1};
        // For each corner, distinct base texels give distinct cells.  One owner word per
        // base cell elects one lane per base texel and round; the winners then apply the four
        // corners' read-modify-writes one corner at a time.  A wave's LDS instructions complete
        // in order, so no atomics are needed; lanes that lost (equal base texel) retry.
        bool pend = live;
        while (__any(pend)) {
          if (pend) owner[c00] = lane;
          wave_lds_sync();
          const bool mine = pend && owner[c00] == lane;
#pragma unroll
          for (int n = 0; n < 4; ++n) {
            if (mine) {
              float4 acc = wg[cells[n]];
              acc.x += v[n * 4 + 0]; acc.y += v[n * 4 + 1]; acc.z += v[n * 4 + 2]; acc.w += v[n * 4 + 3];
              wg[cells[n]] = acc;
            }
            __asm__ volatile("" ::: "memory");   // keep the corners' LDS accesses in program order
          }
          pend = pend && !mine;
        }
        wave_lds_sync();
        // flush and zero: the window's wh rows of row = 4 ww floats are taken 64 consecutive
        // floats per step (flat index p = y row + cc, so an atomic instruction covers one or
        // two pieces of texture rows, and no lane idles at a row's end); y = floor(p / row) is
        // the high word of p m with m = ceil(2^32 / row), exact since p (m row - 2^32) < 2^32
        // for p < 4 kWaveWin and row <= 4 kWaveWin.
        const int32_t row = ww * 4;
        const int32_t nf = wh * row;                                // floats in the window
        const uint32_t m = 0xffffffffu / (uint32_t)row + 1u;       // uniform (scalar)
        const int32_t bi = ri + dmin_i, bj = rj + dmin_j;   // texel of window cell (0, 0), unwrapped
        const bool flat = bi >= 0 && bi + ww <= Wt && bj >= 0 && bj + wh <= Ht;
        if (flat) {   // the window does not wrap: plain strided addresses
          const uint32_t gbase = ((uint32_t)bj * (uint32_t)Wt + (uint32_t)bi) * 4u;
          const uint32_t gstride = (uint32_t)Wt * 4u;
          for (int32_t p = lane; p < nf; p += 64) {
            const uint32_t y = __umulhi((uint32_t)p, m);
            const uint32_t cc = (uint32_t)p - y * (uint32_t)row;
            const float val = win[p];
            win[p] = 0.0f;
            if (val != 0.0f) grad_add(G, gbase + y * gstride + cc, val);
          }
        } else {
          // wrapped (repeat) or outside the texture (clamp: only zeros land there)
          for (int32_t p = lane; p < nf; p += 64) {
            const int32_t y = (int32_t)__umulhi((uint32_t)p, m);
            const int32_t cc = p - y * row;
            const float val = win[p];
            win[p] = 0.0f;
            if (val != 0.0f) {
              const int32_t tj = abs_index(rj, dmin_j + y, Ht, wrap);
              const int32_t ti = abs_index(ri, dmin_i + (cc >> 2), Wt, wrap);
              grad_add(G, ((uint32_t)tj * (uint32_t)Wt + (uint32_t)ti) * 4u + (uint32_t)(cc & 3), val);
            }
          }
        }
        wave_lds_sync();   // the window is reused by the next pass or layer
      } else if (npass == 1) {
        npass = 2;      // retry by halves
        pass = -1;
      } else if (npass == 2) {
        npass = 4;      // this half again as two quarters, and the halves after it as quarters
        pass = 2 * pass - 1;
      } else {
        direct = direct || live;
        ++n_path[3];
      }
    }
    // rare (minified texels, pole fans): kept out of the passes above so that its
    // address arithmetic is not hoisted into the common path
    if (__any(direct)) {
      if (direct) {
        const int32_t i1 = next_index(i0, Wt, wrap), j1 = next_index(j0, Ht, wrap);
        const uint32_t w = (uint32_t)Wt;
        const uint32_t q[4] = {((uint32_t)j0 * w + (uint32_t)i0) * 4u, ((uint32_t)j0 * w + (uint32_t)i1) * 4u,
                               ((uint32_t)j1 * w + (uint32_t)i0) * 4u, ((uint32_t)j1 * w + (uint32_t)i1) * 4u};
#pragma unroll
        for (int n = 0; n < 4; ++n) {
#pragma unroll
          for (int ch = 0; ch < 4; ++ch) grad_add(G, q[n] + (uint32_t)ch, v[n * 4 + ch]);
        }
      }
    }
  }
  if (count_paths && lane == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (n_path[q]) atomicAdd(status + VS_STAT_SCATTER_WAVE + q, (unsigned long long)n_path[q]);
  }
  if (sse) {
    // block reduction of the squared error, one atomic per block
    double sv = my_sse;
    for (int off = 32; off > 0; off >>= 1) sv += __shfl_xor(sv, off);
    if (lane == 0) sred[tid >> 6] = sv;
    __syncthreads();
    if (tid == 0) unsafeAtomicAdd(sse, (sred[0] + sred[1]) + (sred[2] + sred[3]));
  }
}

}  // namespace vs

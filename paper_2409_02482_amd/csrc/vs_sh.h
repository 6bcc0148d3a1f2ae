// Forward shading with the paper's baked appearance: 8-bit spherical-harmonic
// coefficient textures at mixed resolution, decoded with the view direction
// (Sec. 4.3 "Texturing Meshes", "Mixed Resolutions", "Squeezing and
// Quantization", "Baking Textures"), optional grazing-angle alpha weight
// (Sec. 4.2 "Transparency Attenuation"), blended like k_shade_fwd (Eq. 6).
#pragma once

#include "vs_shade.h"

namespace vs {

constexpr int kShLevels = 4;   // SH degrees 0..3, one texture level each

// Per layer: the packed coefficient bytes and, per level, its size, byte
// offset and reciprocal sizes (for the FP64 wrap of split_coord).
struct ShTable {
  const uint8_t* data[kMaxLayers];
  int32_t w[kMaxLayers][kShLevels], h[kMaxLayers][kShLevels];
  int64_t off[kMaxLayers][kShLevels];
  double inv_w[kMaxLayers][kShLevels], inv_h[kMaxLayers][kShLevels];
};

struct ShParams {
  float mid, scale;   // decoded value = mid + scale * (q - 127.5)
  float eps_T;
  int wrap, view_alpha;
};

// Real orthonormal spherical harmonics up to degree DEG of a unit direction,
// index l^2 + l + m; Y_1^{-1}, Y_1^0, Y_1^1 are proportional to y, z, x.
template <int DEG>
__device__ inline void sh_basis(float x, float y, float z, float (&Y)[16]) {
  Y[0] = 0.28209479177387814f;
  if (DEG >= 1) {
    Y[1] = 0.48860251190291992f * y;
    Y[2] = 0.48860251190291992f * z;
    Y[3] = 0.48860251190291992f * x;
  }
  if (DEG >= 2) {
    Y[4] = 1.0925484305920792f * x * y;
    Y[5] = 1.0925484305920792f * y * z;
    Y[6] = 0.31539156525252005f * (3.0f * z * z - 1.0f);
    Y[7] = 1.0925484305920792f * x * z;
    Y[8] = 0.54627421529603959f * (x * x - y * y);
  }
  if (DEG >= 3) {
    Y[9] = 0.59004358992664352f * y * (3.0f * x * x - y * y);
    Y[10] = 2.8906114426405538f * x * y * z;
    Y[11] = 0.45704579946446572f * y * (5.0f * z * z - 1.0f);
    Y[12] = 0.37317633259011540f * z * (5.0f * z * z - 3.0f);
    Y[13] = 0.45704579946446572f * x * (5.0f * z * z - 1.0f);
    Y[14] = 1.4453057213202769f * z * (x * x - y * y);
    Y[15] = 0.59004358992664352f * x * (x * x - 3.0f * y * y);
  }
}

__device__ inline float sigmoidf(float x) { return 1.0f / (1.0f + __expf(-x)); }

// Unit face normal of triangle t (world space), dotted with the unit ray d: |d.n|.
__device__ inline float abs_cos_face(const float* __restrict__ xyz, const int32_t* __restrict__ tri, uint32_t t,
                                     float dx, float dy, float dz) {
  const Tri3 id = elem_at<Tri3>(tri, t);
  const float ax = xyz[3 * id.a], ay = xyz[3 * id.a + 1], az = xyz[3 * id.a + 2];
  const float e1x = xyz[3 * id.b] - ax, e1y = xyz[3 * id.b + 1] - ay, e1z = xyz[3 * id.b + 2] - az;
  const float e2x = xyz[3 * id.c] - ax, e2y = xyz[3 * id.c + 1] - ay, e2z = xyz[3 * id.c + 2] - az;
  const float nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
  const float len2 = nx * nx + ny * ny + nz * nz;
  if (!(len2 > 0.0f)) return 0.0f;
  return fabsf(nx * dx + ny * dy + nz * dz) * rsqrtf(len2);
}

// One thread per pixel, same tiling and XCD order as k_shade_fwd.  Per hit
// layer: UV in FP64, then per degree l the footprint in that level (FP64
// coordinates, as for RGBA textures) and the 2l+1 coefficient words of the
// four corners; the decode and the bilinear weights are folded into the
// harmonic sum (all linear):
//   raw_c = mid * sum_i Y_i + scale * sum_l [ sum_corner w_corner sum_m Y_lm q_lm,c - 127.5 sum_m Y_lm ],
// q the raw bytes (FP32 sums of exact byte values).  The bytes of a texel's coefficients of one degree
// are adjacent, so a corner costs 2l+1 consecutive words.
// At degree 3 the register budget is held to 4 wavefronts per SIMD (a few
// bytes of spill cost less than the lost latency hiding).
template <int DEG>
__global__ void __launch_bounds__(256, DEG == 3 ? 4 : 1) k_shade_sh(const vs_view* __restrict__ views, int n_views,
                                                  const int32_t* __restrict__ tile_view, int64_t n_tiles,
                                                  LayerTable L, ShTable S, const ProjVert* __restrict__ proj,
                                                  int64_t vpv, const uint64_t* __restrict__ vis,
                                                  float4* __restrict__ out, ShParams prm,
                                                  unsigned long long* __restrict__ status) {
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
  // view ray through the pixel centre, world space: R^T ((x + 1/2 - cx) / fx, (y + 1/2 - cy) / fy, 1)
  float dx, dy, dz;
  {
    const double xc = ((double)c.x + 0.5 - V.cam.cx) / V.cam.fx, yc = ((double)c.y + 0.5 - V.cam.cy) / V.cam.fy;
    const double* R = V.cam.R;
    const double wx = R[0] * xc + R[3] * yc + R[6], wy = R[1] * xc + R[4] * yc + R[7];
    const double wz = R[2] * xc + R[5] * yc + R[8];
    const double inv = 1.0 / sqrt(wx * wx + wy * wy + wz * wz);
    dx = (float)(wx * inv); dy = (float)(wy * inv); dz = (float)(wz * inv);
  }
  float Y[16];
  sh_basis<DEG>(dx, dy, dz, Y);
  float sumY = 0.0f;
#pragma unroll
  for (int i = 0; i < (DEG + 1) * (DEG + 1); ++i) sumY += Y[i];
  float Cr = 0.f, Cg = 0.f, Cb = 0.f, T = c.valid ? 1.0f : 0.0f;
  for (int l = 0; l < k; ++l) {
    const uint64_t key = c.valid ? vrow[l * P] : kEmpty;
    double u, v;
    if (key != kEmpty && slot_uv(L.tri[l], L.n_tri[l], L.n_vert[l], pview + L.vert_off[l],
                                 reinterpret_cast<const float2*>(L.uv[l]), key, px, py, u, v, status)) {
      float acc[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int d = 0; d <= DEG; ++d) {
        const int32_t Wl = S.w[l][d], Hl = S.h[l][d];
        int32_t i0, i1, j0, j1;
        float fx, fy;
        split_coord(u * (double)Wl - 0.5, Wl, S.inv_w[l][d], prm.wrap, i0, i1, fx);
        split_coord(v * (double)Hl - 0.5, Hl, S.inv_h[l][d], prm.wrap, j0, j1, fy);
        const float gx = 1.0f - fx, gy = 1.0f - fy;
        const float w00 = gx * gy, w01 = fx * gy, w10 = gx * fy, w11 = fx * fy;
        const int n = 2 * d + 1;
        const uint32_t* base = reinterpret_cast<const uint32_t*>(S.data[l] + S.off[l][d]);
        const uint32_t* p00 = base + ((int64_t)j0 * Wl + i0) * n;
        const uint32_t* p01 = base + ((int64_t)j0 * Wl + i1) * n;
        const uint32_t* p10 = base + ((int64_t)j1 * Wl + i0) * n;
        const uint32_t* p11 = base + ((int64_t)j1 * Wl + i1) * n;
        // per corner, the harmonic sum of this degree's raw bytes; then the corners' weights
        float s00[4] = {0.f, 0.f, 0.f, 0.f}, s01[4] = {0.f, 0.f, 0.f, 0.f};
        float s10[4] = {0.f, 0.f, 0.f, 0.f}, s11[4] = {0.f, 0.f, 0.f, 0.f};
        float ysum = 0.f;
#pragma unroll
        for (int m = 0; m < n; ++m) {
          const uint32_t q00 = p00[m], q01 = p01[m], q10 = p10[m], q11 = p11[m];
          const float y = Y[d * d + m];
          ysum += y;
#pragma unroll
          for (int ch = 0; ch < 4; ++ch) {
            const int sh = 8 * ch;
            s00[ch] += y * (float)((q00 >> sh) & 0xffu);
            s01[ch] += y * (float)((q01 >> sh) & 0xffu);
            s10[ch] += y * (float)((q10 >> sh) & 0xffu);
            s11[ch] += y * (float)((q11 >> sh) & 0xffu);
          }
        }
        // the weights sum to 1, so the byte offset 127.5 comes off once per degree
#pragma unroll
        for (int ch = 0; ch < 4; ++ch)
          acc[ch] += (w00 * s00[ch] + w01 * s01[ch] + w10 * s10[ch] + w11 * s11[ch]) - 127.5f * ysum;
      }
      float a = sigmoidf(prm.mid * sumY + prm.scale * acc[3]);
      if (prm.view_alpha) {
        const float vn = abs_cos_face(L.xyz[l], L.tri[l], (uint32_t)(key & 0xffffffffu), dx, dy, dz);
        a *= 2.0f * sigmoidf(10.0f * vn) - 1.0f;
      }
      const float ta = T * a;
      Cr += ta * sigmoidf(prm.mid * sumY + prm.scale * acc[0]);
      Cg += ta * sigmoidf(prm.mid * sumY + prm.scale * acc[1]);
      Cb += ta * sigmoidf(prm.mid * sumY + prm.scale * acc[2]);
      T *= (1.0f - a);
    }
    if (prm.eps_T > 0.f && __all(T < prm.eps_T)) break;
  }
  if (c.valid) out[V.pix_offset + pix] = make_float4(Cr, Cg, Cb, 1.0f - T);
}

}  // namespace vs

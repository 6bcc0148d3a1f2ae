// k-SDF volume rendering (Sec. 4.1 "k-SDF", Sec. 4.2 "Surfaces Blending",
// Sec. 4.4 "Occupancy Grid" and "Importance Sampling").
//
// Fields live on vertex grids over the cube [lo, hi]^3 ([z][y][x] order) and
// are read trilinearly.  The occupancy grid is one thread per voxel, decided in
// FP64 and packed to bits with a wavefront ballot.  Rendering is one pixel ray
// per half wavefront (32 lanes): the ray's march steps are spread over the
// lanes (a lane owns a contiguous run of steps, so occupied-length ranks are a
// prefix sum of per-lane counts), and the ray's samples sit one per lane in up
// to four slots (sample i in lane i % 32, slot i / 32).  Transmittance is a multiplicative
// scan across lanes, the importance CDF an additive scan, inversion a binary
// search over the CDF in the wave's LDS, and the merge of new samples a rank
// computation (existing samples first on ties) followed by a scatter in LDS.
// Ray set-up, marching, sample positions and SDF values are FP64 (the
// occupancy decisions and march steps match a plain FP64 evaluation exactly);
// weights, appearance and blending are FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vs.h"

namespace vs {

constexpr int kKsdfWaves = 4;      // wavefronts per 256-thread block
constexpr int kKsdfRays = 2 * kKsdfWaves;   // rays per block (two per wavefront)
constexpr int kKsdfMaxN = VS_KSDF_MAX_SAMPLES;

struct KsdfParams {
  const float* sdf;
  const float4* rgba;
  int32_t sdf_res, rgba_res, occ_res;
  double lo, hi, h_occ;
  double inv_sdf, inv_rgba, inv_occ;       // R / (hi - lo) of each grid
  float cexp[2][VS_KSDF_MAX_SURFACES];     // exp(-beta_r o_j) for beta_r = beta / 2 (round 0) and beta
  int32_t factor;                          // 1: every |beta o_j| <= 60, so exp(-beta_r (d + o_j)) = E cexp
  int32_t k;
  double off[VS_KSDF_MAX_SURFACES];
  double beta, occ_threshold, half_diag;
  int32_t n, m, steps;
  float pdf_floor;
};

// Grid element at a 32-bit element index (grids are limited to 2^32 bytes, so
// the byte offset is a 32-bit unsigned value added to a scalar base address).
__device__ inline float ksdf_at(const float* __restrict__ g, uint32_t i) {
  return *(const float*)((const char*)g + (i << 2));
}
__device__ inline float4 ksdf_at4(const float4* __restrict__ g, uint32_t i) {
  return *(const float4*)((const char*)g + (i << 4));
}

// Cell of a point along one axis: base vertex and weight (FP64).
__device__ inline void ksdf_cell(double p, double lo, double inv, int R, uint32_t& b, double& f) {
  const double c = fmin(fmax((p - lo) * inv, 0.0), (double)R);
  const double bb = fmin(floor(c), (double)(R - 1));
  b = (uint32_t)bb;
  f = c - bb;
}

// Trilinear lookup of the SDF grid in FP64 (the accumulation order of a plain
// evaluation: corners z-major, then y, then x).
__device__ inline double ksdf_sdf(const KsdfParams& P, double px, double py, double pz) {
  const int R = P.sdf_res;
  uint32_t ix, iy, iz;
  double fx, fy, fz;
  ksdf_cell(px, P.lo, P.inv_sdf, R, ix, fx);
  ksdf_cell(py, P.lo, P.inv_sdf, R, iy, fy);
  ksdf_cell(pz, P.lo, P.inv_sdf, R, iz, fz);
  const uint32_t R1 = R + 1;
  double acc = 0.0;
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const double w = ((dx ? fx : 1.0 - fx) * (dy ? fy : 1.0 - fy)) * (dz ? fz : 1.0 - fz);
        const uint32_t idx = ((iz + dz) * R1 + (iy + dy)) * R1 + (ix + dx);
        acc += w * (double)ksdf_at(P.sdf, idx);
      }
  return acc;
}

// Gradient of the trilinear SDF inside the cell that holds p (the cell of
// ksdf_sdf): along each axis, the corner differences of the cell's 4 grid
// lines weighted by the other two axes' weights.
__device__ inline void ksdf_sdf_grad(const KsdfParams& P, double px, double py, double pz, double& gx, double& gy,
                                     double& gz) {
  const int R = P.sdf_res;
  uint32_t ix, iy, iz;
  double fx, fy, fz;
  ksdf_cell(px, P.lo, P.inv_sdf, R, ix, fx);
  ksdf_cell(py, P.lo, P.inv_sdf, R, iy, fy);
  ksdf_cell(pz, P.lo, P.inv_sdf, R, iz, fz);
  const uint32_t R1 = R + 1, base = (iz * R1 + iy) * R1 + ix;
  double g[2][2][2];
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) g[dz][dy][dx] = (double)ksdf_at(P.sdf, base + (dz * R1 + dy) * R1 + dx);
  const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
  double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      sx += (wy[a] * wz[b]) * (g[b][a][1] - g[b][a][0]);
      sy += (wx[a] * wz[b]) * (g[b][1][a] - g[b][0][a]);
      sz += (wx[a] * wy[b]) * (g[1][b][a] - g[0][b][a]);
    }
  gx = sx * P.inv_sdf;
  gy = sy * P.inv_sdf;
  gz = sz * P.inv_sdf;
}

// Trilinear lookup of the RGBA grid: FP64 cell coordinates, FP32 weights and sum.
__device__ inline float4 ksdf_rgba(const KsdfParams& P, double px, double py, double pz) {
  const int R = P.rgba_res;
  uint32_t ix, iy, iz;
  double dfx, dfy, dfz;
  ksdf_cell(px, P.lo, P.inv_rgba, R, ix, dfx);
  ksdf_cell(py, P.lo, P.inv_rgba, R, iy, dfy);
  ksdf_cell(pz, P.lo, P.inv_rgba, R, iz, dfz);
  const float fx = (float)dfx, fy = (float)dfy, fz = (float)dfz;
  const uint32_t R1 = R + 1;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const float w = ((dx ? fx : 1.f - fx) * (dy ? fy : 1.f - fy)) * (dz ? fz : 1.f - fz);
        const float4 g = ksdf_at4(P.rgba, ((iz + dz) * R1 + (iy + dy)) * R1 + (ix + dx));
        acc.x += w * g.x;
        acc.y += w * g.y;
        acc.z += w * g.z;
        acc.w += w * g.w;
      }
  return acc;
}

// ---------------------------------------------------------------------------
// occupancy grid
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_ksdf_occupancy(KsdfParams P, uint32_t* __restrict__ occ, int64_t n_vox,
                                                        int64_t n_words) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool bit = false;
  if (i < n_vox) {
    const int64_t R = P.occ_res;
    const int64_t x = i % R, y = (i / R) % R, z = i / (R * R);
    const double cx = P.lo + ((double)x + 0.5) * P.h_occ;
    const double cy = P.lo + ((double)y + 0.5) * P.h_occ;
    const double cz = P.lo + ((double)z + 0.5) * P.h_occ;
    const double dc = ksdf_sdf(P, cx, cy, cz);
    for (int j = 0; j < P.k; ++j) {
      const double delta = fmax(fabs(dc + P.off[j]) - P.half_diag, 0.0);
      const double e = exp(-P.beta * fabs(delta));
      const double phi = P.beta * e / ((1.0 + e) * (1.0 + e));
      bit = bit || phi > P.occ_threshold;
    }
  }
  const uint64_t b = __ballot(bit);
  const int lane = threadIdx.x & 63;
  const int64_t word = i >> 5;
  if ((lane & 31) == 0 && word < n_words) occ[word] = (uint32_t)(lane ? b >> 32 : b);
}

// ---------------------------------------------------------------------------
// half-wavefront helpers: a wavefront renders two rays, one per 32-lane half
// (DPP row shifts within 16-lane rows, a row broadcast from row 0 to row 1 and
// from row 2 to row 3, whole-wave shifts by one lane with the half edges
// patched)
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK = 0xf>
__device__ inline float ksdf_dpp(float old, float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), CTRL, ROW_MASK, 0xf, false));
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ inline int ksdf_dpp_i(int old, int x) {
  return __builtin_amdgcn_update_dpp(old, x, CTRL, ROW_MASK, 0xf, false);
}

// Inclusive prefix sum / product within each half.
__device__ inline int ksdf_hscan_add_i(int x) {
  x += ksdf_dpp_i<0x111>(0, x);
  x += ksdf_dpp_i<0x112>(0, x);
  x += ksdf_dpp_i<0x114>(0, x);
  x += ksdf_dpp_i<0x118>(0, x);
  x += ksdf_dpp_i<0x142, 0xa>(0, x);
  return x;
}
__device__ inline float ksdf_hscan_add(float x) {
  x += ksdf_dpp<0x111>(0.f, x);
  x += ksdf_dpp<0x112>(0.f, x);
  x += ksdf_dpp<0x114>(0.f, x);
  x += ksdf_dpp<0x118>(0.f, x);
  x += ksdf_dpp<0x142, 0xa>(0.f, x);
  return x;
}
__device__ inline float ksdf_hscan_mul(float x) {
  x *= ksdf_dpp<0x111>(1.f, x);
  x *= ksdf_dpp<0x112>(1.f, x);
  x *= ksdf_dpp<0x114>(1.f, x);
  x *= ksdf_dpp<0x118>(1.f, x);
  x *= ksdf_dpp<0x142, 0xa>(1.f, x);
  return x;
}

// Value of lane l of this lane's half.
__device__ inline float ksdf_hlane(float x, int l, int h) {
  const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
  const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32 + l));
  return h ? b : a;
}
__device__ inline int ksdf_hlane_i(int x, int l, int h) {
  const int a = __builtin_amdgcn_readlane(x, l), b = __builtin_amdgcn_readlane(x, 32 + l);
  return h ? b : a;
}

// Sum over this lane's half.
__device__ inline float ksdf_hsum(float x, int h) { return ksdf_hlane(ksdf_hscan_add(x), 31, h); }

// Value of lane - 1 of the half (old at the half's first lane) and of lane + 1 (nxt at its last lane).
__device__ inline float ksdf_hbelow(float old, float x, int l) {
  const float y = ksdf_dpp<0x138>(old, x);
  return l == 0 ? old : y;
}
__device__ inline float ksdf_habove(float nxt, float x, int l) {
  const float y = ksdf_dpp<0x130>(nxt, x);
  return l == 31 ? nxt : y;
}

__device__ inline void ksdf_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS of one ray (half a wavefront).
struct KsdfLds {
  double t[kKsdfMaxN];      // sorted sample parameters
  double d[kKsdfMaxN];      // their SDF values
  float cdf[kKsdfMaxN];     // importance CDF c_0..c_{N-1}
  double tn[64];            // samples of the current importance round
  double dn[64];
  uint64_t mask[32];        // march: occupied-step bits per lane
  int32_t pre[32];          // march: exclusive prefix of occupied steps per lane
};

// NeuS opacity of the interval between two samples from E = exp(-beta d_j) at
// both ends: 1 - Phi_{i+1}/Phi_i = (E_{i+1} - E_i) / (1 + E_{i+1}), 0 where
// Phi_i = 0 (E_i infinite), 1 where only Phi_{i+1} = 0.
__device__ inline float ksdf_alpha(float e, float en, bool valid) {
  if (!valid || isinf(e)) return 0.f;
  if (isinf(en)) return 1.f;
  return fmaxf((en - e) * __builtin_amdgcn_rcpf(1.f + en), 0.f);
}

// exp(-beta_r (d + o_j)) per slot: E cexp_j from E = exp(-beta_r d) shared by
// all surfaces, or one exponential per surface when the offsets are too large
// for the factor to stay a normal float.
__device__ inline float ksdf_surface_exp(const KsdfParams& P, int round, int j, double beta_r, double d, float E) {
  return P.factor ? E * P.cexp[round][j] : expf(-(float)(beta_r * (d + P.off[j])));
}

// NeuS interval weights of one surface over the NS slots of this half's ray,
// w_i = a_i prod_{l<i} (1 - a_l) (a multiplicative scan per slot, carried
// from slot to slot).
template <int NSL>
__device__ inline void ksdf_weights(const float (&e)[NSL], float (&w)[NSL], int NS, int N, int l, int h) {
  float carry = 1.f;
#pragma unroll
  for (int sl = 0; sl < NSL; ++sl) {
    if (sl < NS) {
      const float nxt = sl + 1 < NSL && sl + 1 < NS ? ksdf_hlane(e[sl + 1 < NSL ? sl + 1 : sl], 0, h) : e[sl];
      const float en = ksdf_habove(nxt, e[sl], l);
      const float a = ksdf_alpha(e[sl], en, 32 * sl + l < N - 1);
      const float c = ksdf_hscan_mul(1.f - a) * carry;
      w[sl] = ksdf_hbelow(carry, c, l) * a;
      carry = ksdf_hlane(c, 31, h);
    } else {
      w[sl] = 0.f;
    }
  }
}

// Block b -> a contiguous run of rays per XCD (blocks are dealt round-robin to the 8 XCDs).
__device__ inline int64_t ksdf_block() {
  const int64_t chunk = (int64_t)gridDim.x / 8;
  return ((int64_t)blockIdx.x % 8) * chunk + (int64_t)blockIdx.x / 8;
}

// Two rays per wavefront, 32 lanes each: the 96 samples of the paper's
// 64 + 32 fill three slots of 32 exactly (NSL = slots per lane, from the
// sample count).  Blocks of 256 threads (8 rays), four per CU: the register
// budget of four blocks holds the per-ray state without spilling to scratch
// (five blocks per CU render as fast but spill, which writes gigabytes of
// scratch traffic per launch).
template <int NSL>
__global__ void __launch_bounds__(256, 4) k_ksdf_render(const vs_view* __restrict__ views, int n_views, int64_t total,
                                                     KsdfParams P, const uint32_t* __restrict__ occ,
                                                     float4* __restrict__ out, float4* __restrict__ layers,
                                                     double* __restrict__ samples) {
  __shared__ KsdfLds lds_all[kKsdfRays];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, h = lane >> 5, l = lane & 31;
  KsdfLds& L = lds_all[2 * wv + h];
  const int64_t ray = (ksdf_block() * kKsdfWaves + wv) * 2 + h;
  const bool real = ray < total;
  if (__builtin_amdgcn_readlane((int)real, 0) == 0) return;      // both halves past the end (ray grows with h)
  const int N = P.n + P.m, m2 = P.m / 2;

  // this half's camera ray
  const int64_t rr = real ? ray : total - 1;
  int lo_v = 0, hi_v = n_views - 1;
  while (lo_v < hi_v) {
    const int mid = (lo_v + hi_v + 1) / 2;
    if (views[mid].pix_offset <= rr) lo_v = mid; else hi_v = mid - 1;
  }
  const vs_camera& C = views[lo_v].cam;
  const int64_t pix = rr - views[lo_v].pix_offset;
  const int64_t pi = pix % C.width, pj = pix / C.width;
  double o[3], v[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) o[q] = -((C.R[q] * C.t[0] + C.R[3 + q] * C.t[1]) + C.R[6 + q] * C.t[2]);
  const double xc = (((double)pi + 0.5) - C.cx) / C.fx, yc = (((double)pj + 0.5) - C.cy) / C.fy;
#pragma unroll
  for (int q = 0; q < 3; ++q) v[q] = (C.R[q] * xc + C.R[3 + q] * yc) + C.R[6 + q];
  const double vn = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
#pragma unroll
  for (int q = 0; q < 3; ++q) v[q] = v[q] / vn;

  // slab interval in the cube, t >= 0
  double t_in = 0.0, t_out = INFINITY;
  bool hit = real;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (v[a] != 0.0) {
      const double t1 = (P.lo - o[a]) / v[a], t2 = (P.hi - o[a]) / v[a];
      t_in = fmax(t_in, fmin(t1, t2));
      t_out = fmin(t_out, fmax(t1, t2));
    } else {
      hit = hit && o[a] >= P.lo && o[a] <= P.hi;
    }
  }
  hit = hit && t_out > t_in;

  // march: lane l of the half owns steps [l sp, (l + 1) sp)
  const int sp = P.steps / 32;
  const double D = hit ? (t_out - t_in) / (double)P.steps : 0.0;
  uint64_t mask = 0;
  if (hit) {
    const int Ro = P.occ_res;
    double A[3], B[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      A[a] = (o[a] - P.lo) * P.inv_occ;
      B[a] = v[a] * P.inv_occ;
    }
#pragma unroll 4
    for (int q = 0; q < sp; ++q) {
      const int s = l * sp + q;
      const double tm = t_in + ((double)s + 0.5) * D;
      uint32_t vox[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        // floor, then clamp to [0, Ro - 1] (the coordinate stays within a rounding of [0, Ro])
        vox[a] = (uint32_t)min(max((int)floor(A[a] + tm * B[a]), 0), Ro - 1);
      }
      const uint32_t idx = (vox[2] * (uint32_t)Ro + vox[1]) * (uint32_t)Ro + vox[0];
      const uint32_t word = *(const uint32_t*)((const char*)occ + ((idx >> 5) << 2));
      mask |= (uint64_t)((word >> (idx & 31)) & 1u) << q;
    }
  }
  const int cnt = __popcll(mask);
  const int incl = ksdf_hscan_add_i(cnt);
  const int M = ksdf_hlane_i(incl, 31, h);
  const bool live = M > 0;
  if (__builtin_amdgcn_readlane((int)live, 0) == 0 && __builtin_amdgcn_readlane((int)live, 32) == 0) {
    if (real && l == 0) out[ray] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (real && layers)
      for (int j = l; j < P.k; j += 32) layers[(int64_t)j * total + ray] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (real && samples)
      for (int i = l; i < N; i += 32) samples[ray * N + i] = -1.0;
    return;
  }
  L.pre[l] = incl - cnt;
  L.mask[l] = mask;
  ksdf_wave_sync();

  // uniform samples in occupied length (a ray without any: parameter 0 and a far-outside SDF, no weight)
  double ts[NSL], ds[NSL];
#pragma unroll
  for (int sl = 0; sl < NSL; ++sl) {
    ts[sl] = 0.0;
    ds[sl] = 1e30;
    const int i = 32 * sl + l;
    if (i < P.n) {
      if (live) {
        const double rho = (((double)i + 0.5) * (double)M) / (double)P.n;
        const double qf = floor(rho);
        const int qi = (int)qf;
        int a = 0, b = 31;                  // largest lane with pre <= qi
        while (a < b) {
          const int mid = (a + b + 1) / 2;
          if (L.pre[mid] <= qi) a = mid; else b = mid - 1;
        }
        uint64_t mk = L.mask[a];
        for (int r = qi - L.pre[a]; r > 0; --r) mk &= mk - 1;
        const int s = a * sp + (int)__builtin_ctzll(mk);
        ts[sl] = t_in + ((double)s + (rho - qf)) * D;
        ds[sl] = ksdf_sdf(P, o[0] + ts[sl] * v[0], o[1] + ts[sl] * v[1], o[2] + ts[sl] * v[2]);
      }
      L.t[i] = ts[sl];
      L.d[i] = ds[sl];
    }
  }
  ksdf_wave_sync();

  // two importance rounds
  int Ncur = P.n;
  for (int round = 0; round < 2 && m2 > 0; ++round) {
    const double beta_r = round == 0 ? P.beta / 2.0 : P.beta;
    const int NS = (Ncur + 31) / 32;
    float E[NSL], W[NSL];
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) {
      E[sl] = sl < NS ? expf(-(float)(beta_r * ds[sl])) : 0.f;
      W[sl] = 0.f;
    }
    for (int j = 0; j < P.k; ++j) {
      float e[NSL], w[NSL];
#pragma unroll
      for (int sl = 0; sl < NSL; ++sl) e[sl] = ksdf_surface_exp(P, round, j, beta_r, ds[sl], E[sl]);
      ksdf_weights(e, w, NS, Ncur, l, h);
#pragma unroll
      for (int sl = 0; sl < NSL; ++sl) W[sl] += w[sl];
    }
    float q[NSL], qs = 0.f;
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) {
      q[sl] = 32 * sl + l < Ncur - 1 ? W[sl] + P.pdf_floor : 0.f;
      qs += q[sl];
    }
    const float rS = 1.f / ksdf_hsum(qs, h);
    float carry = 0.f;
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) {
      if (sl < NS) {
        const float c = ksdf_hscan_add(q[sl] * rS) + carry;
        if (32 * sl + l < Ncur - 1) L.cdf[32 * sl + l + 1] = c;
        carry = ksdf_hlane(c, 31, h);
      }
    }
    if (l == 0) L.cdf[0] = 0.f;
    ksdf_wave_sync();
    double tn[2] = {0.0, 0.0}, dn[2] = {0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int qn = 32 * r + l;
      if (qn < m2) {
        const double u = ((double)qn + 0.5) / (double)m2;
        int a = 0, b = Ncur - 1;              // largest i with cdf[i] <= u
        while (a < b) {
          const int mid = (a + b + 1) / 2;
          if ((double)L.cdf[mid] <= u) a = mid; else b = mid - 1;
        }
        a = min(a, Ncur - 2);
        const double ca = (double)L.cdf[a], cb = (double)L.cdf[a + 1];
        const double fr = cb > ca ? (u - ca) / (cb - ca) : 0.0;
        tn[r] = L.t[a] + fr * (L.t[a + 1] - L.t[a]);
        dn[r] = live ? ksdf_sdf(P, o[0] + tn[r] * v[0], o[1] + tn[r] * v[1], o[2] + tn[r] * v[2]) : 1e30;
        L.tn[qn] = tn[r];
        L.dn[qn] = dn[r];
      }
    }
    ksdf_wave_sync();
    // ranks in the merged order (existing samples first on ties)
    int rk[NSL], rn[2] = {-1, -1};
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) {
      rk[sl] = -1;
      const int i = 32 * sl + l;
      if (sl < NS && i < Ncur) {
        int c = 0;
        for (int qn = 0; qn < m2; ++qn) c += L.tn[qn] < ts[sl];
        rk[sl] = i + c;
      }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int qn = 32 * r + l;
      if (qn < m2) {
        int a = 0, b = Ncur;                  // number of existing samples <= tn
        while (a < b) {
          const int mid = (a + b) / 2;
          if (L.t[mid] <= tn[r]) a = mid + 1; else b = mid;
        }
        rn[r] = qn + a;
      }
    }
    ksdf_wave_sync();
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl)
      if (rk[sl] >= 0) {
        L.t[rk[sl]] = ts[sl];
        L.d[rk[sl]] = ds[sl];
      }
#pragma unroll
    for (int r = 0; r < 2; ++r)
      if (rn[r] >= 0) {
        L.t[rn[r]] = tn[r];
        L.d[rn[r]] = dn[r];
      }
    ksdf_wave_sync();
    Ncur += m2;
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) {
      const int i = 32 * sl + l;
      if (i < Ncur) {
        ts[sl] = L.t[i];
        ds[sl] = L.d[i];
      }
    }
  }

  // appearance and view-dependent attenuation at each interval start
  const int NS = (N + 31) / 32;
  float4 app[NSL];
  float aw[NSL];
#pragma unroll
  for (int sl = 0; sl < NSL; ++sl) {
    app[sl] = make_float4(0.f, 0.f, 0.f, 0.f);
    aw[sl] = 0.f;
    if (32 * sl + l < N - 1) {
      const double px = o[0] + ts[sl] * v[0], py = o[1] + ts[sl] * v[1], pz = o[2] + ts[sl] * v[2];
      app[sl] = ksdf_rgba(P, px, py, pz);
      double gx, gy, gz;
      ksdf_sdf_grad(P, px, py, pz, gx, gy, gz);
      const double gn = sqrt((gx * gx + gy * gy) + gz * gz);
      const double vdn = gn > 0.0 ? fabs(((gx / gn) * v[0] + (gy / gn) * v[1]) + (gz / gn) * v[2]) : 0.0;
      aw[sl] = 2.f / (1.f + expf(-10.f * (float)vdn)) - 1.f;
    }
  }

  // per-surface quadrature and fixed-order blend
  float R = 0.f, G = 0.f, B = 0.f, T = 1.f;
  float E[NSL];
#pragma unroll
  for (int sl = 0; sl < NSL; ++sl) E[sl] = sl < NS ? expf(-(float)(P.beta * ds[sl])) : 0.f;
  for (int j = 0; j < P.k; ++j) {
    float e[NSL], w[NSL];
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) e[sl] = ksdf_surface_exp(P, 1, j, P.beta, ds[sl], E[sl]);
    ksdf_weights(e, w, NS, N, l, h);
    float pr = 0.f, pg = 0.f, pb = 0.f, pa = 0.f;
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) {
      pr += w[sl] * app[sl].x;
      pg += w[sl] * app[sl].y;
      pb += w[sl] * app[sl].z;
      pa += w[sl] * aw[sl] * app[sl].w;
    }
    const float cr = ksdf_hsum(pr, h), cg = ksdf_hsum(pg, h), cb = ksdf_hsum(pb, h), ca = ksdf_hsum(pa, h);
    R += (T * ca) * cr;
    G += (T * ca) * cg;
    B += (T * ca) * cb;
    T *= 1.f - ca;
    if (real && layers && l == 0)
      layers[(int64_t)j * total + ray] = live ? make_float4(cr, cg, cb, ca) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
  if (real && l == 0) out[ray] = live ? make_float4(R, G, B, 1.f - T) : make_float4(0.f, 0.f, 0.f, 0.f);
  if (real && samples) {
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) {
      const int i = 32 * sl + l;
      if (i < N) samples[ray * N + i] = live ? ts[sl] : -1.0;
    }
  }
}

}  // namespace vs

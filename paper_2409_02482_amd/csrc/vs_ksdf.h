// k-SDF volume rendering (Sec. 4.1 "k-SDF", Sec. 4.2 "Surfaces Blending",
// Sec. 4.4 "Occupancy Grid" and "Importance Sampling").
//
// Fields live on vertex grids over the cube [lo, hi]^3 ([z][y][x] order) and
// are read trilinearly.  The occupancy grid is one thread per voxel, decided in
// FP64 and packed to bits with a wavefront ballot.  Rendering is one wavefront
// per pixel ray: the ray's march steps are spread over the 64 lanes (a lane
// owns a contiguous run of steps, so occupied-length ranks are a prefix sum of
// per-lane counts), and the ray's samples sit one per lane in up to two slots
// (sample i in lane i % 64, slot i / 64).  Transmittance is a multiplicative
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

constexpr int kKsdfWaves = 4;      // rays in flight per 256-thread block
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
// wavefront helpers (64 lanes, DPP: row shifts within 16-lane rows, row
// broadcasts across rows, whole-wave shifts by one lane)
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK = 0xf>
__device__ inline float ksdf_dpp(float old, float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), CTRL, ROW_MASK, 0xf, false));
}
template <int CTRL, int ROW_MASK = 0xf>
__device__ inline int ksdf_dpp_i(int old, int x) {
  return __builtin_amdgcn_update_dpp(old, x, CTRL, ROW_MASK, 0xf, false);
}

// Inclusive prefix sum over the wave.
__device__ inline int ksdf_scan_add_i(int x) {
  x += ksdf_dpp_i<0x111>(0, x);
  x += ksdf_dpp_i<0x112>(0, x);
  x += ksdf_dpp_i<0x114>(0, x);
  x += ksdf_dpp_i<0x118>(0, x);
  x += ksdf_dpp_i<0x142, 0xa>(0, x);
  x += ksdf_dpp_i<0x143, 0xc>(0, x);
  return x;
}

__device__ inline float ksdf_scan_add(float x) {
  x += ksdf_dpp<0x111>(0.f, x);
  x += ksdf_dpp<0x112>(0.f, x);
  x += ksdf_dpp<0x114>(0.f, x);
  x += ksdf_dpp<0x118>(0.f, x);
  x += ksdf_dpp<0x142, 0xa>(0.f, x);
  x += ksdf_dpp<0x143, 0xc>(0.f, x);
  return x;
}

// Inclusive prefix product over the wave.
__device__ inline float ksdf_scan_mul(float x) {
  x *= ksdf_dpp<0x111>(1.f, x);
  x *= ksdf_dpp<0x112>(1.f, x);
  x *= ksdf_dpp<0x114>(1.f, x);
  x *= ksdf_dpp<0x118>(1.f, x);
  x *= ksdf_dpp<0x142, 0xa>(1.f, x);
  x *= ksdf_dpp<0x143, 0xc>(1.f, x);
  return x;
}

__device__ inline float ksdf_lane(float x, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l)); }

// Sum over the wave (the same value in every lane).
__device__ inline float ksdf_sum(float x) { return ksdf_lane(ksdf_scan_add(x), 63); }

// Value of lane - 1 (lane 0: old) and of lane + 1 (lane 63: old).
__device__ inline float ksdf_from_below(float old, float x) { return ksdf_dpp<0x138>(old, x); }
__device__ inline float ksdf_from_above(float old, float x) { return ksdf_dpp<0x130>(old, x); }

__device__ inline void ksdf_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct KsdfLds {
  double t[kKsdfMaxN];      // sorted sample parameters
  double d[kKsdfMaxN];      // their SDF values
  float cdf[kKsdfMaxN];     // importance CDF c_0..c_{N-1}
  double tn[64];            // samples of the current importance round
  double dn[64];
  int32_t pre[64];          // march: exclusive prefix of occupied steps per lane
  uint32_t mask[64];        // march: occupied-step bits per lane
};

// NeuS opacity of the interval between two samples from E = exp(-beta d_j) at
// both ends: 1 - Phi_{i+1}/Phi_i = (E_{i+1} - E_i) / (1 + E_{i+1}), 0 where
// Phi_i = 0 (E_i infinite), 1 where only Phi_{i+1} = 0.
__device__ inline float ksdf_alpha(float e, float en, bool valid) {
  if (!valid || isinf(e)) return 0.f;
  if (isinf(en)) return 1.f;
  return fmaxf((en - e) * __builtin_amdgcn_rcpf(1.f + en), 0.f);
}

// exp(-beta_r (d + o_j)) at the two slots: E cexp_j from E = exp(-beta_r d)
// shared by all surfaces, or one exponential per surface when the offsets are
// too large for the factor to stay a normal float.
__device__ inline void ksdf_surface_exp(const KsdfParams& P, int round, int j, double beta_r, double d0, double d1,
                                        float E0, float E1, float& e0, float& e1) {
  if (P.factor) {
    e0 = E0 * P.cexp[round][j];
    e1 = E1 * P.cexp[round][j];
  } else {
    e0 = expf(-(float)(beta_r * (d0 + P.off[j])));
    e1 = expf(-(float)(beta_r * (d1 + P.off[j])));
  }
}

// NeuS interval weights of one surface when all N <= 64 samples sit in slot 0.
__device__ inline float ksdf_weights1(float e0, int N, int lane) {
  const float n0 = ksdf_from_above(e0, e0);
  const float a0 = ksdf_alpha(e0, n0, lane < N - 1);
  return ksdf_from_below(1.f, ksdf_scan_mul(1.f - a0)) * a0;
}

// NeuS interval weights of one surface over the samples held in two slots,
// w_i = a_i prod_{l<i} (1 - a_l), from e = exp(-beta_r d_j) at each sample.
__device__ inline void ksdf_weights(float e0, float e1, int N, int lane, float& w0, float& w1) {
  // the next sample: lane + 1 of the same slot; lane 63 of slot 0 continues with lane 0 of slot 1
  const float n0 = ksdf_from_above(ksdf_lane(e1, 0), e0), n1 = ksdf_from_above(e1, e1);
  const float a0 = ksdf_alpha(e0, n0, lane < N - 1), a1 = ksdf_alpha(e1, n1, lane + 64 < N - 1);
  const float c0 = ksdf_scan_mul(1.f - a0);
  const float tot0 = ksdf_lane(c0, 63);
  const float c1 = ksdf_scan_mul(1.f - a1) * tot0;
  w0 = ksdf_from_below(1.f, c0) * a0;
  w1 = ksdf_from_below(tot0, c1) * a1;
}

// Block b -> a contiguous run of rays per XCD (blocks are dealt round-robin to the 8 XCDs).
__device__ inline int64_t ksdf_block() {
  const int64_t chunk = (int64_t)gridDim.x / 8;
  return ((int64_t)blockIdx.x % 8) * chunk + (int64_t)blockIdx.x / 8;
}

// Five 256-thread blocks per CU (20 waves): the register budget this sets
// (96 VGPRs) costs a few spills but hides more gather latency than four.
__global__ void __launch_bounds__(256, 5) k_ksdf_render(const vs_view* __restrict__ views, int n_views, int64_t total,
                                                     KsdfParams P, const uint32_t* __restrict__ occ,
                                                     float4* __restrict__ out, float4* __restrict__ layers,
                                                     double* __restrict__ samples) {
  __shared__ KsdfLds lds_all[kKsdfWaves];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  KsdfLds& L = lds_all[wv];
  const int64_t ray = ksdf_block() * kKsdfWaves + wv;
  if (ray >= total) return;
  const int N = P.n + P.m, m2 = P.m / 2;

  int lo_v = 0, hi_v = n_views - 1;      // the view holding this ray
  while (lo_v < hi_v) {
    const int mid = (lo_v + hi_v + 1) / 2;
    if (views[mid].pix_offset <= ray) lo_v = mid; else hi_v = mid - 1;
  }
  const vs_camera& C = views[lo_v].cam;
  const int64_t pix = ray - views[lo_v].pix_offset;
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
  bool hit = true;
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

  // march: lane owns steps [lane sp, (lane + 1) sp)
  int M = 0;
  uint32_t mask = 0;
  int pre = 0;
  double D = 0.0;
  const int sp = P.steps / 64;
  if (hit) {
    D = (t_out - t_in) / (double)P.steps;
    const int Ro = P.occ_res;
    double A[3], B[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      A[a] = (o[a] - P.lo) * P.inv_occ;
      B[a] = v[a] * P.inv_occ;
    }
#pragma unroll 4
    for (int q = 0; q < sp; ++q) {
      const int s = lane * sp + q;
      const double tm = t_in + ((double)s + 0.5) * D;
      uint32_t vox[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        // floor, then clamp to [0, Ro - 1] (the coordinate stays within a rounding of [0, Ro])
        vox[a] = (uint32_t)min(max((int)floor(A[a] + tm * B[a]), 0), Ro - 1);
      }
      const uint32_t idx = (vox[2] * (uint32_t)Ro + vox[1]) * (uint32_t)Ro + vox[0];
      mask |= ((*(const uint32_t*)((const char*)occ + ((idx >> 5) << 2)) >> (idx & 31)) & 1u) << q;
    }
    const int c = __popc(mask);
    const int incl = ksdf_scan_add_i(c);
    pre = incl - c;
    M = __builtin_amdgcn_readlane(incl, 63);
  }
  if (M == 0) {
    if (lane == 0) out[ray] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (layers)
      for (int j = lane; j < P.k; j += 64) layers[(int64_t)j * total + ray] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (samples)
      for (int i = lane; i < N; i += 64) samples[ray * N + i] = -1.0;
    return;
  }
  L.pre[lane] = pre;
  L.mask[lane] = mask;
  ksdf_wave_sync();

  // uniform samples in occupied length
  double ts[2] = {0.0, 0.0}, ds[2] = {0.0, 0.0};
#pragma unroll
  for (int sl = 0; sl < 2; ++sl) {
    const int i = lane + 64 * sl;
    if (i < P.n) {
      const double rho = (((double)i + 0.5) * (double)M) / (double)P.n;
      const double qf = floor(rho);
      const int qi = (int)qf;
      int a = 0, b = 63;                  // largest lane with pre <= qi
      while (a < b) {
        const int mid = (a + b + 1) / 2;
        if (L.pre[mid] <= qi) a = mid; else b = mid - 1;
      }
      uint32_t mk = L.mask[a];
      for (int r = qi - L.pre[a]; r > 0; --r) mk &= mk - 1;
      const int s = a * sp + __builtin_ctz(mk);
      const double t = t_in + ((double)s + (rho - qf)) * D;
      ts[sl] = t;
      ds[sl] = ksdf_sdf(P, o[0] + t * v[0], o[1] + t * v[1], o[2] + t * v[2]);
      L.t[i] = t;
      L.d[i] = ds[sl];
    }
  }
  ksdf_wave_sync();

  // two importance rounds
  int Ncur = P.n;
  for (int round = 0; round < 2 && m2 > 0; ++round) {
    const double beta_r = round == 0 ? P.beta / 2.0 : P.beta;
    const float E0 = expf(-(float)(beta_r * ds[0])), E1 = expf(-(float)(beta_r * ds[1]));
    float W0 = 0.f, W1 = 0.f;
    if (Ncur > 64) {
      for (int j = 0; j < P.k; ++j) {
        float e0, e1, w0, w1;
        ksdf_surface_exp(P, round, j, beta_r, ds[0], ds[1], E0, E1, e0, e1);
        ksdf_weights(e0, e1, Ncur, lane, w0, w1);
        W0 += w0;
        W1 += w1;
      }
    } else {
      for (int j = 0; j < P.k; ++j) {
        float e0, e1;
        ksdf_surface_exp(P, round, j, beta_r, ds[0], ds[1], E0, E1, e0, e1);
        W0 += ksdf_weights1(e0, Ncur, lane);
      }
    }
    const bool v0 = lane < Ncur - 1, v1 = lane + 64 < Ncur - 1;
    const float q0 = v0 ? W0 + P.pdf_floor : 0.f, q1 = v1 ? W1 + P.pdf_floor : 0.f;
    const float S = ksdf_sum(q0 + q1);
    const float rS = 1.f / S;
    const float c0 = ksdf_scan_add(q0 * rS);
    const float c1 = ksdf_scan_add(q1 * rS) + ksdf_lane(c0, 63);
    if (lane == 0) L.cdf[0] = 0.f;
    if (v0) L.cdf[lane + 1] = c0;
    if (v1) L.cdf[lane + 65] = c1;
    ksdf_wave_sync();
    double tn = 0.0, dn = 0.0;
    if (lane < m2) {
      const double u = ((double)lane + 0.5) / (double)m2;
      int a = 0, b = Ncur - 1;              // largest i with cdf[i] <= u
      while (a < b) {
        const int mid = (a + b + 1) / 2;
        if ((double)L.cdf[mid] <= u) a = mid; else b = mid - 1;
      }
      a = min(a, Ncur - 2);
      const double ca = (double)L.cdf[a], cb = (double)L.cdf[a + 1];
      const double fr = cb > ca ? (u - ca) / (cb - ca) : 0.0;
      tn = L.t[a] + fr * (L.t[a + 1] - L.t[a]);
      dn = ksdf_sdf(P, o[0] + tn * v[0], o[1] + tn * v[1], o[2] + tn * v[2]);
      L.tn[lane] = tn;
      L.dn[lane] = dn;
    }
    ksdf_wave_sync();
    // ranks in the merged order (existing samples first on ties)
    int r0 = -1, r1 = -1, rn = -1;
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int i = lane + 64 * sl;
      if (i < Ncur) {
        int cnt = 0;
        for (int q = 0; q < m2; ++q) cnt += L.tn[q] < ts[sl];
        (sl ? r1 : r0) = i + cnt;
      }
    }
    if (lane < m2) {
      int a = 0, b = Ncur;                  // number of existing samples <= tn
      while (a < b) {
        const int mid = (a + b) / 2;
        if (L.t[mid] <= tn) a = mid + 1; else b = mid;
      }
      rn = lane + a;
    }
    ksdf_wave_sync();
    if (r0 >= 0) { L.t[r0] = ts[0]; L.d[r0] = ds[0]; }
    if (r1 >= 0) { L.t[r1] = ts[1]; L.d[r1] = ds[1]; }
    if (rn >= 0) { L.t[rn] = tn; L.d[rn] = dn; }
    ksdf_wave_sync();
    Ncur += m2;
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int i = lane + 64 * sl;
      if (i < Ncur) {
        ts[sl] = L.t[i];
        ds[sl] = L.d[i];
      }
    }
  }

  // appearance and view-dependent attenuation at each interval start
  float4 app[2];
  float aw[2];
#pragma unroll
  for (int sl = 0; sl < 2; ++sl) {
    app[sl] = make_float4(0.f, 0.f, 0.f, 0.f);
    aw[sl] = 0.f;
    const int i = lane + 64 * sl;
    if (i < N - 1) {
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
  const float E0 = expf(-(float)(P.beta * ds[0])), E1 = expf(-(float)(P.beta * ds[1]));
  for (int j = 0; j < P.k; ++j) {
    float e0, e1, w0, w1;
    ksdf_surface_exp(P, 1, j, P.beta, ds[0], ds[1], E0, E1, e0, e1);
    ksdf_weights(e0, e1, N, lane, w0, w1);
    const float cr = ksdf_sum(w0 * app[0].x + w1 * app[1].x);
    const float cg = ksdf_sum(w0 * app[0].y + w1 * app[1].y);
    const float cb = ksdf_sum(w0 * app[0].z + w1 * app[1].z);
    const float ca = ksdf_sum(w0 * aw[0] * app[0].w + w1 * aw[1] * app[1].w);
    R += (T * ca) * cr;
    G += (T * ca) * cg;
    B += (T * ca) * cb;
    T *= 1.f - ca;
    if (layers && lane == 0) layers[(int64_t)j * total + ray] = make_float4(cr, cg, cb, ca);
  }
  if (lane == 0) out[ray] = make_float4(R, G, B, 1.f - T);
  if (samples) {
    if (lane < N) samples[ray * N + lane] = ts[0];
    if (lane + 64 < N) samples[ray * N + lane + 64] = ts[1];
  }
}

}  // namespace vs

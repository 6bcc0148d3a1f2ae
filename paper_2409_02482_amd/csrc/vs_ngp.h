// Neural textures (Sec. 4.3 "Texturing Meshes"): a 2-D multiresolution hash
// grid and a small MLP, grounded to the texture resolution by evaluating them
// at the texel centres only (Fig. 5), so that the renderer samples an ordinary
// RGBA texture.  Per texel (i, j) at u = (i + 1/2)/W, v = (j + 1/2)/H:
//   level l: x = u N_l, y = v N_l (FP64, as the texel coordinates elsewhere),
//            bilinear over the 4 surrounding vertices of 2 features each;
//            vertex index y (N_l + 1) + x when (N_l + 1)^2 <= T, else
//            (x XOR y * 2654435761) mod 2^32 masked to T - 1;
//   e = concat_l features (2L), z1 = W1 e + b1, h1 = relu(z1) (64),
//   z2 = W2 h1 + b2, h2 = relu(z2) (64), o = W3 h2 + b3 (4), texel = sigmoid(o).
// Parameters per layer, flat f32:
//   tables [L][T][2] | W1 [64][2L] | b1 [64] | W2 [64][64] | b2 [64] | W3 [4][64] | b3 [4].
// The per-texel products run on the matrix cores (see k_ngp_bake).  The
// backward pass (two per-texel kernels, to keep each one's registers, and so
// its occupancy, moderate) writes the layer inputs and the deltas of every
// texel to a workspace; the weight gradients are then tall-skinny products
// over texels (k_ngp_wgrad).
#pragma once

#include "vs_common.h"

namespace vs {

constexpr int kNgpHidden = 64;
constexpr int kNgpOut = 4;
constexpr int kNgpMaxLevels = 16;
constexpr uint32_t kNgpPrimeY = 2654435761u;
constexpr int kNgpTile = 16;   // texels per tile side; a block of 256 threads covers one tile
constexpr int kNgpSlots = 400; // LDS vertex sums per level in the table scatter (a 20 x 20 window)

struct NgpShape {
  int32_t levels, log2_table;
  int32_t res[kNgpMaxLevels];
  int32_t dense[kNgpMaxLevels];
  int64_t o_w1, o_b1, o_w2, o_b2, o_w3, o_b3, total;   // o_tab = 0
};

// Per layer buffers and sizes; block_off is the prefix sum of 256-texel tiles
// over layers, and row block_off * 256 + thread is a texel's staging row.
struct NgpTable {
  const float* params[kMaxLayers];
  float* tex[kMaxLayers];
  const float* gtex[kMaxLayers];
  float* gparams[kMaxLayers];
  int32_t w[kMaxLayers], h[kMaxLayers];
  int64_t block_off[kMaxLayers + 1];
  int32_t k;
};

// Staging for the backward, feature-major [feature][R] over R = 256 * tiles
// rows (every access of a wavefront, and every GEMM tile load, is then
// consecutive): A1 = e, A2 = h1, A3 = h2, D1, D2, DO.  Rows of texels outside
// the texture hold zeros.
struct NgpStage {
  float* a1;   // [2L][R]
  float* a2;   // [64][R]
  float* a3;   // [64][R]
  float* d1;   // [64][R]
  float* d2;   // [64][R]
  float* d0;   // [4][R]
  int64_t R;
};

__device__ inline uint32_t ngp_index(uint32_t x, uint32_t y, int32_t N, int32_t dense, uint32_t mask) {
  return dense ? y * (uint32_t)(N + 1) + x : ((x ^ (y * kNgpPrimeY)) & mask);
}

struct NgpTexel {
  int l;
  int32_t i, j;
  bool valid;
  int64_t t;     // texel index within the layer, j W + i
  int64_t row;   // staging row
};

__device__ inline NgpTexel ngp_texel(const NgpTable& T) {
  NgpTexel r;
  const int64_t b = blockIdx.x;
  int l = 0;
  while (l + 1 < T.k && T.block_off[l + 1] <= b) ++l;
  r.l = l;
  const int W = T.w[l], H = T.h[l];
  const int tiles_x = (W + kNgpTile - 1) / kNgpTile;
  const int64_t tb = b - T.block_off[l];
  const int ty = (int)(tb / tiles_x), tx = (int)(tb - (int64_t)ty * tiles_x);
  r.i = tx * kNgpTile + (threadIdx.x & 15);
  r.j = ty * kNgpTile + (threadIdx.x >> 4);
  r.valid = r.i < W && r.j < H;
  r.t = (int64_t)r.j * W + r.i;
  r.row = b * 256 + threadIdx.x;
  return r;
}

// Encoding of one texel centre; also the per-level corner indices and weights.
template <int LMAX>
__device__ inline void ngp_encode(const float* __restrict__ tables, const NgpShape& S, double u, double v, float (&e)[2 * LMAX],
                                  uint32_t (&idx)[LMAX][4], float (&wt)[LMAX][4]) {
  const uint32_t T = 1u << S.log2_table, mask = T - 1u;
#pragma unroll
  for (int lv = 0; lv < LMAX; ++lv) {
    e[2 * lv] = 0.f;
    e[2 * lv + 1] = 0.f;
    if (lv >= S.levels) continue;
    const int32_t N = S.res[lv];
    const double x = u * (double)N, y = v * (double)N;
    const double x0 = floor(x), y0 = floor(y);
    const float fx = (float)(x - x0), fy = (float)(y - y0);
    const uint32_t xi = (uint32_t)x0, yi = (uint32_t)y0;
    const float2* tab = reinterpret_cast<const float2*>(tables) + (int64_t)lv * T;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t dx = c & 1, dy = c >> 1;
      const uint32_t q = ngp_index(xi + dx, yi + dy, N, S.dense[lv], mask);
      const float w = (dx ? fx : 1.0f - fx) * (dy ? fy : 1.0f - fy);
      const float2 f = tab[q];
      e[2 * lv] += w * f.x;
      e[2 * lv + 1] += w * f.y;
      idx[lv][c] = q;
      wt[lv][c] = w;
    }
  }
}

__device__ inline float ngp_sigmoid(float x) { return 1.0f / (1.0f + expf(-x)); }

// texture = sigmoid(MLP(encoding)) at every texel centre of every layer; with
// STAGE the layer inputs e, h1 and h2 are kept for the backward.
//
// The three layers are dense products over the block's 256 texels and run on
// the matrix cores (v_mfma_f32_16x16x4_f32, FP32 in and out) in transposed
// form, Z^T = W X^T + b: the hidden units are the 16-row M tiles, 16 texels
// (one texel row of the tile) the N tile.  An MFMA leaves lane l with
// D[4 (l / 16) + r][l % 16], r = 0..3, and takes its B operand as
// B[k = l / 16][n = l % 16]; issuing the r-th of four MFMAs with the r-th
// register of the previous layer's output therefore feeds that output straight
// back as the next B operand, with the K index permuted to 4 (l / 16) + r; the
// weights (A operands) are laid out in LDS in that permuted order, one 64-lane
// fragment per MFMA.  Encodings go through LDS to become layer 1's B operand.
typedef float ngp_f4 __attribute__((ext_vector_type(4)));

template <int LMAX, bool STAGE>
__global__ void __launch_bounds__(256) k_ngp_bake(NgpTable T, NgpShape S, NgpStage G) {
  constexpr int KIN = 2 * LMAX, KS1 = KIN / 4, EST = KIN + 1;
  __shared__ float w1f[4 * KS1 * 64];     // [mt][ks][lane]: W1[16 mt + lane % 16][4 ks + lane / 16]
  __shared__ float w2f[64 * 64];          // [mt][it][r][lane]: W2[16 mt + lane % 16][16 it + 4 (lane / 16) + r]
  __shared__ float w3f[16 * 64];          // [it][r][lane]: W3[lane % 16][16 it + 4 (lane / 16) + r] (rows >= 4: 0)
  __shared__ float es[4][64 * EST];       // per wave: the encodings of its 64 texels
  const NgpTexel x = ngp_texel(T);
  const int l = x.l, tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const float* P = T.params[l];
  const int nin = 2 * S.levels;
  for (int f = tid; f < 4 * KS1 * 64; f += 256) {
    const int ln = f & 63, fr = f >> 6, mt = fr / KS1, ks = fr - mt * KS1;
    const int m = 16 * mt + (ln & 15), kk = 4 * ks + (ln >> 4);
    w1f[f] = kk < nin ? P[S.o_w1 + m * nin + kk] : 0.f;
  }
  for (int f = tid; f < 64 * 64; f += 256) {
    const int ln = f & 63, fr = f >> 6, mt = fr >> 4, it = (fr >> 2) & 3, r = fr & 3;
    w2f[f] = P[S.o_w2 + (16 * mt + (ln & 15)) * kNgpHidden + 16 * it + 4 * (ln >> 4) + r];
  }
  for (int f = tid; f < 16 * 64; f += 256) {
    const int ln = f & 63, fr = f >> 6, it = fr >> 2, r = fr & 3, m = ln & 15;
    w3f[f] = m < kNgpOut ? P[S.o_w3 + m * kNgpHidden + 16 * it + 4 * (ln >> 4) + r] : 0.f;
  }
  // this thread's encoding (zeros outside the texture)
  float e[KIN];
  uint32_t idx[LMAX][4];
  float wt[LMAX][4];
#pragma unroll
  for (int q = 0; q < KIN; ++q) e[q] = 0.f;
  if (x.valid) {
    const double u = ((double)x.i + 0.5) / (double)T.w[l], v = ((double)x.j + 0.5) / (double)T.h[l];
    ngp_encode<LMAX>(P, S, u, v, e, idx, wt);
  }
  float* ew = es[wv];
#pragma unroll
  for (int q = 0; q < KIN; ++q) ew[lane * EST + q] = e[q];
  if (STAGE) {
    const uint32_t row = (uint32_t)x.row, R = (uint32_t)G.R;
#pragma unroll
    for (int q = 0; q < KIN; ++q)
      if (q < nin) G.a1[q * R + row] = e[q];
  }
  __syncthreads();

  const int g = lane >> 4, n = lane & 15;
  const float* b1 = P + S.o_b1;
  const float* b2 = P + S.o_b2;
  const float* b3 = P + S.o_b3;
  const int W = T.w[l], H = T.h[l];
#pragma unroll 1
  for (int it_n = 0; it_n < 4; ++it_n) {
    // N tile: texels 16 it_n + n of this wave = texel row 4 wv + it_n of the tile
    const int nb = 64 * wv + 16 * it_n + n;
    const int ti = x.i - (tid & 15) + (nb & 15), tj = x.j - (tid >> 4) + (nb >> 4);
    const bool valid = ti < W && tj < H;
    ngp_f4 h[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) h[mt][r] = b1[16 * mt + 4 * g + r];
#pragma unroll
    for (int ks = 0; ks < KS1; ++ks) {
      const float bop = ew[(16 * it_n + n) * EST + 4 * ks + g];
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
        h[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(w1f[(mt * KS1 + ks) * 64 + lane], bop, h[mt], 0, 0, 0);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) h[mt][r] = fmaxf(h[mt][r], 0.f);
    ngp_f4 z[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) z[mt][r] = b2[16 * mt + 4 * g + r];
#pragma unroll
    for (int it = 0; it < 4; ++it)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
          z[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(w2f[((mt * 4 + it) * 4 + r) * 64 + lane], h[it][r], z[mt], 0, 0,
                                                       0);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) z[mt][r] = fmaxf(z[mt][r], 0.f);
    ngp_f4 o;
#pragma unroll
    for (int r = 0; r < 4; ++r) o[r] = g == 0 ? b3[r] : 0.f;
#pragma unroll
    for (int it = 0; it < 4; ++it)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        o = __builtin_amdgcn_mfma_f32_16x16x4f32(w3f[(it * 4 + r) * 64 + lane], z[it][r], o, 0, 0, 0);
    if (g == 0 && valid)
      reinterpret_cast<float4*>(T.tex[l])[(int64_t)tj * W + ti] =
          make_float4(ngp_sigmoid(o[0]), ngp_sigmoid(o[1]), ngp_sigmoid(o[2]), ngp_sigmoid(o[3]));
    if (STAGE) {
      // 32-bit element offsets (the workspace holds < 2^31 floats per array)
      const uint32_t row = (uint32_t)(blockIdx.x * 256 + nb), R = (uint32_t)G.R;
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t m = 16 * mt + 4 * g + r;
          G.a2[m * R + row] = valid ? h[mt][r] : 0.f;
          G.a3[m * R + row] = valid ? z[mt][r] : 0.f;
        }
    }
  }
}

// Adds (v0, v1) into the feature pair q of a table for every active lane,
// summing lanes that share q first when the level is coarse (many texels per
// cell): one leader per distinct index and round, the others' values reduced
// across the wavefront.
__device__ inline void ngp_table_add(float* __restrict__ g, uint32_t q, float v0, float v1, bool active, bool merge) {
  if (!merge) {
    if (active) {
      unsafeAtomicAdd(g + 2 * (int64_t)q, v0);
      unsafeAtomicAdd(g + 2 * (int64_t)q + 1, v1);
    }
    return;
  }
  uint64_t pend = __ballot(active);
  while (pend) {
    const int leader = __builtin_ctzll(pend);
    const uint32_t k0 = __builtin_amdgcn_readlane(q, leader);
    const bool same = active && q == k0;
    float s0 = same ? v0 : 0.0f, s1 = same ? v1 : 0.0f;
    for (int off = 32; off > 0; off >>= 1) {
      s0 += __shfl_xor(s0, off);
      s1 += __shfl_xor(s1, off);
    }
    if ((int)__lane_id() == leader) {
      unsafeAtomicAdd(g + 2 * (int64_t)k0, s0);
      unsafeAtomicAdd(g + 2 * (int64_t)k0 + 1, s1);
    }
    pend &= ~__ballot(same);
  }
}

// Backward, first half, per texel (after a staging bake of the same
// parameters): do = dL/dtex * t (1 - t) from the baked texel t, and
// d2 = (W3^T do) [h2 > 0] (h2 > 0 exactly where z2 > 0); both staged.
__global__ void __launch_bounds__(256) k_ngp_texel_bwd1(NgpTable T, NgpShape S, NgpStage G) {
#pragma clang fp contract(fast)
  const NgpTexel x = ngp_texel(T);
  const int l = x.l;
  const float* P = T.params[l];
  const uint32_t r = (uint32_t)x.row, R = (uint32_t)G.R;
  float d0[4] = {0.f, 0.f, 0.f, 0.f};
  if (x.valid) {
    const float4 g = reinterpret_cast<const float4*>(T.gtex[l])[x.t];
    const float4 t = reinterpret_cast<const float4*>(T.tex[l])[x.t];
    d0[0] = g.x * t.x * (1.0f - t.x); d0[1] = g.y * t.y * (1.0f - t.y);
    d0[2] = g.z * t.z * (1.0f - t.z); d0[3] = g.w * t.w * (1.0f - t.w);
  }
  const float* W3 = P + S.o_w3;
#pragma unroll
  for (int j = 0; j < kNgpHidden; ++j) {
    float acc = 0.f;
#pragma unroll
    for (int c = 0; c < kNgpOut; ++c) acc += W3[c * kNgpHidden + j] * d0[c];
    G.d2[j * R + r] = G.a3[j * R + r] > 0.0f ? acc : 0.0f;
  }
#pragma unroll
  for (int c = 0; c < kNgpOut; ++c) G.d0[c * R + r] = d0[c];
}

// Backward, second half, per texel: d1 = (W2^T d2) [h1 > 0] (staged), de = W1^T d1,
// and de scattered into the hash tables through the encoding's corners and weights.
// The two products run on the matrix cores as in the bake (transposed form,
// 16 texels per N tile, d1 chained into the de product through a permuted K);
// de goes through LDS back to its texel's thread for the scatter.
template <int LMAX>
__global__ void __launch_bounds__(256) k_ngp_texel_bwd2(NgpTable T, NgpShape S, NgpStage G) {
  constexpr int KIN = 2 * LMAX, MT1 = (KIN + 15) / 16, DST = KIN + 1;
  constexpr int W2N = 64 * 64, W1N = MT1 * 16 * 64, DEN = 256 * DST;
  // one LDS buffer, two phases: the products' operands and de, then the per-level vertex sums
  __shared__ float lds[W2N + W1N + DEN];
  static_assert(LMAX * kNgpSlots * 2 <= W2N + W1N + DEN, "vertex sums must fit the product buffers");
  float* w2t = lds;                      // [mt][ks][lane]: W2[4 ks + lane / 16][16 mt + lane % 16]
  float* w1t = lds + W2N;                // [mt][it][r][lane]: W1[16 it + 4 (lane / 16) + r][16 mt + lane % 16]
  float* des = lds + W2N + W1N;          // de per texel of the block
  const NgpTexel x = ngp_texel(T);
  const int l = x.l, tid = threadIdx.x, wv = tid >> 6, lane = tid & 63, g = lane >> 4, n = lane & 15;
  const float* P = T.params[l];
  const int nin = 2 * S.levels;
  const uint32_t R = (uint32_t)G.R;
  for (int f = tid; f < 64 * 64; f += 256) {
    const int ln = f & 63, fr = f >> 6, mt = fr >> 4, ks = fr & 15;
    w2t[f] = P[S.o_w2 + (4 * ks + (ln >> 4)) * kNgpHidden + 16 * mt + (ln & 15)];
  }
  for (int f = tid; f < MT1 * 16 * 64; f += 256) {
    const int ln = f & 63, fr = f >> 6, mt = fr >> 4, it = (fr >> 2) & 3, r = fr & 3;
    const int q = 16 * mt + (ln & 15), j = 16 * it + 4 * (ln >> 4) + r;
    w1t[f] = q < nin ? P[S.o_w1 + j * nin + q] : 0.f;
  }
  __syncthreads();
#pragma unroll 1
  for (int it_n = 0; it_n < 4; ++it_n) {
    const int nb = 64 * wv + 16 * it_n + n;
    const uint32_t row = (uint32_t)(blockIdx.x * 256 + nb);
    ngp_f4 d1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) d1[mt] = ngp_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      const float bop = G.d2[(4 * ks + g) * R + row];   // zero outside the texture
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
        d1[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(w2t[(mt * 16 + ks) * 64 + lane], bop, d1[mt], 0, 0, 0);
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t q = 16 * mt + 4 * g + r;
        d1[mt][r] = G.a2[q * R + row] > 0.0f ? d1[mt][r] : 0.0f;
        G.d1[q * R + row] = d1[mt][r];
      }
    ngp_f4 de[MT1];
#pragma unroll
    for (int mt = 0; mt < MT1; ++mt) de[mt] = ngp_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int it = 0; it < 4; ++it)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int mt = 0; mt < MT1; ++mt)
          de[mt] = __builtin_amdgcn_mfma_f32_16x16x4f32(w1t[((mt * 4 + it) * 4 + r) * 64 + lane], d1[it][r], de[mt], 0,
                                                        0, 0);
#pragma unroll
    for (int mt = 0; mt < MT1; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int q = 16 * mt + 4 * g + r;
        if (q < KIN) des[nb * DST + q] = de[mt][r];
      }
  }
  __syncthreads();
  float de[KIN];
#pragma unroll
  for (int q = 0; q < KIN; ++q) de[q] = des[tid * DST + q];
  __syncthreads();
  // Scatter of de into the tables.  The block's 16 x 16 texels touch a small
  // window of each level's vertices; their contributions are summed per vertex
  // in LDS (float atomics) and each window vertex is then added to its table
  // entry once: neighbouring texels share corners, so this issues a quarter or
  // less of the global atomics.  A level whose window does not fit uses
  // direct global atomics.
  const int W = T.w[l], H = T.h[l];
  const double u = ((double)x.i + 0.5) / (double)W, v = ((double)x.j + 0.5) / (double)H;
  const int i_first = x.i - (tid & 15), j_first = x.j - (tid >> 4);
  const uint32_t TT = 1u << S.log2_table, mask = TT - 1u;
  float* gtab = T.gparams[l];
  float* vs = lds;                       // [level][kNgpSlots][2]
  for (int e = tid; e < LMAX * kNgpSlots * 2; e += 256) vs[e] = 0.f;
  __syncthreads();
  uint32_t vx0[LMAX], vy0[LMAX];
  int ex[LMAX], ey[LMAX];
#pragma unroll
  for (int lv = 0; lv < LMAX; ++lv) {
    ex[lv] = ey[lv] = 0;
    vx0[lv] = vy0[lv] = 0;
    if (lv >= S.levels) continue;
    const int32_t N = S.res[lv];
    // the window: vertices of the first and last texel of the tile along each axis (monotone in the texel)
    const double xa = floor(((double)i_first + 0.5) / (double)W * (double)N);
    const double xb = floor(((double)(i_first + 15) + 0.5) / (double)W * (double)N);
    const double ya = floor(((double)j_first + 0.5) / (double)H * (double)N);
    const double yb = floor(((double)(j_first + 15) + 0.5) / (double)H * (double)N);
    vx0[lv] = (uint32_t)xa;
    vy0[lv] = (uint32_t)ya;
    ex[lv] = (int)(xb - xa) + 2;
    ey[lv] = (int)(yb - ya) + 2;
    const bool windowed = (int64_t)ex[lv] * ey[lv] <= kNgpSlots;
    const double xx = u * (double)N, yy = v * (double)N;
    const double x0 = floor(xx), y0 = floor(yy);
    const float fx = (float)(xx - x0), fy = (float)(yy - y0);
    const uint32_t xi = (uint32_t)x0, yi = (uint32_t)y0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t dx = c & 1, dy = c >> 1;
      const float w = (dx ? fx : 1.0f - fx) * (dy ? fy : 1.0f - fy);
      if (windowed) {
        if (x.valid) {
          const int slot = (int)(yi + dy - vy0[lv]) * ex[lv] + (int)(xi + dx - vx0[lv]);
          atomicAdd(&vs[(lv * kNgpSlots + slot) * 2], w * de[2 * lv]);
          atomicAdd(&vs[(lv * kNgpSlots + slot) * 2 + 1], w * de[2 * lv + 1]);
        }
      } else {
        const uint32_t q = x.valid ? ngp_index(xi + dx, yi + dy, N, S.dense[lv], mask) : 0u;
        ngp_table_add(gtab + (int64_t)lv * TT * 2, q, w * de[2 * lv], w * de[2 * lv + 1], x.valid, false);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int lv = 0; lv < LMAX; ++lv) {
    if (lv >= S.levels || (int64_t)ex[lv] * ey[lv] > kNgpSlots) continue;
    const int32_t N = S.res[lv];
    for (int sl = tid; sl < ex[lv] * ey[lv]; sl += 256) {
      const float a0 = vs[(lv * kNgpSlots + sl) * 2], a1 = vs[(lv * kNgpSlots + sl) * 2 + 1];
      if (a0 != 0.0f || a1 != 0.0f) {
        const uint32_t vx = vx0[lv] + (uint32_t)(sl % ex[lv]), vy = vy0[lv] + (uint32_t)(sl / ex[lv]);
        const uint32_t q = ngp_index(vx, vy, N, S.dense[lv], mask);
        float* gq = gtab + (int64_t)lv * TT * 2 + 2 * (int64_t)q;
        unsafeAtomicAdd(gq, a0);
        unsafeAtomicAdd(gq + 1, a1);
      }
    }
  }
}

// One weight-gradient product of one layer: C[m][n] = sum_r D[m][r] A[n][r]
// over the layer's staging rows (feature-major, row stride R), m < M (<= 64),
// n < K (<= 64); the bias gradient is sum_r D[m][r].  Blocks split the rows;
// each thread owns a 4 x 4 tile of outputs (m = 4 (tid / 16) ..,
// n = 4 (tid % 16) ..) and the threads of the first column tile also the 4
// bias sums; partial sums are added to the gradient (weights row-major
// [M][K], then the bias [M]).
struct NgpGemm {
  const float* D[3 * kMaxLayers];
  const float* A[3 * kMaxLayers];
  float* gw[3 * kMaxLayers];
  float* gb[3 * kMaxLayers];
  int64_t rows[3 * kMaxLayers];
  int32_t M[3 * kMaxLayers], K[3 * kMaxLayers];
  int64_t R;
  int32_t n_gemm, blocks_per_gemm;
};

__global__ void __launch_bounds__(256) k_ngp_wgrad(NgpGemm Q) {
#pragma clang fp contract(fast)
  // rows padded to 65 floats: the staging writes (64 lanes, 64 consecutive rows of one feature) then fall
  // on distinct banks instead of all on one
  __shared__ float sD[64][65];
  __shared__ float sA[64][65];
  const int gi = blockIdx.x / Q.blocks_per_gemm, part = blockIdx.x - gi * Q.blocks_per_gemm;
  if (gi >= Q.n_gemm) return;
  const int M = Q.M[gi], K = Q.K[gi];
  const int64_t rows = Q.rows[gi], R = Q.R;
  const int64_t per = ((rows + Q.blocks_per_gemm - 1) / Q.blocks_per_gemm + 63) / 64 * 64;
  const int64_t r0 = (int64_t)part * per, r1 = min(rows, r0 + per);
  const int tid = threadIdx.x, mb = (tid >> 4) * 4, nb = (tid & 15) * 4;
  float acc[4][4], bacc[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    bacc[a] = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
  }
  for (int64_t rb = r0; rb < r1; rb += 64) {
    const int nr = (int)min((int64_t)64, r1 - rb);
    __syncthreads();
    for (int p = tid; p < 64 * 64; p += 256) {
      const int rr = p & 63, cc = p >> 6;   // consecutive threads read consecutive rows of one feature
      sD[rr][cc] = (rr < nr && cc < M) ? Q.D[gi][cc * R + rb + rr] : 0.f;
      sA[rr][cc] = (rr < nr && cc < K) ? Q.A[gi][cc * R + rb + rr] : 0.f;
    }
    __syncthreads();
    for (int rr = 0; rr < nr; ++rr) {
      const float dv[4] = {sD[rr][mb], sD[rr][mb + 1], sD[rr][mb + 2], sD[rr][mb + 3]};
      const float aw[4] = {sA[rr][nb], sA[rr][nb + 1], sA[rr][nb + 2], sA[rr][nb + 3]};
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        bacc[a] += dv[a];
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] += dv[a] * aw[b];
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int m = mb + a;
    if (m >= M) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int n = nb + b;
      if (n < K && acc[a][b] != 0.0f) unsafeAtomicAdd(Q.gw[gi] + (int64_t)m * K + n, acc[a][b]);
    }
    if (nb == 0 && bacc[a] != 0.0f) unsafeAtomicAdd(Q.gb[gi] + m, bacc[a]);
  }
}

}  // namespace vs

// Texture fitting kernels: fused Adam step + projection to [lo, hi] + gradient
// reset, and the per-iteration bookkeeping that keeps the loss history on the
// device (so an iteration can be replayed from a HIP graph without host sync).
#pragma once

#include "vs_common.h"

namespace vs {

struct AdamTable {
  float* p[kMaxLayers];
  float* g[kMaxLayers];
  float* m[kMaxLayers];
  float* v[kMaxLayers];
  int64_t off[kMaxLayers + 1];   // prefix of element counts
  int32_t k;
};

// One Adam step over every texel scalar of every layer.  The step number t is
// read from the device (t = *step + 1) so that graph replays advance it.
// After the update the parameter is projected to [lo, hi] and the gradient
// is reset to 0 for the next accumulation.
__global__ void __launch_bounds__(256) k_adam(AdamTable A, float lr, float b1, float b2, float eps, float lo,
                                              float hi, const int32_t* __restrict__ step) {
  const int64_t n = A.off[A.k];
  const int t = *step + 1;
  const float c1 = 1.0f / (1.0f - (float)pow((double)b1, (double)t));
  const float c2 = 1.0f / (1.0f - (float)pow((double)b2, (double)t));
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; i < n; i += stride) {
    int l = 0;
    while (l + 1 < A.k && A.off[l + 1] <= i) ++l;
    const int64_t j = i - A.off[l];
    // every layer holds a multiple of 4 scalars (RGBA), so a float4 never straddles layers
    float4 g = *reinterpret_cast<float4*>(A.g[l] + j);
    float4 m = *reinterpret_cast<float4*>(A.m[l] + j);
    float4 v = *reinterpret_cast<float4*>(A.v[l] + j);
    float4 p = *reinterpret_cast<float4*>(A.p[l] + j);
    float* gp = &g.x;
    float* mp = &m.x;
    float* vp = &v.x;
    float* pp = &p.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      mp[q] = b1 * mp[q] + (1.0f - b1) * gp[q];
      vp[q] = b2 * vp[q] + (1.0f - b2) * gp[q] * gp[q];
      const float mh = mp[q] * c1, vh = vp[q] * c2;
      pp[q] = fminf(fmaxf(pp[q] - lr * mh / (sqrtf(vh) + eps), lo), hi);
    }
    *reinterpret_cast<float4*>(A.m[l] + j) = m;
    *reinterpret_cast<float4*>(A.v[l] + j) = v;
    *reinterpret_cast<float4*>(A.p[l] + j) = p;
    *reinterpret_cast<float4*>(A.g[l] + j) = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// Squeezing and quantisation (Sec. 4.3): the texture value of a logit is
// q(sigmoid(theta)), q(x) = round(levels x) / levels with ties to even
// (levels = 0: no quantisation).  Decided in FP64, so that a code does not
// hinge on the FP32 rounding of the sigmoid.
__device__ inline float squeeze_quantize(float theta, int levels) {
  const double s = 1.0 / (1.0 + exp(-(double)theta));
  return levels ? (float)(rint((double)levels * s) / (double)levels) : (float)s;
}

struct TexOut {
  float* t[kMaxLayers];
};

// tex = q(sigmoid(params)) over every scalar of every layer.
__global__ void __launch_bounds__(256) k_squeeze(AdamTable A, TexOut T, int levels) {
  const int64_t n = A.off[A.k];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; i < n; i += stride) {
    int l = 0;
    while (l + 1 < A.k && A.off[l + 1] <= i) ++l;
    const int64_t j = i - A.off[l];
    const float4 p = *reinterpret_cast<const float4*>(A.p[l] + j);
    *reinterpret_cast<float4*>(T.t[l] + j) = make_float4(squeeze_quantize(p.x, levels), squeeze_quantize(p.y, levels),
                                                         squeeze_quantize(p.z, levels), squeeze_quantize(p.w, levels));
  }
}

// Adam on the logits of a squeezed, quantised texture.  The gradient arrives
// as dL/dtex; quantisation is passed straight through, so
// dL/dtheta = dL/dtex * s (1 - s), s = sigmoid(theta).  After the update the
// texture is re-derived from the logit and the gradient is reset.
__global__ void __launch_bounds__(256) k_adam_squeezed(AdamTable A, TexOut T, float lr, float b1, float b2, float eps,
                                                       int levels, const int32_t* __restrict__ step) {
  const int64_t n = A.off[A.k];
  const int t = *step + 1;
  const float c1 = 1.0f / (1.0f - (float)pow((double)b1, (double)t));
  const float c2 = 1.0f / (1.0f - (float)pow((double)b2, (double)t));
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; i < n; i += stride) {
    int l = 0;
    while (l + 1 < A.k && A.off[l + 1] <= i) ++l;
    const int64_t j = i - A.off[l];
    float4 g = *reinterpret_cast<float4*>(A.g[l] + j);
    float4 m = *reinterpret_cast<float4*>(A.m[l] + j);
    float4 v = *reinterpret_cast<float4*>(A.v[l] + j);
    float4 p = *reinterpret_cast<float4*>(A.p[l] + j);
    float4 tx;
    float* gp = &g.x;
    float* mp = &m.x;
    float* vp = &v.x;
    float* pp = &p.x;
    float* tp = &tx.x;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float sg = 1.0f / (1.0f + expf(-pp[q]));
      const float gq = gp[q] * sg * (1.0f - sg);
      mp[q] = b1 * mp[q] + (1.0f - b1) * gq;
      vp[q] = b2 * vp[q] + (1.0f - b2) * gq * gq;
      const float mh = mp[q] * c1, vh = vp[q] * c2;
      pp[q] = pp[q] - lr * mh / (sqrtf(vh) + eps);
      tp[q] = squeeze_quantize(pp[q], levels);
    }
    *reinterpret_cast<float4*>(A.m[l] + j) = m;
    *reinterpret_cast<float4*>(A.v[l] + j) = v;
    *reinterpret_cast<float4*>(A.p[l] + j) = p;
    *reinterpret_cast<float4*>(T.t[l] + j) = tx;
    *reinterpret_cast<float4*>(A.g[l] + j) = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// history[*step] = *sse (if room), *sse = 0, ++*step.  One thread.
__global__ void k_fit_bookkeep(double* __restrict__ sse, double* __restrict__ history, int32_t hist_len,
                               int32_t* __restrict__ step) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int32_t t = *step;
  if (sse) {
    if (history && t >= 0 && t < hist_len) history[t] = *sse;
    *sse = 0.0;
  }
  *step = t + 1;
}

// Order-independent checksum of a visibility buffer (autotune cross-check):
// sum over slots of a mix of (key, slot index), wrapping.
__global__ void __launch_bounds__(256) k_vis_checksum(const uint64_t* __restrict__ vis, int64_t n,
                                                      unsigned long long* __restrict__ out) {
  unsigned long long acc = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    uint64_t x = vis[i] ^ ((uint64_t)i * 0x9E3779B97F4A7C15ull);
    x ^= x >> 31;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 29;
    acc += x;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(out, acc);
}

}  // namespace vs

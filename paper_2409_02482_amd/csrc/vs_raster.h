// Visibility kernels (steps 1-3): vertex projection and per-layer
// rasterisation into 64-bit (depth, triangle id) keys.
//
// Binned pipeline (one call of vs_raster_layers):
//   k_project      snapped screen positions and w = 1/z for every (view, layer, vertex)
//   k_bin_count    per triangle: setup, cull, bounding box -> screen tiles of
//                  B x bin_rows(B) pixels; reserve the triangle's place in its
//                  first bin = (view, tile, layer), count it in its other bins,
//                  and record its packed tile span and place
//   k_scan_*       exclusive prefix sum of the bins' entry counts -> list offsets
//   k_bin_scatter  write triangle ids into the bin lists (front faces first)
//   k_raster_bins  one block per bin: an LDS tile of keys starts EMPTY, the
//                  bin's triangles take 64-bit LDS minima, and the finished
//                  tile is stored once, coalesced (so no clear pass is needed);
//                  a fragment whose depth lower bound already loses to the
//                  tile's key skips the exact FP64 depth, and a back-facing
//                  triangle whose bound loses everywhere in its bounding box
//                  is skipped whole
// First-bin reservations are aggregated per wavefront: lanes whose first bin
// and side agree elect one lane that reserves for the whole group.
#pragma once

#include "vs_common.h"

namespace vs {

constexpr int kRasterThreads = 256;

// Bins are B pixels wide and bin_rows(B) high (a whole number of 8-row
// sub-tiles): 64-pixel bins are 56 rows high, so that a block's 64-bit key
// tile (28 KiB) and back-face queue leave room for five blocks per CU (a
// 64 x 64 tile alone, 32 KiB, fits only four).  Metric scene / k = 9 scene,
// raster phase: 56 rows 5.31 / 8.78 ms; 48 rows (still five blocks) 5.67 /
// 8.78 ms; 40 rows (six blocks) 5.63 / 8.47 ms.
__host__ __device__ constexpr int bin_rows(int B) { return B == 64 ? 56 : B; }
constexpr int kSmallSpan = 16384;   // small-triangle path: bbox extents <= 64 px, so edge values fit int32
constexpr int kSmallArea = 256;     // ... and at most this many candidate pixels in the tile

// Fill n u64 words with a value (grid-stride).
__global__ void __launch_bounds__(256) k_fill_u64(uint64_t* __restrict__ p, int64_t n, uint64_t val) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = val;
}

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t val) {
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

// Pixel-centre range covered by the triangle's fixed-point bounding box, clipped to the view.
struct PixRange { int i0, i1, j0, j1; };

__device__ inline PixRange pixel_range(const TriSetup& T, int W, int H) {
  const double mnx = fmin(T.X[0], fmin(T.X[1], T.X[2])), mxx = fmax(T.X[0], fmax(T.X[1], T.X[2]));
  const double mny = fmin(T.Y[0], fmin(T.Y[1], T.Y[2])), mxy = fmax(T.Y[0], fmax(T.Y[1], T.Y[2]));
  PixRange r;
  r.i0 = max((int)ceil((mnx - 128.0) * (1.0 / 256.0)), 0);
  r.i1 = min((int)floor((mxx - 128.0) * (1.0 / 256.0)), W - 1);
  r.j0 = max((int)ceil((mny - 128.0) * (1.0 / 256.0)), 0);
  r.j1 = min((int)floor((mxy - 128.0) * (1.0 / 256.0)), H - 1);
  return r;
}

__device__ inline int cull_slot(int r) {
  return r == kTriInvalid ? VS_STAT_CULLED_INVALID : r == kTriDegenerate ? VS_STAT_CULLED_DEGENERATE
                                                                        : VS_STAT_BAD_INDEX;
}

// Record of one (view, layer, triangle) written by k_bin_count: its pixel
// bounding box clipped to the view, packed in 64 bits,
//   i0 | i1 << 13 | j0 << 26 | j1 << 39 | front << 52 | valid << 53,
// and the depth bits of its lower-bound key (depth_lower_key >> 32).
// "front" marks a negative screen area before orientation normalisation,
// which is the front side of an outward, counter-clockwise wound closed mesh
// under this camera convention (y down).  It orders the bin lists, front
// faces first; the raster uses the box and the bound to skip, without
// loading its vertices, a back-facing triangle that cannot lower any key.
constexpr uint64_t kSpanValid = 1ull << 53;
constexpr uint64_t kSpanFront = 1ull << 52;

struct alignas(16) SpanRec {
  uint64_t box;
  uint32_t zlo;    // high word of the triangle's depth lower-bound key
  uint32_t rank;   // entries of the same side of its first bin reserved before it
};

__device__ inline uint64_t pack_box(int i0, int i1, int j0, int j1, bool front) {
  return (uint64_t)i0 | ((uint64_t)i1 << 13) | ((uint64_t)j0 << 26) | ((uint64_t)j1 << 39) |
         (front ? kSpanFront : 0ull) | kSpanValid;
}

__device__ inline void unpack_box(uint64_t b, int& i0, int& i1, int& j0, int& j1) {
  i0 = (int)(b & 8191); i1 = (int)((b >> 13) & 8191); j0 = (int)((b >> 26) & 8191); j1 = (int)((b >> 39) & 8191);
}

// Triangles per thread in the count and scatter launches.  Count: the vertex
// ids of all four are requested first, then the vertex records two at a time,
// the next one's loads issued as soon as a record slot is free (four records
// loaded up front needed 97 registers and were slower); the four first-bin
// reservations are in flight together and the records are written once they
// return.  Scatter: the records and first-bin list ranges of all four are read
// together; only a triangle's other bins still take a returning atomic there.
// Eight per thread in the scatter: 102 registers, metric raster phase 5.00
// against 4.98 ms, k = 9 scene 7.96 against 7.67 ms.
constexpr int kCountReps = 4;
constexpr int kScatterReps = 4;

// Grid of a count/scatter launch with R triangles per thread: x = blocks of
// R x 256 padded triangles of one view (each layer's range rounded up to 64,
// so that a wavefront never spans two layers), rounded up to a multiple of
// the XCD count; y = view.
template <int R>
__host__ __device__ inline uint32_t bin_grid_x(int64_t n_tri_padded) {
  return (uint32_t)((((n_tri_padded + 255) / 256 + R - 1) / R + 7) / 8 * 8);
}

// Block of 256 padded triangles that repetition r of this block handles.
// Blocks are dealt round-robin to the 8 XCDs, and gridDim.x is a multiple of
// 8, so blockIdx.x % 8 is the XCD: the remap gives each XCD a contiguous
// eighth of the view's triangles (triangles that share vertices share that
// XCD's L2).
template <int R>
__device__ inline uint32_t bin_block(int r) {
  const uint32_t chunk = gridDim.x >> 3;
  return ((blockIdx.x & 7u) * chunk + (blockIdx.x >> 3)) * R + r;
}

// Which (layer, triangle) of view blockIdx.y this thread handles in block vb;
// g is the triangle's index over all layers of the view.  The layer is the
// same on every lane of a wavefront, so the layer search and its table
// entries are scalar.
__device__ inline bool bin_thread(const LayerTable& L, uint32_t vb, int& l, int32_t& t, int64_t& g) {
  const int k = L.k;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t gw = (int64_t)vb * 256 + wave * 64;   // the wavefront's first padded index
  int lw = 0;
  while (lw + 1 < k && L.tri_pad[lw + 1] <= gw) ++lw;
  l = lw;
  t = 0;
  g = 0;
  const int64_t gp = gw + (threadIdx.x & 63);
  if (gp >= L.tri_pad[k]) return false;
  t = (int32_t)(gp - L.tri_pad[l]);
  if (t >= L.n_tri[l]) return false;   // padding
  g = L.tri_off[l] + t;
  return true;
}

// Bins of one view: (tile, layer) pairs, tile-major, starting at
// tile_offset[slot] * k in the counters of all views (so a view's bin index
// fits 32 bits: at most 1024^2 tiles times 16 layers).
__device__ inline int64_t view_bins_base(const vs_view& V, int slot, int k) {
  return (int64_t)V.tile_offset[slot] * k;
}

// Per triangle: reserve its place among the entries of its side (front-facing
// or not) in its first bin, count it in its other bins, and record its box,
// depth bound and that place.
template <int B>
__global__ void __launch_bounds__(256) k_bin_count(const vs_view* __restrict__ views, LayerTable L,
                                                   const ProjVert* __restrict__ proj, int64_t vpv, int slot,
                                                   uint32_t* __restrict__ count, uint32_t* __restrict__ cursor,
                                                   SpanRec* __restrict__ spans,
                                                   unsigned long long* __restrict__ status) {
  constexpr int R = kCountReps;
  constexpr int BH = bin_rows(B);
  const int v = blockIdx.y;
  const int k = L.k;
  const vs_view& V = views[v];
  const int W = V.cam.width, H = V.cam.height;
  const int ntx = (W + B - 1) / B;
  uint32_t* cv = count + view_bins_base(V, slot, k);
  uint32_t* uv = cursor + 2 * view_bins_base(V, slot, k);   // per bin: front, other side
  const ProjVert* pview = proj + (int64_t)v * vpv;
  SpanRec* sview = spans + (int64_t)v * L.tri_off[k];
  bool ok[R];
  int l[R];
  int32_t t[R];
  int64_t g[R];
  int3 ids[R];
  // ids of every repetition first (small); vertex records two at a time, the
  // next record's loads issued as soon as a record slot is free
#pragma unroll
  for (int r = 0; r < R; ++r) {
    ok[r] = bin_thread(L, bin_block<R>(r), l[r], t[r], g[r]);
    ids[r] = make_int3(0, 0, 0);
    if (ok[r]) ids[r] = load_ids(L.tri[l[r]], (uint32_t)t[r]);
  }
  auto fetch = [&](int r, TriLoad& q) {
    // defined on every lane: left undefined, the records stay live across the
    // divergent loads and cost about 16 more registers
    q.a = q.b = q.c = make_int4(0, 0, 0, 0);
    q.id[0] = q.id[1] = q.id[2] = 0;
    q.bad = false;
    if (ok[r]) load_vertices(ids[r], L.n_vert[l[r]], pview + L.vert_off[l[r]], q);
  };
  TriLoad qa, qb;
  fetch(0, qa);
  if (R > 1) fetch(1, qb);
  const int lane = (int)__lane_id();
  const uint64_t lt = __lanemask_lt();
  uint64_t boxes[R];   // the records' box and bound words (zero for a culled or off-screen triangle),
  uint32_t zlos[R];    // written once the places are known
  uint32_t base[R], rank[R];
  int leader_of[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    TriLoad& qr = (r & 1) ? qb : qa;
    int tx0 = 0, tx1 = 0, ty0 = 0, ty1 = 0;
    bool live = ok[r], front = false;
    if (live) {
      TriSetup T;
      const int st = setup_loaded(qr, T);
      SpanRec span;
      span.box = 0; span.zlo = 0; span.rank = 0;
      if (st != kTriOk) {
        atomicAdd(status + cull_slot(st), 1ull);
        live = false;
      } else {
        const PixRange pr = pixel_range(T, W, H);
        if (pr.i0 > pr.i1 || pr.j0 > pr.j1) {
          live = false;
        } else {
          tx0 = pr.i0 / B; tx1 = pr.i1 / B; ty0 = pr.j0 / BH; ty1 = pr.j1 / BH;
          front = T.orig_sign < 0;
          span.box = pack_box(pr.i0, pr.i1, pr.j0, pr.j1, front);
          span.zlo = (uint32_t)(depth_lower_key(T, (uint32_t)t[r]) >> 32);
        }
      }
      boxes[r] = span.box;
      zlos[r] = span.zlo;
    }
    if (r + 2 < R) fetch(r + 2, qr);   // this record slot is free now
    // first bin of every lane, and its side: lanes of the same (bin, side) class
    // elect one lane (register exchanges only), which reserves their places
    // among the bin's entries of that side (the scan adds these reservations to
    // the bin's count); every lane's place is the reservation plus its rank
    const int32_t b0 = live ? (ty0 * ntx + tx0) * k + l[r] : -1;
    const int32_t c0 = live ? 2 * b0 + (front ? 0 : 1) : -1;
    uint64_t active = __ballot(c0 >= 0);
    uint32_t group = 0;
    rank[r] = 0;
    leader_of[r] = lane;
    while (active) {
      const int leader = (int)__builtin_ctzll(active);
      const int32_t lc = __builtin_amdgcn_readlane(c0, leader);
      const uint64_t same = __ballot(c0 == lc);
      if (c0 == lc) {
        leader_of[r] = leader;
        rank[r] = (uint32_t)__popcll(same & lt);
      }
      if (lane == leader) group = (uint32_t)__popcll(same);
      active &= ~same;
    }
    base[r] = 0;
    if (group) base[r] = atomicAdd(uv + c0, group);
    if (live) {
      for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) {
          if (ty == ty0 && tx == tx0) continue;
          atomicAdd(cv + (ty * ntx + tx) * k + l[r], 1u);
        }
    }
  }
  // the reservations of every repetition were in flight together; each record
  // is written once (a 16-byte store), with its place
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t e = __shfl(base[r], leader_of[r]) + rank[r];
    if (ok[r]) {
      SpanRec span;
      span.box = boxes[r];
      span.zlo = zlos[r];
      span.rank = e;
      sview[g[r]] = span;
    }
  }
}

// Exclusive scan of the per-bin entry counts into 64-bit list offsets (the
// total can pass 2^32 when triangles cover many bins; a bin's own count stays
// below 2^30 because n_views * triangles does).
// Pass 1: each block takes 1024 bins.  A bin's entries are those counted in
// count (triangles for which it is not the first bin) plus the places its
// first-bin triangles reserved on both sides (first[2 b], first[2 b + 1]);
// the sum is written back to count, then the local prefixes and the block's
// total.
__global__ void __launch_bounds__(256) k_scan_local(uint32_t* __restrict__ count, const uint32_t* __restrict__ first,
                                                    uint64_t* __restrict__ out, uint64_t* __restrict__ partial,
                                                    int64_t n) {
  __shared__ uint64_t s[256];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * 1024 + tid * 4;
  uint32_t v[4];
  uint64_t sum = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    v[q] = base + q < n ? count[base + q] + first[2 * (base + q)] + first[2 * (base + q) + 1] : 0u;
    if (base + q < n) count[base + q] = v[q];
    sum += v[q];
  }
  s[tid] = sum;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint64_t add = tid >= off ? s[tid - off] : 0u;
    __syncthreads();
    s[tid] += add;
    __syncthreads();
  }
  uint64_t run = s[tid] - sum;  // exclusive prefix of this thread
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (base + q < n) out[base + q] = run;
    run += v[q];
  }
  if (tid == 255) partial[blockIdx.x] = s[255];
}

// Pass 2: one block scans the block totals in place (exclusive), carrying across chunks.
__global__ void __launch_bounds__(1024) k_scan_partials(uint64_t* __restrict__ partial, int64_t n) {
  __shared__ uint64_t s[1024];
  __shared__ uint64_t carry;
  const int tid = threadIdx.x;
  if (tid == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < n; base += 1024) {
    const uint64_t v = base + tid < n ? partial[base + tid] : 0u;
    s[tid] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const uint64_t add = tid >= off ? s[tid - off] : 0u;
      __syncthreads();
      s[tid] += add;
      __syncthreads();
    }
    if (base + tid < n) partial[base + tid] = carry + s[tid] - v;
    __syncthreads();
    if (tid == 1023) carry += s[1023];
    __syncthreads();
  }
}

// Pass 3: add the block prefixes.
__global__ void __launch_bounds__(256) k_scan_add(uint64_t* __restrict__ out, const uint64_t* __restrict__ partial,
                                                  int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += partial[i / 1024];
}

// Write triangle ids into the bin lists: front-facing triangles from the
// head of a bin's list, the others from its tail.  A triangle's place in its
// first bin (most triangles have only one) was reserved by the count, so it
// takes no atomic here; its other bins are reserved here, after every
// first-bin entry of the same side.  A bin whose list would end
// past the capacity is left unwritten; the raster of that bin then scans every
// triangle of its layer instead (slow but exact) and the overflow is counted.
template <int B>
__global__ void __launch_bounds__(256) k_bin_scatter(const vs_view* __restrict__ views, LayerTable L, int slot,
                                                     const SpanRec* __restrict__ spans,
                                                     const uint32_t* __restrict__ count,
                                                     const uint64_t* __restrict__ offset,
                                                     uint32_t* __restrict__ cursor, int32_t* __restrict__ list,
                                                     uint64_t capacity) {
  constexpr int R = kScatterReps;
  constexpr int BH = bin_rows(B);
  const int v = blockIdx.y;
  const int k = L.k;
  const vs_view& V = views[v];
  const int ntx = (V.cam.width + B - 1) / B;
  const int64_t vb = view_bins_base(V, slot, k);
  const uint32_t* cv = count + vb;
  const uint64_t* ov = offset + vb;
  uint32_t* uv = cursor + 2 * vb;   // per bin: [2 b] front entries from the head, [2 b + 1] the others from the tail
  const SpanRec* sview = spans + (int64_t)v * L.tri_off[k];
  bool ok[R];
  int l[R];
  int32_t t[R];
  int64_t g[R];
  uint64_t span[R];
  uint32_t rank[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    ok[r] = bin_thread(L, bin_block<R>(r), l[r], t[r], g[r]);
    uint4 rec = make_uint4(0u, 0u, 0u, 0u);
    if (ok[r]) rec = reinterpret_cast<const uint4*>(sview)[g[r]];
    span[r] = (uint64_t)rec.x | ((uint64_t)rec.y << 32);
    rank[r] = rec.w;
  }
  // the first bins' list ranges, all in flight together
  int32_t b0[R];
  uint64_t off[R];
  uint32_t cnt[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    ok[r] = ok[r] && (span[r] & kSpanValid);
    b0[r] = -1;
    off[r] = 0;
    cnt[r] = 0;
    if (ok[r]) {
      int i0, i1, j0, j1;
      unpack_box(span[r], i0, i1, j0, j1);
      b0[r] = ((j0 / BH) * ntx + i0 / B) * k + l[r];
      off[r] = ov[b0[r]];
      cnt[r] = cv[b0[r]];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (!ok[r]) continue;
    const bool front = (span[r] & kSpanFront) != 0;
    const uint64_t end = off[r] + cnt[r];
    // first bin: the place reserved by the count
    if (end <= capacity) list[front ? off[r] + rank[r] : end - 1 - rank[r]] = t[r];
    // the span's other bins, four at a time: their list ranges and reservations
    // are all in flight before any entry is written
    int i0, i1, j0, j1;
    unpack_box(span[r], i0, i1, j0, j1);
    const int tx0 = i0 / B, tx1 = i1 / B, ty0 = j0 / BH, ty1 = j1 / BH;
    int tx = tx0, ty = ty0;   // the bin before the next one to take
    int left = (tx1 - tx0 + 1) * (ty1 - ty0 + 1) - 1;
    while (left > 0) {
      int32_t bq[4];
      uint64_t oq[4];
      uint32_t cq[4], rq[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        bq[e] = -1;
        if (e < left) {
          if (++tx > tx1) {
            tx = tx0;
            ++ty;
          }
          bq[e] = (ty * ntx + tx) * k + l[r];
        }
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        oq[e] = 0;
        cq[e] = 0;
        rq[e] = 0;
        if (bq[e] >= 0) {
          oq[e] = ov[bq[e]];
          cq[e] = cv[bq[e]];
          rq[e] = atomicAdd(uv + 2 * bq[e] + (front ? 0 : 1), 1u);
        }
      }
      // one wait for all four reservations (the empty statement uses them on every
      // lane), so that the stores below issue back to back
      __asm__ volatile("" ::"v"(rq[0]), "v"(rq[1]), "v"(rq[2]), "v"(rq[3]), "v"(cq[0]), "v"(cq[1]), "v"(cq[2]),
                       "v"(cq[3]));
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint64_t bend = oq[e] + cq[e];
        if (bq[e] >= 0 && bend <= capacity) list[front ? oq[e] + rq[e] : bend - 1 - rq[e]] = t[r];
      }
      left -= 4;
    }
  }
}

// tile_view[g] = view owning tile g of the given tile-size slot.
__global__ void __launch_bounds__(256) k_tile_view_slot(const vs_view* __restrict__ views, int n_views,
                                                        int32_t* __restrict__ tile_view, int64_t n_tiles, int slot) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_tiles) return;
  tile_view[g] = find_view_tile(views, n_views, g, slot);
}

// One block per bin.  Small triangles (bounding box <= 64 px on each side and
// few candidate pixels) are walked by one lane with exact int32 edge values;
// larger ones are tested by the lane's whole wavefront, each lane owning
// B*bin_rows(B)/64 pixels, with exact FP64 edge values.  Wavefronts work independently
// on the LDS tile (64-bit atomic minimum).
//
// The bin's list holds its front-facing triangles first.  They are drawn
// first; then the tile's largest key per 8 x 8 sub-tile is taken, and a
// back-facing triangle whose depth lower bound (a key no larger than any key it
// can produce) is at least every sub-tile maximum under its bounding box is
// skipped: every pixel it could reach already holds a key no larger than any
// of its own, so the minimum cannot change (keys only decrease).  On a closed
// shell seen from outside, the back faces lie behind the front faces covering
// the same pixels, so most of them are skipped without a pixel walk.  An empty
// pixel keeps its sub-tile maximum at EMPTY, so nothing is skipped there.  With
// fragment counting on, nothing is skipped (the count covers every covered
// pixel of every triangle).
template <int B>
__global__ void __launch_bounds__(kRasterThreads) k_raster_bins(
    const vs_view* __restrict__ views, const int32_t* __restrict__ bin_view, int64_t n_tiles, LayerTable L,
    const ProjVert* __restrict__ proj, int64_t vpv, int slot, const uint32_t* __restrict__ count,
    const uint64_t* __restrict__ offset, const uint32_t* __restrict__ cursor, const int32_t* __restrict__ list,
    const SpanRec* __restrict__ spans, uint64_t capacity, unsigned long long* __restrict__ vis,
    unsigned long long* __restrict__ status, int count_frags) {
  constexpr int BH = bin_rows(B);              // bin rows
  constexpr int kSub = B < 8 ? B : 8;          // sub-tile edge of the depth bound
  constexpr int kNs = B / kSub;                // sub-tiles per row
  constexpr int kNsY = BH / kSub;              // sub-tile rows
  static_assert(B % kSub == 0 && BH % kSub == 0, "bins must be whole sub-tiles");
  __shared__ __align__(16) unsigned long long tile[B * BH];
  __shared__ unsigned long long smax[kNs * kNsY];
  __shared__ int32_t queue[2 * kRasterThreads];   // back-facing triangles that may lower a key
  __shared__ uint32_t qn;
  const int k = L.k;
  const int64_t n_bins = n_tiles * k;
  // XCD-contiguous remap of the block index
  const int64_t chunk = (n_bins + 7) / 8;
  const int64_t bid = ((int64_t)blockIdx.x % 8) * chunk + (int64_t)blockIdx.x / 8;
  if (bid >= n_bins) return;
  const int64_t g = bid / k;
  const int l = (int)(bid - g * k);
  const int v = bin_view[g];
  const vs_view& V = views[v];
  const int W = V.cam.width, H = V.cam.height;
  const int ntx = (W + B - 1) / B;
  const int64_t tl = g - V.tile_offset[slot];
  const int ty = (int)(tl / ntx), tx = (int)(tl - (int64_t)ty * ntx);
  const int x0 = tx * B, y0 = ty * BH;
  const int x1 = min(x0 + B, W) - 1, y1 = min(y0 + BH, H) - 1;
  const int tid = threadIdx.x, lane = tid & 63;
  for (int p = tid; p < B * BH / 2; p += kRasterThreads)   // 16-byte stores
    reinterpret_cast<ulonglong2*>(tile)[p] = make_ulonglong2(kEmpty, kEmpty);
  const ProjVert* P = proj + (int64_t)v * vpv + L.vert_off[l];
  const int32_t* tri = L.tri[l];
  const int32_t nvert = L.n_vert[l];
  const uint32_t cnt = count[bid];
  const bool overflow = offset[bid] + cnt > capacity;
  const uint32_t n = overflow ? (uint32_t)L.n_tri[l] : cnt;
  const int32_t* lst = list + (overflow ? 0 : offset[bid]);
  const SpanRec* srec = spans + (int64_t)v * L.tri_off[k] + L.tri_off[l];   // records of this view and layer
  // front-facing entries head the list (an overflowing bin scans its whole layer in one phase)
  const uint32_t n_front = (overflow || count_frags) ? n : min(cursor[2 * bid], cnt);
  unsigned long long frags = 0;
  __syncthreads();
  // Draw triangle t of this layer (t < 0: nothing).  Called by every thread of the block in
  // step (the wavefront path for large triangles loops over the wavefront's lanes).
  auto draw = [&](int32_t tq) {
    int32_t big = -1;   // a triangle for the whole wavefront
    TriSetup T;
    if (tq >= 0 && setup_triangle<true>(tri, (uint32_t)tq, nvert, P, T) == kTriOk) {
      const int32_t t = tq;
      PixRange pr = pixel_range(T, W, H);
      const int ci0 = max(pr.i0, x0), ci1 = min(pr.i1, x1), cj0 = max(pr.j0, y0), cj1 = min(pr.j1, y1);
      if (ci0 <= ci1 && cj0 <= cj1) {
        const unsigned long long lbkey = depth_lower_key(T, (uint32_t)t);
        const double spanx = fmax(T.X[0], fmax(T.X[1], T.X[2])) - fmin(T.X[0], fmin(T.X[1], T.X[2]));
        const double spany = fmax(T.Y[0], fmax(T.Y[1], T.Y[2])) - fmin(T.Y[0], fmin(T.Y[1], T.Y[2]));
        const int area = (ci1 - ci0 + 1) * (cj1 - cj0 + 1);
        if (spanx <= kSmallSpan && spany <= kSmallSpan && area <= kSmallArea) {
          // exact int32 edge walk: every edge value inside the bbox is below 2^30 in magnitude
          double E[3];
          edge_values(T, 256.0 * ci0 + 128.0, 256.0 * cj0 + 128.0, E);
          int32_t er0 = (int32_t)E[0] - (int32_t)T.th[0];
          int32_t er1 = (int32_t)E[1] - (int32_t)T.th[1];
          int32_t er2 = (int32_t)E[2] - (int32_t)T.th[2];
          const int32_t ax0 = (int32_t)(-(T.Y[2] - T.Y[1]) * 256.0), ay0 = (int32_t)((T.X[2] - T.X[1]) * 256.0);
          const int32_t ax1 = (int32_t)(-(T.Y[0] - T.Y[2]) * 256.0), ay1 = (int32_t)((T.X[0] - T.X[2]) * 256.0);
          const int32_t ax2 = (int32_t)(-(T.Y[1] - T.Y[0]) * 256.0), ay2 = (int32_t)((T.X[1] - T.X[0]) * 256.0);
          for (int j = cj0; j <= cj1; ++j) {
            int32_t e0 = er0, e1 = er1, e2 = er2;
            for (int i = ci0; i <= ci1; ++i) {
              if ((e0 | e1 | e2) >= 0) {
                unsigned long long* slotp = &tile[(j - y0) * B + (i - x0)];
                // keys only decrease, so a single-copy-atomic read at or below the bound proves a loss
                if (__hip_atomic_load(slotp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) > lbkey) {
                  const double E0 = (double)e0 + T.th[0], E1 = (double)e1 + T.th[1], E2 = (double)e2 + T.th[2];
                  atomicMin(slotp, (unsigned long long)depth_key(T, E0, E1, E2, (uint32_t)t));
                }
                ++frags;
              }
              e0 += ax0; e1 += ax1; e2 += ax2;
            }
            er0 += ay0; er1 += ay1; er2 += ay2;
          }
        } else {
          big = t;
        }
      }
    }
    for (uint64_t bm = __ballot(big >= 0); bm; bm &= bm - 1) {
      const int32_t t = __builtin_amdgcn_readlane(big, __builtin_ctzll(bm));
      TriSetup Tb;
      setup_triangle<true>(tri, (uint32_t)t, nvert, P, Tb);
      const unsigned long long lbkey = depth_lower_key(Tb, (uint32_t)t);
      for (int p = lane; p < B * BH; p += 64) {
        const int i = x0 + (p % B), j = y0 + (p / B);
        if (i > x1 || j > y1) continue;
        double E[3];
        edge_values(Tb, 256.0 * i + 128.0, 256.0 * j + 128.0, E);
        if (E[0] >= Tb.th[0] && E[1] >= Tb.th[1] && E[2] >= Tb.th[2]) {
          if (__hip_atomic_load(&tile[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) > lbkey)
            atomicMin(&tile[p], (unsigned long long)depth_key(Tb, E[0], E[1], E[2], (uint32_t)t));
          ++frags;
        }
      }
    }
  };
  // The first two chunks of back-facing entries and their records are requested before the
  // front-facing phase, so that their latency hides behind it.
  const uint4* srec4 = reinterpret_cast<const uint4*>(srec);
  const uint32_t cp0 = n_front + tid, cp1 = n_front + kRasterThreads + tid;
  const int32_t pt0 = cp0 < n ? lst[cp0] : -1, pt1 = cp1 < n ? lst[cp1] : -1;
  const uint4 pr0 = pt0 >= 0 ? srec4[pt0] : make_uint4(0u, 0u, 0u, 0u);
  const uint4 pr1 = pt1 >= 0 ? srec4[pt1] : make_uint4(0u, 0u, 0u, 0u);
  // phase 1: front-facing entries (every entry of an overflowing bin, or with fragment counting)
  for (uint32_t c0 = 0; c0 < n_front; c0 += kRasterThreads) {
    const uint32_t c = c0 + tid;
    draw(c < n_front ? (overflow ? (int32_t)c : lst[c]) : -1);
  }
  if (n_front < n) {   // uniform: back-facing entries follow
    if (tid == 0) qn = 0;
    __syncthreads();
    {
      // sub-tile maxima without LDS atomics: the kThr consecutive lanes of a sub-tile
      // each take kPer of its keys (whole row pieces) and combine by lane exchange
      constexpr int kSubs = kNs * kNsY;
      constexpr int kThr = kSubs * 64 <= kRasterThreads ? 64 : kSubs * 16 <= kRasterThreads ? 16 : 4;   // per sub-tile
      constexpr int kPer = kSub * kSub / kThr;                                                          // keys per thread
      static_assert(kSubs * kThr <= kRasterThreads && kSub * kSub % kThr == 0, "sub-tile reduction shape");
      if (tid < kSubs * kThr) {   // whole wavefronts
        const int sub = tid / kThr, u = tid % kThr;
        const int sx = sub % kNs, sy = sub / kNs;
        unsigned long long m = 0ull;
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
          const int kk = u * kPer + e;
          m = max(m, tile[(sy * kSub + kk / kSub) * B + sx * kSub + kk % kSub]);
        }
#pragma unroll
        for (int off = kThr / 2; off > 0; off >>= 1) m = max(m, (unsigned long long)__shfl_xor(m, off));
        if (u == 0) smax[sub] = m;
      }
    }
    __syncthreads();
    // phase 2: each back-facing entry is tested from its record (box and depth bound) alone;
    // the ones that may lower a key are queued in LDS and drawn 256 at a time, so that the
    // skipped majority costs no vertex loads and leaves no idle lanes behind.
    for (uint32_t c0 = n_front, chunk = 0; c0 < n; c0 += kRasterThreads, ++chunk) {
      const uint32_t c = c0 + tid;
      bool keep = false;
      int32_t t = 0;
      if (c < n) {
        uint4 r;
        if (chunk < 2) {   // uniform
          t = chunk == 0 ? pt0 : pt1;
          r = chunk == 0 ? pr0 : pr1;
        } else {
          t = lst[c];
          r = srec4[t];
        }
        int i0, i1, j0, j1;
        unpack_box((uint64_t)r.x | ((uint64_t)r.y << 32), i0, i1, j0, j1);
        const unsigned long long lb = ((unsigned long long)r.z << 32) | (uint32_t)t;
        const int ci0 = max(i0, x0), ci1 = min(i1, x1), cj0 = max(j0, y0), cj1 = min(j1, y1);
        for (int sj = (cj0 - y0) / kSub; sj <= (cj1 - y0) / kSub; ++sj)
          for (int si = (ci0 - x0) / kSub; si <= (ci1 - x0) / kSub; ++si)
            keep = keep || smax[sj * kNs + si] > lb;
      }
      const uint64_t kb = __ballot(keep);
      uint32_t base = 0;
      if (lane == 0 && kb) base = atomicAdd(&qn, (uint32_t)__popcll(kb));
      base = __builtin_amdgcn_readfirstlane(base);
      if (keep) queue[base + (uint32_t)__popcll(kb & __lanemask_lt())] = t;
      __syncthreads();
      uint32_t q = qn;
      const bool last = c0 + kRasterThreads >= n;
      while (q >= kRasterThreads || (last && q > 0)) {   // uniform
        draw(tid < (int)q ? queue[tid] : -1);
        const uint32_t rest = q > kRasterThreads ? q - kRasterThreads : 0;
        const int32_t moved = tid < (int)rest ? queue[kRasterThreads + tid] : 0;
        __syncthreads();
        if (tid < (int)rest) queue[tid] = moved;
        if (tid == 0) qn = rest;
        __syncthreads();
        q = rest;
      }
    }
  }
  __syncthreads();
  // coalesced store of the finished tile: pairs of keys as 16-byte stores when
  // every row of the bin starts 16-byte aligned (even view width and plane
  // start; x0 is even), single keys otherwise
  unsigned long long* plane = vis + (int64_t)k * V.pix_offset + (int64_t)l * W * H;
  if (B >= 2 && (W & 1) == 0 && (reinterpret_cast<uintptr_t>(plane) & 15) == 0) {   // uniform
    const ulonglong2* tile2 = reinterpret_cast<const ulonglong2*>(tile);
    for (int p = tid; p < B * BH / 2; p += kRasterThreads) {
      const int i = x0 + (2 * p) % B, j = y0 + (2 * p) / B;
      if (j > y1) continue;
      const ulonglong2 kv = tile2[p];
      unsigned long long* dst = plane + (int64_t)j * W + i;
      if (i + 1 <= x1) *reinterpret_cast<ulonglong2*>(dst) = kv;   // x1 - x0 + 1 is even unless W ends the row
      else if (i <= x1) dst[0] = kv.x;
    }
  } else {
    for (int p = tid; p < B * BH; p += kRasterThreads) {
      const int i = x0 + (p % B), j = y0 + (p / B);
      if (i <= x1 && j <= y1) plane[(int64_t)j * W + i] = tile[p];
    }
  }
  if (count_frags) {
    for (int off = 32; off > 0; off >>= 1) frags += __shfl_xor(frags, off);
    if ((tid & 63) == 0 && frags) atomicAdd(status + VS_STAT_FRAGMENTS, frags);
  }
  if (tid == 0 && overflow) atomicAdd(status + VS_STAT_BIN_OVERFLOW, 1ull);
}

// Steps 2-3, direct form (reference path for tests): one thread per (view,
// layer, triangle) walks its bounding box and takes 64-bit atomic minima in
// the visibility plane, which must hold EMPTY before.
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
  const int r = setup_triangle(L.tri[l], (uint32_t)t, L.n_vert[l], P, T);
  if (r != kTriOk) {
    atomicAdd(status + cull_slot(r), 1ull);
    return;
  }
  const PixRange pr = pixel_range(T, W, H);
  if (pr.i0 > pr.i1 || pr.j0 > pr.j1) return;
  unsigned long long* plane = vis + (int64_t)k * V.pix_offset + (int64_t)l * W * H;
  const double dx0 = -(T.Y[2] - T.Y[1]) * 256.0, dy0 = (T.X[2] - T.X[1]) * 256.0;
  const double dx1 = -(T.Y[0] - T.Y[2]) * 256.0, dy1 = (T.X[0] - T.X[2]) * 256.0;
  const double dx2 = -(T.Y[1] - T.Y[0]) * 256.0, dy2 = (T.X[1] - T.X[0]) * 256.0;
  double Er[3];
  edge_values(T, 256.0 * pr.i0 + 128.0, 256.0 * pr.j0 + 128.0, Er);
  unsigned long long frags = 0;
  for (int j = pr.j0; j <= pr.j1; ++j) {
    double E0 = Er[0], E1 = Er[1], E2 = Er[2];
    for (int i = pr.i0; i <= pr.i1; ++i) {
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

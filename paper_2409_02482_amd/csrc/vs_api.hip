// Host side of the C ABI declared in include/vs.h: argument validation,
// workspace layout and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "vs.h"
#include "vs_common.h"
#include "vs_raster.h"
#include "vs_shade.h"
#include "vs_sh.h"
#include "vs_fit.h"
#include "vs_ngp.h"
#include "vs_ksdf.h"

namespace {

thread_local std::string g_last_error;

vs_status fail(vs_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

vs_status ok() {
  g_last_error.clear();
  return VS_OK;
}

vs_status check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(VS_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  return VS_OK;
}

// Tile sizes of the four tile_offset slots: 16-pixel tiles shade, and the raster bins
// of size B are B wide and vs::bin_rows(B) high.
const int kTileW[4] = {8, 16, 32, 64};
const int kTileH[4] = {vs::bin_rows(8), vs::bin_rows(16), vs::bin_rows(32), vs::bin_rows(64)};

vs_status check_camera(const vs_camera& c, int v) {
  if (c.width < 1 || c.height < 1 || c.width > VS_MAX_VIEW_DIM || c.height > VS_MAX_VIEW_DIM)
    return fail(VS_ERR_SIZE, "view %d: size %dx%d outside 1..%d", v, c.width, c.height, VS_MAX_VIEW_DIM);
  const double vals[] = {c.fx, c.fy, c.cx, c.cy, c.z_near};
  for (double x : vals)
    if (!std::isfinite(x)) return fail(VS_ERR_ARG, "view %d: non-finite intrinsics", v);
  for (double x : c.R)
    if (!std::isfinite(x)) return fail(VS_ERR_ARG, "view %d: non-finite rotation", v);
  for (double x : c.t)
    if (!std::isfinite(x)) return fail(VS_ERR_ARG, "view %d: non-finite translation", v);
  if (!(c.z_near > 0.0)) return fail(VS_ERR_ARG, "view %d: z_near must be > 0", v);
  return VS_OK;
}

// Validate the view table: host copy consistent with its own cameras.
vs_status check_views(const vs_views* views) {
  if (!views || !views->host || !views->dev) return fail(VS_ERR_ARG, "views: null table");
  if (views->n_views < 1) return fail(VS_ERR_ARG, "views: n_views must be >= 1");
  int64_t pix = 0, tiles[4] = {0, 0, 0, 0};
  for (int v = 0; v <= views->n_views; ++v) {
    const vs_view& r = views->host[v];
    if (r.pix_offset != pix) return fail(VS_ERR_ARG, "views: record %d pix_offset mismatch (not prepared?)", v);
    for (int s = 0; s < 4; ++s)
      if (r.tile_offset[s] != tiles[s]) return fail(VS_ERR_ARG, "views: record %d tile_offset mismatch", v);
    if (v == views->n_views) break;
    vs_status st = check_camera(r.cam, v);
    if (st) return st;
    pix += (int64_t)r.cam.width * r.cam.height;
    for (int s = 0; s < 4; ++s)
      tiles[s] += (int64_t)((r.cam.width + kTileW[s] - 1) / kTileW[s]) * ((r.cam.height + kTileH[s] - 1) / kTileH[s]);
  }
  return VS_OK;
}

vs_status build_layers(const vs_mesh* layers, int32_t k, vs::LayerTable& L) {
  if (!layers) return fail(VS_ERR_ARG, "layers: null");
  if (k < 1 || k > VS_MAX_LAYERS) return fail(VS_ERR_SIZE, "k = %d outside 1..%d", k, VS_MAX_LAYERS);
  std::memset(&L, 0, sizeof(L));
  L.k = k;
  for (int l = 0; l < k; ++l) {
    const vs_mesh& m = layers[l];
    if (!m.xyz || !m.uv || !m.tri) return fail(VS_ERR_ARG, "layer %d: null mesh pointer", l);
    if (m.n_vert < 1 || m.n_tri < 1) return fail(VS_ERR_SIZE, "layer %d: empty mesh", l);
    if (m.n_vert > VS_MAX_LAYER_ELEMS || m.n_tri > VS_MAX_LAYER_ELEMS)
      return fail(VS_ERR_SIZE, "layer %d: more than %d vertices or triangles", l, VS_MAX_LAYER_ELEMS);
    L.xyz[l] = m.xyz;
    L.uv[l] = m.uv;
    L.tri[l] = m.tri;
    L.n_vert[l] = m.n_vert;
    L.n_tri[l] = m.n_tri;
    L.vert_off[l + 1] = L.vert_off[l] + m.n_vert;
    L.tri_off[l + 1] = L.tri_off[l] + m.n_tri;
    L.tri_pad[l + 1] = L.tri_pad[l] + ((int64_t)m.n_tri + 63) / 64 * 64;
  }
  for (int l = k + 1; l <= VS_MAX_LAYERS; ++l) {
    L.vert_off[l] = L.vert_off[k];
    L.tri_off[l] = L.tri_off[k];
    L.tri_pad[l] = L.tri_pad[k];
  }
  return VS_OK;
}

vs_status build_textures(const vs_texture* tex, int32_t k, vs::TexTable& X) {
  if (!tex) return fail(VS_ERR_ARG, "textures: null");
  std::memset(&X, 0, sizeof(X));
  for (int l = 0; l < k; ++l) {
    if (!tex[l].rgba) return fail(VS_ERR_ARG, "texture %d: null", l);
    if (tex[l].width < 1 || tex[l].height < 1 || tex[l].width > VS_MAX_TEX_DIM || tex[l].height > VS_MAX_TEX_DIM)
      return fail(VS_ERR_SIZE, "texture %d: size %dx%d outside 1..%d", l, tex[l].width, tex[l].height,
                  VS_MAX_TEX_DIM);
    X.tex[l] = reinterpret_cast<const float4*>(tex[l].rgba);
    X.w[l] = tex[l].width;
    X.h[l] = tex[l].height;
    X.inv_w[l] = 1.0 / tex[l].width;
    X.inv_h[l] = 1.0 / tex[l].height;
  }
  return VS_OK;
}

int bin_slot(int bin) { return bin == 8 ? 0 : bin == 16 ? 1 : bin == 32 ? 2 : bin == 64 ? 3 : -1; }

constexpr int kDefaultBin = 64;

vs::WsLayout ws_layout(const vs::LayerTable& L, const vs_views* views, int bin, int64_t capacity = 0) {
  vs::WsLayout w;
  const int n_views = views->n_views;
  w.bin = bin ? bin : kDefaultBin;
  w.slot = bin_slot(w.bin);
  const vs_view& tot = views->host[n_views];
  w.n_tiles16 = tot.tile_offset[1];
  w.n_tiles_bin = w.slot >= 0 ? tot.tile_offset[w.slot] : 0;
  w.n_bins = w.n_tiles_bin * L.k;
  w.n_partial = (w.n_bins + 1023) / 1024;
  const uint64_t tris = (uint64_t)n_views * (uint64_t)L.tri_off[L.k];
  const uint64_t factor = w.bin == 8 ? 4 : w.bin == 16 ? 3 : 2;
  w.capacity = capacity > 0 ? (uint64_t)capacity : std::max<uint64_t>(tris * factor, 1u << 20);
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += vs::align_up(bytes, 256); return o; };
  w.status = take(256);
  w.tile_view = take((size_t)w.n_tiles16 * 4);
  w.proj = take((size_t)n_views * (size_t)L.vert_off[L.k] * sizeof(vs::ProjVert));
  // everything below depends on the bin size; render and backward read only the part above
  w.bin_view = take((size_t)w.n_tiles_bin * 4);
  w.count = take((size_t)w.n_bins * 4);
  w.offset = take((size_t)w.n_bins * 8);
  w.cursor = take((size_t)w.n_bins * 8);
  w.spans = take((size_t)n_views * (size_t)L.tri_off[L.k] * sizeof(vs::SpanRec));
  w.partial = take((size_t)w.n_partial * 8);
  w.list = take((size_t)w.capacity * 4);
  w.total = off;
  return w;
}

vs_status check_ws(const void* ws, size_t ws_bytes, size_t need) {
  if (!ws) return fail(VS_ERR_WORKSPACE, "workspace: null");
  if ((uintptr_t)ws % 256) return fail(VS_ERR_WORKSPACE, "workspace: not 256-byte aligned");
  if (ws_bytes < need) return fail(VS_ERR_WORKSPACE, "workspace: %zu bytes given, %zu needed", ws_bytes, need);
  return VS_OK;
}

int64_t total_tiles(const vs_views* views, int slot) { return views->host[views->n_views].tile_offset[slot]; }

unsigned grid_1d(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

extern "C" {

const char* vs_version(void) { return "volsurf-gfx950 0.1"; }

const char* vs_last_error(void) { return g_last_error.c_str(); }

const char* vs_status_string(vs_status s) {
  switch (s) {
    case VS_OK: return "VS_OK";
    case VS_ERR_ARG: return "VS_ERR_ARG";
    case VS_ERR_SIZE: return "VS_ERR_SIZE";
    case VS_ERR_WORKSPACE: return "VS_ERR_WORKSPACE";
    case VS_ERR_HIP: return "VS_ERR_HIP";
    case VS_ERR_UNSUPPORTED: return "VS_ERR_UNSUPPORTED";
    default: return "VS_ERR_UNKNOWN";
  }
}

vs_status vs_views_prepare(const vs_camera* cams, int32_t n_views, vs_view* out) {
  if (!cams || !out) return fail(VS_ERR_ARG, "vs_views_prepare: null pointer");
  if (n_views < 1) return fail(VS_ERR_ARG, "vs_views_prepare: n_views must be >= 1");
  int64_t pix = 0, tiles[4] = {0, 0, 0, 0};
  for (int v = 0; v <= n_views; ++v) {
    vs_view& r = out[v];
    std::memset(&r, 0, sizeof(r));
    if (v < n_views) {
      vs_status st = check_camera(cams[v], v);
      if (st) return st;
      r.cam = cams[v];
    }
    r.pix_offset = pix;
    for (int s = 0; s < 4; ++s) r.tile_offset[s] = tiles[s];
    if (v == n_views) break;
    pix += (int64_t)cams[v].width * cams[v].height;
    for (int s = 0; s < 4; ++s)
      tiles[s] += (int64_t)((cams[v].width + kTileW[s] - 1) / kTileW[s]) *
                  ((cams[v].height + kTileH[s] - 1) / kTileH[s]);
  }
  return ok();
}

size_t vs_raster_workspace_bytes(const vs_mesh* layers, int32_t k, const vs_views* views,
                                 const vs_raster_opts* opts) {
  vs::LayerTable L;
  if (build_layers(layers, k, L) || check_views(views)) return 0;
  const int bin = opts ? opts->bin : 0;
  if (bin && bin_slot(bin) < 0) return 0;
  if (opts && opts->list_capacity < 0) return 0;
  return ws_layout(L, views, bin, opts ? opts->list_capacity : 0).total;
}

vs_status vs_raster_layers(const vs_mesh* layers, int32_t k, const vs_views* views, uint64_t* vis, void* ws,
                           size_t ws_bytes, const vs_raster_opts* opts, void* stream) {
  vs::LayerTable L;
  vs_status st = build_layers(layers, k, L);
  if (st) return st;
  if ((st = check_views(views))) return st;
  if (!vis) return fail(VS_ERR_ARG, "vis: null");
  const int bin = opts ? opts->bin : 0;
  if (bin && bin_slot(bin) < 0) return fail(VS_ERR_UNSUPPORTED, "bin = %d (use 0, 8, 16, 32 or 64)", bin);
  if ((uint64_t)views->n_views * (uint64_t)L.tri_off[k] >= (1ull << 30))
    return fail(VS_ERR_SIZE, "n_views * total triangles must be below 2^30");
  const int64_t cap = opts ? opts->list_capacity : 0;
  if (cap < 0 || cap >= (1ll << 32)) return fail(VS_ERR_SIZE, "list_capacity must be in [0, 2^32)");
  const vs::WsLayout lay = ws_layout(L, views, bin, cap);
  if ((st = check_ws(ws, ws_bytes, lay.total))) return st;
  const int flags = opts ? opts->flags : 0;
  const int count_frags = flags & VS_RASTER_COUNT_FRAGMENTS;
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  auto* status = (unsigned long long*)(base + lay.status);
  auto* proj = (vs::ProjVert*)(base + lay.proj);
  auto* tile_view = (int32_t*)(base + lay.tile_view);
  auto* bin_view = (int32_t*)(base + lay.bin_view);
  auto* count = (uint32_t*)(base + lay.count);
  auto* offset = (uint64_t*)(base + lay.offset);
  auto* cursor = (uint32_t*)(base + lay.cursor);
  auto* spans = (vs::SpanRec*)(base + lay.spans);
  auto* partial = (uint64_t*)(base + lay.partial);
  auto* list = (int32_t*)(base + lay.list);
  const int64_t vpv = L.vert_off[k];
  const int nv = views->n_views;
  const int64_t ntri = L.tri_off[k];
  hipLaunchKernelGGL(vs::k_fill_u64, dim3(1), dim3(256), 0, s, (uint64_t*)status, (int64_t)VS_STAT_COUNT, 0ull);
  hipLaunchKernelGGL(vs::k_tile_view, dim3(grid_1d(lay.n_tiles16, 256)), dim3(256), 0, s, views->dev, nv, tile_view,
                     lay.n_tiles16);
  hipLaunchKernelGGL(vs::k_project, dim3(grid_1d(vpv, 256), nv), dim3(256), 0, s, views->dev, L, proj, vpv);
  if (flags & VS_RASTER_DIRECT) {
    const int64_t total_slots = (int64_t)k * views->host[nv].pix_offset;
    hipLaunchKernelGGL(vs::k_fill_u64, dim3((unsigned)std::min<int64_t>(grid_1d(total_slots, 256), 65536)),
                       dim3(256), 0, s, vis, total_slots, (uint64_t)VS_EMPTY);
    hipLaunchKernelGGL(vs::k_raster_direct, dim3(grid_1d(ntri, 256), nv), dim3(256), 0, s, views->dev, L,
                       (const vs::ProjVert*)proj, vpv, (unsigned long long*)vis, status, count_frags);
    if ((st = check_launch("vs_raster_layers"))) return st;
    return ok();
  }
  const int B = lay.bin, slot = lay.slot;
  const unsigned fill_grid = (unsigned)std::min<int64_t>(grid_1d(lay.n_bins, 256), 65536);
  hipLaunchKernelGGL(vs::k_tile_view_slot, dim3(grid_1d(lay.n_tiles_bin, 256)), dim3(256), 0, s, views->dev, nv,
                     bin_view, lay.n_tiles_bin, slot);
  hipLaunchKernelGGL(vs::k_fill_u32, dim3(fill_grid), dim3(256), 0, s, count, lay.n_bins, 0u);
  hipLaunchKernelGGL(vs::k_fill_u32, dim3(fill_grid), dim3(256), 0, s, cursor, 2 * lay.n_bins, 0u);
  const dim3 count_grid(vs::bin_grid_x<vs::kCountReps>(L.tri_pad[k]), (unsigned)nv);
  const dim3 scatter_grid(vs::bin_grid_x<vs::kScatterReps>(L.tri_pad[k]), (unsigned)nv);
  auto bin_count = [&](auto kern) {
    hipLaunchKernelGGL(kern, count_grid, dim3(256), 0, s, views->dev, L, (const vs::ProjVert*)proj, vpv, slot, count,
                       cursor, spans, status);
  };
  auto bin_scatter = [&](auto kern) {
    hipLaunchKernelGGL(kern, scatter_grid, dim3(256), 0, s, views->dev, L, slot, (const vs::SpanRec*)spans,
                       (const uint32_t*)count, (const uint64_t*)offset, cursor, list, lay.capacity);
  };
  switch (B) {
    case 8: bin_count(vs::k_bin_count<8>); break;
    case 16: bin_count(vs::k_bin_count<16>); break;
    case 32: bin_count(vs::k_bin_count<32>); break;
    default: bin_count(vs::k_bin_count<64>); break;
  }
  hipLaunchKernelGGL(vs::k_scan_local, dim3((unsigned)lay.n_partial), dim3(256), 0, s, count,
                     (const uint32_t*)cursor, offset, partial, lay.n_bins);
  hipLaunchKernelGGL(vs::k_scan_partials, dim3(1), dim3(1024), 0, s, partial, lay.n_partial);
  hipLaunchKernelGGL(vs::k_scan_add, dim3(grid_1d(lay.n_bins, 256)), dim3(256), 0, s, offset,
                     (const uint64_t*)partial, lay.n_bins);
  switch (B) {
    case 8: bin_scatter(vs::k_bin_scatter<8>); break;
    case 16: bin_scatter(vs::k_bin_scatter<16>); break;
    case 32: bin_scatter(vs::k_bin_scatter<32>); break;
    default: bin_scatter(vs::k_bin_scatter<64>); break;
  }
  const unsigned nblk = (unsigned)((lay.n_bins + 7) / 8 * 8);
  auto raster = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(nblk), dim3(vs::kRasterThreads), 0, s, views->dev, (const int32_t*)bin_view,
                       lay.n_tiles_bin, L, (const vs::ProjVert*)proj, vpv, slot, (const uint32_t*)count,
                       (const uint64_t*)offset, (const uint32_t*)cursor, (const int32_t*)list,
                       (const vs::SpanRec*)spans, lay.capacity, (unsigned long long*)vis, status, count_frags);
  };
  switch (B) {
    case 8: raster(vs::k_raster_bins<8>); break;
    case 16: raster(vs::k_raster_bins<16>); break;
    case 32: raster(vs::k_raster_bins<32>); break;
    default: raster(vs::k_raster_bins<64>); break;
  }
  if ((st = check_launch("vs_raster_layers"))) return st;
  return ok();
}

vs_status vs_render(const vs_mesh* layers, const vs_texture* tex, int32_t k, const vs_views* views,
                    const uint64_t* vis, const void* ws, size_t ws_bytes, float* out_rgba,
                    const vs_shade_opts* opts, void* stream) {
  vs::LayerTable L;
  vs::TexTable X;
  vs_status st = build_layers(layers, k, L);
  if (st) return st;
  if ((st = build_textures(tex, k, X))) return st;
  if ((st = check_views(views))) return st;
  if (!vis || !out_rgba) return fail(VS_ERR_ARG, "vis/out_rgba: null");
  const vs::WsLayout lay = ws_layout(L, views, 0);
  if ((st = check_ws(ws, ws_bytes, lay.proj + (size_t)views->n_views * L.vert_off[k] * sizeof(vs::ProjVert))))
    return st;
  const float eps = opts ? opts->eps_T : 0.0f;
  const int wrap = opts ? opts->wrap : 0;
  if (wrap != 0 && wrap != 1) return fail(VS_ERR_UNSUPPORTED, "wrap = %d", wrap);
  if (!(eps >= 0.0f && eps < 1.0f)) return fail(VS_ERR_ARG, "eps_T must be in [0, 1)");
  const char* base = (const char*)ws;
  auto* status = (unsigned long long*)(base + lay.status);
  const auto* proj = (const vs::ProjVert*)(base + lay.proj);
  hipStream_t s = (hipStream_t)stream;
  const int64_t tiles = total_tiles(views, vs::kShadeTileSlot);
  const auto* tile_view = (const int32_t*)(base + lay.tile_view);
  hipLaunchKernelGGL(vs::k_shade_fwd, dim3((unsigned)vs::shade_grid_blocks(tiles)), dim3(256), 0, s, views->dev,
                     views->n_views, tile_view, tiles, L, X, proj, L.vert_off[k], vis, (float4*)out_rgba, eps, wrap,
                     status);
  if ((st = check_launch("vs_render"))) return st;
  return ok();
}

}  // extern "C"

// ------------------------------------------------------------------ no-alloc entry point

// The workspace of vs_render_noalloc.  In host code this name is only a
// stand-in for the device symbol: kernels and copies get the per-device
// address that hipGetSymbolAddress returns, never the name itself.
static __device__ __align__(256) unsigned char scratch[VS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];   // device address of `scratch` on each device, looked up once

vs_status scratch_for_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(VS_ERR_HIP, "vs_render_noalloc: hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(VS_ERR_HIP, "vs_render_noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(VS_ERR_HIP, "vs_render_noalloc: hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    if ((uintptr_t)p % 256) return fail(VS_ERR_HIP, "vs_render_noalloc: scratch not 256-byte aligned");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return VS_OK;
}

}  // namespace

extern "C" {

vs_status vs_render_noalloc(const vs_mesh* layers, const vs_texture* tex, int32_t k, const vs_views* views,
                            uint64_t* vis, float* out_rgba, const vs_raster_opts* raster_opts,
                            const vs_shade_opts* shade_opts, void* stream) {
  // everything both calls check is checked here first, so that an error enqueues nothing
  vs::LayerTable L;
  vs::TexTable X;
  vs_status st = build_layers(layers, k, L);
  if (st) return st;
  if ((st = build_textures(tex, k, X))) return st;
  if ((st = check_views(views))) return st;
  if (!vis || !out_rgba) return fail(VS_ERR_ARG, "vis/out_rgba: null");
  const int bin = raster_opts ? raster_opts->bin : 0;
  if (bin && bin_slot(bin) < 0) return fail(VS_ERR_UNSUPPORTED, "bin = %d (use 0, 8, 16, 32 or 64)", bin);
  const int64_t cap = raster_opts ? raster_opts->list_capacity : 0;
  if (cap < 0 || cap >= (1ll << 32)) return fail(VS_ERR_SIZE, "list_capacity must be in [0, 2^32)");
  if ((uint64_t)views->n_views * (uint64_t)L.tri_off[k] >= (1ull << 30))
    return fail(VS_ERR_SIZE, "n_views * total triangles must be below 2^30");
  const int wrap = shade_opts ? shade_opts->wrap : 0;
  if (wrap != 0 && wrap != 1) return fail(VS_ERR_UNSUPPORTED, "wrap = %d", wrap);
  const float eps = shade_opts ? shade_opts->eps_T : 0.0f;
  if (!(eps >= 0.0f && eps < 1.0f)) return fail(VS_ERR_ARG, "eps_T must be in [0, 1)");
  const size_t need = ws_layout(L, views, bin, cap).total;
  if (need > (size_t)VS_NOALLOC_SCRATCH_BYTES)
    return fail(VS_ERR_WORKSPACE, "vs_render_noalloc: %zu workspace bytes needed, the static scratch holds %llu",
                need, (unsigned long long)VS_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  if ((st = scratch_for_current_device(&ws))) return st;
  if ((st = vs_raster_layers(layers, k, views, vis, ws, (size_t)VS_NOALLOC_SCRATCH_BYTES, raster_opts, stream)))
    return st;
  if ((st = vs_render(layers, tex, k, views, vis, ws, (size_t)VS_NOALLOC_SCRATCH_BYTES, out_rgba, shade_opts,
                      stream)))
    return st;
  return ok();
}

vs_status vs_render_sh(const vs_mesh* layers, const vs_sh_texture* tex, int32_t k, const vs_views* views,
                       const uint64_t* vis, const void* ws, size_t ws_bytes, float* out_rgba,
                       const vs_sh_opts* opts, void* stream) {
  vs::LayerTable L;
  vs_status st = build_layers(layers, k, L);
  if (st) return st;
  if ((st = check_views(views))) return st;
  if (!vis || !out_rgba) return fail(VS_ERR_ARG, "vis/out_rgba: null");
  if (!opts) return fail(VS_ERR_ARG, "vs_render_sh: opts must not be NULL");
  if (!tex) return fail(VS_ERR_ARG, "SH textures: null");
  const int deg = opts->degree;
  if (deg < 0 || deg > 3) return fail(VS_ERR_UNSUPPORTED, "SH degree %d outside 0..3", deg);
  if (opts->wrap != 0 && opts->wrap != 1) return fail(VS_ERR_UNSUPPORTED, "wrap = %d", opts->wrap);
  if (opts->view_alpha != 0 && opts->view_alpha != 1) return fail(VS_ERR_ARG, "view_alpha must be 0 or 1");
  if (!(opts->eps_T >= 0.0f && opts->eps_T < 1.0f)) return fail(VS_ERR_ARG, "eps_T must be in [0, 1)");
  if (!(std::isfinite(opts->vmin) && std::isfinite(opts->vmax) && opts->vmin < opts->vmax))
    return fail(VS_ERR_ARG, "need finite vmin < vmax");
  vs::ShTable S;
  std::memset(&S, 0, sizeof(S));
  for (int l = 0; l < k; ++l) {
    const vs_sh_texture& t = tex[l];
    if (!t.data) return fail(VS_ERR_ARG, "SH texture %d: null", l);
    if ((uintptr_t)t.data % 4) return fail(VS_ERR_ARG, "SH texture %d: data not 4-byte aligned", l);
    if (t.width < 1 || t.height < 1 || t.width > VS_MAX_TEX_DIM || t.height > VS_MAX_TEX_DIM)
      return fail(VS_ERR_SIZE, "SH texture %d: size %dx%d outside 1..%d", l, t.width, t.height, VS_MAX_TEX_DIM);
    S.data[l] = t.data;
    int64_t off = 0;
    for (int d = 0; d < vs::kShLevels; ++d) {
      const int32_t w = std::max(1, t.width >> d), h = std::max(1, t.height >> d);
      S.w[l][d] = w;
      S.h[l][d] = h;
      S.off[l][d] = off;
      S.inv_w[l][d] = 1.0 / w;
      S.inv_h[l][d] = 1.0 / h;
      off += (int64_t)w * h * (2 * d + 1) * 4;
    }
  }
  const vs::WsLayout lay = ws_layout(L, views, 0);
  if ((st = check_ws(ws, ws_bytes, lay.proj + (size_t)views->n_views * L.vert_off[k] * sizeof(vs::ProjVert))))
    return st;
  vs::ShParams prm;
  prm.mid = 0.5f * (opts->vmin + opts->vmax);
  prm.scale = (opts->vmax - opts->vmin) / 255.0f;
  prm.eps_T = opts->eps_T;
  prm.wrap = opts->wrap;
  prm.view_alpha = opts->view_alpha;
  const char* base = (const char*)ws;
  auto* status = (unsigned long long*)(base + lay.status);
  const auto* proj = (const vs::ProjVert*)(base + lay.proj);
  const auto* tile_view = (const int32_t*)(base + lay.tile_view);
  hipStream_t s = (hipStream_t)stream;
  const int64_t tiles = total_tiles(views, vs::kShadeTileSlot);
  auto launch = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)vs::shade_grid_blocks(tiles)), dim3(256), 0, s, views->dev,
                       views->n_views, tile_view, tiles, L, S, proj, L.vert_off[k], vis, (float4*)out_rgba, prm,
                       status);
  };
  switch (deg) {
    case 0: launch(vs::k_shade_sh<0>); break;
    case 1: launch(vs::k_shade_sh<1>); break;
    case 2: launch(vs::k_shade_sh<2>); break;
    default: launch(vs::k_shade_sh<3>); break;
  }
  if ((st = check_launch("vs_render_sh"))) return st;
  return ok();
}

vs_status vs_render_backward(const vs_mesh* layers, const vs_texture* tex, int32_t k, const vs_views* views,
                             const uint64_t* vis, const void* ws, size_t ws_bytes, const float* grad_rgba,
                             float* const* grad_tex, float* out_rgba, double* sse, const vs_shade_opts* opts,
                             void* stream) {
  vs::LayerTable L;
  vs::TexTable X;
  vs_status st = build_layers(layers, k, L);
  if (st) return st;
  if ((st = build_textures(tex, k, X))) return st;
  if ((st = check_views(views))) return st;
  if (!vis) return fail(VS_ERR_ARG, "vis: null");
  if (!grad_tex) return fail(VS_ERR_ARG, "grad_tex: null");
  for (int l = 0; l < k; ++l) {
    if (!grad_tex[l]) return fail(VS_ERR_ARG, "grad_tex[%d]: null", l);
    X.grad[l] = grad_tex[l];
  }
  const float* target = opts ? opts->target : nullptr;
  if (!target && !grad_rgba) return fail(VS_ERR_ARG, "need grad_rgba or opts->target");
  const float scale = opts ? opts->loss_scale : 1.0f;
  const int wrap = opts ? opts->wrap : 0;
  if (wrap != 0 && wrap != 1) return fail(VS_ERR_UNSUPPORTED, "wrap = %d", wrap);
  const int loss = opts ? opts->loss : VS_LOSS_L2;
  if (loss != VS_LOSS_L2 && loss != VS_LOSS_L1) return fail(VS_ERR_UNSUPPORTED, "loss = %d", loss);
  const float eps = opts ? opts->eps_T : 0.0f;
  if (!(eps >= 0.0f && eps < 1.0f)) return fail(VS_ERR_ARG, "eps_T must be in [0, 1)");
  const int sflags = opts ? opts->flags : 0;
  if (sflags & ~VS_SHADE_COUNT_PATHS) return fail(VS_ERR_UNSUPPORTED, "shade flags = %d", sflags);
  const vs::WsLayout lay = ws_layout(L, views, 0);
  if ((st = check_ws(ws, ws_bytes, lay.proj + (size_t)views->n_views * L.vert_off[k] * sizeof(vs::ProjVert))))
    return st;
  const char* base = (const char*)ws;
  auto* status = (unsigned long long*)(base + lay.status);
  const auto* proj = (const vs::ProjVert*)(base + lay.proj);
  hipStream_t s = (hipStream_t)stream;
  const int64_t tiles = total_tiles(views, vs::kShadeTileSlot);
  const auto* tile_view = (const int32_t*)(base + lay.tile_view);
  const int count_paths = sflags & VS_SHADE_COUNT_PATHS;
  auto launch = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)vs::shade_grid_blocks(tiles)), dim3(256), 0, s, views->dev,
                       views->n_views, tile_view, tiles, L, X, proj,
                       L.vert_off[k], vis, (const float4*)grad_rgba, (const float4*)target, scale, loss,
                       (float4*)out_rgba, target ? sse : nullptr, wrap, eps, status, count_paths);
  };
  // per-layer state lives in registers, so the common layer counts get their own instantiation
  if (k <= 4) launch(vs::k_shade_bwd<4>);
  else if (k <= 7) launch(vs::k_shade_bwd<7>);
  else if (k <= 8) launch(vs::k_shade_bwd<8>);
  else if (k <= 9) launch(vs::k_shade_bwd<9>);
  else launch(vs::k_shade_bwd<16>);
  if ((st = check_launch("vs_render_backward"))) return st;
  return ok();
}

vs_status vs_read_status(const void* ws, size_t ws_bytes, int64_t* out, void* stream) {
  if (!ws || !out) return fail(VS_ERR_ARG, "vs_read_status: null pointer");
  if (ws_bytes < 256) return fail(VS_ERR_WORKSPACE, "workspace too small");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(out, ws, VS_STAT_COUNT * sizeof(int64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(VS_ERR_HIP, "vs_read_status: %s", hipGetErrorString(e));
  return ok();
}

}  // extern "C"

// ------------------------------------------------------------------ autotune

namespace {

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

uint64_t problem_key(const vs::LayerTable& L, const vs_views* views) {
  uint64_t h = 1469598103934665603ull;
  h = fnv1a(h, &L.k, sizeof(L.k));
  for (int l = 0; l < L.k; ++l) {
    h = fnv1a(h, &L.n_vert[l], 4);
    h = fnv1a(h, &L.n_tri[l], 4);
  }
  h = fnv1a(h, &views->n_views, 4);
  for (int v = 0; v < views->n_views; ++v) {
    h = fnv1a(h, &views->host[v].cam.width, 4);
    h = fnv1a(h, &views->host[v].cam.height, 4);
  }
  return h;
}

int cache_lookup(const char* path, uint64_t key) {
  if (!path) return 0;
  std::ifstream f(path);
  std::string line;
  int found = 0;
  while (std::getline(f, line)) {
    std::istringstream ss(line);
    std::string hex;
    int bin = 0;
    if (ss >> hex >> bin && std::strtoull(hex.c_str(), nullptr, 16) == key && bin_slot(bin) >= 0) found = bin;
  }
  return found;
}

}  // namespace

extern "C" vs_status vs_autotune(const vs_mesh* layers, int32_t k, const vs_views* views, uint64_t* vis, void* ws,
                                 size_t ws_bytes, vs_raster_opts* inout, const char* cache_path, void* stream) {
  vs::LayerTable L;
  vs_status st = build_layers(layers, k, L);
  if (st) return st;
  if ((st = check_views(views))) return st;
  if (!inout || !vis || !ws) return fail(VS_ERR_ARG, "vs_autotune: null pointer");
  const uint64_t key = problem_key(L, views);
  const int cached = cache_lookup(cache_path, key);
  if (cached) {
    inout->bin = cached;
    return ok();
  }
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(VS_ERR_HIP, "vs_autotune: hipEventCreate failed");
  const int cands[4] = {8, 16, 32, 64};
  float best_ms = 1e30f;
  int best = 0;
  unsigned long long ref_sum = 0;
  bool have_ref = false;
  const int64_t n_slots = (int64_t)k * views->host[views->n_views].pix_offset;
  // checksum scratch: the last 8 bytes of the 256-byte status slot (beyond the VS_STAT_COUNT counters)
  auto* sum_dev = (unsigned long long*)((char*)ws + 31 * sizeof(unsigned long long));
  vs_status result = VS_OK;
  for (int ci = 0; ci < 4 && result == VS_OK; ++ci) {
    vs_raster_opts o = *inout;
    o.bin = cands[ci];
    o.flags &= ~VS_RASTER_DIRECT;
    if (ws_layout(L, views, o.bin, o.list_capacity).total > ws_bytes) continue;
    float ms = 1e30f;
    for (int rep = 0; rep < 4 && result == VS_OK; ++rep) {
      if (hipEventRecord(e0, s) != hipSuccess) { result = fail(VS_ERR_HIP, "vs_autotune: event record failed"); break; }
      result = vs_raster_layers(layers, k, views, vis, ws, ws_bytes, &o, stream);
      if (result != VS_OK) break;
      float t = 0.f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&t, e0, e1) != hipSuccess)
        result = fail(VS_ERR_HIP, "vs_autotune: event timing failed");
      if (rep > 0) ms = std::min(ms, t);
    }
    if (result != VS_OK) break;
    hipLaunchKernelGGL(vs::k_fill_u64, dim3(1), dim3(64), 0, s, (uint64_t*)sum_dev, (int64_t)1, 0ull);
    hipLaunchKernelGGL(vs::k_vis_checksum, dim3(1024), dim3(256), 0, s, (const uint64_t*)vis, n_slots, sum_dev);
    unsigned long long sum = 0;
    if (hipMemcpyAsync(&sum, sum_dev, 8, hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
      result = fail(VS_ERR_HIP, "vs_autotune: checksum copy failed");
    if (result != VS_OK) break;
    if (!have_ref) { ref_sum = sum; have_ref = true; }
    else if (sum != ref_sum) result = fail(VS_ERR_HIP, "vs_autotune: bin %d gives a different visibility buffer", o.bin);
    if (ms < best_ms) { best_ms = ms; best = o.bin; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (result != VS_OK) return result;
  if (!best) return fail(VS_ERR_WORKSPACE, "vs_autotune: no bin size fits the workspace");
  // leave vis holding the chosen configuration's result (identical for every bin)
  inout->bin = best;
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::app);
    char line[64];
    snprintf(line, sizeof(line), "%016llx %d\n", (unsigned long long)key, best);
    f << line;
  }
  return ok();
}

// ------------------------------------------------------------------ fitting

namespace {

// Per-layer buffers of a fitting step; any of the pointer arrays may be absent (NULL) when unused.
vs_status build_adam(const char* who, float* const* params, float* const* grads, float* const* m, float* const* v,
                     float* const* tex, const int64_t* counts, int32_t k, vs::AdamTable& A, vs::TexOut& T) {
  if (!params || !counts) return fail(VS_ERR_ARG, "%s: null pointer", who);
  if (k < 1 || k > VS_MAX_LAYERS) return fail(VS_ERR_SIZE, "%s: k = %d", who, k);
  std::memset(&A, 0, sizeof(A));
  std::memset(&T, 0, sizeof(T));
  A.k = k;
  for (int l = 0; l < k; ++l) {
    const float* bufs[5] = {params[l], grads ? grads[l] : nullptr, m ? m[l] : nullptr, v ? v[l] : nullptr,
                            tex ? tex[l] : nullptr};
    const bool need[5] = {true, grads != nullptr, m != nullptr, v != nullptr, tex != nullptr};
    for (int b = 0; b < 5; ++b) {
      if (!need[b]) continue;
      if (!bufs[b]) return fail(VS_ERR_ARG, "%s: layer %d null", who, l);
      if ((uintptr_t)bufs[b] % 16) return fail(VS_ERR_ARG, "%s: layer %d buffer not 16-byte aligned", who, l);
    }
    if (counts[l] <= 0 || counts[l] % 4) return fail(VS_ERR_SIZE, "%s: count %d not a positive multiple of 4", who, l);
    A.p[l] = params[l];
    if (grads) A.g[l] = grads[l];
    if (m) A.m[l] = m[l];
    if (v) A.v[l] = v[l];
    if (tex) T.t[l] = tex[l];
    A.off[l + 1] = A.off[l] + counts[l];
  }
  for (int l = k + 1; l <= VS_MAX_LAYERS; ++l) A.off[l] = A.off[k];
  return VS_OK;
}

vs_status check_adam_opts(const char* who, const vs_adam_opts* opts) {
  if (!opts) return fail(VS_ERR_ARG, "%s: null opts", who);
  if (!(opts->lr >= 0.f) || !(opts->beta1 >= 0.f && opts->beta1 < 1.f) || !(opts->beta2 >= 0.f && opts->beta2 < 1.f) ||
      !(opts->eps > 0.f) || !(opts->lo <= opts->hi))
    return fail(VS_ERR_ARG, "%s: bad hyper-parameters", who);
  return VS_OK;
}

unsigned adam_grid(const vs::AdamTable& A) {
  return (unsigned)std::min<int64_t>(grid_1d(A.off[A.k] / 4, 256), 8192);
}

}  // namespace

extern "C" vs_status vs_adam_step(float* const* params, float* const* grads, float* const* m, float* const* v,
                                  const int64_t* counts, int32_t k, const vs_adam_opts* opts, int32_t* step,
                                  double* sse, double* history, int32_t hist_len, void* stream) {
  if (!grads || !m || !v || !step) return fail(VS_ERR_ARG, "vs_adam_step: null pointer");
  vs::AdamTable A;
  vs::TexOut T;
  vs_status st = build_adam("vs_adam_step", params, grads, m, v, nullptr, counts, k, A, T);
  if (st) return st;
  if ((st = check_adam_opts("vs_adam_step", opts))) return st;
  if (history && hist_len < 0) return fail(VS_ERR_ARG, "vs_adam_step: hist_len < 0");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(vs::k_adam, dim3(adam_grid(A)), dim3(256), 0, s, A, opts->lr, opts->beta1, opts->beta2, opts->eps,
                     opts->lo, opts->hi, (const int32_t*)step);
  hipLaunchKernelGGL(vs::k_fit_bookkeep, dim3(1), dim3(64), 0, s, sse, history, hist_len, step);
  if ((st = check_launch("vs_adam_step"))) return st;
  return ok();
}

extern "C" vs_status vs_squeeze(const float* const* params, float* const* tex, const int64_t* counts, int32_t k,
                                int32_t levels, void* stream) {
  if (!tex) return fail(VS_ERR_ARG, "vs_squeeze: null tex");
  if (levels < 0 || levels > 65535) return fail(VS_ERR_ARG, "vs_squeeze: levels = %d outside 0..65535", levels);
  vs::AdamTable A;
  vs::TexOut T;
  vs_status st = build_adam("vs_squeeze", const_cast<float* const*>(params), nullptr, nullptr, nullptr, tex, counts, k,
                            A, T);
  if (st) return st;
  hipLaunchKernelGGL(vs::k_squeeze, dim3(adam_grid(A)), dim3(256), 0, (hipStream_t)stream, A, T, (int)levels);
  if ((st = check_launch("vs_squeeze"))) return st;
  return ok();
}

extern "C" vs_status vs_adam_step_squeezed(float* const* params, float* const* grads, float* const* m, float* const* v,
                                           float* const* tex, const int64_t* counts, int32_t k, int32_t levels,
                                           const vs_adam_opts* opts, int32_t* step, double* sse, double* history,
                                           int32_t hist_len, void* stream) {
  if (!grads || !m || !v || !tex || !step) return fail(VS_ERR_ARG, "vs_adam_step_squeezed: null pointer");
  if (levels < 0 || levels > 65535) return fail(VS_ERR_ARG, "vs_adam_step_squeezed: levels = %d outside 0..65535", levels);
  vs::AdamTable A;
  vs::TexOut T;
  vs_status st = build_adam("vs_adam_step_squeezed", params, grads, m, v, tex, counts, k, A, T);
  if (st) return st;
  if ((st = check_adam_opts("vs_adam_step_squeezed", opts))) return st;
  if (history && hist_len < 0) return fail(VS_ERR_ARG, "vs_adam_step_squeezed: hist_len < 0");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(vs::k_adam_squeezed, dim3(adam_grid(A)), dim3(256), 0, s, A, T, opts->lr, opts->beta1,
                     opts->beta2, opts->eps, (int)levels, (const int32_t*)step);
  hipLaunchKernelGGL(vs::k_fit_bookkeep, dim3(1), dim3(64), 0, s, sse, history, hist_len, step);
  if ((st = check_launch("vs_adam_step_squeezed"))) return st;
  return ok();
}

// ------------------------------------------------------------------ neural textures

namespace {

vs_status ngp_shape(const vs_ngp_config* cfg, vs::NgpShape& S) {
  if (!cfg) return fail(VS_ERR_ARG, "vs_ngp: null config");
  if (cfg->levels < 1 || cfg->levels > VS_NGP_MAX_LEVELS) return fail(VS_ERR_SIZE, "vs_ngp: levels = %d", cfg->levels);
  if (cfg->log2_table < 4 || cfg->log2_table > 24) return fail(VS_ERR_SIZE, "vs_ngp: log2_table = %d", cfg->log2_table);
  std::memset(&S, 0, sizeof(S));
  S.levels = cfg->levels;
  S.log2_table = cfg->log2_table;
  const int64_t T = (int64_t)1 << cfg->log2_table;
  for (int l = 0; l < cfg->levels; ++l) {
    const int32_t n = cfg->resolution[l];
    if (n < 1 || n > 65535) return fail(VS_ERR_SIZE, "vs_ngp: resolution[%d] = %d outside 1..65535", l, n);
    S.res[l] = n;
    S.dense[l] = (int64_t)(n + 1) * (n + 1) <= T;
  }
  const int64_t H = vs::kNgpHidden, O = vs::kNgpOut, in = 2 * (int64_t)cfg->levels;
  S.o_w1 = (int64_t)cfg->levels * T * 2;
  S.o_b1 = S.o_w1 + H * in;
  S.o_w2 = S.o_b1 + H;
  S.o_b2 = S.o_w2 + H * H;
  S.o_w3 = S.o_b2 + H;
  S.o_b3 = S.o_w3 + O * H;
  S.total = S.o_b3 + O;
  return VS_OK;
}

vs_status ngp_table(const char* who, const float* const* params, int32_t k, const int32_t* width,
                    const int32_t* height, vs::NgpTable& T) {
  if (!params || !width || !height) return fail(VS_ERR_ARG, "%s: null pointer", who);
  if (k < 1 || k > VS_MAX_LAYERS) return fail(VS_ERR_SIZE, "%s: k = %d", who, k);
  std::memset(&T, 0, sizeof(T));
  T.k = k;
  for (int l = 0; l < k; ++l) {
    if (!params[l]) return fail(VS_ERR_ARG, "%s: params[%d] null", who, l);
    if ((uintptr_t)params[l] % 16) return fail(VS_ERR_ARG, "%s: params[%d] not 16-byte aligned", who, l);
    if (width[l] < 1 || height[l] < 1 || width[l] > VS_MAX_TEX_DIM || height[l] > VS_MAX_TEX_DIM)
      return fail(VS_ERR_SIZE, "%s: texture %d size %dx%d", who, l, width[l], height[l]);
    T.params[l] = params[l];
    T.w[l] = width[l];
    T.h[l] = height[l];
    const int64_t tiles = (int64_t)((width[l] + vs::kNgpTile - 1) / vs::kNgpTile) *
                          ((height[l] + vs::kNgpTile - 1) / vs::kNgpTile);
    T.block_off[l + 1] = T.block_off[l] + tiles;
  }
  for (int l = k + 1; l <= VS_MAX_LAYERS; ++l) T.block_off[l] = T.block_off[k];
  return VS_OK;
}

struct NgpWs {
  size_t a1, a2, a3, d1, d2, d0, total;
};

// rows: 256 per texel tile of every layer
NgpWs ngp_ws(const vs::NgpShape& S, int64_t rows) {
  NgpWs w;
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += (bytes + 255) / 256 * 256; return o; };
  w.a1 = take((size_t)rows * 2 * S.levels * 4);
  w.a2 = take((size_t)rows * vs::kNgpHidden * 4);
  w.a3 = take((size_t)rows * vs::kNgpHidden * 4);
  w.d1 = take((size_t)rows * vs::kNgpHidden * 4);
  w.d2 = take((size_t)rows * vs::kNgpHidden * 4);
  w.d0 = take((size_t)rows * vs::kNgpOut * 4);
  w.total = off;
  return w;
}

int64_t ngp_rows(const int32_t* width, const int32_t* height, int32_t k) {
  int64_t rows = 0;
  for (int l = 0; l < k; ++l)
    rows += (int64_t)((std::max(width[l], 0) + vs::kNgpTile - 1) / vs::kNgpTile) *
            ((std::max(height[l], 0) + vs::kNgpTile - 1) / vs::kNgpTile) * 256;
  return rows;
}

}  // namespace

extern "C" int64_t vs_ngp_param_count(const vs_ngp_config* cfg) {
  vs::NgpShape S;
  if (ngp_shape(cfg, S)) return -1;
  return S.total;
}

extern "C" size_t vs_ngp_workspace_bytes(const vs_ngp_config* cfg, int32_t k, const int32_t* width,
                                         const int32_t* height) {
  vs::NgpShape S;
  if (ngp_shape(cfg, S) || !width || !height || k < 1 || k > VS_MAX_LAYERS) return 0;
  return ngp_ws(S, ngp_rows(width, height, k)).total;
}

vs::NgpStage ngp_stage(void* ws, const NgpWs& w, int64_t rows) {
  char* base = (char*)ws;
  vs::NgpStage G;
  G.R = rows;
  G.a1 = (float*)(base + w.a1);
  G.a2 = (float*)(base + w.a2);
  G.a3 = (float*)(base + w.a3);
  G.d1 = (float*)(base + w.d1);
  G.d2 = (float*)(base + w.d2);
  G.d0 = (float*)(base + w.d0);
  return G;
}

extern "C" vs_status vs_ngp_bake(const float* const* params, const vs_ngp_config* cfg, int32_t k, const int32_t* width,
                                 const int32_t* height, float* const* tex, void* ws, size_t ws_bytes, void* stream) {
  vs::NgpShape S;
  vs::NgpTable T;
  vs_status st = ngp_shape(cfg, S);
  if (st) return st;
  if ((st = ngp_table("vs_ngp_bake", params, k, width, height, T))) return st;
  if (!tex) return fail(VS_ERR_ARG, "vs_ngp_bake: null tex");
  for (int l = 0; l < k; ++l) {
    if (!tex[l] || (uintptr_t)tex[l] % 16) return fail(VS_ERR_ARG, "vs_ngp_bake: tex[%d] null or misaligned", l);
    T.tex[l] = tex[l];
  }
  vs::NgpStage G;
  std::memset(&G, 0, sizeof(G));
  if (ws) {
    const int64_t rows = T.block_off[k] * 256;
    if (rows * vs::kNgpHidden >= ((int64_t)1 << 31)) return fail(VS_ERR_SIZE, "vs_ngp_bake: too many texels to stage");
    const NgpWs w = ngp_ws(S, rows);
    if ((st = check_ws(ws, ws_bytes, w.total))) return st;
    G = ngp_stage(ws, w, rows);
  }
  hipStream_t s = (hipStream_t)stream;
  const unsigned grid = (unsigned)T.block_off[k];
  auto launch = [&](auto kern) { hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, s, T, S, G); };
  if (S.levels <= 8) {
    if (ws) launch(vs::k_ngp_bake<8, true>); else launch(vs::k_ngp_bake<8, false>);
  } else {
    if (ws) launch(vs::k_ngp_bake<16, true>); else launch(vs::k_ngp_bake<16, false>);
  }
  if ((st = check_launch("vs_ngp_bake"))) return st;
  return ok();
}

extern "C" vs_status vs_ngp_backward(const float* const* params, const vs_ngp_config* cfg, int32_t k,
                                     const int32_t* width, const int32_t* height, const float* const* tex,
                                     const float* const* grad_tex, float* const* grad_params, void* ws,
                                     size_t ws_bytes, void* stream) {
  vs::NgpShape S;
  vs::NgpTable T;
  vs_status st = ngp_shape(cfg, S);
  if (st) return st;
  if ((st = ngp_table("vs_ngp_backward", params, k, width, height, T))) return st;
  if (!grad_tex || !grad_params || !tex) return fail(VS_ERR_ARG, "vs_ngp_backward: null pointer");
  for (int l = 0; l < k; ++l) {
    if (!tex[l] || (uintptr_t)tex[l] % 16) return fail(VS_ERR_ARG, "vs_ngp_backward: tex[%d] null or misaligned", l);
    T.tex[l] = const_cast<float*>(tex[l]);
    if (!grad_tex[l] || (uintptr_t)grad_tex[l] % 16)
      return fail(VS_ERR_ARG, "vs_ngp_backward: grad_tex[%d] null or misaligned", l);
    if (!grad_params[l] || (uintptr_t)grad_params[l] % 16)
      return fail(VS_ERR_ARG, "vs_ngp_backward: grad_params[%d] null or misaligned", l);
    T.gtex[l] = grad_tex[l];
    T.gparams[l] = grad_params[l];
  }
  const int64_t R = T.block_off[k] * 256;
  if (R * vs::kNgpHidden >= ((int64_t)1 << 31)) return fail(VS_ERR_SIZE, "vs_ngp_backward: too many texels");
  const NgpWs w = ngp_ws(S, R);
  if ((st = check_ws(ws, ws_bytes, w.total))) return st;
  const vs::NgpStage G = ngp_stage(ws, w, R);
  hipStream_t s = (hipStream_t)stream;
  const unsigned grid = (unsigned)T.block_off[k];
  hipLaunchKernelGGL(vs::k_ngp_texel_bwd1, dim3(grid), dim3(256), 0, s, T, S, G);
  if (S.levels <= 8) hipLaunchKernelGGL(vs::k_ngp_texel_bwd2<8>, dim3(grid), dim3(256), 0, s, T, S, G);
  else hipLaunchKernelGGL(vs::k_ngp_texel_bwd2<16>, dim3(grid), dim3(256), 0, s, T, S, G);
  if ((st = check_launch("vs_ngp_backward"))) return st;
  // weight products: per layer dW1, db1 from (D1, e), dW2, db2 from (D2, h1), dW3, db3 from (D0, h2)
  vs::NgpGemm Q;
  std::memset(&Q, 0, sizeof(Q));
  const int nin = 2 * S.levels;
  int64_t max_rows = 0;
  for (int l = 0; l < k; ++l) {
    const int64_t r0 = T.block_off[l] * 256, rows = (T.block_off[l + 1] - T.block_off[l]) * 256;
    max_rows = std::max(max_rows, rows);
    float* gp = grad_params[l];
    const int g0 = 3 * l;
    Q.D[g0] = G.d1 + r0; Q.A[g0] = G.a1 + r0; Q.gw[g0] = gp + S.o_w1; Q.gb[g0] = gp + S.o_b1;
    Q.M[g0] = vs::kNgpHidden; Q.K[g0] = nin;
    Q.D[g0 + 1] = G.d2 + r0; Q.A[g0 + 1] = G.a2 + r0; Q.gw[g0 + 1] = gp + S.o_w2; Q.gb[g0 + 1] = gp + S.o_b2;
    Q.M[g0 + 1] = vs::kNgpHidden; Q.K[g0 + 1] = vs::kNgpHidden;
    Q.D[g0 + 2] = G.d0 + r0; Q.A[g0 + 2] = G.a3 + r0; Q.gw[g0 + 2] = gp + S.o_w3; Q.gb[g0 + 2] = gp + S.o_b3;
    Q.M[g0 + 2] = vs::kNgpOut; Q.K[g0 + 2] = vs::kNgpHidden;
    for (int q = 0; q < 3; ++q) Q.rows[g0 + q] = rows;
  }
  Q.R = R;
  Q.n_gemm = 3 * k;
  // enough blocks to fill the chip, each with at least a few 64-row tiles
  Q.blocks_per_gemm = (int32_t)std::max<int64_t>(1, std::min<int64_t>(256, max_rows / 512));
  hipLaunchKernelGGL(vs::k_ngp_wgrad, dim3((unsigned)(Q.n_gemm * Q.blocks_per_gemm)), dim3(256), 0, s, Q);
  if ((st = check_launch("vs_ngp_backward (weights)"))) return st;
  return ok();
}

// ------------------------------------------------------------------ graphs

struct vs_graph_s {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

// ---------------------------------------------------------------------------
// k-SDF volume rendering
// ---------------------------------------------------------------------------
namespace {

vs_status ksdf_params(const char* who, const vs_ksdf_field* f, const vs_ksdf_opts* o, vs::KsdfParams& P) {
  if (!f || !o) return fail(VS_ERR_ARG, "%s: null field or opts", who);
  if (!f->sdf || !f->rgba) return fail(VS_ERR_ARG, "%s: null field grid", who);
  if ((uintptr_t)f->rgba % 16) return fail(VS_ERR_ARG, "%s: rgba grid not 16-byte aligned", who);
  if (f->sdf_res < 1 || f->sdf_res > 1023 || f->rgba_res < 1 || f->rgba_res > 644)
    return fail(VS_ERR_SIZE, "%s: grid resolutions %d, %d outside 1..1023, 1..644", who, f->sdf_res, f->rgba_res);
  if (!(std::isfinite(f->lo) && std::isfinite(f->hi) && f->lo < f->hi))
    return fail(VS_ERR_ARG, "%s: need finite lo < hi", who);
  if (o->k < 1 || o->k > VS_KSDF_MAX_SURFACES) return fail(VS_ERR_ARG, "%s: k = %d outside 1..%d", who, o->k,
                                                            VS_KSDF_MAX_SURFACES);
  for (int j = 0; j < o->k; ++j) {
    if (!std::isfinite(o->offsets[j])) return fail(VS_ERR_ARG, "%s: offset %d not finite", who, j);
    if (j && o->offsets[j] < o->offsets[j - 1]) return fail(VS_ERR_ARG, "%s: offsets must not decrease", who);
  }
  if (!(std::isfinite(o->beta) && o->beta > 0.0)) return fail(VS_ERR_ARG, "%s: beta must be > 0", who);
  if (!(std::isfinite(o->occ_threshold) && o->occ_threshold > 0.0))
    return fail(VS_ERR_ARG, "%s: occ_threshold must be > 0", who);
  if (o->occ_res < 1 || o->occ_res > 1024) return fail(VS_ERR_SIZE, "%s: occ_res %d outside 1..1024", who, o->occ_res);
  if (o->n_uniform < 2 || o->n_importance < 0 || o->n_importance % 2 ||
      o->n_uniform + o->n_importance > VS_KSDF_MAX_SAMPLES)
    return fail(VS_ERR_ARG, "%s: need n_uniform >= 2, even n_importance >= 0, total <= %d", who, VS_KSDF_MAX_SAMPLES);
  if (o->march_steps < 64 || o->march_steps > 2048 || o->march_steps % 64)
    return fail(VS_ERR_ARG, "%s: march_steps must be a multiple of 64 in 64..2048", who);
  if (!(std::isfinite(o->pdf_floor) && o->pdf_floor > 0.0)) return fail(VS_ERR_ARG, "%s: pdf_floor must be > 0", who);
  std::memset(&P, 0, sizeof(P));
  P.sdf = f->sdf;
  P.rgba = (const float4*)f->rgba;
  P.sdf_res = f->sdf_res;
  P.rgba_res = f->rgba_res;
  P.occ_res = o->occ_res;
  P.lo = f->lo;
  P.hi = f->hi;
  P.h_occ = (f->hi - f->lo) / o->occ_res;
  P.inv_sdf = f->sdf_res / (f->hi - f->lo);
  P.inv_rgba = f->rgba_res / (f->hi - f->lo);
  P.inv_occ = o->occ_res / (f->hi - f->lo);
  P.k = o->k;
  P.factor = 1;
  for (int j = 0; j < o->k; ++j) {
    P.off[j] = o->offsets[j];
    if (!(std::fabs(o->beta * o->offsets[j]) <= 60.0)) P.factor = 0;
    P.cexp[0][j] = (float)std::exp(-(o->beta / 2.0) * o->offsets[j]);
    P.cexp[1][j] = (float)std::exp(-o->beta * o->offsets[j]);
  }
  P.beta = o->beta;
  P.occ_threshold = o->occ_threshold;
  P.half_diag = std::sqrt(3.0) * P.h_occ / 2.0;
  P.n = o->n_uniform;
  P.m = o->n_importance;
  P.steps = o->march_steps;
  P.pdf_floor = (float)o->pdf_floor;
  return VS_OK;
}

}  // namespace

extern "C" int64_t vs_ksdf_occupancy_words(int32_t occ_res) {
  if (occ_res < 1 || occ_res > 1024) return 0;
  return ((int64_t)occ_res * occ_res * occ_res + 31) / 32;
}

extern "C" vs_status vs_ksdf_occupancy(const vs_ksdf_field* field, const vs_ksdf_opts* opts, uint32_t* occ,
                                       void* stream) {
  vs::KsdfParams P;
  vs_status st = ksdf_params("vs_ksdf_occupancy", field, opts, P);
  if (st) return st;
  if (!occ) return fail(VS_ERR_ARG, "vs_ksdf_occupancy: null occ");
  const int64_t n_vox = (int64_t)P.occ_res * P.occ_res * P.occ_res;
  const int64_t words = vs_ksdf_occupancy_words(P.occ_res);
  hipLaunchKernelGGL(vs::k_ksdf_occupancy, dim3((unsigned)((n_vox + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                     P, occ, n_vox, words);
  if ((st = check_launch("vs_ksdf_occupancy"))) return st;
  return ok();
}

extern "C" vs_status vs_ksdf_render(const vs_ksdf_field* field, const vs_ksdf_opts* opts, const uint32_t* occ,
                                    const vs_views* views, float* out_rgba, float* layers, double* samples,
                                    void* stream) {
  vs::KsdfParams P;
  vs_status st = ksdf_params("vs_ksdf_render", field, opts, P);
  if (st) return st;
  if ((st = check_views(views))) return st;
  if (!occ || !out_rgba) return fail(VS_ERR_ARG, "vs_ksdf_render: null occ or out_rgba");
  if ((uintptr_t)out_rgba % 16 || (layers && (uintptr_t)layers % 16) || (samples && (uintptr_t)samples % 8))
    return fail(VS_ERR_ARG, "vs_ksdf_render: misaligned output");
  const int64_t total = views->host[views->n_views].pix_offset;
  const int64_t blocks = ((total + vs::kKsdfRays - 1) / vs::kKsdfRays + 7) / 8 * 8;
  if (blocks > INT32_MAX) return fail(VS_ERR_SIZE, "vs_ksdf_render: too many pixels");
  auto launch = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, views->dev, views->n_views,
                       total, P, occ, (float4*)out_rgba, (float4*)layers, samples);
  };
  const int n_total = P.n + P.m;
  if (n_total <= 64) launch(vs::k_ksdf_render<2>);
  else if (n_total <= 96) launch(vs::k_ksdf_render<3>);
  else launch(vs::k_ksdf_render<4>);
  if ((st = check_launch("vs_ksdf_render"))) return st;
  return ok();
}

extern "C" vs_status vs_graph_begin(void* stream) {
  if (!stream) return fail(VS_ERR_ARG, "vs_graph_begin: the null stream cannot be captured");
  const hipError_t e = hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return fail(VS_ERR_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e));
  return ok();
}

extern "C" vs_status vs_graph_end(void* stream, vs_graph* out) {
  if (!stream || !out) return fail(VS_ERR_ARG, "vs_graph_end: null pointer");
  *out = nullptr;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture((hipStream_t)stream, &g);
  if (e != hipSuccess) return fail(VS_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(VS_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  *out = new vs_graph_s{g, x};
  return ok();
}

extern "C" vs_status vs_graph_launch(vs_graph g, void* stream) {
  if (!g) return fail(VS_ERR_ARG, "vs_graph_launch: null graph");
  const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
  if (e != hipSuccess) return fail(VS_ERR_HIP, "hipGraphLaunch: %s", hipGetErrorString(e));
  return ok();
}

extern "C" vs_status vs_graph_destroy(vs_graph g) {
  if (!g) return ok();
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  delete g;
  return ok();
}

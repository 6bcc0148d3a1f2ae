// Host side of the C ABI declared in include/vs.h: argument validation,
// workspace layout and kernel launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "vs.h"
#include "vs_common.h"
#include "vs_raster.h"
#include "vs_shade.h"

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

const int kTileSizes[4] = {8, 16, 32, 64};

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
    for (int s = 0; s < 4; ++s) {
      const int S = kTileSizes[s];
      tiles[s] += (int64_t)((r.cam.width + S - 1) / S) * ((r.cam.height + S - 1) / S);
    }
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
    L.xyz[l] = m.xyz;
    L.uv[l] = m.uv;
    L.tri[l] = m.tri;
    L.n_vert[l] = m.n_vert;
    L.n_tri[l] = m.n_tri;
    L.vert_off[l + 1] = L.vert_off[l] + m.n_vert;
    L.tri_off[l + 1] = L.tri_off[l] + m.n_tri;
  }
  for (int l = k + 1; l <= VS_MAX_LAYERS; ++l) {
    L.vert_off[l] = L.vert_off[k];
    L.tri_off[l] = L.tri_off[k];
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
  }
  return VS_OK;
}

vs::WsLayout ws_layout(const vs::LayerTable& L, int n_views) {
  vs::WsLayout w;
  size_t off = 0;
  w.status = off;
  off += 256;
  w.proj = off;
  off += vs::align_up((size_t)n_views * (size_t)L.vert_off[L.k] * sizeof(vs::ProjVert), 256);
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
    for (int s = 0; s < 4; ++s) {
      const int S = kTileSizes[s];
      tiles[s] += (int64_t)((cams[v].width + S - 1) / S) * ((cams[v].height + S - 1) / S);
    }
  }
  return ok();
}

size_t vs_raster_workspace_bytes(const vs_mesh* layers, int32_t k, const vs_views* views,
                                 const vs_raster_opts* opts) {
  (void)opts;
  vs::LayerTable L;
  if (build_layers(layers, k, L) || check_views(views)) return 0;
  return ws_layout(L, views->n_views).total;
}

vs_status vs_raster_layers(const vs_mesh* layers, int32_t k, const vs_views* views, uint64_t* vis, void* ws,
                           size_t ws_bytes, const vs_raster_opts* opts, void* stream) {
  vs::LayerTable L;
  vs_status st = build_layers(layers, k, L);
  if (st) return st;
  if ((st = check_views(views))) return st;
  if (!vis) return fail(VS_ERR_ARG, "vis: null");
  const vs::WsLayout lay = ws_layout(L, views->n_views);
  if ((st = check_ws(ws, ws_bytes, lay.total))) return st;
  const int count_frags = opts ? (opts->flags & VS_RASTER_COUNT_FRAGMENTS) : 0;
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)ws;
  auto* status = (unsigned long long*)(base + lay.status);
  auto* proj = (vs::ProjVert*)(base + lay.proj);
  const int64_t vpv = L.vert_off[k];
  const int64_t total_slots = (int64_t)k * views->host[views->n_views].pix_offset;
  const int nv = views->n_views;
  hipLaunchKernelGGL(vs::k_fill_u64, dim3(1), dim3(256), 0, s, (uint64_t*)status, (int64_t)VS_STAT_COUNT, 0ull);
  hipLaunchKernelGGL(vs::k_fill_u64, dim3((unsigned)std::min<int64_t>(grid_1d(total_slots, 256), 65536)), dim3(256),
                     0, s, vis, total_slots, (uint64_t)VS_EMPTY);
  hipLaunchKernelGGL(vs::k_project, dim3(grid_1d(vpv, 256), nv), dim3(256), 0, s, views->dev, L, proj, vpv);
  hipLaunchKernelGGL(vs::k_raster_direct, dim3(grid_1d(L.tri_off[k], 256), nv), dim3(256), 0, s, views->dev, L,
                     (const vs::ProjVert*)proj, vpv, (unsigned long long*)vis, status, count_frags);
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
  const vs::WsLayout lay = ws_layout(L, views->n_views);
  if ((st = check_ws(ws, ws_bytes, lay.total))) return st;
  const float eps = opts ? opts->eps_T : 0.0f;
  const int wrap = opts ? opts->wrap : 0;
  if (wrap != 0 && wrap != 1) return fail(VS_ERR_UNSUPPORTED, "wrap = %d", wrap);
  if (!(eps >= 0.0f && eps < 1.0f)) return fail(VS_ERR_ARG, "eps_T must be in [0, 1)");
  const char* base = (const char*)ws;
  auto* status = (unsigned long long*)(base + lay.status);
  const auto* proj = (const vs::ProjVert*)(base + lay.proj);
  hipStream_t s = (hipStream_t)stream;
  const int64_t tiles = total_tiles(views, vs::kShadeTileSlot);
  hipLaunchKernelGGL(vs::k_shade_fwd, dim3((unsigned)tiles), dim3(256), 0, s, views->dev, views->n_views, L, X, proj,
                     L.vert_off[k], vis, (float4*)out_rgba, eps, wrap, status);
  if ((st = check_launch("vs_render"))) return st;
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
  const vs::WsLayout lay = ws_layout(L, views->n_views);
  if ((st = check_ws(ws, ws_bytes, lay.total))) return st;
  const char* base = (const char*)ws;
  auto* status = (unsigned long long*)(base + lay.status);
  const auto* proj = (const vs::ProjVert*)(base + lay.proj);
  hipStream_t s = (hipStream_t)stream;
  const int64_t tiles = total_tiles(views, vs::kShadeTileSlot);
  auto launch = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3((unsigned)tiles), dim3(256), 0, s, views->dev, views->n_views, L, X, proj,
                       L.vert_off[k], vis, (const float4*)grad_rgba, (const float4*)target, scale,
                       (float4*)out_rgba, target ? sse : nullptr, wrap, status);
  };
  if (k <= 4) launch(vs::k_shade_bwd<4>);
  else if (k <= 8) launch(vs::k_shade_bwd<8>);
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

/*
 * vs.h -- C ABI of the MI355X (gfx950) layered-mesh renderer.
 *
 * The library renders k nested, semi-transparent, UV-textured triangle-mesh
 * shells in a fixed order with no sorting, and differentiates the result with
 * respect to the textures (Volumetric Surfaces, arXiv 2409.02482):
 *
 *   mesh shells + UV textures + cameras  ->  image
 *
 * Per layer the triangles are rasterised to find the first intersection of
 * each pixel ray with that shell (Fig. 2c; sampling locations found by
 * rasterisation, Sec. 1), the UVs are interpolated, the layer's RGBA texture
 * is read bilinearly from the four surrounding texel centres (Fig. 5,
 * Sec. 4.3 "Texturing Meshes"), and the layers are alpha-blended front to
 * back from the outermost shell inward (Sec. 4.2, Eq. 6, read with the
 * product over the layers in front of layer i, j < i).  The adjoint returns
 * texture gradients only: geometry is fixed while textures are fit
 * (Sec. 4.3).
 *
 * Conventions
 *   - Layer 0 is the OUTERMOST shell.  Layers are independent: each keeps its
 *     own nearest hit, and there is no depth test across layers.
 *   - Cameras: OpenCV pinhole, world->camera (R row-major, t), x right,
 *     y down, z forward; pixel (i, j) has its centre at (i + 1/2, j + 1/2).
 *   - Screen positions snap to 1/256 pixel (round half to even); a triangle
 *     with a vertex at or in front of z_near, beyond +-2^16 pixels, or not
 *     finite, is culled (no clipping) and counted in the status block.
 *   - Fill rule: a pixel centre on an edge belongs to the triangle only if
 *     the edge is a top or a left edge.
 *   - Visibility key of a slot = (bits of float(z) << 32) | triangle id, z the
 *     perspective-correct camera depth; the slot keeps the minimum key
 *     (nearest, ties to the smaller id).  VS_EMPTY where nothing covers.
 *   - Textures: f32 straight (not premultiplied) RGBA, [H][W][4]; texel (i, j)
 *     centred at ((i+1/2)/W, (j+1/2)/H); row 0 holds v in [0, 1/H).
 *   - Output: f32 [sum_v H_v W_v][4], RGB over black, A = 1 - transmittance.
 *
 * Memory and streams
 *   - Every buffer is owned by the caller.  Pointers documented "device" must
 *     be device memory of the current HIP device; "host" pointers are read
 *     during the call only.  The library never allocates device memory.
 *   - All work is enqueued on the caller's stream; no call synchronises the
 *     host except vs_read_status and vs_autotune.  No call records a memset
 *     node, so a sequence of calls can be captured in a HIP graph (the host
 *     arrays are read at enqueue time; replays reuse the captured values).
 *
 * Errors
 *   - Every call returns a vs_status.  VS_OK = 0.  Arguments are validated on
 *     the host before anything is enqueued; on error nothing is enqueued and
 *     vs_last_error() (thread-local) holds a message.  Conditions only the
 *     device can see (culled triangles, out-of-range triangle ids found in a
 *     visibility buffer) are counted in the status block inside the
 *     workspace; read it with vs_read_status.
 */
#ifndef VS_H_
#define VS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vs_status;
enum {
  VS_OK = 0,
  VS_ERR_ARG = 1,          /* null pointer, bad count, inconsistent view table */
  VS_ERR_SIZE = 2,         /* a size outside the documented limits */
  VS_ERR_WORKSPACE = 3,    /* workspace missing or too small */
  VS_ERR_HIP = 4,          /* a HIP runtime call failed */
  VS_ERR_UNSUPPORTED = 5   /* option value not supported */
};

#define VS_MAX_LAYERS 16
#define VS_MAX_VIEW_DIM 8192
#define VS_MAX_TEX_DIM 16384
#define VS_MAX_LAYER_ELEMS (1 << 28)   /* vertices, and triangles, of one layer (32-bit byte offsets) */
#define VS_EMPTY 0xFFFFFFFFFFFFFFFFull

/* One shell.  Device pointers.  xyz f32 [n_vert][3] world positions,
 * uv f32 [n_vert][2], tri i32 [n_tri][3] vertex ids.  1 <= n_vert, n_tri <=
 * VS_MAX_LAYER_ELEMS: an empty layer, or a larger one, is rejected
 * (VS_ERR_SIZE). */
typedef struct vs_mesh {
  const float* xyz;
  const float* uv;
  const int32_t* tri;
  int32_t n_vert;             /* 1..VS_MAX_LAYER_ELEMS */
  int32_t n_tri;              /* 1..VS_MAX_LAYER_ELEMS */
} vs_mesh;

/* One layer texture.  Device pointer, f32 [height][width][4] straight RGBA. */
typedef struct vs_texture {
  const float* rgba;
  int32_t width;
  int32_t height;
} vs_texture;

/* A pinhole camera (host record). */
typedef struct vs_camera {
  int32_t width, height;      /* pixels, 1..VS_MAX_VIEW_DIM */
  double fx, fy, cx, cy;      /* pixels */
  double R[9];                /* world->camera rotation, row-major */
  double t[3];                /* world->camera translation */
  double z_near;              /* > 0 */
} vs_camera;

/* A view record: the camera plus the offsets that place the view in the
 * batched buffers.  Built by vs_views_prepare; copy the same bytes to the
 * device.  The array has n_views + 1 records: the last one holds the totals
 * (pix_offset = total pixels, tile_offset[s] = total tiles). */
typedef struct vs_view {
  vs_camera cam;
  int64_t pix_offset;         /* sum_{u<v} W_u H_u */
  int64_t tile_offset[4];     /* sum_{u<v} ceil(W_u/Sw) ceil(H_u/Sh) for Sw x Sh = 8x8, 16x16, 32x32, 64x56 */
} vs_view;

/* The views of one batched call: host and device copies of the same
 * vs_views_prepare output (n_views + 1 records each). */
typedef struct vs_views {
  const vs_view* host;
  const vs_view* dev;
  int32_t n_views;
} vs_views;

/* Raster options.  bin: screen-tile width in pixels, one of 8, 16, 32, 64, or
 * 0 for the library default (64); tiles are square except the 64-pixel ones,
 * which are 56 rows high.  The result is bit-identical for every value.
 * The workspace must have been sized for the same bin value.
 * flags: VS_RASTER_COUNT_FRAGMENTS counts covered (triangle, pixel) pairs in
 * the status block (costs extra atomics); VS_RASTER_DIRECT uses the unbinned
 * one-thread-per-triangle path with global atomics (a slower, independent
 * implementation of the same result, kept for cross-checking). */
#define VS_RASTER_COUNT_FRAGMENTS 1
#define VS_RASTER_DIRECT 2
typedef struct vs_raster_opts {
  int32_t bin;
  int32_t flags;
  int64_t list_capacity;      /* triangle-list entries reserved in the workspace; 0 = automatic.
                                 Bins that do not fit are still rasterised exactly, more slowly,
                                 and counted in VS_STAT_BIN_OVERFLOW. */
} vs_raster_opts;

/* Shading options.
 * eps_T:  a pixel stops reading layers once every pixel of its wavefront has
 *         transmittance below eps_T (0 = always read all k layers).  The
 *         colour changes by at most eps_T * max|c|.
 * wrap:   0 = repeat (the OpenGL default), 1 = clamp to edge.
 * target: device f32 [sum_v H_v W_v][4] or NULL.  When set, the backward
 *         pass uses the fused RGB loss selected by `loss` instead of
 *         grad_rgba (A of the target is ignored):
 *           VS_LOSS_L2: loss_scale * sum_p ||RGB_p - target_p||_2^2
 *           VS_LOSS_L1: loss_scale * sum_p ||RGB_p - target_p||_1  (the
 *                       paper's texturing loss, Sec. 4.3; gradient sign(.),
 *                       0 at a tie)
 * loss_scale: multiplies the fused loss (e.g. 1/number of scalars).
 * flags:  VS_SHADE_COUNT_PATHS makes vs_render_backward count, in the status
 *         block, how each wavefront's texture-gradient scatter was done per
 *         layer: through one LDS window for the whole wavefront, per half or
 *         per quarter wavefront (footprints too large for one window), or by
 *         direct atomics (a quarter still too large); costs a few atomics. */
enum { VS_LOSS_L2 = 0, VS_LOSS_L1 = 1 };
#define VS_SHADE_COUNT_PATHS 1
typedef struct vs_shade_opts {
  float eps_T;
  int32_t wrap;
  const float* target;
  float loss_scale;
  int32_t loss;
  int32_t flags;
} vs_shade_opts;

/* Status block counters (vs_read_status). */
enum {
  VS_STAT_CULLED_INVALID = 0,   /* triangles with a vertex behind z_near, beyond the guard band or NaN */
  VS_STAT_CULLED_DEGENERATE = 1,/* zero-area triangles after snapping */
  VS_STAT_BAD_INDEX = 2,        /* vertex ids outside [0, n_vert) */
  VS_STAT_FRAGMENTS = 3,        /* covered (triangle, pixel) pairs tested by the raster */
  VS_STAT_BAD_KEY = 4,          /* visibility keys naming a triangle id >= n_tri */
  VS_STAT_BIN_OVERFLOW = 5,     /* bins whose triangle list exceeded the workspace (still exact, slower) */
  VS_STAT_SCATTER_WAVE = 6,     /* with VS_SHADE_COUNT_PATHS: layer-wavefronts scattered through one window */
  VS_STAT_SCATTER_HALF = 7,     /*   ... half wavefronts scattered through a window */
  VS_STAT_SCATTER_QUARTER = 8,  /*   ... quarter wavefronts scattered through a window */
  VS_STAT_SCATTER_DIRECT = 9,   /*   ... quarter wavefronts scattered by direct atomics */
  VS_STAT_COUNT = 10
};

/* Library version string. */
const char* vs_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char* vs_last_error(void);

/* Name of a status code. */
const char* vs_status_string(vs_status s);

/* Fill n_views + 1 view records (host memory, out[n_views + 1]) from
 * n_views cameras (host).  Validates each camera. */
vs_status vs_views_prepare(const vs_camera* cams, int32_t n_views, vs_view* out);

/* Workspace needed by vs_raster_layers for these layers and views (bytes).
 * The same workspace is then passed to vs_render / vs_render_backward: it
 * carries the projected vertices and the status block. */
size_t vs_raster_workspace_bytes(const vs_mesh* layers, int32_t k, const vs_views* views,
                                 const vs_raster_opts* opts);

/* Rasterise every layer in every view: the visibility of the method's
 * sampling positions.  Each pixel ray meets each shell once, at the shell's
 * first intersection (Fig. 2c), and those positions are found by
 * rasterising every shell separately (Sec. 1, sampling by rasterisation).
 * Per (view, layer, pixel) the slot keeps the key of the nearest covering
 * triangle (conventions above: snapping, fill rule, key).
 * layers: host array [k] of device meshes, layer 0 outermost.  1 <= k <= 16.
 * n_views * total triangles must be below 2^30.  Bin-list offsets are 64-bit,
 * so any total of (triangle, bin) entries is handled; bins whose list does
 * not fit the reserved capacity (below 2^32 entries) are rasterised by the
 * exact full-layer path and counted in VS_STAT_BIN_OVERFLOW.
 * vis:    device u64 [sum_v k H_v W_v], written in full.  Slot of (view v,
 *         layer l, pixel (x, y)) = k * pix_offset[v] + l * H_v W_v + y W_v + x.
 * ws:     device workspace of at least vs_raster_workspace_bytes bytes,
 *         256-byte aligned.  Its status block is reset by this call.
 * opts:   may be NULL (defaults). */
vs_status vs_raster_layers(const vs_mesh* layers, int32_t k, const vs_views* views, uint64_t* vis, void* ws,
                           size_t ws_bytes, const vs_raster_opts* opts, void* stream);

/* Shade and blend (forward): per slot, the perspective-correct UV of the hit,
 * the layer's RGBA read bilinearly from the four surrounding texel centres
 * (Fig. 5; texel-centre access as in OpenGL, Sec. 4.3 "Texturing Meshes"),
 * and the layers alpha-blended front to back from the outermost shell
 * inward (Sec. 4.2, Eq. 6, with the product over the layers in front,
 * j < i; fixed order without sorting, Sec. 1 and Sec. 4.3 "Baking Textures").
 * tex:  host array [k] of device textures.
 * vis:  the visibility buffer of vs_raster_layers for the same layers/views.
 * ws:   the workspace that vs_raster_layers filled for the same layers/views.
 * out_rgba: device f32 [sum_v H_v W_v][4]. */
vs_status vs_render(const vs_mesh* layers, const vs_texture* tex, int32_t k, const vs_views* views,
                    const uint64_t* vis, const void* ws, size_t ws_bytes, float* out_rgba,
                    const vs_shade_opts* opts, void* stream);

/* Raster and shade in one call WITHOUT ALLOCATING: for callers that cannot
 * allocate device memory or pass a workspace (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The result is that
 * of vs_raster_layers(layers, k, views, vis, ws, ..., raster_opts) followed by
 * vs_render(layers, tex, k, views, vis, ws, ..., out_rgba, shade_opts): the
 * same kernels, with the workspace taken from a static device array of
 * VS_NOALLOC_SCRATCH_BYTES bytes that the library holds on every device it
 * runs on until the process ends (its address is looked up once per device,
 * at the first call on that device).
 * vis:      device u64 [sum_v k H_v W_v], written in full (as vs_raster_layers).
 * out_rgba: device f32 [sum_v H_v W_v][4] (as vs_render).
 * raster_opts, shade_opts: may be NULL (defaults).
 * Errors: VS_ERR_WORKSPACE, before anything is enqueued, when
 * vs_raster_workspace_bytes for these layers, views and raster options
 * exceeds VS_NOALLOC_SCRATCH_BYTES; other argument errors as the two calls.
 * Every call on one device shares that device's array and leaves its
 * contents behind (each call re-initialises what it reads): calls that
 * overlap in time on one device, on any streams, race and must be ordered
 * by the caller. */
#define VS_NOALLOC_SCRATCH_BYTES (64ull << 20)
vs_status vs_render_noalloc(const vs_mesh* layers, const vs_texture* tex, int32_t k, const vs_views* views,
                            uint64_t* vis, float* out_rgba, const vs_raster_opts* raster_opts,
                            const vs_shade_opts* shade_opts, void* stream);

/* Texture adjoint: the derivative of vs_render's image with respect to the
 * texels, which is what the texturing phase optimises on fixed meshes
 * (Sec. 4.3 "Texturing Meshes").  The blend of Sec. 4.2, Eq. 6 is reversed
 * back to front without divisions (dL/dc_l = g a_l T_l,
 * dL/da_l = T_l <g, c_l - S_l> + g_A T_l prod_{m>l} (1 - a_m), S_l the colour
 * blended behind layer l) and each corner texel of the bilinear read (Fig. 5)
 * receives its weight times these.
 * grad_rgba: device f32 [sum_v H_v W_v][4] = dL/d(out_rgba); ignored (may be
 *            NULL) when opts->target is set (fused L2 or L1 loss).
 * opts->eps_T: the forward walk stops where vs_render's does, so the gradient
 *            is that of the image vs_render returns with the same eps_T.
 * grad_tex:  host array [k] of device pointers, f32 [H_l][W_l][4] each,
 *            ACCUMULATED into (+=).  Summation order is not fixed (atomics).
 * out_rgba:  optional device f32 [sum_v H_v W_v][4]: when non-NULL the
 *            forward image is written too (same values as vs_render).
 * sse:       optional device f64 [1]: when non-NULL and opts->target is set,
 *            the unscaled loss sum_p ||RGB_p - target_p||^2 (L2) or
 *            sum_p ||RGB_p - target_p||_1 (L1) is ACCUMULATED into it. */
vs_status vs_render_backward(const vs_mesh* layers, const vs_texture* tex, int32_t k, const vs_views* views,
                             const uint64_t* vis, const void* ws, size_t ws_bytes, const float* grad_rgba,
                             float* const* grad_tex, float* out_rgba, double* sse, const vs_shade_opts* opts,
                             void* stream);

/* ---- baked view-dependent appearance (Sec. 4.3 "Texturing Meshes", "Mixed
 *      Resolutions", "Squeezing and Quantization", "Baking Textures"; Sec. 4.2
 *      "Transparency Attenuation") ---- */

/* One shell's baked spherical-harmonic texture (device memory, 8-bit).
 * With SH degree D (vs_sh_opts.degree, 0..3) a texel carries (D+1)^2
 * coefficients per RGBA channel.  The coefficients of degree l live at level
 * l, of max(1, width >> l) x max(1, height >> l) texels: the base colour at
 * full resolution, each higher degree at half the previous one.  Levels
 * follow each other from level 0; level l is texel-major,
 * [H_l][W_l][2l+1][4] bytes: the 2l+1 coefficients (m = -l..l) of a texel are
 * adjacent, each as R, G, B, A bytes.  Byte q decodes to
 * vmin + (vmax - vmin) q / 255.  Size: sum_{l<=D} W_l H_l (2l+1) 4 bytes,
 * 4-byte aligned. */
typedef struct vs_sh_texture {
  const uint8_t* data;
  int32_t width, height;   /* level-0 size, 1..VS_MAX_TEX_DIM */
} vs_sh_texture;

/* Options of vs_render_sh.
 * vmin, vmax: decoding range of the 8-bit coefficients (the paper uses -15, 15).
 * eps_T, wrap: as in vs_shade_opts.
 * degree:     0..3, the same for every layer.
 * view_alpha: 1 multiplies each layer's alpha by 2 sigmoid(10 |v.n|) - 1
 *             (v the pixel's unit view ray, n the hit triangle's unit
 *             world-space face normal); 0 keeps the decoded alpha. */
typedef struct vs_sh_opts {
  float vmin, vmax;
  float eps_T;
  int32_t wrap;
  int32_t degree;
  int32_t view_alpha;
} vs_sh_opts;

/* Shade and blend with baked SH textures (forward).
 * For each hit layer, every coefficient is read bilinearly at the slot's UV
 * from the four surrounding texel centres of its level (texels decoded
 * first), the layer's RGBA is sigmoid(sum_i sh_i Y_i(v)) with Y_i the real,
 * orthonormal spherical harmonics (index l^2 + l + m, Y_1^{-1}, Y_1^0, Y_1^1
 * proportional to y, z, x: no Condon-Shortley phase) of v, the unit
 * world-space direction from the camera through the pixel centre, and the
 * layers are blended as in vs_render.
 * tex: host array [k] of device textures.  vis, ws, out_rgba and stream as in
 * vs_render.  opts must not be NULL. */
vs_status vs_render_sh(const vs_mesh* layers, const vs_sh_texture* tex, int32_t k, const vs_views* views,
                       const uint64_t* vis, const void* ws, size_t ws_bytes, float* out_rgba,
                       const vs_sh_opts* opts, void* stream);

/* Copy the status block (VS_STAT_COUNT int64 counters) to host memory.
 * Synchronises the stream. */
vs_status vs_read_status(const void* ws, size_t ws_bytes, int64_t* out, void* stream);

/* Pick the raster bin size for these layers and views by timing every bin
 * size whose workspace fits in ws_bytes (size the workspace with bin = 8 to
 * allow all of them) with HIP events on the stream; all candidates must give
 * the same visibility checksum, else VS_ERR_HIP.  On return inout->bin holds
 * the fastest bin (inout->flags and list_capacity are kept).  cache_path
 * (may be NULL): a text file of "key bin" lines; a hit skips the timing, a
 * miss appends.  Synchronises the stream; never call it while capturing.
 * vis and ws are overwritten (vis holds a valid result afterwards). */
vs_status vs_autotune(const vs_mesh* layers, int32_t k, const vs_views* views, uint64_t* vis, void* ws,
                      size_t ws_bytes, vs_raster_opts* inout, const char* cache_path, void* stream);

/* ---- texture fitting (textures are fit on fixed meshes, Sec. 4.3) ---- */

/* Adam hyper-parameters; after each step every texel scalar is projected to [lo, hi]. */
typedef struct vs_adam_opts {
  float lr, beta1, beta2, eps, lo, hi;
} vs_adam_opts;

/* One fused Adam step over k texture planes: params, grads, m, v are host
 * arrays [k] of device pointers to f32 buffers of counts[l] scalars each
 * (counts: host array, multiples of 4, 16-byte aligned buffers).  The step
 * number is read from *step (device int32, t = *step + 1), so a captured graph
 * advances it on every replay.  After the update every gradient scalar is
 * reset to 0.  Then, in stream order: if sse (device f64 [1]) is non-NULL,
 * history[*step] = *sse when *step < hist_len (history: device f64
 * [hist_len] or NULL) and *sse = 0; finally ++*step. */
vs_status vs_adam_step(float* const* params, float* const* grads, float* const* m, float* const* v,
                       const int64_t* counts, int32_t k, const vs_adam_opts* opts, int32_t* step, double* sse,
                       double* history, int32_t hist_len, void* stream);

/* Squeezing and quantisation (Sec. 4.3 "Squeezing and Quantization"): the
 * texture a logit stands for is q(sigmoid(param)) with
 * q(x) = round(levels * x) / levels, ties to even, decided in FP64
 * (levels = 255 for 8-bit storage; 0 = no quantisation).  params and tex:
 * host arrays [k] of device f32 buffers of counts[l] scalars (multiples of
 * 4, 16-byte aligned).  0 <= levels <= 65535. */
vs_status vs_squeeze(const float* const* params, float* const* tex, const int64_t* counts, int32_t k,
                     int32_t levels, void* stream);

/* Quantisation-aware fitting step: Adam on the logits of squeezed, quantised
 * textures.  grads hold dL/dtex (e.g. from vs_render_backward on tex); the
 * quantiser is passed straight through, so the logit gradient is
 * dL/dtex * s (1 - s), s = sigmoid(param).  After the update tex is rewritten
 * as vs_squeeze does, the gradient is reset and the bookkeeping of
 * vs_adam_step runs.  opts->lo and opts->hi are not used (logits are
 * unbounded).  Other arguments as in vs_adam_step. */
vs_status vs_adam_step_squeezed(float* const* params, float* const* grads, float* const* m, float* const* v,
                                float* const* tex, const int64_t* counts, int32_t k, int32_t levels,
                                const vs_adam_opts* opts, int32_t* step, double* sse, double* history,
                                int32_t hist_len, void* stream);

/* ---- neural textures (Sec. 4.3 "Texturing Meshes") ----
 * A neural texture is a 2-D multiresolution hash grid followed by an MLP,
 * grounded to the texture resolution by evaluating it at the texel centres
 * ((i + 1/2)/W, (j + 1/2)/H) only (Sec. 4.3, Fig. 5): baking gives an ordinary
 * RGBA texture for vs_render / vs_render_backward, and the texture gradient
 * those return is carried back to the network by vs_ngp_backward.
 * Level l of L has resolution N_l: its vertices are the integer points
 * 0..N_l of (u N_l, v N_l) (FP64), each holding 2 features, read bilinearly;
 * a level with (N_l + 1)^2 <= T is stored densely (index y (N_l + 1) + x),
 * otherwise at (x XOR y * 2654435761) mod 2^32 masked to T - 1, T = 2^log2_table.
 * MLP (hidden width 64, FP32): z1 = W1 e + b1, h1 = relu(z1); z2 = W2 h1 + b2,
 * h2 = relu(z2); o = W3 h2 + b3; texel RGBA = sigmoid(o), e the 2L features.
 * Parameters of one layer: one f32 array of vs_ngp_param_count floats,
 *   tables [L][T][2] | W1 [64][2L] | b1 [64] | W2 [64][64] | b2 [64] | W3 [4][64] | b3 [4]. */
#define VS_NGP_MAX_LEVELS 16
typedef struct vs_ngp_config {
  int32_t levels;                          /* 1..16 */
  int32_t log2_table;                      /* 4..24 */
  int32_t resolution[VS_NGP_MAX_LEVELS];   /* N_l, 1..65535 */
} vs_ngp_config;

/* Floats of one layer's parameters, or -1 for an invalid configuration. */
int64_t vs_ngp_param_count(const vs_ngp_config* cfg);

/* Workspace bytes of vs_ngp_backward for k layers of textures width[l] x height[l]. */
size_t vs_ngp_workspace_bytes(const vs_ngp_config* cfg, int32_t k, const int32_t* width, const int32_t* height);

/* Bake: tex[l] (device f32 [height[l]][width[l]][4]) = the neural texture of
 * params[l] at every texel centre.  params, tex: host arrays [k] of device
 * pointers (16-byte aligned); width, height: host arrays [k], 1..VS_MAX_TEX_DIM.
 * ws (device, vs_ngp_workspace_bytes, 256-byte aligned) may be NULL; when
 * given, the network's per-texel activations are kept there for
 * vs_ngp_backward. */
vs_status vs_ngp_bake(const float* const* params, const vs_ngp_config* cfg, int32_t k, const int32_t* width,
                      const int32_t* height, float* const* tex, void* ws, size_t ws_bytes, void* stream);

/* Backward of the last vs_ngp_bake that was given this workspace (same
 * params, sizes and textures tex): with grad_tex[l] = dL/dtex[l] (device f32
 * [height][width][4]) it ACCUMULATES dL/dparams into grad_params[l] (device
 * f32, vs_ngp_param_count floats each; summation order not fixed: atomics). */
vs_status vs_ngp_backward(const float* const* params, const vs_ngp_config* cfg, int32_t k, const int32_t* width,
                          const int32_t* height, const float* const* tex, const float* const* grad_tex,
                          float* const* grad_params, void* ws, size_t ws_bytes, void* stream);

/* ---- k-SDF volume rendering (Sec. 4.1 "k-SDF", Sec. 4.2 "Surfaces
 *      Blending", Sec. 4.4 "Occupancy Grid" and "Importance Sampling";
 *      supplement "Points sampling") ----
 * The implicit stage renders k nested surfaces d_j = d + o_j of a main signed
 * distance d (positive outside) by NeuS quadrature along each pixel ray and
 * blends them in fixed order, surface 0 (the outermost) first.  The fields are
 * given on vertex grids over the cube [lo, hi]^3 and read trilinearly: a grid
 * of resolution R has (R+1)^3 vertices in [z][y][x] order; a point p reads
 * cell coordinate c = (p - lo) * (R / (hi - lo)) (per axis, FP64) clamped to
 * [0, R], base vertex min(floor(c), R - 1), weights c - base.  The occupancy
 * grid uses the same coordinate with R = occ_res: a march step is occupied iff
 * the voxel floor((p - lo) * (occ_res / (hi - lo))) of its midpoint
 * p = o + t v is.  A midpoint within a few ulps of a voxel face may be
 * assigned to either neighbouring voxel. */
#define VS_KSDF_MAX_SURFACES 16
#define VS_KSDF_MAX_SAMPLES 128
typedef struct vs_ksdf_field {
  const float* sdf;     /* device, [(sdf_res+1)^3]: main signed distance d */
  const float* rgba;    /* device, 16-byte aligned, [(rgba_res+1)^3][4]: straight RGB and transparency */
  int32_t sdf_res;      /* 1..1023 (the grid stays below 2^32 bytes) */
  int32_t rgba_res;     /* 1..644 (the grid stays below 2^32 bytes) */
  double lo, hi;        /* lo < hi */
} vs_ksdf_field;

/* Options of the k-SDF calls.
 * k, offsets:   surfaces d + offsets[j], offsets non-decreasing (positive offsets lie inside).
 * beta:         logistic kernel size; density phi(x) = beta e^{-beta x} / (1 + e^{-beta x})^2 (Eq. 2),
 *               CDF Phi(x) = 1 / (1 + e^{-beta x}).
 * occ_threshold, occ_res: a voxel of the occ_res^3 grid over the cube is occupied iff for some j,
 *               phi(max(|d_j(centre)| - sqrt(3) h_o / 2, 0)) > occ_threshold (decided in FP64).
 * n_uniform:    samples placed uniformly in the occupied part of each ray.
 * n_importance: samples added by two importance rounds of n_importance/2 each (kernel size beta/2,
 *               then beta); n_uniform + n_importance <= VS_KSDF_MAX_SAMPLES.
 * march_steps:  equal steps over the ray's interval in the cube that resolve its occupied part
 *               (a step is occupied iff the voxel holding its midpoint is); multiple of 64, <= 2048.
 * pdf_floor:    added to every interval weight before the importance pdf is normalised. */
typedef struct vs_ksdf_opts {
  int32_t k;                                 /* 1..VS_KSDF_MAX_SURFACES */
  double offsets[VS_KSDF_MAX_SURFACES];
  double beta;                               /* > 0 */
  double occ_threshold;                      /* > 0 */
  int32_t occ_res;                           /* 1..1024 */
  int32_t n_uniform;                         /* >= 2 */
  int32_t n_importance;                      /* even, >= 0 */
  int32_t march_steps;
  double pdf_floor;                          /* > 0 */
} vs_ksdf_opts;

/* 32-bit words of an occupancy bit grid of resolution occ_res (0 if invalid):
 * voxel (x, y, z) is bit i & 31 of word i >> 5, i = (z occ_res + y) occ_res + x. */
int64_t vs_ksdf_occupancy_words(int32_t occ_res);

/* Build the occupancy grid (Sec. 4.4) of field and opts into occ (device,
 * vs_ksdf_occupancy_words words; every word is written). */
vs_status vs_ksdf_occupancy(const vs_ksdf_field* field, const vs_ksdf_opts* opts, uint32_t* occ, void* stream);

/* Render every pixel of views (vs_views_prepare output) by k-SDF volume rendering.
 * Per pixel ray (origin -R^T t, direction R^T ((i+.5-cx)/fx, (j+.5-cy)/fy, 1) normalised) over its
 * interval [t_in, t_out] in the cube (t >= 0):
 *   1. march_steps equal steps mark the occupied part; with M occupied steps, uniform sample i sits in
 *      occupied step floor(rho) at fraction rho - floor(rho), rho = (i + 1/2) M / n_uniform;
 *   2. two importance rounds: over the sorted samples, NeuS interval weights of every surface
 *      (a_i = max((Phi(d_j(x_i)) - Phi(d_j(x_{i+1}))) / Phi(d_j(x_i)), 0), w_i = a_i prod_{l<i} (1 - a_l))
 *      are summed over surfaces, floored, normalised and inverted at u_q = (q + 1/2)/(n_importance/2)
 *      (linear within an interval); new samples are merged in order;
 *   3. per surface C_j = sum_i w_ij xi(x_i), A_j = sum_i w_ij alpha_w(x_i) a(x_i), (xi, a) the RGBA
 *      field, alpha_w = 2 sigmoid(10 |v.n|) - 1, n the normalised gradient of d (the derivative of
 *      the trilinear interpolant inside the cell holding x_i);
 *   4. out = (sum_j C_j A_j prod_{l<j} (1 - A_l), 1 - prod_j (1 - A_j)).
 * Rays that miss the cube or meet no occupied step give zeros.
 * occ: from vs_ksdf_occupancy with the same field and opts.
 * out_rgba: device f32 [total pixels][4], 16-byte aligned.
 * layers (may be NULL): device f32 [k][total pixels][4], (C_j, A_j) per surface.
 * samples (may be NULL): device f64 [total pixels][n_uniform + n_importance], the final sorted sample
 *   parameters t, -1 for rays without samples.
 * Weights, appearance and blending are FP32; ray set-up, marching and sample positions FP64. */
vs_status vs_ksdf_render(const vs_ksdf_field* field, const vs_ksdf_opts* opts, const uint32_t* occ,
                         const vs_views* views, float* out_rgba, float* layers, double* samples, void* stream);

/* ---- HIP graphs: capture a sequence of the calls above on one stream ---- */
typedef struct vs_graph_s* vs_graph;

/* Start capturing work enqueued on stream (must not be the null stream). */
vs_status vs_graph_begin(void* stream);
/* End the capture and instantiate it; *out receives the executable graph. */
vs_status vs_graph_end(void* stream, vs_graph* out);
/* Replay a captured graph on stream. */
vs_status vs_graph_launch(vs_graph g, void* stream);
/* Release a graph (NULL is ignored). */
vs_status vs_graph_destroy(vs_graph g);

#ifdef __cplusplus
}
#endif

#endif /* VS_H_ */

/*
 * narvis.h -- C ABI of the NARVis hot path on MI355X (gfx950).
 *
 * The library renders attributed point clouds the way the multi-attribute
 * compute rasterizer of NARVis does (Sec. 3.2): a render stage projects
 * every point, culls it against the view frustum and keeps, per pixel, the
 * point closest to the camera through a depth test on a custom framebuffer;
 * a resolve stage then copies the winning point's attributes into G-buffer
 * planes (no blending of overlapping points).
 *
 * Conventions shared by every entry point
 *  - Every buffer argument is device memory owned by the caller (for example
 *    a torch tensor); the library never allocates, frees or retains it.
 *  - Work is enqueued asynchronously on the HIP stream passed as `stream`
 *    (a hipStream_t, NULL = the default stream).  No call synchronises with
 *    the host; results are visible once the stream reaches that point.
 *  - Arguments are validated on the host before anything is enqueued.  On any
 *    error status nothing has been enqueued and outputs are untouched.
 *    Launch failures reported by the runtime come back as NARVIS_ERR_DEVICE.
 *  - Calls are re-entrant for disjoint output buffers.
 *  - Images are row-major with row 0 at the top; a "plane" is W*H values.
 */
#ifndef NARVIS_H
#define NARVIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NARVIS_OK = 0,
    NARVIS_ERR_INVALID_ARG = -1,
    NARVIS_ERR_OUT_OF_MEMORY = -2,
    NARVIS_ERR_DEVICE = -3,
    NARVIS_ERR_UNSUPPORTED = -4,
    NARVIS_ERR_WORKSPACE = -5
} narvis_status;

/* Element formats of a per-point attribute stream (Sec. 3.2 names uint8 and
 * fp32; uint16 and fp16 are accepted as well). */
typedef enum { NARVIS_U8 = 0, NARVIS_U16 = 1, NARVIS_F16 = 2, NARVIS_F32 = 3 } narvis_dtype;

#define NARVIS_MAX_ATTRS 8
#define NARVIS_KEY_EMPTY 0xFFFFFFFFFFFFFFFFull
/* Screen tiles (at most) of the bounded render. */
#define NARVIS_TILE_BOUNDS_MAX 8192

/* Point positions, structure of arrays: x[n], y[n], z[n] float32, device. */
typedef struct {
    const float *x;
    const float *y;
    const float *z;
} narvis_points;

/* One attribute stream: element i lives at (char*)data + i*stride_bytes.
 * stride_bytes >= element size (1, 2, 2, 4 bytes); AoS layouts are described
 * by a stride larger than the element. */
typedef struct {
    const void *data;
    int32_t dtype;        /* narvis_dtype */
    int32_t stride_bytes;
} narvis_attr;

/* Up to 8 attribute streams ("currently tested up to 8", Sec. 3.2). */
typedef struct {
    int32_t count;
    narvis_attr a[NARVIS_MAX_ATTRS];
} narvis_attrs;

/* Pinhole camera placement.  Vertical field of view in degrees, aspect W/H,
 * right-handed look-at, OpenGL-style perspective (the paper trains with a 60
 * degree field of view, near 0.1 and far 2e5, Sec. 3.3). */
typedef struct {
    double eye[3];
    double target[3];
    double up[3];
    double fovy_deg;
    double znear;
    double zfar;
} narvis_camera;

/* Colour of a point: the G-buffer's rgb plane and the splat renderer. */
typedef enum {
    NARVIS_COLOR_LUT = 0,   /* lut[q] of one attribute (transfer function)     */
    NARVIS_COLOR_RGB8 = 1   /* three uint8 attributes times fp32(1/255)        */
} narvis_color_mode;

/* Output planes of the resolve stage.  `keys` is required; every other plane
 * pointer may be NULL to skip it.
 *   keys   uint64[H][W]   per pixel: (fp32 depth bits << 32) | point index of
 *                         the closest point, NARVIS_KEY_EMPTY if none.
 *   depth  float[H][W]    depth of the winner (distance along the viewing
 *                         axis), 0 for an empty pixel.
 *   attr   float[count][H][W]  attribute c of the winner converted exactly to
 *                         fp32 (integers by value, fp16 widened; a half NaN
 *                         becomes the quiet fp32 NaN with the same sign and
 *                         payload), 0 for an empty pixel.
 *   rgb    float[3][H][W] colour of the winner, 0 for an empty pixel; with
 *                         rgb_mode NARVIS_COLOR_LUT the transfer-function
 *                         colour lut[q] of attribute lut_attr,
 *                         q = floor((s - lut_min) * lut_inv_range * 256)
 *                         clamped to [0,255] (NaN -> 0); with
 *                         NARVIS_COLOR_RGB8 the uint8 attributes lut_attr,
 *                         lut_attr+1, lut_attr+2 times fp32(1/255) (each
 *                         product rounded once), as the splat colours them.
 *   vel2d  float[4][H][W] Vel2D of Sec. 4.5.3 from attributes vel_attr,
 *                         vel_attr+1, vel_attr+2 (vx, vy, vz): the derivative
 *                         of normalised device coordinates along v
 *                         (v'x, v'y), then theta = atan2(v'y, v'x)/pi and
 *                         |v'|; 0 for an empty pixel.
 *   lut    float[256][3] device table for rgb.
 *   bounds  optional device scratch of bounds_bytes >=
 *           narvis_raster_bounds_bytes(W, H) bytes (4-byte aligned, contents
 *           overwritten): when given, narvis_rasterize renders in the bounded
 *           mode (see narvis_raster_opts); NULL renders in one pass.  The
 *           keys are the same either way.
 *   hint_keys  optional (with bounds) earlier key buffer uint64[H][W], as
 *           narvis_raster_opts.hint_keys: 8-byte aligned, read only,
 *           overlapping neither keys nor the scratch.
 *   rgb_mode  narvis_color_mode of the rgb plane (0 = LUT).
 *   glyph   optional uint8[n] glyph mask (original point order; nonzero =
 *           glyph point) for the glyph-priority render of narvis_rasterize:
 *           see narvis_raster_opts.glyph.
 *   radius  float[H][W] projected splat radius of the winner in pixels
 *           (Sec. 3.2: the rasterizer computes the projected point radius;
 *           Sec. 4.2: the world radius is the mean distance to the four
 *           nearest neighbours, narvis_knn_radius):
 *           (r * radius_focal_px) / depth with r = fp32 attribute
 *           radius_attr of the winner (each product rounded once); 0 for an
 *           empty pixel.  narvis_rasterize sets radius_focal_px itself
 *           (narvis_camera_focal_px); narvis_raster_resolve takes it from
 *           the struct.
 * The depth, rgb and vel2d planes may be slices of one [8][H][W] tensor in
 * the order r, g, b, depth, v'x, v'y, theta, |v'|: that is the network input
 * narvis_postprocess reads. */
typedef struct {
    uint64_t *keys;
    float *depth;
    float *attr;
    float *rgb;
    float *vel2d;
    const float *lut;
    int32_t lut_attr;
    float lut_min;
    float lut_inv_range;
    int32_t vel_attr;
    void *bounds;
    size_t bounds_bytes;
    const void *hint_keys;
    int32_t rgb_mode;
    const uint8_t *glyph;
    float *radius;
    int32_t radius_attr;
    float radius_focal_px;
} narvis_gbuffer;

/* Render-stage strategy.  Every variant produces the same key buffer; they
 * differ only in how the per-pixel minimum is reached. */
typedef enum {
    NARVIS_RENDER_AUTO = 0,    /* library's choice for the device            */
    NARVIS_RENDER_GLOBAL = 1,  /* atomic min per surviving point, no z-test  */
    NARVIS_RENDER_EARLYZ = 2,  /* read the key first, atomic only if closer  */
    NARVIS_RENDER_LDS = 3      /* fold each workgroup's candidates per pixel
                                  in LDS first, then early-z + atomic once per
                                  touched pixel (scalar path: as EARLYZ)     */
} narvis_render_variant;

/* Bounded render (LDS variant on 16-byte aligned coordinates, when bounds
 * are given, n >= 4096 and W, H < 2^24): the points are taken in chunks of
 * 2048; every 8th chunk is rendered first.  Then, with d(p) the depth bits of
 * the smallest key pixel p holds so far (0xFFFFFFFF if none), the scratch
 * receives
 *   uint16 tile[NARVIS_TILE_BOUNDS_MAX]: for screen tiles of 2^s x 2^s
 *          pixels (the smallest s >= 3 giving at most NARVIS_TILE_BOUNDS_MAX
 *          tiles, row-major), the largest d(p) >> 16 over the tile,
 *   uint32 pixel[H][W]: d(p)  (from byte 2 NARVIS_TILE_BOUNDS_MAX),
 * and the other chunks are rendered, a point being dropped when
 * (bits(w) >> 16) exceeds the bound of its tile or bits(w) that of its pixel.
 * Keys only decrease, so the pixel's key is already smaller than such a
 * point's: the result is the single-pass result, bit for bit.  This is the paper's early
 * z-test (Sec. 3.2), taken against a compact copy of the depth buffer.
 *
 * Hinted bounded render (hint_keys given, with bounds): before the first
 * chunks, every key of the hint buffer that is not empty and whose index
 * (low 32 bits) is below n names a point, which is rendered like any other.
 * In a viewer loop the previous frame's keys name points near the front of
 * the next frame, so the bounds are tighter and fewer points reach the
 * atomics.  Whatever the hint holds, the result is the same bit for bit.
 * Ignored when the bounded render does not apply (see above). */
typedef struct {
    int32_t variant;      /* narvis_render_variant                           */
    int32_t grid_blocks;  /* 0 = automatic, otherwise the number of
                             workgroups (a grid-stride loop covers all points) */
    void *bounds;         /* NULL, or device scratch of bounds_bytes >=
                             narvis_raster_bounds_bytes(W, H) bytes (4-byte
                             aligned, contents overwritten): bounded render */
    size_t bounds_bytes;
    const void *hint_keys; /* NULL, or (with bounds) a device key buffer
                             uint64[H][W] of an earlier render, 8-byte
                             aligned, read only, overlapping neither `keys`
                             nor the scratch: hinted bounded render     */
    const uint8_t *glyph;  /* NULL, or a device uint8[n] glyph mask:
                             glyph-priority render (VisGlyph, Sec. 4.3
                             "Glyph Stylization Support": the frontmost glyph
                             point of a pixel is kept and non-glyph points in
                             front of it are ignored).  A pixel that a point
                             with glyph[i] != 0 reaches keeps the nearest such
                             point; any other pixel keeps the nearest point.
                             The key of a point with glyph[i] == 0 has bit 63
                             set ((bits(w) | 2^31) << 32 | i), so the minimum
                             key is the answer; the resolve's depth drops
                             that bit.  Not with narvis_raster_render_layout. */
} narvis_raster_opts;

/* Parameters of the Gaussian splat renderer. */
typedef struct {
    float sigma_px;         /* standard deviation in pixels, (0, 32]          */
    float opacity;          /* peak opacity, (0, 1]                            */
    int32_t color_mode;     /* narvis_color_mode                               */
    int32_t color_attr;     /* attribute index (first of three for RGB8)       */
    const float *lut;       /* device float[256][3] for NARVIS_COLOR_LUT       */
    float lut_min;
    float lut_inv_range;
    int32_t aniso;          /* 0: isotropic; 1: elongated along the velocity
                               (see narvis_splat)                               */
    int32_t vel_attr;       /* aniso: first of the three velocity attributes   */
    float stretch;          /* aniso: s of S = diag(s, 1, 1), in [1, 1e6]      */
    float focal_px;         /* ignored on input: narvis_splat derives it from
                               the camera (narvis_camera_focal_px)              */
    uint64_t max_pairs;     /* pair capacity of the workspace; 0 = the
                               isotropic worst case (required > 0 for aniso;
                               narvis_splat_count_pairs gives the exact need) */
} narvis_splat_params;

/* Human-readable name of a status code (static storage). */
const char *narvis_status_string(narvis_status s);

/* Compose the clip-space matrix M = P * V of `cam` in FP64 on the host and
 * round each entry once to fp32 (round to nearest even).  vp_rowmajor[16]
 * receives M row-major; *near_f / *far_f receive the fp32 cull bounds.
 * Host only, touches no device.  INVALID_ARG for W or H < 1, eye == target,
 * up parallel to the viewing direction, fovy outside (0,180) or not
 * 0 < znear < zfar. */
narvis_status narvis_camera_matrix(const narvis_camera *cam, int32_t W, int32_t H,
                                   float vp_rowmajor[16], float *near_f, float *far_f);

/* Focal length in pixels of `cam` for an image H pixels high:
 * (H / 2) / tan(fovy / 2), composed in FP64 on the host and rounded once to
 * fp32 (the scale of narvis_gbuffer.radius).  Host only.  INVALID_ARG as
 * narvis_camera_matrix. */
narvis_status narvis_camera_focal_px(const narvis_camera *cam, int32_t H, float *focal_px);

/* Bytes of the bounded render's scratch for a W x H image:
 * 2 NARVIS_TILE_BOUNDS_MAX + 4 W H; 0 for invalid W, H. */
size_t narvis_raster_bounds_bytes(int32_t W, int32_t H);

/* Fill keys[W*H] with NARVIS_KEY_EMPTY. */
narvis_status narvis_raster_clear(uint64_t *keys, int32_t W, int32_t H, void *stream);

/* Render stage (Sec. 3.2: transform to screen space, keep the closest point
 * per pixel by a depth test).  For every point i < n, in fp32 with each
 * operation rounded in the order written (no fused multiply-add):
 *   cx = ((M00 x + M01 y) + M02 z) + M03,  cy likewise with row 1,
 *   w  = ((M30 x + M31 y) + M32 z) + M33   (the depth),
 *   kept iff near_f <= w <= far_f,
 *   sx = ((cx / w) * 0.5 + 0.5) * W,  sy = (0.5 - (cy / w) * 0.5) * H,
 *   kept iff 0 <= sx < W and 0 <= sy < H, pixel = (int)sy * W + (int)sx,
 *   keys[pixel] = min(keys[pixel], (bits(w) << 32) | i).
 * Keys are merged into the existing buffer (clear it first for a new frame).
 * n may be 0; n <= 2^32.  W, H >= 1 and W*H < 2^31.  `opts` may be NULL. */
narvis_status narvis_raster_render(const narvis_points *pts, uint64_t n, const float vp_rowmajor[16],
                                   float near_f, float far_f, int32_t W, int32_t H, uint64_t *keys,
                                   const narvis_raster_opts *opts, void *stream);

/* Resolve stage (Sec. 3.2: transfer the winner's attributes to the
 * G-buffers): reads gbuf->keys and writes the requested planes (see
 * narvis_gbuffer).  `pts` and vp_rowmajor are needed only for vel2d (the
 * winner's clip coordinates are recomputed exactly as in the render stage).
 * `attrs` may be NULL when no attribute plane is requested. */
narvis_status narvis_raster_resolve(const narvis_points *pts, const narvis_attrs *attrs, uint64_t n,
                                    const float vp_rowmajor[16], int32_t W, int32_t H,
                                    const narvis_gbuffer *gbuf, void *stream);

/* Whole frame: camera matrix, clear, render, resolve. */
narvis_status narvis_rasterize(const narvis_points *pts, const narvis_attrs *attrs, uint64_t n,
                               const narvis_camera *cam, int32_t W, int32_t H,
                               narvis_gbuffer *gbuf, void *stream);

/* ------------------------------------------------------------------------
 * Spatial layout (Morton order + per-batch boxes) for the batch-culled
 * render.  The compute rasterizer that the paper's rasterizer extends keeps
 * its points sorted along a Morton (Z-order) curve (Sec. 3.2; Sec. 4.3 names
 * its Morton-ordered data); a batch of consecutive points is then a compact
 * piece of space, and its bounding box lets the render skip the whole batch
 * when it lies outside the view volume or behind the depths already drawn.
 * The keys are those of the original order, bit for bit: every key carries
 * the point's original index, so ties still go to the lowest original index.
 * ------------------------------------------------------------------------ */

/* Points per batch of a layout (one box each). */
#define NARVIS_LAYOUT_BATCH 2048

/* A layout of n points, caller-owned device memory (16-byte aligned):
 *   x, y, z  float[n]       coordinates in layout order;
 *   index    uint32[n]      original index of each point (a permutation);
 *   boxes    float[nb][8]   per batch b of points [2048 b, 2048 (b+1)) the
 *                           box of its points with finite coordinates:
 *                           xmin, ymin, zmin, 0, xmax, ymax, zmax, 0
 *                           (+inf ... -inf when it has none),
 *                           nb = narvis_layout_batches(n);
 * and, optionally (all five or none), the render's depth sample: every 8th
 * point of the layout order (positions 0, 8, 16, ...), ns =
 * narvis_layout_samples(n) points, which the bounded render draws first so
 * that its depth bounds cover the whole cloud evenly:
 *   sx, sy, sz float[ns], sindex uint32[ns]  as x, y, z, index at 8 j,
 *   sboxes   float[nsb][8]  boxes of the sample's batches of 2048,
 *                           nsb = narvis_layout_batches(ns).
 * Without the sample the render draws every 8th batch first instead; in
 * layout order a batch is a compact piece of space, so those leave whole
 * screen regions without bounds on views that see the whole cloud.
 * Order (narvis_layout_build): the stable sort by the 30-bit Morton code of
 * each point's cell in a 1024^3 grid over the box [lo, hi] of all points
 * with finite coordinates: per axis t = (a - lo) * (1024 / (hi - lo)) in fp32
 * (each operation rounded; scale 0 when hi == lo), cell 0 if not t > 0, 1023
 * if t >= 1023, else floor(t); bit k of the x, y, z cells goes to bit 3k,
 * 3k + 1, 3k + 2 of the code; a point with a non-finite coordinate gets code
 * 2^30.  Equal codes keep the original order. */
typedef struct {
    float *x;
    float *y;
    float *z;
    uint32_t *index;
    float *boxes;
    float *sx;
    float *sy;
    float *sz;
    uint32_t *sindex;
    float *sboxes;
} narvis_layout;

/* Number of batches (boxes) of a layout of n points: ceil(n / 2048). */
uint64_t narvis_layout_batches(uint64_t n);

/* Points of a layout's depth sample: ceil(n / 8). */
uint64_t narvis_layout_samples(uint64_t n);

/* Device workspace bytes of narvis_layout_build for n points (16 n bytes
 * and a little more); 0 for n >= 2^32. */
size_t narvis_layout_workspace_size(uint64_t n);

/* Build the layout of the n points `pts` (original order, device, 4-byte
 * aligned) into `out` (see narvis_layout; every array 16-byte aligned and
 * disjoint from the input), using the device workspace `ws` (256-byte
 * aligned, caller-owned, contents overwritten).  n < 2^32.  INVALID_ARG on
 * bad arguments, WORKSPACE if ws_bytes is too small.  Asynchronous on
 * `stream`. */
narvis_status narvis_layout_build(const narvis_points *pts, uint64_t n, const narvis_layout *out, void *ws,
                                  size_t ws_bytes, void *stream);

/* Render stage over a layout: the same keys as narvis_raster_render over
 * the points in their original order (each key's low word is the original
 * index), with whole batches skipped when their box cannot hold a kept
 * point.  opts: variant AUTO or LDS only, bounds as for narvis_raster_render
 * (then batches are also skipped when their box's nearest depth exceeds
 * every tile bound under its screen rectangle; with the layout's depth
 * sample the sample is drawn first and then every batch, without it every
 * 8th batch and then the others); hint_keys must be NULL.  n < 2^32.
 * INVALID_ARG otherwise. */
narvis_status narvis_raster_render_layout(const narvis_layout *L, uint64_t n, const float vp_rowmajor[16],
                                          float near_f, float far_f, int32_t W, int32_t H, uint64_t *keys,
                                          const narvis_raster_opts *opts, void *stream);

/* Whole frame over a layout: camera matrix, clear, batch-culled render
 * (bounded when gbuf->bounds is given; gbuf->hint_keys must be NULL), and
 * the resolve of narvis_rasterize, which gathers the winners' attributes by
 * their original index from `attrs` (original order).  `pts` (original
 * order) is needed only for the vel2d planes and may be NULL otherwise. */
narvis_status narvis_rasterize_layout(const narvis_layout *L, const narvis_points *pts, const narvis_attrs *attrs,
                                      uint64_t n, const narvis_camera *cam, int32_t W, int32_t H,
                                      narvis_gbuffer *gbuf, void *stream);

/* ------------------------------------------------------------------------
 * World splat radius of every point: the mean distance to its four nearest
 * neighbours (Sec. 4.2, the hole-filling splat radius of the terrain), the
 * attribute that narvis_gbuffer.radius projects per pixel.  In fp32, each
 * operation rounded in the order written:
 *   d(i, j) = sqrt(((x_j - x_i)^2 + (y_j - y_i)^2) + (z_j - z_i)^2),
 *   r_i = (((d1 + d2) + d3) + d4) * 0.25 with d1 <= d2 <= d3 <= d4 the four
 *   smallest d(i, j) over the other points j with finite coordinates
 *   (duplicates of i count, at distance 0); with m < 4 such points the m
 *   smallest are summed the same way and divided by m; r_i = 0 when m = 0
 *   or when a coordinate of i is not finite.
 * Exact for every point: a uniform grid (cell size chosen from the cloud's
 * box and measured cell occupancy) settles most points within a few rings
 * of cells, and the others are found by a scan of all points.
 * ------------------------------------------------------------------------ */

/* Device workspace bytes of narvis_knn_radius for n points (about 28 n +
 * 12 * 2^ceil(log2(2 n)) bytes); 0 for n >= 2^32. */
size_t narvis_knn_radius_workspace_size(uint64_t n);

/* radius: float[n] device, written for every point.  pts: original order,
 * 4-byte aligned.  n < 2^32.  Synchronises `stream` (the grid is sized on
 * the host from the cloud's box and occupancy, read back during the call).
 * *cell_out (optional, host): the grid's cell edge; *unresolved_out
 * (optional, host): the points settled by the full scan.  INVALID_ARG on bad
 * arguments, WORKSPACE if ws_bytes is too small, DEVICE on a runtime error. */
narvis_status narvis_knn_radius(const narvis_points *pts, uint64_t n, float *radius, void *ws, size_t ws_bytes,
                                float *cell_out, uint32_t *unresolved_out, void *stream);

/* Largest image (in pixels) of narvis_rasterize_static, and the bytes of
 * its static device scratch: narvis_raster_bounds_bytes of that image
 * (3840 x 2160 = 8,294,400 pixels: 33,193,984 bytes per device). */
#define NARVIS_STATIC_MAX_PIXELS (3840u * 2160u)
#define NARVIS_STATIC_SCRATCH_BYTES (2u * NARVIS_TILE_BOUNDS_MAX + 4u * NARVIS_STATIC_MAX_PIXELS)

/* Allocation-free whole frame, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Computes exactly what narvis_rasterize computes in the
 * bounded mode, with the bounds scratch taken from a static device array of
 * NARVIS_STATIC_SCRATCH_BYTES bytes owned by the library instead of
 * gbuf->bounds: each device that the library runs on holds its copy from
 * the library's load until the process ends.  Allocates nothing (no
 * hipMalloc, hipFree or allocating library call); the first call on a
 * device looks the array's address up once.
 *   gbuf->bounds must be NULL (INVALID_ARG otherwise); gbuf->hint_keys is
 *   honoured as in narvis_rasterize.  W * H > NARVIS_STATIC_MAX_PIXELS:
 *   NARVIS_ERR_WORKSPACE, nothing enqueued.  Other errors as narvis_rasterize.
 * Every call on one device shares that device's scratch, and the scratch
 * keeps the last call's contents (each call overwrites every byte it reads,
 * so nothing carries over): calls that can overlap in time on one device
 * (unordered streams, several host threads) race and must be serialised by
 * the caller. */
narvis_status narvis_rasterize_static(const narvis_points *pts, const narvis_attrs *attrs, uint64_t n,
                                      const narvis_camera *cam, int32_t W, int32_t H, narvis_gbuffer *gbuf,
                                      void *stream);

/* Bytes of device workspace narvis_splat needs for n points at W x H
 * (0 if the arguments are invalid).  The size grows linearly with n: point
 * records, tile counts, two ping-pong copies of the (key, index) pairs (at
 * most four tiles per point for sigma <= 1.5 px, more for wider splats), the
 * radix histograms and the per-tile ranges. */
size_t narvis_splat_workspace_size(uint64_t n, int32_t W, int32_t H, const narvis_splat_params *p);

/* Gaussian splat renderer, the target the post-process network learns to
 * reproduce (Sec. 4.2: the forward pass of 3D Gaussian splatting over the
 * points, depth-sorted alpha blending).  Every point that survives the
 * rasterizer's cull becomes an isotropic screen-space Gaussian of standard
 * deviation sigma_px centred on (sx, sy).  Pixel (px, py) samples it at its
 * centre: d2 = ((px + 0.5) - sx)^2 + ((py + 0.5) - sy)^2 (fp32); Gaussians
 * with d2 > (3 sigma)^2 do not reach the pixel.  The Gaussians reaching a
 * pixel are composited nearest first, ties by lower index (the rasterizer's
 * key order): alpha = min(0.99, opacity * exp(-d2 / (2 sigma^2))), skipped
 * when below 1/255; with T = 1 initially, each contributor gives
 * T' = T (1 - alpha) and stops the pixel if T' < 1e-4, otherwise adds
 * colour * alpha * T and sets T = T'.  Background black.
 * img: float[3][H][W] device, written entirely.  workspace: device memory of
 * at least narvis_splat_workspace_size bytes, owned by the caller, contents
 * scratch.  n < 2^30.  INVALID_ARG on bad arguments, WORKSPACE if ws_bytes
 * is too small.
 *
 * Anisotropic splat (p->aniso = 1; the paper's GR for vector fields, Sec. 4.2:
 * Gaussians elongated along the vector v with covariance R diag(s, 1, 1) R^T,
 * R orthonormal with first column v / |v|).  Reading of the base size: the
 * world covariance is rho^2 (I + (s - 1) u u^T), u = v / |v| (0 when |v| is 0
 * or not finite), rho = sigma_px * w / f (the cross-section projects to about
 * sigma_px pixels at the point's depth; f = narvis_camera_focal_px).  The
 * screen covariance is J Sigma J^T, J the Jacobian of (sx, sy).  In fp32,
 * each operation rounded in the order written (M_rc: the clip matrix; c =
 * 0, 1, 2):
 *   ww = w * w;  hx = 0.5 * W;  hy = 0.5 * H
 *   jx_c = (((M0c * w) - (cx * M3c)) / ww) * hx
 *   jy_c = -((((M1c * w) - (cy * M3c)) / ww) * hy)
 *   sxx = (jx_0 jx_0 + jx_1 jx_1) + jx_2 jx_2   (likewise sxy = jx . jy, syy)
 *   vn = sqrt((vx vx + vy vy) + vz vz);  u = v / vn if 0 < vn <= FLT_MAX
 *   ax = (jx_0 u_0 + jx_1 u_1) + jx_2 u_2;  ay likewise with jy;  k = s - 1
 *   rho = (sigma * w) / f;  r2 = rho * rho
 *   S00 = (sxx + k (ax ax)) r2;  S01 = (sxy + k (ax ay)) r2;  S11 = (syy + k (ay ay)) r2
 *   det = (S00 S11) - (S01 S01); the point is dropped unless 0 < det <= FLT_MAX
 *   Q00 = S11 / det;  Q01 = -(S01 / det);  Q11 = S00 / det
 *   half extents rx = 3 sqrt(S00), ry = 3 sqrt(S11) replace 3 sigma in the
 *   footprint rectangle;  a pixel is reached iff
 *   q = ((Q00 dx) dx + ((Q01 dx) dy) 2) + (Q11 dy) dy <= 9, and
 *   alpha = min(0.99, opacity exp(-q / 2)).
 * Pairs beyond p->max_pairs are dropped (the image is then incomplete):
 * size the workspace with narvis_splat_count_pairs. */
narvis_status narvis_splat(const narvis_points *pts, const narvis_attrs *attrs, uint64_t n,
                           const narvis_camera *cam, int32_t W, int32_t H, float *img,
                           const narvis_splat_params *p, void *workspace, size_t ws_bytes, void *stream);

/* Exact number of (tile, point) pairs narvis_splat will emit for these
 * arguments (projection only, 64-bit sum; synchronises `stream`).  The
 * workspace needs narvis_splat_workspace_size(n, W, H, p) bytes for any
 * p->max_pairs (1 keeps it small).  Same errors as narvis_splat. */
narvis_status narvis_splat_count_pairs(const narvis_points *pts, const narvis_attrs *attrs, uint64_t n,
                                       const narvis_camera *cam, int32_t W, int32_t H,
                                       const narvis_splat_params *p, void *workspace, size_t ws_bytes,
                                       uint64_t *pairs, void *stream);

/* Number of (tile, key) pairs that the last narvis_splat call on `workspace`
 * emitted and depth-sorted (with the same n, W, H and *p): for every point
 * that survives the cull, one pair per 16 x 16 pixel tile touched by the
 * pixel rectangle [floor(sx - 3 sigma - 1), floor(sx + 3 sigma + 1)] x
 * [floor(sy - 3 sigma - 1), floor(sy + 3 sigma + 1)] clipped to the image
 * (fp32; the extra pixel covers the rounding of the footprint's ends).
 * Anisotropic: the rectangle uses rx, ry, and only its tiles whose pixel
 * centres the ellipse can reach count: the least q over the tile's centres
 * (exact arithmetic, evaluated in fp32) is at most 9 + 4e-6 M + 1e-3, M the
 * terms' magnitude bound (Q00 U^2 + 2 |Q01| U V + Q11 V^2, U and V the
 * largest offsets); no tile holding a reached pixel is dropped.  For
 * measurement (the sort's keys per second).  Copies one counter from the workspace to *pairs and synchronises
 * `stream`.  INVALID_ARG on bad arguments, WORKSPACE if ws_bytes is too small,
 * DEVICE if the copy fails. */
narvis_status narvis_splat_pair_count(const void *workspace, size_t ws_bytes, uint64_t n, int32_t W, int32_t H,
                                      const narvis_splat_params *p, uint64_t *pairs, void *stream);

/* ------------------------------------------------------------------------
 * Learned post-process (after the U-Net post-processor of Sec. 3.3): a
 * four-level encoder-decoder, 32-64-128-256 channels, two 3x3 conv + ReLU
 * per level, 2x2 average pooling down, bilinear x2 upsampling up with
 * [upsampled, skip] concatenation, a 1x1 head to RGB.  Convolutions run on
 * the matrix cores with bfloat16 operands and fp32 accumulation.
 *
 * Parameter blob (host fp32, narvis_net_param_count() values): for each
 * layer in the order e1a e1b e2a e2b e3a e3b e4a e4b d3a d3b d2a d2b d1a d1b
 * head, the weights [Cout][Cin][k][k] followed by the bias [Cout].  Layer
 * shapes (Cin -> Cout, k): 8->32,3  32->32,3  32->64,3  64->64,3
 * 64->128,3  128->128,3  128->256,3  256->256,3  384->128,3  128->128,3
 * 192->64,3  64->64,3  96->32,3  32->32,3  32->3,1.
 *
 * Network input: planar fp32 [B][8][H][W] G-buffer planes in the order
 * r, g, b, depth, v'x, v'y, theta, |v'| (the RGB+D+Vel2D set of Sec. 4.5.3);
 * the network sees 1/depth (0 where depth is 0).  Output: planar fp32
 * [B][3][H][W].  H and W must be multiples of 8 and at most 32768, and
 * B*W*H < 2^31 (INVALID_ARG otherwise).
 * ------------------------------------------------------------------------ */

typedef enum { NARVIS_PRECISION_BF16 = 0, NARVIS_PRECISION_FP8 = 1 } narvis_precision;

/* Opaque, library-owned network parameters on the device that was current
 * at creation (fp32 master copy, bf16 working copies, Adam moments).  Every
 * call that runs the network must be made with that device current
 * (INVALID_ARG otherwise). */
typedef struct narvis_weights narvis_weights;

/* Number of floats in the parameter blob. */
size_t narvis_net_param_count(void);

/* Create a parameter handle from a host blob of exactly
 * narvis_net_param_count() finite floats.  Allocates device memory and
 * synchronises the device.  INVALID_ARG on a wrong count or non-finite
 * values, OUT_OF_MEMORY if the allocation fails. */
narvis_status narvis_weights_create(const float *host_blob, size_t count, narvis_weights **out);

/* Release a handle (synchronises its device).  NULL is ignored. */
void narvis_weights_destroy(narvis_weights *w);

/* Copy the fp32 master parameters back to a host blob (synchronises). */
narvis_status narvis_weights_read(const narvis_weights *w, float *host_blob, size_t count);

/* Device workspace bytes for narvis_postprocess on B images of W x H
 * (0 if the dimensions are invalid). */
size_t narvis_postprocess_workspace_size(int32_t B, int32_t W, int32_t H);

/* Forward pass: feat [B][8][H][W] fp32 -> img [B][3][H][W] fp32 (device).
 * precision: NARVIS_PRECISION_BF16, or NARVIS_PRECISION_FP8 after
 * narvis_weights_calibrate_fp8 (UNSUPPORTED before it, and again after a
 * training step changed the parameters).  WORKSPACE if ws_bytes is too
 * small. */
narvis_status narvis_postprocess(const narvis_weights *w, const float *feat, int32_t B, int32_t W, int32_t H,
                                 float *img, int32_t precision, void *ws, size_t ws_bytes, void *stream);

/* Prepare FP8 inference (OCP e4m3 on the matrix cores, fp32 accumulation)
 * from the calibration batch feat [B][8][H][W] (training views, not the
 * images to be processed): run the bfloat16 forward, take each layer's input
 * max-abs as its static activation scale (max/448) and quantise each layer's
 * weights with one scale per output channel (max |W[co]| / 448).  Then choose
 * the layers that run in FP8 (e4m3 keeps three significand bits, and how far
 * a layer's rounding moves the image depends on the trained weights after
 * it): candidates are the ten layers below full resolution (the
 * full-resolution layers and the 1x1 head always stay in bfloat16); each
 * candidate alone in FP8 is scored by max |image - bfloat16 image| over the
 * calibration batch, and candidates are added in ascending order of that
 * score while the whole set's score stays within 0.025.  Needs
 * narvis_train_workspace_size(B, W, H) bytes of workspace; synchronises the
 * stream (the scales and scores are read back). */
narvis_status narvis_weights_calibrate_fp8(narvis_weights *w, const float *feat, int32_t B, int32_t W, int32_t H,
                                           void *ws, size_t ws_bytes, void *stream);

/* Layers chosen by the last narvis_weights_calibrate_fp8 (bit l set: layer l
 * in blob order runs in FP8).  UNSUPPORTED before a calibration. */
narvis_status narvis_weights_fp8_layers(const narvis_weights *w, uint32_t *mask);

/* Device workspace bytes for narvis_train_step / narvis_train_gradients. */
size_t narvis_train_workspace_size(int32_t B, int32_t W, int32_t H);

/* One training step on a batch: forward (activations kept in the
 * workspace), loss = mean squared error against target [B][3][H][W] plus
 * lam_tv * (mean |horizontal difference| + mean |vertical difference|) of
 * the output (Eq. 1 without its perceptual term), backward through every
 * layer, and an Adam update (beta 0.9 / 0.999, eps 1e-8, bias-corrected) of
 * the fp32 master parameters with learning rate lr.  The loss value is
 * written to *loss_out (device float).  Weight gradients are reduced in a
 * fixed order, so a step is bit-reproducible. */
narvis_status narvis_train_step(narvis_weights *w, const float *feat, const float *target, int32_t B, int32_t W,
                                int32_t H, float lr, float lam_tv, float *loss_out, void *ws, size_t ws_bytes,
                                void *stream);

/* The same forward, loss and backward without the update: the gradient of
 * the loss with respect to every parameter is written to grad_out (device
 * fp32, blob order) and the loss to *loss_out. */
narvis_status narvis_train_gradients(narvis_weights *w, const float *feat, const float *target, int32_t B, int32_t W,
                                     int32_t H, float lam_tv, float *grad_out, float *loss_out, void *ws,
                                     size_t ws_bytes, void *stream);

/* Where the training calls keep one tensor of the forward and backward
 * passes inside their workspace (for B images of W x H), so that a caller
 * can inspect it after narvis_train_step / narvis_train_gradients returned
 * (tests feed each layer's stored input, output and upstream gradient to a
 * reference and compare element by element).  Host only.
 * name: "feat" (network input, depth inverted), the layer outputs "e1a",
 * "sk1" (= e1b), "e2a", "sk2", "e3a", "sk3", "e4a", "e4b", "d3a", "d3b",
 * "d2a", "d2b", "d1a", "d1b", the pooled "pool1".."pool3", the upsampled
 * "up3", "up2", "up1", the head output "out", and the gradients "gy" (of the
 * loss with respect to "out"), "g_<layer>" (with respect to that layer's
 * output), "g_cat1".."g_cat3" (with respect to a decoder layer's
 * concatenated input [upsampled, skip]) and "g_pool1".."g_pool3".
 * *offset: byte offset in the workspace; *channels, *height, *width: the
 * tensor's shape per image; *dtype 0: bfloat16 NHWC [B][height][width][channels]
 * ("gy" holds 8 channels, the last 5 zero), 1: fp32 planar
 * [B][channels][height][width].  INVALID_ARG for an unknown name or invalid
 * dimensions. */
narvis_status narvis_train_tensor(int32_t B, int32_t W, int32_t H, const char *name, size_t *offset,
                                  int32_t *channels, int32_t *height, int32_t *width, int32_t *dtype);

/* ------------------------------------------------------------------------
 * The paper's own post-processor (Sec. 3.3, Fig. 4, Eq. 1): a U-Net with
 * gated convolutions.  Readings where the paper is silent:
 *   descriptors  d_0 = conv1x1(x_0) (8 -> 8 channels, bias), downscaled by
 *                2x2 average pooling to five scales d_0..d_4;
 *   encoder      level l = 0..4 (widths w_l, the paper's 64-128-256-512-1024
 *                by default): z = conv3x3([x_l | d_l]) (zero padding 1,
 *                bias) with 2 w_l outputs, y_l = ELU(z[:w_l]) *
 *                sigmoid(z[w_l:]), x_{l+1} = avgpool2(y_l); x_0 = the
 *                network input of narvis_postprocess (depth as 1/depth);
 *   decoder      level l = 3..0: u = transposed 2x2 stride-2 convolution
 *                (w_{l+1} -> w_l, bias) of the level above (y_4, then the
 *                decoder outputs): u[2i+a][2j+b][c] = sum_k in[i][j][k] *
 *                T[a][b][c][k] + bias[c]; z = conv3x3([u | y_l]) with 2 w_l
 *                outputs, y'_l = gate(z);
 *   head         conv1x1(w_0 -> 3), linear.
 * Parameter blob (fp32), per layer: desc (W [8][8], b [8]), enc0..enc4
 * (W [2 w_l][c_in][3][3], b [2 w_l], c_in = 16 for level 0, w_{l-1} + 8
 * otherwise), then for l = 3, 2, 1, 0: up_l (T [2][2][w_l][w_{l+1}],
 * b [w_l]) and dec_l (W [2 w_l][2 w_l][3][3], b [2 w_l]), then head
 * (W [3][w_0], b [3]).  Every w_l a multiple of 32 in [32, 4096].
 * Inference takes any H x W: the network runs on the grid padded to the next
 * multiples of 16 (the padded pixels are empty pixels, every input channel
 * 0) and the top-left H x W of its output is returned.  Training frames are
 * whole multiples of 16.  Activations bf16 NHWC, fp32 accumulation.
 * Training: the loss and Adam of narvis_train_step.
 * Parameters live on the device current at narvis_unet_create; the forward
 * and training calls must be made with that device current (INVALID_ARG
 * otherwise).
 * ------------------------------------------------------------------------ */
typedef struct narvis_unet narvis_unet;

/* Floats in the parameter blob for these widths (0 if invalid). */
size_t narvis_unet_param_count(const int32_t widths[5]);
/* Create (allocates device memory, synchronises).  INVALID_ARG on bad
 * widths, a wrong count or non-finite values; OUT_OF_MEMORY. */
narvis_status narvis_unet_create(const int32_t widths[5], const float *host_blob, size_t count, narvis_unet **out);
void narvis_unet_destroy(narvis_unet *u);
narvis_status narvis_unet_read(const narvis_unet *u, float *host_blob, size_t count);
/* Workspace bytes for B images of W x H; train != 0 for the training calls. */
size_t narvis_unet_workspace_size(const narvis_unet *u, int32_t B, int32_t W, int32_t H, int32_t train);
/* feat [B][8][H][W] fp32 (the network input of narvis_postprocess) ->
 * img [B][3][H][W] fp32. */
narvis_status narvis_unet_forward(const narvis_unet *u, const float *feat, int32_t B, int32_t W, int32_t H,
                                  float *img, void *ws, size_t ws_bytes, void *stream);
/* One training step (forward, loss, backward, Adam), as narvis_train_step. */
narvis_status narvis_unet_train_step(narvis_unet *u, const float *feat, const float *target, int32_t B, int32_t W,
                                     int32_t H, float lr, float lam_tv, float *loss_out, void *ws, size_t ws_bytes,
                                     void *stream);
/* Forward, loss and backward without the update: every parameter's gradient
 * to grad_out (device fp32, blob order), the loss to *loss_out. */
narvis_status narvis_unet_gradients(narvis_unet *u, const float *feat, const float *target, int32_t B, int32_t W,
                                    int32_t H, float lam_tv, float *grad_out, float *loss_out, void *ws,
                                    size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* NARVIS_H */

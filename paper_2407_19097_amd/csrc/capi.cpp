// C-ABI glue: argument validation, device facts and stage sequencing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "internal.h"
#include "narvis.h"

namespace narvis {

DeviceInfo device_info()
{
    static std::mutex mu;
    static std::vector<DeviceInfo> cache;
    static std::vector<bool> have;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)cache.size() <= dev) {
        cache.resize(dev + 1);
        have.resize(dev + 1, false);
    }
    if (!have[dev]) {
        DeviceInfo d{256, 8};
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) d.cus = v;
        // gfx950 (MI355X) and gfx942 carry 8 XCDs per device in single-partition mode;
        // with fewer compute units (a partitioned device) fall back to one.
        d.xcds = d.cus >= 64 ? 8 : 1;
        cache[dev] = d;
        have[dev] = true;
    }
    return cache[dev];
}

}  // namespace narvis

using namespace narvis;

namespace {

constexpr int64_t kMaxPixels = (int64_t(1) << 31) - 1;
constexpr int32_t kMaxSide = 1 << 24;
constexpr uint64_t kMaxPoints = uint64_t(1) << 32;

bool image_ok(int32_t W, int32_t H)
{
    return W >= 1 && H >= 1 && W <= kMaxSide && H <= kMaxSide && (int64_t)W * (int64_t)H <= kMaxPixels;
}

bool points_ok(const narvis_points *pts, uint64_t n)
{
    if (n > kMaxPoints) return false;
    if (n == 0) return true;
    return pts && pts->x && pts->y && pts->z;
}

bool matrix_ok(const float vp[16], float near_f, float far_f)
{
    if (!vp) return false;
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(vp[k])) return false;
    return std::isfinite(near_f) && std::isfinite(far_f) && near_f > 0.0f && near_f <= far_f;
}

int dtype_size(int32_t dt)
{
    switch (dt) {
    case NARVIS_U8: return 1;
    case NARVIS_U16: return 2;
    case NARVIS_F16: return 2;
    case NARVIS_F32: return 4;
    default: return 0;
    }
}

bool pack_attrs(const narvis_attrs *attrs, uint64_t n, AttrPack &out)
{
    out = AttrPack{};
    if (!attrs) return true;
    if (attrs->count < 0 || attrs->count > NARVIS_MAX_ATTRS) return false;
    out.count = attrs->count;
    for (int c = 0; c < attrs->count; ++c) {
        const narvis_attr &a = attrs->a[c];
        const int sz = dtype_size(a.dtype);
        if (sz == 0 || a.stride_bytes < sz) return false;
        if (n > 0 && !a.data) return false;
        // element alignment is required for the typed loads
        if ((reinterpret_cast<uintptr_t>(a.data) | (uintptr_t)a.stride_bytes) & (uintptr_t)(sz - 1)) return false;
        out.a[c].p = static_cast<const unsigned char *>(a.data);
        out.a[c].dtype = a.dtype;
        out.a[c].stride = a.stride_bytes;
    }
    return true;
}

narvis_status from_hip(hipError_t e) { return e == hipSuccess ? NARVIS_OK : NARVIS_ERR_DEVICE; }

// the rgb plane's colour source: a table over one attribute, or three uint8
// attributes
bool rgb_ok(const narvis_gbuffer &g, const AttrPack &pack)
{
    if (!g.rgb) return true;
    if (g.rgb_mode == NARVIS_COLOR_LUT) return g.lut && g.lut_attr >= 0 && g.lut_attr < pack.count;
    if (g.rgb_mode != NARVIS_COLOR_RGB8 || g.lut_attr < 0 || g.lut_attr + 2 >= pack.count) return false;
    for (int c = 0; c < 3; ++c)
        if (pack.a[g.lut_attr + c].dtype != NARVIS_U8) return false;
    return true;
}

}  // namespace

extern "C" const char *narvis_status_string(narvis_status s)
{
    switch (s) {
    case NARVIS_OK: return "ok";
    case NARVIS_ERR_INVALID_ARG: return "invalid argument";
    case NARVIS_ERR_OUT_OF_MEMORY: return "out of memory";
    case NARVIS_ERR_DEVICE: return "device error";
    case NARVIS_ERR_UNSUPPORTED: return "unsupported";
    case NARVIS_ERR_WORKSPACE: return "workspace too small";
    default: return "unknown status";
    }
}

extern "C" narvis_status narvis_raster_clear(uint64_t *keys, int32_t W, int32_t H, void *stream)
{
    if (!keys || !image_ok(W, H) || (reinterpret_cast<uintptr_t>(keys) & 7u)) return NARVIS_ERR_INVALID_ARG;
    return from_hip(launch_clear(keys, (int64_t)W * H, static_cast<hipStream_t>(stream)));
}

// a hint needs the bounded render's scratch, 8-byte alignment, and no
// overlap with the keys or the scratch (it is read while they are written)
// the radius plane reads attribute radius_attr with a finite focal length
static bool radius_ok(const narvis_gbuffer &g, const AttrPack &pack)
{
    if (!g.radius) return true;
    return g.radius_attr >= 0 && g.radius_attr < pack.count;
}

static bool hint_ok(const void *hint, const void *keys, const void *bounds, size_t bounds_bytes, int32_t W, int32_t H)
{
    if (!hint) return true;
    const uintptr_t h0 = reinterpret_cast<uintptr_t>(hint), h1 = h0 + 8 * (uintptr_t)W * (uintptr_t)H;
    const uintptr_t k0 = reinterpret_cast<uintptr_t>(keys), k1 = k0 + 8 * (uintptr_t)W * (uintptr_t)H;
    const uintptr_t b0 = reinterpret_cast<uintptr_t>(bounds), b1 = b0 + bounds_bytes;
    return bounds && !(h0 & 7u) && !(h0 < k1 && k0 < h1) && !(h0 < b1 && b0 < h1);
}

extern "C" size_t narvis_raster_bounds_bytes(int32_t W, int32_t H)
{
    if (!image_ok(W, H)) return 0;
    return 2 * (size_t)NARVIS_TILE_BOUNDS_MAX + 4 * (size_t)W * (size_t)H;
}

extern "C" narvis_status narvis_raster_render(const narvis_points *pts, uint64_t n, const float vp[16],
                                              float near_f, float far_f, int32_t W, int32_t H, uint64_t *keys,
                                              const narvis_raster_opts *opts, void *stream)
{
    if (!keys || !image_ok(W, H) || !points_ok(pts, n) || !matrix_ok(vp, near_f, far_f))
        return NARVIS_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(keys) & 7u) return NARVIS_ERR_INVALID_ARG;
    int32_t variant = opts ? opts->variant : NARVIS_RENDER_AUTO;
    int32_t grid = opts ? opts->grid_blocks : 0;
    void *bounds = opts ? opts->bounds : nullptr;
    if (variant < NARVIS_RENDER_AUTO || variant > NARVIS_RENDER_LDS || grid < 0) return NARVIS_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(bounds) & 3u) return NARVIS_ERR_INVALID_ARG;
    if (bounds && opts->bounds_bytes < narvis_raster_bounds_bytes(W, H)) return NARVIS_ERR_WORKSPACE;
    const uint64_t *hint = opts ? static_cast<const uint64_t *>(opts->hint_keys) : nullptr;
    if (!hint_ok(hint, keys, bounds, bounds ? opts->bounds_bytes : 0, W, H)) return NARVIS_ERR_INVALID_ARG;
    if (n > 0 && ((reinterpret_cast<uintptr_t>(pts->x) | reinterpret_cast<uintptr_t>(pts->y) |
                   reinterpret_cast<uintptr_t>(pts->z)) & 3u))
        return NARVIS_ERR_INVALID_ARG;
    const uint8_t *glyph = (opts && n > 0) ? opts->glyph : nullptr;
    const Proj P = make_proj(vp, near_f, far_f, W, H);
    return from_hip(launch_render(n ? pts->x : nullptr, n ? pts->y : nullptr, n ? pts->z : nullptr, n, P, keys,
                                  variant, grid, static_cast<uint16_t *>(bounds), hint, static_cast<hipStream_t>(stream),
                                  LayoutArgs{nullptr, nullptr, glyph}));
}

extern "C" narvis_status narvis_raster_resolve(const narvis_points *pts, const narvis_attrs *attrs, uint64_t n,
                                               const float vp[16], int32_t W, int32_t H,
                                               const narvis_gbuffer *gbuf, void *stream)
{
    if (!gbuf || !gbuf->keys || !image_ok(W, H) || (reinterpret_cast<uintptr_t>(gbuf->keys) & 7u))
        return NARVIS_ERR_INVALID_ARG;
    AttrPack pack;
    if (!pack_attrs(attrs, n, pack)) return NARVIS_ERR_INVALID_ARG;
    if (gbuf->attr && pack.count == 0) return NARVIS_ERR_INVALID_ARG;
    if (!rgb_ok(*gbuf, pack) || !radius_ok(*gbuf, pack)) return NARVIS_ERR_INVALID_ARG;
    if (gbuf->radius && !std::isfinite(gbuf->radius_focal_px)) return NARVIS_ERR_INVALID_ARG;
    if (gbuf->vel2d) {
        if (gbuf->vel_attr < 0 || gbuf->vel_attr + 2 >= pack.count) return NARVIS_ERR_INVALID_ARG;
        if (!points_ok(pts, n) || !vp) return NARVIS_ERR_INVALID_ARG;
        for (int k = 0; k < 16; ++k)
            if (!std::isfinite(vp[k])) return NARVIS_ERR_INVALID_ARG;
    }
    if (n > kMaxPoints) return NARVIS_ERR_INVALID_ARG;
    float ident[16] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1};
    const Proj P = make_proj(vp ? vp : ident, 1.0f, 1.0f, W, H);
    const bool need_pts = gbuf->vel2d != nullptr && n > 0;
    return from_hip(launch_resolve(need_pts ? pts->x : nullptr, need_pts ? pts->y : nullptr,
                                   need_pts ? pts->z : nullptr, n, P, pack, *gbuf,
                                   static_cast<hipStream_t>(stream)));
}

namespace {

// Whole frame with the bounds scratch `bounds` (NULL: single pass).
narvis_status rasterize_frame(const narvis_points *pts, const narvis_attrs *attrs, uint64_t n,
                              const narvis_camera *cam, int32_t W, int32_t H, const narvis_gbuffer *gbuf,
                              void *bounds, size_t bounds_bytes, void *stream)
{
    float vp[16], near_f = 0.0f, far_f = 0.0f;
    narvis_status st = narvis_camera_matrix(cam, W, H, vp, &near_f, &far_f);
    if (st != NARVIS_OK) return st;
    if (!gbuf || !gbuf->keys || !image_ok(W, H) || !points_ok(pts, n)) return NARVIS_ERR_INVALID_ARG;
    AttrPack pack;
    if (!pack_attrs(attrs, n, pack)) return NARVIS_ERR_INVALID_ARG;
    if (!matrix_ok(vp, near_f, far_f)) return NARVIS_ERR_INVALID_ARG;
    // validate the resolve arguments before enqueuing anything
    if (gbuf->attr && pack.count == 0) return NARVIS_ERR_INVALID_ARG;
    if (!rgb_ok(*gbuf, pack) || !radius_ok(*gbuf, pack)) return NARVIS_ERR_INVALID_ARG;
    if (gbuf->vel2d && (gbuf->vel_attr < 0 || gbuf->vel_attr + 2 >= pack.count)) return NARVIS_ERR_INVALID_ARG;
    narvis_gbuffer g = *gbuf;
    if (g.radius && narvis_camera_focal_px(cam, H, &g.radius_focal_px) != NARVIS_OK) return NARVIS_ERR_INVALID_ARG;
    if (n > 0 && ((reinterpret_cast<uintptr_t>(pts->x) | reinterpret_cast<uintptr_t>(pts->y) |
                   reinterpret_cast<uintptr_t>(pts->z)) & 3u))
        return NARVIS_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(gbuf->keys) & 7u) || (reinterpret_cast<uintptr_t>(bounds) & 3u))
        return NARVIS_ERR_INVALID_ARG;
    if (bounds && bounds_bytes < narvis_raster_bounds_bytes(W, H)) return NARVIS_ERR_WORKSPACE;
    if (!hint_ok(gbuf->hint_keys, gbuf->keys, bounds, bounds_bytes, W, H)) return NARVIS_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = from_hip(launch_clear(gbuf->keys, (int64_t)W * H, s));
    if (st != NARVIS_OK) return st;
    const Proj P = make_proj(vp, near_f, far_f, W, H);
    st = from_hip(launch_render(n ? pts->x : nullptr, n ? pts->y : nullptr, n ? pts->z : nullptr, n, P,
                                gbuf->keys, NARVIS_RENDER_AUTO, 0, static_cast<uint16_t *>(bounds),
                                static_cast<const uint64_t *>(gbuf->hint_keys), s,
                                LayoutArgs{nullptr, nullptr, n ? gbuf->glyph : nullptr}));
    if (st != NARVIS_OK) return st;
    return from_hip(launch_resolve(n ? pts->x : nullptr, n ? pts->y : nullptr, n ? pts->z : nullptr, n, P, pack, g,
                                   s));
}

}  // namespace

extern "C" narvis_status narvis_rasterize(const narvis_points *pts, const narvis_attrs *attrs, uint64_t n,
                                          const narvis_camera *cam, int32_t W, int32_t H, narvis_gbuffer *gbuf,
                                          void *stream)
{
    if (!gbuf) return NARVIS_ERR_INVALID_ARG;
    return rasterize_frame(pts, attrs, n, cam, W, H, gbuf, gbuf->bounds, gbuf->bounds_bytes, stream);
}

extern "C" narvis_status narvis_rasterize_static(const narvis_points *pts, const narvis_attrs *attrs, uint64_t n,
                                                 const narvis_camera *cam, int32_t W, int32_t H,
                                                 narvis_gbuffer *gbuf, void *stream)
{
    if (!gbuf || gbuf->bounds) return NARVIS_ERR_INVALID_ARG;
    if (!image_ok(W, H)) return NARVIS_ERR_INVALID_ARG;
    if ((uint64_t)W * (uint64_t)H > (uint64_t)NARVIS_STATIC_MAX_PIXELS) return NARVIS_ERR_WORKSPACE;
    void *scratch = nullptr;
    const narvis_status st = from_hip(static_scratch(&scratch));
    if (st != NARVIS_OK) return st;
    return rasterize_frame(pts, attrs, n, cam, W, H, gbuf, scratch, NARVIS_STATIC_SCRATCH_BYTES, stream);
}

// ---------------------------------------------------------------------------
// spatial layout
// ---------------------------------------------------------------------------

extern "C" uint64_t narvis_layout_batches(uint64_t n) { return (n + NARVIS_LAYOUT_BATCH - 1) / NARVIS_LAYOUT_BATCH; }

extern "C" uint64_t narvis_layout_samples(uint64_t n) { return (n + 7) / 8; }

extern "C" size_t narvis_layout_workspace_size(uint64_t n)
{
    if (n >= (uint64_t(1) << 32)) return 0;
    return (size_t)layout_workspace(n).bytes;
}

namespace {

bool aligned16(const void *p) { return !(reinterpret_cast<uintptr_t>(p) & 15u); }

// a layout of n points: every array given and 16-byte aligned; the depth
// sample's five arrays all given (and aligned) or all null
bool layout_ok(const narvis_layout *L, uint64_t n)
{
    if (!L || n >= (uint64_t(1) << 32)) return false;
    const int given = !!L->sx + !!L->sy + !!L->sz + !!L->sindex + !!L->sboxes;
    if (given != 0 && given != 5) return false;
    if (n == 0) return true;
    if (given && !(aligned16(L->sx) && aligned16(L->sy) && aligned16(L->sz) && aligned16(L->sindex) &&
                   aligned16(L->sboxes)))
        return false;
    return L->x && L->y && L->z && L->index && L->boxes && aligned16(L->x) && aligned16(L->y) && aligned16(L->z) &&
           aligned16(L->index) && aligned16(L->boxes);
}

}  // namespace

extern "C" narvis_status narvis_layout_build(const narvis_points *pts, uint64_t n, const narvis_layout *out, void *ws,
                                             size_t ws_bytes, void *stream)
{
    if (!points_ok(pts, n) || !layout_ok(out, n)) return NARVIS_ERR_INVALID_ARG;
    if (n > 0 && ((reinterpret_cast<uintptr_t>(pts->x) | reinterpret_cast<uintptr_t>(pts->y) |
                   reinterpret_cast<uintptr_t>(pts->z)) & 3u))
        return NARVIS_ERR_INVALID_ARG;
    if (!ws || ws_bytes < narvis_layout_workspace_size(n)) return NARVIS_ERR_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) & 255u) return NARVIS_ERR_INVALID_ARG;
    if (n == 0) return NARVIS_OK;
    // the outputs must not overlap the inputs (the gather reads them)
    const uintptr_t in[3] = {reinterpret_cast<uintptr_t>(pts->x), reinterpret_cast<uintptr_t>(pts->y),
                             reinterpret_cast<uintptr_t>(pts->z)};
    const uintptr_t o[3] = {reinterpret_cast<uintptr_t>(out->x), reinterpret_cast<uintptr_t>(out->y),
                            reinterpret_cast<uintptr_t>(out->z)};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (o[a] < in[b] + 4 * n && in[b] < o[a] + 4 * n) return NARVIS_ERR_INVALID_ARG;
    // the sample is gathered from the layout's own arrays: no overlap with them
    if (out->sx) {
        const uint64_t ns = narvis_layout_samples(n);
        const uintptr_t so[4] = {reinterpret_cast<uintptr_t>(out->sx), reinterpret_cast<uintptr_t>(out->sy),
                                 reinterpret_cast<uintptr_t>(out->sz), reinterpret_cast<uintptr_t>(out->sindex)};
        const uintptr_t lo[4] = {o[0], o[1], o[2], reinterpret_cast<uintptr_t>(out->index)};
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                if (so[a] < lo[b] + 4 * n && lo[b] < so[a] + 4 * ns) return NARVIS_ERR_INVALID_ARG;
    }
    return from_hip(launch_layout(pts->x, pts->y, pts->z, n, out->x, out->y, out->z, out->index, out->boxes, out->sx,
                                  out->sy, out->sz, out->sindex, out->sboxes, ws, static_cast<hipStream_t>(stream)));
}

extern "C" size_t narvis_knn_radius_workspace_size(uint64_t n)
{
    if (n >= (uint64_t(1) << 32)) return 0;
    return (size_t)knn_workspace(n).bytes;
}

extern "C" narvis_status narvis_knn_radius(const narvis_points *pts, uint64_t n, float *radius, void *ws,
                                           size_t ws_bytes, float *cell_out, uint32_t *unresolved_out, void *stream)
{
    if (!points_ok(pts, n) || n >= (uint64_t(1) << 32) || (n > 0 && !radius)) return NARVIS_ERR_INVALID_ARG;
    if (n > 0 && ((reinterpret_cast<uintptr_t>(pts->x) | reinterpret_cast<uintptr_t>(pts->y) |
                   reinterpret_cast<uintptr_t>(pts->z) | reinterpret_cast<uintptr_t>(radius)) & 3u))
        return NARVIS_ERR_INVALID_ARG;
    if (!ws || ws_bytes < narvis_knn_radius_workspace_size(n) || (reinterpret_cast<uintptr_t>(ws) & 255u))
        return NARVIS_ERR_WORKSPACE;
    KnnStats st{};
    const narvis_status r = from_hip(launch_knn(n ? pts->x : nullptr, n ? pts->y : nullptr, n ? pts->z : nullptr, n,
                                                radius, ws, static_cast<hipStream_t>(stream), &st));
    if (r != NARVIS_OK) return r;
    if (cell_out) *cell_out = st.cell;
    if (unresolved_out) *unresolved_out = st.unresolved;
    return NARVIS_OK;
}

namespace {

LayoutArgs layout_args(const narvis_layout *L, uint64_t n)
{
    LayoutArgs a{n ? L->index : nullptr, n ? reinterpret_cast<const float4 *>(L->boxes) : nullptr, nullptr};
    if (n && L->sx) {
        a.sx = L->sx;
        a.sy = L->sy;
        a.sz = L->sz;
        a.six = L->sindex;
        a.sbox = reinterpret_cast<const float4 *>(L->sboxes);
        a.ns = narvis_layout_samples(n);
    }
    return a;
}

}  // namespace

extern "C" narvis_status narvis_raster_render_layout(const narvis_layout *L, uint64_t n, const float vp[16],
                                                     float near_f, float far_f, int32_t W, int32_t H, uint64_t *keys,
                                                     const narvis_raster_opts *opts, void *stream)
{
    if (!keys || !image_ok(W, H) || !layout_ok(L, n) || !matrix_ok(vp, near_f, far_f)) return NARVIS_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(keys) & 7u) return NARVIS_ERR_INVALID_ARG;
    const int32_t variant = opts ? opts->variant : NARVIS_RENDER_AUTO;
    const int32_t grid = opts ? opts->grid_blocks : 0;
    void *bounds = opts ? opts->bounds : nullptr;
    if ((variant != NARVIS_RENDER_AUTO && variant != NARVIS_RENDER_LDS) || grid < 0) return NARVIS_ERR_INVALID_ARG;
    if (opts && (opts->hint_keys || opts->glyph)) return NARVIS_ERR_INVALID_ARG;
    if (reinterpret_cast<uintptr_t>(bounds) & 3u) return NARVIS_ERR_INVALID_ARG;
    if (bounds && opts->bounds_bytes < narvis_raster_bounds_bytes(W, H)) return NARVIS_ERR_WORKSPACE;
    const Proj P = make_proj(vp, near_f, far_f, W, H);
    return from_hip(launch_render(n ? L->x : nullptr, n ? L->y : nullptr, n ? L->z : nullptr, n, P, keys,
                                  NARVIS_RENDER_LDS, grid, static_cast<uint16_t *>(bounds), nullptr,
                                  static_cast<hipStream_t>(stream), layout_args(L, n)));
}

extern "C" narvis_status narvis_rasterize_layout(const narvis_layout *L, const narvis_points *pts,
                                                 const narvis_attrs *attrs, uint64_t n, const narvis_camera *cam,
                                                 int32_t W, int32_t H, narvis_gbuffer *gbuf, void *stream)
{
    float vp[16], near_f = 0.0f, far_f = 0.0f;
    narvis_status st = narvis_camera_matrix(cam, W, H, vp, &near_f, &far_f);
    if (st != NARVIS_OK) return st;
    if (!gbuf || !gbuf->keys || !image_ok(W, H) || !layout_ok(L, n)) return NARVIS_ERR_INVALID_ARG;
    if (gbuf->hint_keys || gbuf->glyph) return NARVIS_ERR_INVALID_ARG;
    AttrPack pack;
    if (!pack_attrs(attrs, n, pack)) return NARVIS_ERR_INVALID_ARG;
    if (!matrix_ok(vp, near_f, far_f)) return NARVIS_ERR_INVALID_ARG;
    if (gbuf->attr && pack.count == 0) return NARVIS_ERR_INVALID_ARG;
    if (!rgb_ok(*gbuf, pack) || !radius_ok(*gbuf, pack)) return NARVIS_ERR_INVALID_ARG;
    narvis_gbuffer g = *gbuf;
    if (g.radius && narvis_camera_focal_px(cam, H, &g.radius_focal_px) != NARVIS_OK) return NARVIS_ERR_INVALID_ARG;
    if (gbuf->vel2d) {
        if (gbuf->vel_attr < 0 || gbuf->vel_attr + 2 >= pack.count || !points_ok(pts, n)) return NARVIS_ERR_INVALID_ARG;
        if (n > 0 && ((reinterpret_cast<uintptr_t>(pts->x) | reinterpret_cast<uintptr_t>(pts->y) |
                       reinterpret_cast<uintptr_t>(pts->z)) & 3u))
            return NARVIS_ERR_INVALID_ARG;
    }
    if ((reinterpret_cast<uintptr_t>(gbuf->keys) & 7u) || (reinterpret_cast<uintptr_t>(gbuf->bounds) & 3u))
        return NARVIS_ERR_INVALID_ARG;
    if (gbuf->bounds && gbuf->bounds_bytes < narvis_raster_bounds_bytes(W, H)) return NARVIS_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = from_hip(launch_clear(gbuf->keys, (int64_t)W * H, s));
    if (st != NARVIS_OK) return st;
    const Proj P = make_proj(vp, near_f, far_f, W, H);
    st = from_hip(launch_render(n ? L->x : nullptr, n ? L->y : nullptr, n ? L->z : nullptr, n, P, gbuf->keys,
                                NARVIS_RENDER_LDS, 0, static_cast<uint16_t *>(gbuf->bounds), nullptr, s,
                                layout_args(L, n)));
    if (st != NARVIS_OK) return st;
    const bool need_pts = gbuf->vel2d != nullptr && n > 0;
    return from_hip(launch_resolve(need_pts ? pts->x : nullptr, need_pts ? pts->y : nullptr,
                                   need_pts ? pts->z : nullptr, n, P, pack, g, s));
}

namespace {

bool splat_params_ok(const narvis_splat_params *p, const AttrPack &pack)
{
    if (!p) return false;
    if (!(p->sigma_px > 0.0f && p->sigma_px <= 32.0f)) return false;
    if (!(p->opacity > 0.0f && p->opacity <= 1.0f)) return false;
    if (p->color_mode == NARVIS_COLOR_LUT) {
        if (!p->lut || p->color_attr < 0 || p->color_attr >= pack.count) return false;
        if (!std::isfinite(p->lut_min) || !std::isfinite(p->lut_inv_range)) return false;
    } else if (p->color_mode == NARVIS_COLOR_RGB8) {
        if (p->color_attr < 0 || p->color_attr + 2 >= pack.count) return false;
        for (int c = 0; c < 3; ++c)
            if (pack.a[p->color_attr + c].dtype != NARVIS_U8) return false;
    } else {
        return false;
    }
    if (p->aniso != 0 && p->aniso != 1) return false;
    if (p->aniso) {
        if (p->vel_attr < 0 || p->vel_attr + 2 >= pack.count || p->max_pairs == 0) return false;
        if (!(p->stretch >= 1.0f && p->stretch <= 1e6f)) return false;
    }
    return true;
}

bool splat_size_ok(uint64_t n, int32_t W, int32_t H, const narvis_splat_params *p)
{
    if (!image_ok(W, H) || n >= (uint64_t(1) << 30) || !p || !(p->sigma_px > 0.0f && p->sigma_px <= 32.0f)) return false;
    const SplatLayout L = splat_layout(n, W, H, p->sigma_px, p->aniso != 0, p->max_pairs);
    return L.cap < (uint64_t(1) << 32) && L.nblk < (uint64_t(1) << 31);
}

}  // namespace

extern "C" size_t narvis_splat_workspace_size(uint64_t n, int32_t W, int32_t H, const narvis_splat_params *p)
{
    if (!splat_size_ok(n, W, H, p)) return 0;
    return (size_t)splat_layout(n, W, H, p->sigma_px, p->aniso != 0, p->max_pairs).bytes;
}

extern "C" narvis_status narvis_splat(const narvis_points *pts, const narvis_attrs *attrs, uint64_t n,
                                      const narvis_camera *cam, int32_t W, int32_t H, float *img,
                                      const narvis_splat_params *p, void *workspace, size_t ws_bytes, void *stream)
{
    float vp[16], near_f = 0.0f, far_f = 0.0f;
    narvis_status st = narvis_camera_matrix(cam, W, H, vp, &near_f, &far_f);
    if (st != NARVIS_OK) return st;
    if (!img || !points_ok(pts, n) || !matrix_ok(vp, near_f, far_f) || !splat_size_ok(n, W, H, p))
        return NARVIS_ERR_INVALID_ARG;
    AttrPack pack;
    if (!pack_attrs(attrs, n, pack) || !splat_params_ok(p, pack)) return NARVIS_ERR_INVALID_ARG;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255u) ||
        (reinterpret_cast<uintptr_t>(img) & 3u))
        return NARVIS_ERR_INVALID_ARG;
    if (ws_bytes < (size_t)splat_layout(n, W, H, p->sigma_px, p->aniso != 0, p->max_pairs).bytes)
        return NARVIS_ERR_WORKSPACE;
    narvis_splat_params q = *p;
    if (narvis_camera_focal_px(cam, H, &q.focal_px) != NARVIS_OK) return NARVIS_ERR_INVALID_ARG;
    const Proj P = make_proj(vp, near_f, far_f, W, H);
    return from_hip(launch_splat(n ? pts->x : nullptr, n ? pts->y : nullptr, n ? pts->z : nullptr, n, P, pack, q, img,
                                 workspace, static_cast<hipStream_t>(stream)));
}

extern "C" narvis_status narvis_splat_pair_count(const void *workspace, size_t ws_bytes, uint64_t n, int32_t W,
                                                 int32_t H, const narvis_splat_params *p, uint64_t *pairs,
                                                 void *stream)
{
    if (!workspace || !pairs || !splat_size_ok(n, W, H, p) || (reinterpret_cast<uintptr_t>(workspace) & 255u))
        return NARVIS_ERR_INVALID_ARG;
    const SplatLayout L = splat_layout(n, W, H, p->sigma_px, p->aniso != 0, p->max_pairs);
    if (ws_bytes < (size_t)L.bytes) return NARVIS_ERR_WORKSPACE;
    // the exclusive scan of the tile counts in depth order leaves the total at scnt[n]
    uint32_t total = 0;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const char *src = static_cast<const char *>(workspace) + L.off_scnt + n * sizeof(uint32_t);
    if (hipMemcpyAsync(&total, src, sizeof(total), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return NARVIS_ERR_DEVICE;
    *pairs = total < L.cap ? total : L.cap;
    return NARVIS_OK;
}

extern "C" narvis_status narvis_splat_count_pairs(const narvis_points *pts, const narvis_attrs *attrs, uint64_t n,
                                                  const narvis_camera *cam, int32_t W, int32_t H,
                                                  const narvis_splat_params *p, void *workspace, size_t ws_bytes,
                                                  uint64_t *pairs, void *stream)
{
    float vp[16], near_f = 0.0f, far_f = 0.0f;
    narvis_status st = narvis_camera_matrix(cam, W, H, vp, &near_f, &far_f);
    if (st != NARVIS_OK) return st;
    if (!pairs || !points_ok(pts, n) || !matrix_ok(vp, near_f, far_f) || !splat_size_ok(n, W, H, p))
        return NARVIS_ERR_INVALID_ARG;
    AttrPack pack;
    if (!pack_attrs(attrs, n, pack) || !splat_params_ok(p, pack)) return NARVIS_ERR_INVALID_ARG;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255u)) return NARVIS_ERR_INVALID_ARG;
    if (ws_bytes < (size_t)splat_layout(n, W, H, p->sigma_px, p->aniso != 0, p->max_pairs).bytes)
        return NARVIS_ERR_WORKSPACE;
    narvis_splat_params q = *p;
    if (narvis_camera_focal_px(cam, H, &q.focal_px) != NARVIS_OK) return NARVIS_ERR_INVALID_ARG;
    const Proj P = make_proj(vp, near_f, far_f, W, H);
    return from_hip(launch_splat_count(n ? pts->x : nullptr, n ? pts->y : nullptr, n ? pts->z : nullptr, n, P, pack,
                                       q, workspace, static_cast<hipStream_t>(stream), pairs));
}

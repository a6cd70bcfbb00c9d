/*
 * CPU oracle for the multi-attribute point rasterizer -- TEST INFRASTRUCTURE.
 *
 * Only the test-suite, the package's smoke check and the CPU-baseline leg of
 * the benchmark may load this file's library.  It shares no code with the GPU
 * library and is written to be checked against the paper by eye: one loop
 * over points, one loop over pixels, every floating-point operation rounded to
 * fp32 in the order written (build with -O2 -ffp-contract=off, SSE scalar
 * arithmetic, no fast-math, denormals kept).
 *
 * What it computes (NARVis, Sec. 3.2 "Multi-Attribute Compute Rasterizer"):
 *   render  -- every point is transformed from world to screen space; the
 *              point closest to the camera wins its pixel through a z-test
 *              on a custom framebuffer.  The framebuffer word is the 64-bit
 *              key (fp32 depth bits << 32 | point index): depth is positive
 *              inside the frustum, so unsigned key order is depth order, and
 *              equal depths fall to the lower index.
 *   resolve -- the winning point's attributes are copied into per-pixel
 *              G-buffer planes; no averaging of overlapping points.
 *   derived -- optional channels used as network input (Sec. 4.5.3): a colour
 *              from a 256-entry transfer-function table, and Vel2D =
 *              (v'x, v'y, theta, |v'|) of the perspective-projected velocity.
 *
 * Readings where the paper is silent (each is also listed in the design notes):
 *   depth       = clip w = distance along the view axis, fp32;
 *   cull        = keep iff near <= w <= far and the screen position falls
 *                 inside [0,W) x [0,H); NaN fails every comparison;
 *   pixel       = (int)sy * W + (int)sx, row 0 at the top of the image;
 *   empty pixel = key 0xFFFFFFFFFFFFFFFF, depth 0, every channel 0;
 *   attributes  = exact conversion to fp32 (u8, u16 values; f16 widened
 *                 exactly; a half NaN becomes the quiet fp32 NaN with the
 *                 same sign and payload);
 *   Vel2D       = derivative of the normalised device coordinates along v,
 *                 theta = atan2(v'y, v'x) / pi (the one inexact channel).
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define ORACLE_EMPTY 0xFFFFFFFFFFFFFFFFull

enum { OR_U8 = 0, OR_U16 = 1, OR_F16 = 2, OR_F32 = 3 };

static uint32_t bits_of(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static float float_of(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }

/* World -> screen for one point.  Returns 1 when the point survives the cull,
 * with its pixel, its depth w and its clip-space cx, cy. */
static int project(const float *M, float near_f, float far_f, int32_t W, int32_t H,
                   float x, float y, float z,
                   int64_t *pix, float *w_out, float *cx_out, float *cy_out)
{
    float cx = M[0] * x;
    cx = cx + M[1] * y;
    cx = cx + M[2] * z;
    cx = cx + M[3];
    float cy = M[4] * x;
    cy = cy + M[5] * y;
    cy = cy + M[6] * z;
    cy = cy + M[7];
    float w = M[12] * x;
    w = w + M[13] * y;
    w = w + M[14] * z;
    w = w + M[15];
    if (!(w >= near_f && w <= far_f)) return 0;
    float nx = cx / w;
    float ny = cy / w;
    float sx = nx * 0.5f;
    sx = sx + 0.5f;
    sx = sx * (float)W;
    float sy = ny * 0.5f;
    sy = 0.5f - sy;
    sy = sy * (float)H;
    if (!(sx >= 0.0f && sx < (float)W && sy >= 0.0f && sy < (float)H)) return 0;
    *pix = (int64_t)(int32_t)sy * (int64_t)W + (int64_t)(int32_t)sx;
    *w_out = w;
    *cx_out = cx;
    *cy_out = cy;
    return 1;
}

/* Render stage: keys[H*W] receives, per pixel, the minimum key of the points
 * that land there (or the empty key). */
void oracle_render(const float *x, const float *y, const float *z, uint64_t n,
                   const float *M, float near_f, float far_f, int32_t W, int32_t H,
                   uint64_t *keys)
{
    const int64_t npx = (int64_t)W * (int64_t)H;
    for (int64_t p = 0; p < npx; ++p) keys[p] = ORACLE_EMPTY;
    for (uint64_t i = 0; i < n; ++i) {
        int64_t p;
        float w, cx, cy;
        if (!project(M, near_f, far_f, W, H, x[i], y[i], z[i], &p, &w, &cx, &cy)) continue;
        uint64_t key = ((uint64_t)bits_of(w) << 32) | (uint64_t)(uint32_t)i;
        if (key < keys[p]) keys[p] = key;
    }
}

/* Glyph-priority render (the paper's VisGlyph, Sec. 4.3 "Glyph Stylization
 * Support": the frontmost glyph point is rendered and non-glyph points in
 * front of it are ignored).  Reading: a pixel that some glyph point reaches
 * keeps the nearest glyph point; a pixel that no glyph point reaches keeps
 * the nearest point, as in the plain render.  glyph[i] != 0 marks glyph
 * points.  The ranking (not a glyph, depth, index) is packed in the key by
 * setting bit 63 for non-glyph points: depth bits never use bit 31 (w > 0). */
void oracle_render_glyph(const float *x, const float *y, const float *z, uint64_t n,
                         const float *M, float near_f, float far_f, int32_t W, int32_t H,
                         const uint8_t *glyph, uint64_t *keys)
{
    const int64_t npx = (int64_t)W * (int64_t)H;
    for (int64_t p = 0; p < npx; ++p) keys[p] = ORACLE_EMPTY;
    for (uint64_t i = 0; i < n; ++i) {
        int64_t p;
        float w, cx, cy;
        if (!project(M, near_f, far_f, W, H, x[i], y[i], z[i], &p, &w, &cx, &cy)) continue;
        uint64_t rank = glyph[i] ? 0u : 1u;
        uint64_t key = (rank << 63) | ((uint64_t)bits_of(w) << 32) | (uint64_t)(uint32_t)i;
        if (key < keys[p]) keys[p] = key;
    }
}

/* The same render restricted to points [i0, i1), merging into an existing key
 * buffer (used to time bounded samples; min is order-free, so rendering a
 * range into a buffer that already holds other ranges gives the same result). */
void oracle_render_range(const float *x, const float *y, const float *z, uint64_t i0, uint64_t i1,
                         const float *M, float near_f, float far_f, int32_t W, int32_t H,
                         uint64_t *keys)
{
    for (uint64_t i = i0; i < i1; ++i) {
        int64_t p;
        float w, cx, cy;
        if (!project(M, near_f, far_f, W, H, x[i], y[i], z[i], &p, &w, &cx, &cy)) continue;
        uint64_t key = ((uint64_t)bits_of(w) << 32) | (uint64_t)(uint32_t)i;
        if (key < keys[p]) keys[p] = key;
    }
}

/* Project a single point; exposed so tests can pin the transform directly.
 * Returns the pixel index or -1 when culled; writes w. */
int64_t oracle_project_point(const float *M, float near_f, float far_f, int32_t W, int32_t H,
                             float x, float y, float z, float *w_out)
{
    int64_t p;
    float w, cx, cy;
    if (!project(M, near_f, far_f, W, H, x, y, z, &p, &w, &cx, &cy)) return -1;
    *w_out = w;
    return p;
}

static float half_to_float(uint16_t h)
{
    uint32_t sign = (uint32_t)(h >> 15) << 31;
    uint32_t e = (h >> 10) & 0x1F;
    uint32_t m = h & 0x3FF;
    if (e == 0) {
        /* zero or subnormal: m * 2^-24, exact in fp32 */
        float v = ldexpf((float)m, -24);
        return (h >> 15) ? -v : v;
    }
    if (e == 31) {
        if (m == 0) return float_of(sign | 0x7F800000u);
        return float_of(sign | 0x7FC00000u | (m << 13));
    }
    return float_of(sign | ((e - 15 + 127) << 23) | (m << 13));
}

typedef struct {
    const void *data;
    int32_t dtype;
    int32_t stride_bytes;
} oracle_attr;

static float attr_value(const oracle_attr *a, uint64_t i)
{
    const unsigned char *base = (const unsigned char *)a->data + (size_t)i * (size_t)a->stride_bytes;
    switch (a->dtype) {
    case OR_U8: return (float)(*(const uint8_t *)base);
    case OR_U16: { uint16_t v; memcpy(&v, base, 2); return (float)v; }
    case OR_F16: { uint16_t v; memcpy(&v, base, 2); return half_to_float(v); }
    default: { float v; memcpy(&v, base, 4); return v; }
    }
}

/* Projected splat radius of each pixel's winner (Sec. 3.2: MACR computes
 * the projected point radius; Sec. 4.2: the world radius is the mean distance
 * to the four nearest neighbours): radius_px = (r * focal_px) / depth, with r
 * the winner's world radius (fp32 attribute), focal_px = (H / 2) / tan(fovy / 2)
 * and depth the winner's w; 0 for an empty pixel. */
void oracle_resolve_radius(const uint64_t *keys, int32_t W, int32_t H, const float *r_world, float focal_px,
                           float *out)
{
    const int64_t npx = (int64_t)W * (int64_t)H;
    for (int64_t p = 0; p < npx; ++p) {
        uint64_t k = keys[p];
        if (k == ORACLE_EMPTY) {
            out[p] = 0.0f;
            continue;
        }
        float w = float_of((uint32_t)(k >> 32) & 0x7FFFFFFFu);
        float r = r_world[k & 0xFFFFFFFFull];
        float t = r * focal_px;
        out[p] = t / w;
    }
}

/* Resolve stage plus optional derived channels.
 *   depth  [H*W]        or NULL
 *   chan   [nattr][H*W] or NULL   raw attributes of the winner
 *   rgb    [3][H*W]     or NULL   rgb_mode 0: lut[q][c] with q the 256-bin index of attribute
 *                                 lut_attr; rgb_mode 1: attribute lut_attr + c (uint8) times
 *                                 the fp32 value of 1/255
 *   vel2d  [4][H*W]     or NULL   (v'x, v'y, theta/pi, |v'|) from attributes vel_attr..+2
 */
void oracle_resolve(const uint64_t *keys, int32_t W, int32_t H,
                    const float *x, const float *y, const float *z, const float *M,
                    const oracle_attr *attrs, int32_t nattr,
                    float *depth, float *chan,
                    float *rgb, const float *lut, int32_t lut_attr, float lut_min, float lut_inv_range,
                    float *vel2d, int32_t vel_attr, int32_t rgb_mode)
{
    const int64_t npx = (int64_t)W * (int64_t)H;
    const float pi_f = 3.14159265358979323846f;
    for (int64_t p = 0; p < npx; ++p) {
        uint64_t k = keys[p];
        int empty = (k == ORACLE_EMPTY);
        uint64_t i = k & 0xFFFFFFFFull;
        if (depth) depth[p] = empty ? 0.0f : float_of((uint32_t)(k >> 32) & 0x7FFFFFFFu);
        if (chan)
            for (int32_t c = 0; c < nattr; ++c)
                chan[(int64_t)c * npx + p] = empty ? 0.0f : attr_value(&attrs[c], i);
        if (rgb && rgb_mode == 1) {
            const float inv255 = 1.0f / 255.0f;
            for (int c = 0; c < 3; ++c)
                rgb[(int64_t)c * npx + p] = empty ? 0.0f : attr_value(&attrs[lut_attr + c], i) * inv255;
        } else if (rgb) {
            int q = 0;
            if (!empty) {
                float t = attr_value(&attrs[lut_attr], i) - lut_min;
                t = t * lut_inv_range;
                t = t * 256.0f;
                if (!(t > 0.0f)) q = 0;
                else if (t >= 255.0f) q = 255;
                else q = (int)t;
            }
            for (int c = 0; c < 3; ++c)
                rgb[(int64_t)c * npx + p] = empty ? 0.0f : lut[q * 3 + c];
        }
        if (vel2d) {
            float o0 = 0.0f, o1 = 0.0f, o2 = 0.0f, o3 = 0.0f;
            if (!empty) {
                float px = x[i], py = y[i], pz = z[i];
                float cx = M[0] * px; cx = cx + M[1] * py; cx = cx + M[2] * pz; cx = cx + M[3];
                float cy = M[4] * px; cy = cy + M[5] * py; cy = cy + M[6] * pz; cy = cy + M[7];
                float w = M[12] * px; w = w + M[13] * py; w = w + M[14] * pz; w = w + M[15];
                float vx = attr_value(&attrs[vel_attr], i);
                float vy = attr_value(&attrs[vel_attr + 1], i);
                float vz = attr_value(&attrs[vel_attr + 2], i);
                float dcx = M[0] * vx; dcx = dcx + M[1] * vy; dcx = dcx + M[2] * vz;
                float dcy = M[4] * vx; dcy = dcy + M[5] * vy; dcy = dcy + M[6] * vz;
                float dw = M[12] * vx; dw = dw + M[13] * vy; dw = dw + M[14] * vz;
                float ww = w * w;
                float ax = dcx * w; float bx = cx * dw; float nxv = ax - bx;
                float ay = dcy * w; float by = cy * dw; float nyv = ay - by;
                o0 = nxv / ww;
                o1 = nyv / ww;
                float m2 = o0 * o0; m2 = m2 + o1 * o1;
                o3 = sqrtf(m2);
                o2 = (float)atan2((double)o1, (double)o0) / pi_f;
            }
            vel2d[0 * npx + p] = o0;
            vel2d[1 * npx + p] = o1;
            vel2d[2 * npx + p] = o2;
            vel2d[3 * npx + p] = o3;
        }
    }
}

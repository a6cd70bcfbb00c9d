/*
 * CPU oracle for the Gaussian splat renderer -- TEST INFRASTRUCTURE.
 *
 * Only the test-suite, the package's smoke check and the CPU-baseline leg of
 * the benchmark may load this file's library; it shares no code with the GPU
 * library.
 *
 * What it computes.  The paper's target renderer is the forward pass of 3D
 * Gaussian splatting applied to the points (Sec. 4.2, "Gaussian Renderer"):
 * each point becomes a Gaussian, the Gaussians covering a pixel are sorted by
 * depth and alpha-blended front to back.  This build uses the isotropic
 * screen-space form: a Gaussian of standard deviation sigma pixels centred
 * on the point's projected position.  Steps, per frame:
 *   1. project every point exactly as the rasterizer does (fp32, same cull);
 *      its centre is (sx, sy) in continuous pixel units;
 *   2. a pixel (px, py) samples at its centre: dx = (px + 0.5) - sx,
 *      dy = (py + 0.5) - sy, d2 = dx*dx + dy*dy (fp32, as the GPU), and the
 *      Gaussian reaches the pixel only if d2 <= (3 sigma)^2;
 *   3. alpha = min(0.99, opacity * exp(-d2 / (2 sigma^2))), skipped when
 *      alpha < 1/255;
 *   4. contributors are taken in ascending order of the rasterizer's key
 *      (depth bits << 32 | index): nearest first, ties to the lower index;
 *   5. T starts at 1; for each contributor T' = T (1 - alpha); if T' < 1e-4
 *      the pixel is finished and this contributor is dropped, otherwise
 *      C += colour * alpha * T and T = T';
 *   6. the background is black.
 * The clamp at 0.99, the 1/255 skip and the 1e-4 termination are the
 * conventions of the published 3DGS forward rasterizer.  Blending is done in
 * fp64; the discrete choices that depend only on exact fp32 quantities (cull,
 * footprint) are taken in fp32 exactly as the GPU does.
 *
 * The optional `fragile` output marks pixels where one of these decisions
 * (the 1/255 skip, the 1e-4 termination) was taken within a relative 1e-5 of
 * its threshold: there an fp32 evaluation may legitimately decide the other
 * way, and a comparison with fp32 code must allow for that.
 *
 * Colour of a point: mode 0 looks its attribute `lut_attr` up in a 256-entry
 * table (same binning as the rasterizer's colour plane); mode 1 reads three
 * uint8 attributes and divides by 255.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t key;
    float sx, sy;
    uint32_t idx;
} splat_rec;

typedef struct {
    const void *data;
    int32_t dtype;
    int32_t stride_bytes;
} splat_attr;

static uint32_t fbits(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }

static float half_value(uint16_t h)
{
    int e = (h >> 10) & 0x1F, m = h & 0x3FF;
    float v;
    if (e == 0) v = ldexpf((float)m, -24);
    else if (e == 31) v = m ? NAN : INFINITY;
    else v = ldexpf((float)(m | 0x400), e - 25);
    return (h & 0x8000) ? -v : v;
}

static float attr_at(const splat_attr *a, uint64_t i)
{
    const unsigned char *p = (const unsigned char *)a->data + (size_t)i * (size_t)a->stride_bytes;
    switch (a->dtype) {
    case 0: return (float)p[0];
    case 1: { uint16_t v; memcpy(&v, p, 2); return (float)v; }
    case 2: { uint16_t v; memcpy(&v, p, 2); return half_value(v); }
    default: { float v; memcpy(&v, p, 4); return v; }
    }
}

static int cmp_rec(const void *a, const void *b)
{
    uint64_t ka = ((const splat_rec *)a)->key, kb = ((const splat_rec *)b)->key;
    return ka < kb ? -1 : (ka > kb ? 1 : 0);
}

/* Returns 0 on success, -1 if memory could not be obtained. img is [3][H*W] doubles. */
int oracle_splat(const float *x, const float *y, const float *z, uint64_t n,
                 const float *M, float near_f, float far_f, int32_t W, int32_t H,
                 float sigma, float opacity, int32_t color_mode,
                 const splat_attr *attrs, int32_t nattr,
                 const float *lut, int32_t lut_attr, float lut_min, float lut_inv_range,
                 double *img, unsigned char *fragile)
{
    (void)nattr;
    const int64_t npx = (int64_t)W * H;
    splat_rec *rec = (splat_rec *)malloc((n ? n : 1) * sizeof(splat_rec));
    double *T = (double *)malloc(npx * sizeof(double));
    unsigned char *done = (unsigned char *)calloc(npx, 1);
    if (!rec || !T || !done) { free(rec); free(T); free(done); return -1; }
    uint64_t m = 0;
    for (uint64_t i = 0; i < n; ++i) {
        float cx = M[0] * x[i]; cx = cx + M[1] * y[i]; cx = cx + M[2] * z[i]; cx = cx + M[3];
        float cy = M[4] * x[i]; cy = cy + M[5] * y[i]; cy = cy + M[6] * z[i]; cy = cy + M[7];
        float w = M[12] * x[i]; w = w + M[13] * y[i]; w = w + M[14] * z[i]; w = w + M[15];
        if (!(w >= near_f && w <= far_f)) continue;
        float nx = cx / w, ny = cy / w;
        float sx = nx * 0.5f; sx = sx + 0.5f; sx = sx * (float)W;
        float sy = ny * 0.5f; sy = 0.5f - sy; sy = sy * (float)H;
        if (!(sx >= 0.0f && sx < (float)W && sy >= 0.0f && sy < (float)H)) continue;
        rec[m].key = ((uint64_t)fbits(w) << 32) | (uint32_t)i;
        rec[m].sx = sx;
        rec[m].sy = sy;
        rec[m].idx = (uint32_t)i;
        ++m;
    }
    qsort(rec, m, sizeof(splat_rec), cmp_rec);
    for (int64_t p = 0; p < npx; ++p) T[p] = 1.0;
    for (int64_t p = 0; p < 3 * npx; ++p) img[p] = 0.0;
    if (fragile) memset(fragile, 0, (size_t)npx);
    const float reach = 3.0f * sigma;
    const float cut2 = reach * reach;
    const double inv2s2 = 1.0 / (2.0 * (double)sigma * (double)sigma);
    const int R = (int)ceilf(reach) + 1;
    for (uint64_t k = 0; k < m; ++k) {
        const uint64_t i = rec[k].idx;
        double col[3];
        if (color_mode == 0) {
            float t = attr_at(&attrs[lut_attr], i) - lut_min;
            t = t * lut_inv_range;
            t = t * 256.0f;
            int q = !(t > 0.0f) ? 0 : (t >= 255.0f ? 255 : (int)t);
            for (int c = 0; c < 3; ++c) col[c] = (double)lut[q * 3 + c];
        } else {
            for (int c = 0; c < 3; ++c) col[c] = (double)attr_at(&attrs[c], i) / 255.0;
        }
        const float sx = rec[k].sx, sy = rec[k].sy;
        const int cxp = (int)sx, cyp = (int)sy;
        for (int py = cyp - R; py <= cyp + R; ++py) {
            if (py < 0 || py >= H) continue;
            for (int px = cxp - R; px <= cxp + R; ++px) {
                if (px < 0 || px >= W) continue;
                const int64_t p = (int64_t)py * W + px;
                if (done[p]) continue;
                float dx = ((float)px + 0.5f) - sx;
                float dy = ((float)py + 0.5f) - sy;
                float d2 = dx * dx;
                d2 = d2 + dy * dy;
                if (!(d2 <= cut2)) continue;
                double a = (double)opacity * exp(-(double)d2 * inv2s2);
                if (a > 0.99) a = 0.99;
                if (fragile && fabs(a - 1.0 / 255.0) <= 1e-5 / 255.0) fragile[p] = 1;
                if (a < 1.0 / 255.0) continue;
                double Tn = T[p] * (1.0 - a);
                if (fragile && fabs(Tn - 1e-4) <= 1e-9) fragile[p] = 1;
                if (Tn < 1e-4) { done[p] = 1; continue; }
                for (int c = 0; c < 3; ++c) img[c * npx + p] += col[c] * a * T[p];
                T[p] = Tn;
            }
        }
    }
    free(rec);
    free(T);
    free(done);
    return 0;
}

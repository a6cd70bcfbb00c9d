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

/* Anisotropic splat (the paper's GR for vector fields, Sec. 4.2: Gaussians
 * elongated along the vector v, covariance R diag(s, 1, 1) R^T).  Reading of
 * the base size: world covariance rho^2 (I + (s - 1) u u^T) with u = v / |v|
 * (0 when |v| is 0 or not finite) and rho = sigma w / f, f the focal length in
 * pixels, so that the cross-section covers about sigma pixels at the point's
 * depth.  The screen covariance is J Sigma J^T, J the Jacobian of the screen
 * position (sx, sy) with respect to the world position.  The footprint (the
 * inverse covariance and the 3-sigma extents) is computed in fp32, operation
 * by operation, as the library's header states it; the blending is fp64.
 * A pixel is reached when q = dx^T Sigma^-1 dx <= 9 (3 sigma), with
 * alpha = min(0.99, opacity exp(-q / 2)); everything else (order, skip,
 * termination, colour) as oracle_splat.  window (optional): {x0, y0, x1, y1},
 * only the pixels of [x0, x1) x [y0, y1) are composited (the others stay 0),
 * for checks of large frames on a region. */
static int footprint(const float *M, float w, float cx, float cy, int32_t W, int32_t H, float vx, float vy,
                     float vz, float sigma, float k, float focal, float q[3], float ext[2])
{
    const float ww = w * w;
    const float hx = 0.5f * (float)W, hy = 0.5f * (float)H;
    float jx[3], jy[3];
    for (int c = 0; c < 3; ++c) {
        float a = M[c] * w;          /* row 0 */
        float b = cx * M[12 + c];    /* row 3 */
        float t = a - b;
        t = t / ww;
        jx[c] = t * hx;
        a = M[4 + c] * w;            /* row 1 */
        b = cy * M[12 + c];
        t = a - b;
        t = t / ww;
        t = t * hy;
        jy[c] = -t;
    }
    float sxx = jx[0] * jx[0]; sxx = sxx + jx[1] * jx[1]; sxx = sxx + jx[2] * jx[2];
    float sxy = jx[0] * jy[0]; sxy = sxy + jx[1] * jy[1]; sxy = sxy + jx[2] * jy[2];
    float syy = jy[0] * jy[0]; syy = syy + jy[1] * jy[1]; syy = syy + jy[2] * jy[2];
    float vn = vx * vx; vn = vn + vy * vy; vn = vn + vz * vz;
    vn = sqrtf(vn);
    float ux = 0.0f, uy = 0.0f, uz = 0.0f;
    if (vn > 0.0f && vn <= 3.40282347e38f) { ux = vx / vn; uy = vy / vn; uz = vz / vn; }
    float ax = jx[0] * ux; ax = ax + jx[1] * uy; ax = ax + jx[2] * uz;
    float ay = jy[0] * ux; ay = ay + jy[1] * uy; ay = ay + jy[2] * uz;
    float rho = sigma * w; rho = rho / focal;
    const float r2 = rho * rho;
    float s00 = ax * ax; s00 = k * s00; s00 = sxx + s00; s00 = s00 * r2;
    float s01 = ax * ay; s01 = k * s01; s01 = sxy + s01; s01 = s01 * r2;
    float s11 = ay * ay; s11 = k * s11; s11 = syy + s11; s11 = s11 * r2;
    float det = s00 * s11;
    float e = s01 * s01;
    det = det - e;
    if (!(det > 0.0f && det <= 3.40282347e38f)) return 0;
    q[0] = s11 / det;
    q[1] = -(s01 / det);
    q[2] = s00 / det;
    ext[0] = 3.0f * sqrtf(s00);
    ext[1] = 3.0f * sqrtf(s11);
    return ext[0] <= 3.40282347e38f && ext[1] <= 3.40282347e38f;
}

typedef struct {
    uint64_t key;
    float sx, sy;
    float q[3], ext[2];
    uint32_t idx;
} aniso_rec;

static int cmp_arec(const void *a, const void *b)
{
    uint64_t ka = ((const aniso_rec *)a)->key, kb = ((const aniso_rec *)b)->key;
    return ka < kb ? -1 : (ka > kb ? 1 : 0);
}

int oracle_splat_aniso(const float *x, const float *y, const float *z, uint64_t n,
                       const float *M, float near_f, float far_f, int32_t W, int32_t H,
                       float sigma, float opacity, int32_t color_mode,
                       const splat_attr *attrs, int32_t nattr,
                       const float *lut, int32_t lut_attr, float lut_min, float lut_inv_range,
                       int32_t vel_attr, float stretch, float focal, const int32_t *window,
                       double *img, unsigned char *fragile)
{
    (void)nattr;
    const int64_t npx = (int64_t)W * H;
    aniso_rec *rec = (aniso_rec *)malloc((n ? n : 1) * sizeof(aniso_rec));
    double *T = (double *)malloc(npx * sizeof(double));
    unsigned char *done = (unsigned char *)calloc(npx, 1);
    if (!rec || !T || !done) { free(rec); free(T); free(done); return -1; }
    const float k = stretch - 1.0f;
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
        aniso_rec *r = &rec[m];
        if (!footprint(M, w, cx, cy, W, H, attr_at(&attrs[vel_attr], i), attr_at(&attrs[vel_attr + 1], i),
                       attr_at(&attrs[vel_attr + 2], i), sigma, k, focal, r->q, r->ext))
            continue;
        r->key = ((uint64_t)fbits(w) << 32) | (uint32_t)i;
        r->sx = sx;
        r->sy = sy;
        r->idx = (uint32_t)i;
        ++m;
    }
    qsort(rec, m, sizeof(aniso_rec), cmp_arec);
    for (int64_t p = 0; p < npx; ++p) T[p] = 1.0;
    for (int64_t p = 0; p < 3 * npx; ++p) img[p] = 0.0;
    if (fragile) memset(fragile, 0, (size_t)npx);
    for (uint64_t r = 0; r < m; ++r) {
        const aniso_rec *a = &rec[r];
        const uint64_t i = a->idx;
        double col[3];
        if (color_mode == 0) {
            float t = attr_at(&attrs[lut_attr], i) - lut_min;
            t = t * lut_inv_range;
            t = t * 256.0f;
            int q = !(t > 0.0f) ? 0 : (t >= 255.0f ? 255 : (int)t);
            for (int c = 0; c < 3; ++c) col[c] = (double)lut[q * 3 + c];
        } else {
            for (int c = 0; c < 3; ++c) col[c] = (double)attr_at(&attrs[lut_attr + c], i) / 255.0;
        }
        /* every pixel whose centre can be reached lies in this rectangle */
        int x0 = (int)fmax(floor((double)a->sx - (double)a->ext[0]) - 1.0, 0.0);
        int x1 = (int)fmin(floor((double)a->sx + (double)a->ext[0]) + 1.0, (double)(W - 1));
        int y0 = (int)fmax(floor((double)a->sy - (double)a->ext[1]) - 1.0, 0.0);
        int y1 = (int)fmin(floor((double)a->sy + (double)a->ext[1]) + 1.0, (double)(H - 1));
        if (window) {  /* only the pixels [x0, x1) x [y0, y1) of the window are computed */
            if (x0 < window[0]) x0 = window[0];
            if (x1 > window[2] - 1) x1 = window[2] - 1;
            if (y0 < window[1]) y0 = window[1];
            if (y1 > window[3] - 1) y1 = window[3] - 1;
        }
        for (int py = y0; py <= y1; ++py) {
            for (int px = x0; px <= x1; ++px) {
                const int64_t p = (int64_t)py * W + px;
                if (done[p]) continue;
                float dx = ((float)px + 0.5f) - a->sx;
                float dy = ((float)py + 0.5f) - a->sy;
                float t0 = a->q[0] * dx; t0 = t0 * dx;
                float t1 = a->q[1] * dx; t1 = t1 * dy; t1 = t1 + t1;
                float t2 = a->q[2] * dy; t2 = t2 * dy;
                float qf = t0 + t1; qf = qf + t2;
                if (!(qf <= 9.0f)) continue;
                double al = (double)opacity * exp(-0.5 * (double)qf);
                if (al > 0.99) al = 0.99;
                if (fragile && fabs(al - 1.0 / 255.0) <= 1e-5 / 255.0) fragile[p] = 1;
                if (al < 1.0 / 255.0) continue;
                double Tn = T[p] * (1.0 - al);
                if (fragile && fabs(Tn - 1e-4) <= 1e-9) fragile[p] = 1;
                if (Tn < 1e-4) { done[p] = 1; continue; }
                for (int c = 0; c < 3; ++c) img[c * npx + p] += col[c] * al * T[p];
                T[p] = Tn;
            }
        }
    }
    free(rec);
    free(T);
    free(done);
    return 0;
}

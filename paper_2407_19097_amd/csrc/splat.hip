// Screen-space Gaussian splat renderer for gfx950.
//
// The paper's target renderer is the forward pass of 3D Gaussian splatting
// applied to the points (Sec. 4.2, "Gaussian Renderer"): each point becomes a
// Gaussian, the Gaussians reaching a pixel are taken nearest first and
// alpha-blended front to back.  Here every point is a screen-space Gaussian of
// standard deviation sigma pixels at its projected position (isotropic), or
// one elongated along the point's velocity (anisotropic).  Pipeline:
//   project -- same fp32 transform and cull as the rasterizer; the Gaussian's
//              3-sigma footprint gives a rectangle of screen tiles (an
//              elongated one keeps only the rectangle's tiles its ellipse
//              can reach);
//   order   -- stable radix sort of the points by depth bits (culled points
//              last): equal depths keep the index order, so this is the order
//              of the rasterizer's (depth, index) key.  Three 8-bit passes
//              when the kept depths span under 2^24 - 1 ulps (bits taken
//              relative to the nearest), else four; chosen on the device;
//   scan    -- exclusive prefix sum of the tile counts in that order;
//   emit    -- one (tile, point index) pair per covered tile, in that order;
//   sort    -- stable radix sort of the pairs by tile (two passes of up to 8
//              bits for up to 65536 tiles): within a tile the list keeps the
//              depth order;
//   ranges  -- first and one-past-last pair of every tile;
//   blend   -- one workgroup per 16x16 tile, one thread per pixel, each wave
//              an 8x8 quarter walking the tile's list on its own: entries that
//              can reach its open pixels are staged through LDS and composited
//              front to back (alpha = min(0.99, o exp(-d^2 / 2 sigma^2)),
//              skipped below 1/255, stop once transmittance would fall under
//              1e-4).
// No step needs the host: counts stay on the device and kernels whose size
// depends on them are launched for the worst case and read the count.
#include <hip/hip_runtime.h>

#include "internal.h"

#pragma clang fp contract(off)

namespace narvis {

namespace {

constexpr int kT = 256;            // threads per workgroup everywhere here
constexpr int kScanItems = 16;     // elements per thread in the scans
constexpr int kScanTile = kT * kScanItems;
constexpr int kSortItems = 16;     // elements per thread in the radix sort passes
constexpr int kSortTile = kT * kSortItems;
constexpr int kTile = 16;          // splat screen tile edge in pixels
constexpr int kRangeParts = 256;   // workgroups folding the projection's depth ranges

__device__ __forceinline__ bool project(const Proj &P, float x, float y, float z, float &sx, float &sy, float &w,
                                        float &cx_out, float &cy_out)
{
    float cx = P.m00 * x;
    cx = cx + P.m01 * y;
    cx = cx + P.m02 * z;
    cx = cx + P.m03;
    float cy = P.m10 * x;
    cy = cy + P.m11 * y;
    cy = cy + P.m12 * z;
    cy = cy + P.m13;
    float ww = P.m30 * x;
    ww = ww + P.m31 * y;
    ww = ww + P.m32 * z;
    ww = ww + P.m33;
    if (!(ww >= P.near_f && ww <= P.far_f)) return false;
    float nx = cx / ww;
    float ny = cy / ww;
    float a = nx * 0.5f;
    a = a + 0.5f;
    a = a * P.Wf;
    float b = ny * 0.5f;
    b = 0.5f - b;
    b = b * P.Hf;
    if (!(a >= 0.0f && a < P.Wf && b >= 0.0f && b < P.Hf)) return false;
    sx = a;
    sy = b;
    w = ww;
    cx_out = cx;
    cy_out = cy;
    return true;
}

__device__ __forceinline__ float attr_f32(const AttrArg &a, uint32_t i)
{
    const unsigned char *p = a.p + (size_t)i * (size_t)a.stride;
    switch (a.dtype) {
    case NARVIS_U8: return (float)(*p);
    case NARVIS_U16: return (float)(*reinterpret_cast<const uint16_t *>(p));
    case NARVIS_F16: return (float)(*reinterpret_cast<const _Float16 *>(p));
    default: return *reinterpret_cast<const float *>(p);
    }
}

struct SplatArgs {
    const float *X, *Y, *Z;
    uint64_t n;
    Proj P;
    AttrPack A;
    int32_t color_mode, color_attr;
    const float *lut;
    float lut_min, lut_inv;
    float reach;          // 3 sigma, in pixels
    int32_t tiles_x, tiles_y;
    float2 *ctr;          // [n] centre
    float4 *col;          // [n] colour
    uint32_t *wbits;      // [n] depth bits
    uint32_t *cnt;        // [n + 1] tile counts, scanned in place to offsets
    uint2 *brange;        // [project workgroups] least and greatest kept depth bits
    uint64_t cap;         // capacity of the pair arrays
    // anisotropic footprint (aniso != 0)
    int32_t aniso, vel_attr;
    float sigma, stretch_k, focal;  // sigma_px, s - 1, focal length in pixels
    float4 *conic;        // [n] Q00, Q01, Q11 of the inverse screen covariance
    float2 *ext;          // [n] 3-sigma half extents of the footprint in x and y
};

// Screen-space footprint of a Gaussian elongated along the point's velocity
// (Sec. 4.2: covariance R diag(s, 1, 1) R^T whose dominant axis is v).  World
// covariance rho^2 (I + (s - 1) u u^T) with u = v / |v| and rho = sigma w / f,
// projected by the Jacobian J of the screen position: J Sigma J^T.  Every
// operation is rounded to fp32 in the order written (the host header spells
// the same sequence out).  False when the covariance is not positive
// definite or not finite (the point is then dropped).
__device__ __forceinline__ bool aniso_footprint(const SplatArgs &S, float cx, float cy, float w, float vx, float vy,
                                                float vz, float4 &q, float2 &ext)
{
    const Proj &P = S.P;
    const float ww = w * w;
    const float hx = 0.5f * P.Wf, hy = 0.5f * P.Hf;
    const float m0[3] = {P.m00, P.m01, P.m02}, m1[3] = {P.m10, P.m11, P.m12}, m3[3] = {P.m30, P.m31, P.m32};
    float jx[3], jy[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float a = m0[c] * w;
        float b = cx * m3[c];
        float t = a - b;
        t = t / ww;
        jx[c] = t * hx;
        a = m1[c] * w;
        b = cy * m3[c];
        t = a - b;
        t = t / ww;
        t = t * hy;
        jy[c] = -t;
    }
    float sxx = jx[0] * jx[0];
    sxx = sxx + jx[1] * jx[1];
    sxx = sxx + jx[2] * jx[2];
    float sxy = jx[0] * jy[0];
    sxy = sxy + jx[1] * jy[1];
    sxy = sxy + jx[2] * jy[2];
    float syy = jy[0] * jy[0];
    syy = syy + jy[1] * jy[1];
    syy = syy + jy[2] * jy[2];
    float vn = vx * vx;
    vn = vn + vy * vy;
    vn = vn + vz * vz;
    vn = sqrtf(vn);
    float ux = 0.0f, uy = 0.0f, uz = 0.0f;
    if (vn > 0.0f && vn <= 3.40282347e38f) {
        ux = vx / vn;
        uy = vy / vn;
        uz = vz / vn;
    }
    float ax = jx[0] * ux;
    ax = ax + jx[1] * uy;
    ax = ax + jx[2] * uz;
    float ay = jy[0] * ux;
    ay = ay + jy[1] * uy;
    ay = ay + jy[2] * uz;
    float rho = S.sigma * w;
    rho = rho / S.focal;
    const float r2 = rho * rho;
    float s00 = ax * ax;
    s00 = S.stretch_k * s00;
    s00 = sxx + s00;
    s00 = s00 * r2;
    float s01 = ax * ay;
    s01 = S.stretch_k * s01;
    s01 = sxy + s01;
    s01 = s01 * r2;
    float s11 = ay * ay;
    s11 = S.stretch_k * s11;
    s11 = syy + s11;
    s11 = s11 * r2;
    float det = s00 * s11;
    const float e = s01 * s01;
    det = det - e;
    if (!(det > 0.0f && det <= 3.40282347e38f)) return false;
    q = make_float4(s11 / det, -(s01 / det), s00 / det, 0.0f);
    ext = make_float2(3.0f * sqrtf(s00), 3.0f * sqrtf(s11));
    return ext.x <= 3.40282347e38f && ext.y <= 3.40282347e38f;
}

// footprint rectangle in pixels, clipped to the image (conservative: every
// pixel whose centre can be within `reach` of (sx, sy) is inside)
__device__ __forceinline__ void pixel_rect(int W, int H, float sx, float sy, float rx, float ry, int &x0, int &x1,
                                           int &y0, int &y1)
{
    // clamped in float first: an anisotropic extent can exceed the int range
    x0 = (int)fmaxf(floorf(sx - rx - 1.0f), -1.0f);
    x1 = (int)fminf(floorf(sx + rx + 1.0f), (float)W);
    y0 = (int)fmaxf(floorf(sy - ry - 1.0f), -1.0f);
    y1 = (int)fminf(floorf(sy + ry + 1.0f), (float)H);
    x0 = max(x0, 0);
    y0 = max(y0, 0);
    x1 = min(x1, W - 1);
    y1 = min(y1, H - 1);
}

// the same rectangle in tiles
__device__ __forceinline__ void tile_rect(const SplatArgs &S, float sx, float sy, float rx, float ry, int &tx0,
                                          int &tx1, int &ty0, int &ty1)
{
    int x0, x1, y0, y1;
    pixel_rect(S.P.W, S.P.H, sx, sy, rx, ry, x0, x1, y0, y1);
    tx0 = x0 / kTile;
    tx1 = x1 / kTile;
    ty0 = y0 / kTile;
    ty1 = y1 / kTile;
}

// Whether a Gaussian of conic (A, B, C) = (Q00, Q01, Q11) can reach a pixel
// whose centre lies at an offset (dx, dy) in [u0, u1] x [v0, v1] from the
// Gaussian's centre: the least q over the box (zero when the box holds the
// centre, else on an edge, at the edge's clamped stationary point) against 9
// plus a margin that covers the fp32 rounding of the pixel test (under 8
// ulps of the terms' magnitudes at any offset of the box) and of this
// evaluation, doubled.  Never false for a box holding a pixel that the
// pixel test takes; true when anything overflows.  kA = -(B / A) and
// kC = -(B / C) (per Gaussian) place the edges' stationary points; their
// rounding moves the edge minima by far less than the margin.
__device__ __forceinline__ bool conic_meets_box(float A, float B, float C, float kA, float kC, float u0, float u1,
                                                float v0, float v1)
{
    if (u0 <= 0.0f && u1 >= 0.0f && v0 <= 0.0f && v1 >= 0.0f) return true;
    auto qf = [&](float u, float v) {
        float t0 = A * u;
        t0 = t0 * u;
        float t1 = B * u;
        t1 = t1 * v;
        t1 = t1 + t1;
        float t2 = C * v;
        t2 = t2 * v;
        float q = t0 + t1;
        return q + t2;
    };
    float best = INFINITY;
    const float us[2] = {u0, u1}, vs[2] = {v0, v1};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float v = fminf(fmaxf(kC * us[k], v0), v1);
        best = fminf(best, qf(us[k], v));
        const float u = fminf(fmaxf(kA * vs[k], u0), u1);
        best = fminf(best, qf(u, vs[k]));
    }
    const float U = fmaxf(fabsf(u0), fabsf(u1)), V = fmaxf(fabsf(v0), fabsf(v1));
    float M = A * U;
    M = M * U;
    float Mb = fabsf(B) * U;
    Mb = Mb * V;
    M = M + (Mb + Mb);
    float Mc = C * V;
    Mc = Mc * V;
    M = M + Mc;
    if (!(best < INFINITY) || !(M < INFINITY)) return true;
    return best <= 9.0f + 4e-6f * M + 1e-3f;
}

// screen tile (tx, ty) against the conic centred at (sx, sy)
__device__ __forceinline__ bool conic_meets_tile(const float4 &q, float kA, float kC, float sx, float sy, int tx,
                                                 int ty)
{
    const float ax = (float)(tx * kTile) + 0.5f, ay = (float)(ty * kTile) + 0.5f;
    return conic_meets_box(q.x, q.y, q.z, kA, kC, ax - sx, (ax + (float)(kTile - 1)) - sx, ay - sy,
                           (ay + (float)(kTile - 1)) - sy);
}

// least and greatest over the workgroup (every thread gets both)
__device__ __forceinline__ void block_range(uint32_t &lo, uint32_t &hi, uint32_t *lo4, uint32_t *hi4)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) {
        lo = min(lo, (uint32_t)__shfl_xor(lo, d));
        hi = max(hi, (uint32_t)__shfl_xor(hi, d));
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        lo4[wid] = lo;
        hi4[wid] = hi;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kT / 64; ++k) {
        lo = min(lo, lo4[k]);
        hi = max(hi, hi4[k]);
    }
}

// one point: footprint, colour, depth bits and tile count; false when culled
// (its count is then 0)
__device__ __forceinline__ bool project_point(const SplatArgs &S, uint64_t i, uint32_t &wb)
{
    float sx, sy, w, cx, cy;
    if (!project(S.P, S.X[i], S.Y[i], S.Z[i], sx, sy, w, cx, cy)) {
        S.cnt[i] = 0;
        return false;
    }
    float rx = S.reach, ry = S.reach;
    float4 q = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (S.aniso) {
        float2 ext;
        const float vx = attr_f32(S.A.a[S.vel_attr], (uint32_t)i), vy = attr_f32(S.A.a[S.vel_attr + 1], (uint32_t)i),
                    vz = attr_f32(S.A.a[S.vel_attr + 2], (uint32_t)i);
        if (!aniso_footprint(S, cx, cy, w, vx, vy, vz, q, ext)) {
            S.cnt[i] = 0;
            return false;
        }
        S.conic[i] = q;
        S.ext[i] = ext;
        rx = ext.x;
        ry = ext.y;
    }
    float4 c;
    if (S.color_mode == NARVIS_COLOR_LUT) {
        float t = attr_f32(S.A.a[S.color_attr], (uint32_t)i) - S.lut_min;
        t = t * S.lut_inv;
        t = t * 256.0f;
        int q;
        if (!(t > 0.0f)) q = 0;
        else if (t >= 255.0f) q = 255;
        else q = (int)t;
        c = make_float4(S.lut[q * 3], S.lut[q * 3 + 1], S.lut[q * 3 + 2], 0.0f);
    } else {
        const float s = 1.0f / 255.0f;
        c = make_float4(attr_f32(S.A.a[S.color_attr], (uint32_t)i) * s,
                        attr_f32(S.A.a[S.color_attr + 1], (uint32_t)i) * s,
                        attr_f32(S.A.a[S.color_attr + 2], (uint32_t)i) * s, 0.0f);
    }
    int tx0, tx1, ty0, ty1;
    tile_rect(S, sx, sy, rx, ry, tx0, tx1, ty0, ty1);
    uint32_t tiles = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
    if (S.aniso) {  // only the rectangle's tiles that the ellipse can reach
        tiles = 0;
        const float kA = -(q.y / q.x), kC = -(q.y / q.z);
        for (int ty = ty0; ty <= ty1; ++ty)
            for (int tx = tx0; tx <= tx1; ++tx) tiles += conic_meets_tile(q, kA, kC, sx, sy, tx, ty) ? 1u : 0u;
    }
    S.ctr[i] = make_float2(sx, sy);
    S.col[i] = c;
    wb = __float_as_uint(w);
    S.wbits[i] = wb;
    S.cnt[i] = tiles;
    return tiles > 0;
}

// Projection of every point, plus the least and greatest depth bits of the
// workgroup's kept points (all ones and zero when it keeps none), from which
// the point sort picks its pass count.
__global__ __launch_bounds__(kT) void k_splat_project(SplatArgs S)
{
    __shared__ uint32_t lo4[kT / 64], hi4[kT / 64];
    const uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    uint32_t wb = 0;
    bool kept = false;
    if (i < S.n) kept = project_point(S, i, wb);
    else if (i == S.n) S.cnt[i] = 0;  // the scan's extra slot, so that cnt[n] becomes the total
    uint32_t lo = kept ? wb : 0xFFFFFFFFu, hi = kept ? wb : 0u;
    block_range(lo, hi, lo4, hi4);
    if (threadIdx.x == 0) S.brange[blockIdx.x] = make_uint2(lo, hi);
}

// The point sort's pass count, chosen on the device.  k_range_partial folds
// the projection's per-workgroup depth ranges into one per workgroup of its
// own, k_depth_plan folds those and writes plan[0] = least kept depth bits and
// plan[1] = 1 when the kept depths span at most 2^24 - 2 ulps: three 8-bit
// passes over the bits relative to plan[0] then order the kept points, and
// all ones in the low 24 bits (a culled point) still sorts after every one of
// them.
__global__ __launch_bounds__(kT) void k_range_partial(const uint2 *br, uint64_t nb, uint2 *part)
{
    __shared__ uint32_t lo4[kT / 64], hi4[kT / 64];
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    for (uint64_t k = (uint64_t)blockIdx.x * kT + threadIdx.x; k < nb; k += (uint64_t)gridDim.x * kT) {
        const uint2 r = br[k];
        lo = min(lo, r.x);
        hi = max(hi, r.y);
    }
    block_range(lo, hi, lo4, hi4);
    if (threadIdx.x == 0) part[blockIdx.x] = make_uint2(lo, hi);
}

__global__ __launch_bounds__(kT) void k_depth_plan(const uint2 *part, uint32_t np, uint32_t *plan)
{
    __shared__ uint32_t lo4[kT / 64], hi4[kT / 64];
    uint32_t lo = 0xFFFFFFFFu, hi = 0u;
    for (uint32_t k = threadIdx.x; k < np; k += kT) {
        const uint2 r = part[k];
        lo = min(lo, r.x);
        hi = max(hi, r.y);
    }
    block_range(lo, hi, lo4, hi4);
    if (threadIdx.x == 0) {
        const bool none = lo > hi;  // nothing kept
        plan[0] = none ? 0u : lo;
        plan[1] = (none || hi - lo <= 0xFFFFFEu) ? 1u : 0u;
    }
}

// tile counts in depth order (scnt[n] = 0: the scan's total slot).  With three
// passes the count sits in the sorted key's top byte; 255 there means "255 or
// more, or culled", read from cnt.
__global__ __launch_bounds__(kT) void k_gather_counts(const uint32_t *cnt, const uint32_t *order,
                                                      const uint32_t *keys, const uint32_t *plan, uint64_t n,
                                                      uint32_t *scnt)
{
    const uint64_t j = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (j > n) return;
    uint32_t c = 0u;
    if (j < n) {
        c = plan[1] ? keys[j] >> 24 : 255u;
        if (c == 255u) {
            const uint32_t i = order[j];
            c = (uint64_t)i < n ? cnt[i] : 0u;  // a permutation of [0, n); guards the read regardless
        }
    }
    scnt[j] = c;
}

// sorted position j: the pairs of point order[j] at [scnt[j], scnt[j + 1]).
// The workgroup's points own one contiguous range of pairs; an isotropic
// range of up to kEmitStage pairs is assembled in LDS and written out with
// consecutive threads on consecutive pairs.
constexpr int kEmitStage = 2048;

__global__ __launch_bounds__(kT) void k_splat_emit(SplatArgs S, const uint32_t *order, const uint32_t *scnt,
                                                   uint32_t *keys, uint32_t *vals)
{
    __shared__ uint32_t sk[kEmitStage], sv[kEmitStage];
    const uint64_t j0 = (uint64_t)blockIdx.x * kT;
    const uint64_t j1 = j0 + kT < S.n ? j0 + kT : S.n;
    const uint32_t wbeg = scnt[j0], wend = scnt[j1];  // uniform
    const bool stage = !S.aniso && wend >= wbeg && wend - wbeg <= (uint32_t)kEmitStage;
    const uint64_t j = j0 + threadIdx.x;
    uint32_t start = 0, stop = 0, i = 0;
    if (j < S.n) {
        start = scnt[j];
        stop = scnt[j + 1];
        if (start != stop) {
            i = order[j];
            if ((uint64_t)i >= S.n) stop = start;  // a permutation of [0, n); guards the reads regardless
        }
    }
    if (start != stop) {
        const float2 c = S.ctr[i];
        const float2 ext = S.aniso ? S.ext[i] : make_float2(S.reach, S.reach);
        int tx0, tx1, ty0, ty1;
        tile_rect(S, c.x, c.y, ext.x, ext.y, tx0, tx1, ty0, ty1);
        uint32_t o = start;
        if (S.aniso) {  // the tiles the projection counted, in the same order
            const float4 q = S.conic[i];
            const float kA = -(q.y / q.x), kC = -(q.y / q.z);
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx) {
                    if (!conic_meets_tile(q, kA, kC, c.x, c.y, tx, ty)) continue;
                    if (o < stop && o < S.cap) {  // the count bounds the tiles; guard anyway
                        keys[o] = (uint32_t)(ty * S.tiles_x + tx);
                        vals[o] = i;
                    }
                    ++o;
                }
        } else {
            for (int ty = ty0; ty <= ty1; ++ty)
                for (int tx = tx0; tx <= tx1; ++tx, ++o) {
                    if (o >= stop) continue;  // the count bounds the rectangle; guard anyway
                    const uint32_t key = (uint32_t)(ty * S.tiles_x + tx);
                    if (stage) {
                        sk[o - wbeg] = key;
                        sv[o - wbeg] = i;
                    } else if (o < S.cap) {
                        keys[o] = key;
                        vals[o] = i;
                    }
                }
        }
    }
    if (!stage) return;  // uniform
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < wend - wbeg; k += kT)
        if (wbeg + k < S.cap) {
            keys[wbeg + k] = sk[k];
            vals[wbeg + k] = sv[k];
        }
}

// ---------------------------------------------------------------------------
// exclusive prefix sum of uint32 (three passes: tile sums, scan of sums,
// apply); each thread takes kScanItems consecutive elements as 16-byte loads
// and stores (every array scanned here is 256-byte aligned)
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// block-wide exclusive scan of one value per thread; returns the block total in *total
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *lds4, uint32_t *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63) lds4[wid] = inc;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kT / 64; ++k) {
        const uint32_t s = lds4[k];
        if (k < wid) before += s;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__global__ __launch_bounds__(kT) void k_scan_sums(const uint32_t *in, uint64_t len, uint32_t *sums)
{
    __shared__ uint32_t lds4[kT / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
    if (base + kScanItems <= len) {
        const uint4 *q = reinterpret_cast<const uint4 *>(in + base);
#pragma unroll
        for (int k = 0; k < kScanItems / 4; ++k) {
            const uint4 v = q[k];
            s += (v.x + v.y) + (v.z + v.w);
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + k < len) s += in[base + k];
    }
    uint32_t total;
    block_excl_scan(s, lds4, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kT) void k_scan_top(uint32_t *sums, uint32_t nb)
{
    __shared__ uint32_t lds4[kT / 64];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t base = 0; base < nb; base += kT) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < nb ? sums[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_excl_scan(v, lds4, &total);
        const uint32_t c = carry;
        if (i < nb) sums[i] = c + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + total;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kT) void k_scan_apply(const uint32_t *in, uint32_t *out, uint64_t len, const uint32_t *sums)
{
    __shared__ uint32_t lds4[kT / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
    const bool full = base + kScanItems <= len;
    if (full) {
        const uint4 *q = reinterpret_cast<const uint4 *>(in + base);
#pragma unroll
        for (int k = 0; k < kScanItems / 4; ++k) {
            const uint4 x = q[k];
            v[4 * k] = x.x;
            v[4 * k + 1] = x.y;
            v[4 * k + 2] = x.z;
            v[4 * k + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k) v[k] = base + k < len ? in[base + k] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) s += v[k];
    uint32_t total;
    uint32_t run = block_excl_scan(s, lds4, &total) + sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const uint32_t x = v[k];
        v[k] = run;
        run += x;
    }
    if (full) {
        uint4 *q = reinterpret_cast<uint4 *>(out + base);
#pragma unroll
        for (int k = 0; k < kScanItems / 4; ++k) q[k] = make_uint4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < kScanItems; ++k)
            if (base + k < len) out[base + k] = v[k];
    }
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8-bit digits, 4096 elements per workgroup
// ---------------------------------------------------------------------------

// Where a pass takes its elements from.  ArraySrc: the caller's or the
// previous pass's arrays, digit position fixed on the host.
template <typename K>
struct ArraySrc {
    const K *k;
    const uint32_t *v;
    int sh;
    uint32_t msk;  // digit mask: 2^(digit bits) - 1, at most 255
    __device__ void init() {}
    __device__ int shift() const { return sh; }
    __device__ uint32_t mask() const { return msk; }
    __device__ K key(uint64_t e) const { return k[e]; }
    __device__ uint32_t val(uint64_t e) const { return v[e]; }
};

// The point sort by depth, four slots of which the plan (k_depth_plan) runs
// four, over the fp32 depth bits, or the last three, over the bits relative
// to plan[0] with the tile count (saturated at 255) in the key's top byte,
// where the count gather after the sort finds it in order.  The first slot
// that runs builds its keys from the projection (all ones for a culled point,
// which sorts it last) and numbers the values; the later ones read the
// previous slot's output.  Slots 1 to 3 write the same buffers in both cases,
// so the sorted order always ends in slot 3's output.
struct DepthSrc {
    const uint32_t *k, *v;        // previous slot's output (slots 1 to 3)
    const uint32_t *wbits, *cnt;  // projection: depth bits and tile counts
    const uint32_t *plan;
    int slot;
    uint32_t base;
    bool three, first;
    __device__ void init()
    {
        three = plan[1] != 0u;
        base = plan[0];
        first = slot == (three ? 1 : 0);
    }
    __device__ int shift() const { return three ? (slot ? 8 * (slot - 1) : -1) : 8 * slot; }
    __device__ uint32_t mask() const { return 255u; }
    __device__ uint32_t key(uint64_t e) const
    {
        if (!first) return k[e];
        const uint32_t c = cnt[e];
        if (!c) return 0xFFFFFFFFu;
        const uint32_t w = wbits[e];
        return three ? ((w - base) | (min(c, 255u) << 24)) : w;
    }
    __device__ uint32_t val(uint64_t e) const { return first ? (uint32_t)e : v[e]; }
};

// Sort block of this workgroup, a permutation of the grid.  Workgroups go to
// the eight XCDs in turn (workgroup w on XCD w % 8).  Of the blocks that hold
// elements (their count rounded up to a multiple of 8, which the grid, also
// a multiple of 8, covers), XCD x takes the x-th eighth in order, so that
// neighbouring histogram columns and offsets are written and read through one
// L2 and every XCD has work; the empty blocks beyond keep their own number.
__device__ __forceinline__ uint32_t sort_block(uint64_t N)
{
    const uint32_t act = (uint32_t)(((N + kSortTile - 1) / kSortTile + 7) & ~uint64_t(7));
    const uint32_t b = blockIdx.x;
    return b >= act ? b : (b & 7u) * (act >> 3) + (b >> 3);
}

// digit counts of one sort block per workgroup, hist[digit * nblk + block]
// for the digits under the source's mask (skipped, like its scatter, when
// the source's shift is negative)
template <typename K, typename Src>
__global__ __launch_bounds__(kT) void k_radix_hist(Src src, const uint32_t *count, uint64_t cap, uint32_t *hist,
                                                   uint32_t nblk)
{
    __shared__ uint32_t h[256];
    src.init();
    const int shift = src.shift();
    if (shift < 0) return;  // uniform for the grid
    const uint32_t mask = src.mask();
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t N = min((uint64_t)*count, cap);
    const uint32_t blk = sort_block(N);
    const uint64_t base = (uint64_t)blk * kSortTile + threadIdx.x;
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint64_t e = base + (uint64_t)r * kT;
        if (e < N) atomicAdd(&h[(uint32_t)(src.key(e) >> shift) & mask], 1u);
    }
    __syncthreads();
    if (threadIdx.x <= mask) hist[(uint64_t)threadIdx.x * nblk + blk] = h[threadIdx.x];
}

// One LSD pass: each workgroup moves its kSortTile elements to the offsets
// the histogram scan gave its digits, in element order (a stable sort).  Wave
// w ranks the contiguous sub-range [w, w + 1) * kSortTile / 4 of the block,
// 64 elements per round: an element's rank is the number of equal digits in
// the wave's earlier rounds (a running per-wave count in LDS, updated by the
// first lane of each digit group: a wave's LDS operations complete in order,
// so no barrier is needed) plus the equal digits at lower lanes of its round
// (ballot match on the 8 digit bits).  The per-wave counts are then combined
// into block offsets, the block is reordered in LDS, and written out with
// consecutive threads on consecutive destinations.  The block's 256 output
// offsets are read once, early, so that their latency overlaps the ranking.
template <typename K, typename Src>
__global__ __launch_bounds__(kT) void k_radix_scatter(Src src, K *kout, uint32_t *vout, const uint32_t *count,
                                                      uint64_t cap, const uint32_t *offs, uint32_t nblk)
{
    constexpr int NW = kT / 64;
    constexpr int PER_WAVE = kSortTile / NW;
    __shared__ K skey[kSortTile];
    __shared__ uint32_t sval[kSortTile];
    __shared__ uint32_t wcnt[NW][256];  // running digit counts of each wave, then each wave's offset
    __shared__ uint32_t bstart[256];
    __shared__ uint32_t sdst[256];
    __shared__ uint32_t lds4[NW];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    src.init();
    const int shift = src.shift();
    if (shift < 0) return;  // uniform for the grid
    const uint32_t mask = src.mask();
    const uint64_t N = min((uint64_t)*count, cap);
    const uint32_t blk = sort_block(N);
    const uint64_t base = (uint64_t)blk * kSortTile;
    if (base >= N) return;  // uniform for the workgroup
#pragma unroll
    for (int w = 0; w < NW; ++w) wcnt[w][threadIdx.x] = 0u;
    const uint32_t myoff = offs[(uint64_t)threadIdx.x * nblk + blk];  // digit threadIdx.x
    K k[kSortItems];
    uint32_t v[kSortItems], rank[kSortItems], dig[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint64_t e = base + (uint64_t)wid * PER_WAVE + (uint64_t)r * 64 + lane;
        const bool ok = e < N;
        k[r] = ok ? src.key(e) : (K)0;
        v[r] = ok ? src.val(e) : 0u;
        dig[r] = ok ? ((uint32_t)(k[r] >> shift) & mask) : 256u;
    }
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    __syncthreads();
    uint32_t *cnt = wcnt[wid];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint32_t d = dig[r];
        unsigned long long m = __ballot(d < 256u);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            if (!((mask >> b) & 1u)) break;  // uniform: the digit has no more bits
            const unsigned long long bb = __ballot((d >> b) & 1u);
            m &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t inwave = (uint32_t)__popcll(m & below);
        const uint32_t before = d < 256u ? cnt[d] : 0u;
        rank[r] = before + inwave;
        // the group's first lane advances the count after every lane has read it
        __builtin_amdgcn_wave_barrier();
        if (d < 256u && inwave == 0) cnt[d] = before + (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit (thread = digit): offsets of the waves, and the digit's total
    uint32_t tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint32_t c = wcnt[w][threadIdx.x];
        wcnt[w][threadIdx.x] = tot;
        tot += c;
    }
    uint32_t total;
    const uint32_t bs = block_excl_scan(tot, lds4, &total);
    bstart[threadIdx.x] = bs;
    sdst[threadIdx.x] = myoff - bs;  // output index = sdst[digit] + position in the reordered block
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        if (dig[r] < 256u) {
            const uint32_t pos = bstart[dig[r]] + cnt[dig[r]] + rank[r];
            if (pos < (uint32_t)kSortTile) {
                skey[pos] = k[r];
                sval[pos] = v[r];
            }
        }
    }
    __syncthreads();
    const uint32_t inblock = (uint32_t)min((uint64_t)kSortTile, N - base);
    for (uint32_t i = threadIdx.x; i < inblock; i += kT) {
        const K key = skey[i];
        const uint32_t d = (uint32_t)(key >> shift) & mask;
        const uint64_t dst = (uint64_t)(sdst[d] + i);
        if (dst < N) {  // always true for a consistent histogram; guards the buffer regardless
            kout[dst] = key;
            vout[dst] = sval[i];
        }
    }
}

// ---------------------------------------------------------------------------
// tile ranges and blending
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kT) void k_fill_u32(uint32_t *p, uint64_t cnt, uint32_t v)
{
    const uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (i < cnt) p[i] = v;
}

// First and one-past-last position of every tile in the sorted pair keys.
// Each thread reads kRangeItems consecutive keys; the neighbours across
// threads come from the adjacent lanes, and the wave's end lanes read theirs.
constexpr int kRangeItems = 16;

__global__ __launch_bounds__(kT) void k_tile_ranges(const uint32_t *keys, const uint32_t *count, uint64_t cap,
                                                    uint32_t *range, uint32_t ntiles)
{
    const uint64_t N = min((uint64_t)*count, cap);
    if ((uint64_t)blockIdx.x * kT * kRangeItems >= N) return;  // uniform for the workgroup
    const uint64_t p0 = ((uint64_t)blockIdx.x * kT + threadIdx.x) * kRangeItems;
    uint32_t t[kRangeItems];
    if (p0 + kRangeItems <= N) {
        // 64-byte aligned: the key array is 256-byte aligned and p0 a multiple of 16
        const uint4 *q = reinterpret_cast<const uint4 *>(keys + p0);
#pragma unroll
        for (int k = 0; k < kRangeItems / 4; ++k) {
            const uint4 v = q[k];
            t[4 * k] = v.x;
            t[4 * k + 1] = v.y;
            t[4 * k + 2] = v.z;
            t[4 * k + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kRangeItems; ++k) t[k] = p0 + k < N ? keys[p0 + k] : 0xFFFFFFFFu;
    }
    const int lane = threadIdx.x & 63;
    uint32_t prev = __shfl_up(t[kRangeItems - 1], 1), next = __shfl_down(t[0], 1);
    if (lane == 0) prev = p0 > 0 && p0 - 1 < N ? keys[p0 - 1] : 0xFFFFFFFFu;
    if (lane == 63) next = p0 + kRangeItems < N ? keys[p0 + kRangeItems] : 0xFFFFFFFFu;
#pragma unroll
    for (int k = 0; k < kRangeItems; ++k) {
        const uint64_t p = p0 + k;
        const uint32_t cur = t[k];
        if (p >= N || cur >= ntiles) continue;
        const uint32_t before = k ? t[k - 1] : prev;
        const uint32_t after = k + 1 < kRangeItems ? t[k + 1] : next;
        if (p == 0 || before != cur) range[2 * cur] = (uint32_t)p;
        if (p + 1 == N || after != cur) range[2 * cur + 1] = (uint32_t)(p + 1);
    }
}

struct BlendArgs {
    uint64_t n, cap;
    const uint32_t *count;
    const uint32_t *range;
    const uint32_t *vals;
    const float2 *ctr;
    const float4 *col;
    const float4 *conic;  // ANISO: per point Q00, Q01, Q11
    const float2 *ext;    // ANISO: per point footprint half extents
    float *img;
    int32_t W, H, tiles_x;
    float reach, cut2, inv2s2, opacity;
};

// ANISO: a Gaussian reaches a pixel when its quadratic form
// q = ((Q00 dx) dx + ((Q01 dx) dy) 2) + (Q11 dy) dy is at most 9 (3 sigma),
// alpha = min(0.99, opacity exp(-q / 2)); otherwise d2 = dx^2 + dy^2 against
// (3 sigma)^2 and alpha = min(0.99, opacity exp(-d2 / 2 sigma^2)).
//
// One workgroup per 16x16 tile, each wave an 8x8 quarter of it, and the
// waves independent of each other: each walks the tile's list 64 entries at
// a time, one per lane (the list entry read two batches ahead, the point
// gathered one ahead, so that the loads overlap the compositing), keeps the
// entries that can reach a pixel of its quarter not yet done (tested against
// the bounding box of those pixels -- isotropic: the disc against the box's
// nearest pixel centre; anisotropic: the footprint rectangle and the conic's
// least q over the box; neither drops an entry that reaches a pixel of the
// box), copies them into its LDS list in list order and composites them,
// until every pixel of its quarter is done.  No barrier
// ties a wave to the others, so a wave whose pixels terminate early leaves.
template <bool ANISO>
__global__ __launch_bounds__(kT) void k_splat_blend(BlendArgs B)
{
    constexpr int NW = kT / 64;
    __shared__ float2 lc[NW][64];    // per wave: centres of the batch entries that can reach its quarter
    __shared__ float4 lcol[NW][64];  // their colours
    __shared__ float4 lq[ANISO ? NW : 1][ANISO ? 64 : 1];  // their conics
    const int tile = blockIdx.x;
    const int tx = tile % B.tiles_x, ty = tile / B.tiles_x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int qx = tx * kTile + (wid & 1) * 8, qy = ty * kTile + (wid >> 1) * 8;  // the wave's quarter
    const int px = qx + (lane & 7), py = qy + (lane >> 3);
    const bool inside = px < B.W && py < B.H;
    const uint32_t N = (uint32_t)min((uint64_t)*B.count, B.cap);
    const uint32_t start = B.range[2 * tile], stop = min(B.range[2 * tile + 1], N);
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    const float ax = (float)qx + 0.5f, ay = (float)qy + 0.5f;  // the quarter's first pixel centre
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    float T = 1.0f, r = 0.0f, g = 0.0f, b = 0.0f;
    bool done = !inside;
    float2 c = make_float2(0.0f, 0.0f), ex = make_float2(0.0f, 0.0f);
    float4 col = make_float4(0.0f, 0.0f, 0.0f, 0.0f), cq = col;
    bool have = false, nhave = false;
    uint32_t nidx = 0u;
    auto read_index = [&](uint32_t s0) {
        const uint32_t e = s0 + (uint32_t)lane;
        nhave = e < stop;
        nidx = nhave ? B.vals[e] : 0u;
    };
    auto gather = [&]() {
        have = nhave && nidx < B.n;  // the index test is always true for consistent lists
        if (have) {
            c = B.ctr[nidx];
            col = B.col[nidx];
            if (ANISO) {
                cq = B.conic[nidx];
                ex = B.ext[nidx];
            }
        }
    };
    if (start < stop) {
        read_index(start);
        gather();
        if (start + 64 < stop) read_index(start + 64);
    }
    for (uint32_t s0 = start; s0 < stop; s0 += 64) {
        if (!__any(!done)) break;  // every pixel of the quarter is done
        // the bounding box of the quarter's pixels still open
        int lx = done ? 0x7FFF : px & 7, hx = done ? -1 : px & 7;
        int ly = done ? 0x7FFF : py & 7, hy = done ? -1 : py & 7;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            lx = min(lx, __shfl_xor(lx, d));
            hx = max(hx, __shfl_xor(hx, d));
            ly = min(ly, __shfl_xor(ly, d));
            hy = max(hy, __shfl_xor(hy, d));
        }
        const float oax = ax + (float)lx, obx = ax + (float)hx;  // its first and last pixel centres
        const float oay = ay + (float)ly, oby = ay + (float)hy;
        bool reach = false;
        if (have) {
            if (!ANISO) {
                // the open box's pixel centre nearest to the centre, in the
                // pixel test's own arithmetic: no open pixel gets a smaller
                // d2 (rounding is monotonic)
                const float dx = c.x < oax ? oax - c.x : (c.x > obx ? c.x - obx : 0.0f);
                const float dy = c.y < oay ? oay - c.y : (c.y > oby ? c.y - oby : 0.0f);
                float d2 = dx * dx;
                d2 = d2 + dy * dy;
                reach = d2 <= B.cut2;
            } else {
                int x0, x1, y0, y1;
                pixel_rect(B.W, B.H, c.x, c.y, ex.x, ex.y, x0, x1, y0, y1);
                reach = x0 <= qx + hx && x1 >= qx + lx && y0 <= qy + hy && y1 >= qy + ly &&
                        conic_meets_box(cq.x, cq.y, cq.z, -(cq.y / cq.x), -(cq.y / cq.z), oax - c.x, obx - c.x,
                                        oay - c.y, oby - c.y);
            }
        }
        const unsigned long long m = __ballot(reach);
        if (reach) {
            const uint32_t off = (uint32_t)__popcll(m & below);
            lc[wid][off] = c;
            lcol[wid][off] = col;
            if (ANISO) lq[wid][off] = cq;
        }
        if (s0 + 64 < stop) {
            gather();
            if (s0 + 128 < stop) read_index(s0 + 128);
        }
        // a wave's LDS operations complete in order: the list is written
        // before it is read, and read before the next batch overwrites it
        __builtin_amdgcn_wave_barrier();
        const uint32_t mine = (uint32_t)__popcll(m);
        for (uint32_t k0 = 0; k0 < mine && !done; k0 += 2) {
            // the alphas of two entries (independent of T) first, then both composited in order
            float av[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const uint32_t k = k0 + u;
                float a = 0.0f;
                if (k < mine) {
                    const float2 cc = lc[wid][k];
                    const float dx = fx - cc.x;
                    const float dy = fy - cc.y;
                    bool reach;
                    float e;
                    if (ANISO) {
                        const float4 q = lq[wid][k];
                        float t0 = q.x * dx;
                        t0 = t0 * dx;
                        float t1 = q.y * dx;
                        t1 = t1 * dy;
                        t1 = t1 + t1;
                        float t2 = q.z * dy;
                        t2 = t2 * dy;
                        float qf = t0 + t1;
                        qf = qf + t2;
                        reach = qf <= 9.0f;
                        e = -0.5f * qf;
                    } else {
                        float d2 = dx * dx;
                        d2 = d2 + dy * dy;
                        reach = d2 <= B.cut2;
                        e = -d2 * B.inv2s2;
                    }
                    a = B.opacity * expf(e);
                    a = fminf(a, 0.99f);
                    if (!reach) a = 0.0f;
                }
                av[u] = a;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const float a = av[u];
                if (done || a < 1.0f / 255.0f) continue;
                const float Tn = T * (1.0f - a);
                if (Tn < 1e-4f) {
                    done = true;
                    continue;
                }
                const float4 cc4 = lcol[wid][k0 + u];
                const float at = a * T;
                r = r + cc4.x * at;
                g = g + cc4.y * at;
                b = b + cc4.z * at;
                T = Tn;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (inside) {
        const int64_t npx = (int64_t)B.W * B.H;
        const int64_t p = (int64_t)py * B.W + px;
        B.img[p] = r;
        B.img[npx + p] = g;
        B.img[2 * npx + p] = b;
    }
}

uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

}  // namespace

// Workspace carve-up, shared by the size query and the launcher.
SplatLayout splat_layout(uint64_t n, int32_t W, int32_t H, float sigma, bool aniso, uint64_t max_pairs)
{
    SplatLayout L{};
    // the footprint rectangle spans x1 - x0 <= 2 reach + 3 pixels in exact
    // arithmetic (+1 for fp32 rounding of its ends), so it touches at most
    // floor((2 reach + 4) / kTile) + 2 tiles per axis
    const float reach = 3.0f * sigma;
    const uint64_t per_axis = (uint64_t)((2.0f * reach + 4.0f) / (float)kTile) + 2;
    L.tiles_x = (W + kTile - 1) / kTile;
    L.tiles_y = (H + kTile - 1) / kTile;
    L.cap = max_pairs ? max_pairs : n * per_axis * per_axis;
    // the pair arrays also hold the point order (n elements) before the pairs
    const uint64_t elems = L.cap > n ? L.cap : n;
    L.nblk = (elems + kSortTile - 1) / kSortTile;
    L.nblk = (L.nblk + 7) & ~uint64_t(7);
    if (L.nblk == 0) L.nblk = 8;
    const uint64_t histlen = L.nblk * 256;
    const uint64_t scanlen = histlen > n + 1 ? histlen : n + 1;
    L.nsums = (scanlen + kScanTile - 1) / kScanTile;
    uint64_t o = 0;
    L.off_ctr = o; o = align256(o + n * sizeof(float2));
    L.off_col = o; o = align256(o + n * sizeof(float4));
    L.off_wbits = o; o = align256(o + n * 4);
    L.off_cnt = o; o = align256(o + (n + 1) * 4);
    L.off_ka = o; o = align256(o + elems * 4);
    L.off_va = o; o = align256(o + elems * 4);
    L.off_kb = o; o = align256(o + elems * 4);
    L.off_vb = o; o = align256(o + elems * 4);
    L.off_scnt = o; o = align256(o + (n + 1) * 4);
    L.off_npts = o; o = align256(o + 4);
    L.off_hist = o; o = align256(o + histlen * 4);
    L.off_sums = o; o = align256(o + L.nsums * 4);
    L.off_range = o; o = align256(o + (uint64_t)L.tiles_x * L.tiles_y * 8);
    L.off_conic = o; o = align256(o + (aniso ? n * sizeof(float4) : 0));
    L.off_ext = o; o = align256(o + (aniso ? n * sizeof(float2) : 0));
    L.off_brange = o; o = align256(o + (n + 1 + kT - 1) / kT * sizeof(uint2));
    L.off_part = o; o = align256(o + kRangeParts * sizeof(uint2));
    L.off_plan = o; o = align256(o + 2 * 4);
    L.bytes = o;
    int bits = 1;
    while ((1ull << bits) < (uint64_t)L.tiles_x * L.tiles_y) ++bits;
    L.key_bits = bits;  // of the pair sort (tile ids)
    return L;
}

static hipError_t scan_excl(const uint32_t *in, uint32_t *out, uint64_t len, uint32_t *sums, hipStream_t s)
{
    const uint64_t nb = (len + kScanTile - 1) / kScanTile;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_sums, dim3((unsigned)nb), dim3(kT), 0, s, in, len, sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kT), 0, s, sums, (uint32_t)nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kT), 0, s, in, out, len, sums);
    return hipGetLastError();
}

__global__ __launch_bounds__(kT) void k_sum_u32(const uint32_t *v, uint64_t n, unsigned long long *sum)
{
    unsigned long long c = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kT) c += v[i];
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(sum, c);
}

hipError_t launch_splat_count(const float *x, const float *y, const float *z, uint64_t n, const Proj &P,
                              const AttrPack &A, const narvis_splat_params &prm, void *ws, hipStream_t s,
                              uint64_t *pairs)
{
    const SplatLayout L = splat_layout(n, P.W, P.H, prm.sigma_px, prm.aniso != 0, prm.max_pairs);
    char *base = static_cast<char *>(ws);
    SplatArgs S{};
    S.X = x;
    S.Y = y;
    S.Z = z;
    S.n = n;
    S.P = P;
    S.A = A;
    S.color_mode = prm.color_mode;
    S.color_attr = prm.color_attr;
    S.lut = prm.lut;
    S.lut_min = prm.lut_min;
    S.lut_inv = prm.lut_inv_range;
    S.reach = 3.0f * prm.sigma_px;
    S.tiles_x = L.tiles_x;
    S.tiles_y = L.tiles_y;
    S.ctr = reinterpret_cast<float2 *>(base + L.off_ctr);
    S.col = reinterpret_cast<float4 *>(base + L.off_col);
    S.wbits = reinterpret_cast<uint32_t *>(base + L.off_wbits);
    S.cnt = reinterpret_cast<uint32_t *>(base + L.off_cnt);
    S.brange = reinterpret_cast<uint2 *>(base + L.off_brange);
    S.cap = L.cap;
    S.aniso = prm.aniso;
    S.vel_attr = prm.vel_attr;
    S.sigma = prm.sigma_px;
    S.stretch_k = prm.stretch - 1.0f;
    S.focal = prm.focal_px;
    S.conic = reinterpret_cast<float4 *>(base + L.off_conic);
    S.ext = reinterpret_cast<float2 *>(base + L.off_ext);
    auto *sum = reinterpret_cast<unsigned long long *>(base + L.off_sums);
    hipLaunchKernelGGL(k_splat_project, dim3((unsigned)((n + 1 + kT - 1) / kT)), dim3(kT), 0, s, S);
    hipError_t e = hipMemsetAsync(sum, 0, 8, s);
    if (e != hipSuccess) return e;
    const uint64_t blocks = (n + kT - 1) / kT;
    hipLaunchKernelGGL(k_sum_u32, dim3((unsigned)(blocks < 4096 ? (blocks ? blocks : 1) : 4096)), dim3(kT), 0, s,
                       S.cnt, n, sum);
    unsigned long long total = 0;
    e = hipMemcpyAsync(&total, sum, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    *pairs = total;
    return hipSuccess;
}

// ceil(key_bits / 8) passes of equal width (the last one takes what is left):
// 13-bit tile ids sort in passes of 7 and 6 bits, whose 128 and 64 digits
// give longer runs per digit in the scatter than 8 and 5 would
template <typename K>
static hipError_t radix_sort(K *ka, uint32_t *va, K *kb, uint32_t *vb, const uint32_t *count, uint64_t cap,
                             int key_bits, uint32_t *hist, uint32_t *sums, hipStream_t s, bool *in_b)
{
    const uint64_t nblk64 = ((cap + kSortTile - 1) / kSortTile + 7) & ~uint64_t(7);
    const uint32_t nblk = (uint32_t)(nblk64 ? nblk64 : 8);
    const int passes = (key_bits + 7) / 8;
    const int width = passes ? (key_bits + passes - 1) / passes : 8;
    bool b = false;
    for (int shift = 0; shift < key_bits; shift += width) {
        const int bits = key_bits - shift < width ? key_bits - shift : width;
        const uint32_t mask = (1u << bits) - 1u;
        const ArraySrc<K> src{b ? kb : ka, b ? vb : va, shift, mask};
        hipLaunchKernelGGL((k_radix_hist<K, ArraySrc<K>>), dim3(nblk), dim3(kT), 0, s, src, count, cap, hist, nblk);
        const hipError_t e = scan_excl(hist, hist, (uint64_t)nblk * (mask + 1u), sums, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_radix_scatter<K, ArraySrc<K>>), dim3(nblk), dim3(kT), 0, s, src, b ? ka : kb,
                           b ? va : vb, count, cap, hist, nblk);
        b = !b;
    }
    *in_b = b;
    return hipGetLastError();
}

hipError_t launch_radix_sort(unsigned long long *ka, uint32_t *va, unsigned long long *kb, uint32_t *vb,
                             const uint32_t *count, uint64_t cap, int key_bits, uint32_t *hist, uint32_t *sums,
                             hipStream_t s, bool *in_b)
{
    return radix_sort(ka, va, kb, vb, count, cap, key_bits, hist, sums, s, in_b);
}

hipError_t launch_radix_sort32(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb, const uint32_t *count,
                               uint64_t cap, int key_bits, uint32_t *hist, uint32_t *sums, hipStream_t s, bool *in_b)
{
    return radix_sort(ka, va, kb, vb, count, cap, key_bits, hist, sums, s, in_b);
}

uint64_t radix_sort_hist_len(uint64_t cap)
{
    const uint64_t nblk = ((cap + kSortTile - 1) / kSortTile + 7) & ~uint64_t(7);
    return (nblk ? nblk : 8) * 256;
}

uint64_t radix_sort_sums_len(uint64_t cap)
{
    return (radix_sort_hist_len(cap) + kScanTile - 1) / kScanTile;
}

hipError_t launch_splat(const float *x, const float *y, const float *z, uint64_t n, const Proj &P, const AttrPack &A,
                        const narvis_splat_params &prm, float *img, void *ws, hipStream_t s)
{
    const SplatLayout L = splat_layout(n, P.W, P.H, prm.sigma_px, prm.aniso != 0, prm.max_pairs);
    char *base = static_cast<char *>(ws);
    SplatArgs S;
    S.X = x;
    S.Y = y;
    S.Z = z;
    S.n = n;
    S.P = P;
    S.A = A;
    S.color_mode = prm.color_mode;
    S.color_attr = prm.color_attr;
    S.lut = prm.lut;
    S.lut_min = prm.lut_min;
    S.lut_inv = prm.lut_inv_range;
    S.reach = 3.0f * prm.sigma_px;
    S.tiles_x = L.tiles_x;
    S.tiles_y = L.tiles_y;
    S.ctr = reinterpret_cast<float2 *>(base + L.off_ctr);
    S.col = reinterpret_cast<float4 *>(base + L.off_col);
    S.wbits = reinterpret_cast<uint32_t *>(base + L.off_wbits);
    S.cnt = reinterpret_cast<uint32_t *>(base + L.off_cnt);
    S.brange = reinterpret_cast<uint2 *>(base + L.off_brange);
    S.cap = L.cap;
    S.aniso = prm.aniso;
    S.vel_attr = prm.vel_attr;
    S.sigma = prm.sigma_px;
    S.stretch_k = prm.stretch - 1.0f;
    S.focal = prm.focal_px;
    S.conic = reinterpret_cast<float4 *>(base + L.off_conic);
    S.ext = reinterpret_cast<float2 *>(base + L.off_ext);
    auto *ka = reinterpret_cast<uint32_t *>(base + L.off_ka);
    auto *kb = reinterpret_cast<uint32_t *>(base + L.off_kb);
    auto *va = reinterpret_cast<uint32_t *>(base + L.off_va);
    auto *vb = reinterpret_cast<uint32_t *>(base + L.off_vb);
    auto *hist = reinterpret_cast<uint32_t *>(base + L.off_hist);
    auto *sums = reinterpret_cast<uint32_t *>(base + L.off_sums);
    auto *range = reinterpret_cast<uint32_t *>(base + L.off_range);
    const uint64_t ntiles = (uint64_t)L.tiles_x * L.tiles_y;

    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((2 * ntiles + kT - 1) / kT)), dim3(kT), 0, s, range, 2 * ntiles, 0u);
    hipLaunchKernelGGL(k_splat_project, dim3((unsigned)((n + 1 + kT - 1) / kT)), dim3(kT), 0, s, S);
    auto *scnt = reinterpret_cast<uint32_t *>(base + L.off_scnt);
    auto *npts = reinterpret_cast<uint32_t *>(base + L.off_npts);
    const uint32_t *total = scnt + n;  // after the scan
    hipError_t e = hipSuccess;
    if (n > 0) {
        // point order by depth (three or four passes, chosen on the device;
        // ends in ka/va)
        const uint64_t nbp = (n + 1 + kT - 1) / kT;  // projection workgroups
        const uint32_t nparts = (uint32_t)(nbp < (uint64_t)kRangeParts ? nbp : (uint64_t)kRangeParts);
        auto *part = reinterpret_cast<uint2 *>(base + L.off_part);
        auto *plan = reinterpret_cast<uint32_t *>(base + L.off_plan);
        hipLaunchKernelGGL(k_range_partial, dim3(nparts), dim3(kT), 0, s, S.brange, nbp, part);
        hipLaunchKernelGGL(k_depth_plan, dim3(1), dim3(kT), 0, s, part, nparts, plan);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kT), 0, s, npts, (uint64_t)1, (uint32_t)n);
        const uint32_t nblk = (uint32_t)((((n + kSortTile - 1) / kSortTile) + 7) & ~uint64_t(7));
        for (int slot = 0; slot < 4; ++slot) {
            // slot 0 writes (kb, vb); then (kb, vb) -> (ka, va) -> (kb, vb) -> (ka, va)
            const bool from_a = slot == 2;
            const DepthSrc src{from_a ? ka : kb, from_a ? va : vb, S.wbits, S.cnt, plan, slot, 0u, false, false};
            uint32_t *ko = (slot & 1) ? ka : kb;
            uint32_t *vo = (slot & 1) ? va : vb;
            hipLaunchKernelGGL((k_radix_hist<uint32_t, DepthSrc>), dim3(nblk), dim3(kT), 0, s, src, npts, n, hist,
                               nblk);
            e = scan_excl(hist, hist, (uint64_t)nblk * 256, sums, s);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL((k_radix_scatter<uint32_t, DepthSrc>), dim3(nblk), dim3(kT), 0, s, src, ko, vo, npts, n,
                               hist, nblk);
        }
        const uint32_t *order = va;
        uint32_t *pk = kb, *pv = vb;  // the free pair of arrays
        hipLaunchKernelGGL(k_gather_counts, dim3((unsigned)((n + 1 + kT - 1) / kT)), dim3(kT), 0, s, S.cnt, order, ka,
                           plan, n, scnt);
        e = scan_excl(scnt, scnt, n + 1, sums, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_splat_emit, dim3((unsigned)((n + kT - 1) / kT)), dim3(kT), 0, s, S, order, scnt, pk, pv);
        // pairs by tile, stable (depth order kept within a tile)
        bool in_b = false;
        e = radix_sort(pk, pv, ka, va, total, L.cap, L.key_bits, hist, sums, s, &in_b);
        if (e != hipSuccess) return e;
        if (!in_b) {
            ka = pk;
            va = pv;
        }
    } else {
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(kT), 0, s, scnt, (uint64_t)1, 0u);
    }
    const uint64_t rblocks = (L.cap + (uint64_t)kT * kRangeItems - 1) / ((uint64_t)kT * kRangeItems);
    hipLaunchKernelGGL(k_tile_ranges, dim3((unsigned)(rblocks ? rblocks : 1)), dim3(kT),
                       0, s, ka, total, L.cap, range, (uint32_t)ntiles);
    BlendArgs B;
    B.n = n;
    B.cap = L.cap;
    B.count = total;
    B.range = range;
    B.vals = va;
    B.ctr = S.ctr;
    B.col = S.col;
    B.conic = S.conic;
    B.ext = S.ext;
    B.img = img;
    B.W = P.W;
    B.H = P.H;
    B.tiles_x = L.tiles_x;
    const float reach = 3.0f * prm.sigma_px;
    B.reach = reach;
    B.cut2 = reach * reach;
    B.inv2s2 = 1.0f / (2.0f * prm.sigma_px * prm.sigma_px);
    B.opacity = prm.opacity;
    if (prm.aniso)
        hipLaunchKernelGGL(k_splat_blend<true>, dim3((unsigned)ntiles), dim3(kT), 0, s, B);
    else
        hipLaunchKernelGGL(k_splat_blend<false>, dim3((unsigned)ntiles), dim3(kT), 0, s, B);
    return hipGetLastError();
}

}  // namespace narvis

// Multi-attribute point rasterizer for gfx950: clear, render, resolve.
//
// Render (Sec. 3.2, "transforms the points from world to screen space and
// renders point depth to a custom framebuffer ... closest visible points ...
// via early z-buffer testing"): every thread streams four consecutive points
// of the SoA x/y/z arrays with 16-byte loads, projects them in fp32 with
// every operation rounded in the written order (this file is compiled with
// FMA contraction off), and merges (depth bits << 32 | index) into the
// per-pixel 64-bit key with an unsigned atomic minimum.  The early-z variant
// first reads the key and skips the atomic when the point cannot win: the key
// buffer only ever decreases, so a stale read can only skip a point that
// would lose anyway.
//
// Resolve (Sec. 3.2, "transfers other corresponding point attributes to the
// final G-buffers"): one thread per pixel gathers the winner's attributes.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>
#include <vector>

#include "internal.h"

#pragma clang fp contract(off)

namespace narvis {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBlock = 256;
constexpr int kQuadsPerThread = 2;

// Correctly rounded reciprocal of a normal w: one Newton step on the hardware
// estimate.  Checked on gfx950 against 1.0f / w for every significand at
// every exponent in [-124, 124].
__device__ __forceinline__ float rcp_rn(float w)
{
    const float y0 = __builtin_amdgcn_rcpf(w);
    return __builtin_fmaf(__builtin_fmaf(-w, y0, 1.0f), y0, y0);
}

// a / w with y = rcp_rn(w): q0 is within an ulp of the quotient, the FMA
// gives the remainder a - w q0 exactly, and the corrected q0 + r y is the
// correctly rounded quotient (Markstein's theorem), i.e. bit-identical to
// a / w whenever the quotient neither overflows nor underflows.  (Where it
// does, the point is culled, or (q / 2 + 1/2) rounds to 1/2 either way.)
__device__ __forceinline__ float div_rcp(float a, float w, float y)
{
    const float q0 = a * y;
    return __builtin_fmaf(__builtin_fmaf(-w, q0, a), y, q0);
}

// RCP: divide by the depth through its reciprocal (shared by both
// coordinates); valid when every kept depth is a normal float with exponent
// in [-124, 124], which the host checks from the near/far bounds.
template <bool RCP = false>
__device__ __forceinline__ bool project(const Proj &P, float x, float y, float z, uint32_t &ix, uint32_t &iy,
                                       float &w)
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
    // evaluated without branches (a culled point's values are discarded), so
    // the independent points of a thread interleave
    float nx, ny;
    if constexpr (RCP) {
        const float r = rcp_rn(ww);
        nx = div_rcp(cx, ww, r);
        ny = div_rcp(cy, ww, r);
    } else {
        nx = cx / ww;
        ny = cy / ww;
    }
    float sx = nx * 0.5f;
    sx = sx + 0.5f;
    sx = sx * P.Wf;
    float sy = ny * 0.5f;
    sy = 0.5f - sy;
    sy = sy * P.Hf;
    // 0 <= sx < W as one unsigned comparison of bit patterns: sx is never -0
    // (u + 0.5 and 0.5 - u are never -0 in round to nearest, and scaling by
    // W >= 1 cannot flush a nonzero value to zero), non-negative floats order
    // like their bits, and every negative value or NaN has a pattern above
    // that of the positive finite W.  Likewise for sy.
    const bool ok = (ww >= P.near_f) & (ww <= P.far_f) & (__float_as_uint(sx) < __float_as_uint(P.Wf)) &
                    (__float_as_uint(sy) < __float_as_uint(P.Hf));
    // clamped before the conversion; equal to sx, sy whenever ok
    const float xs = fminf(fmaxf(sx, 0.0f), P.Wf), ys = fminf(fmaxf(sy, 0.0f), P.Hf);
    ix = (uint32_t)(int32_t)xs;
    iy = (uint32_t)(int32_t)ys;
    w = ww;
    return ok;
}

template <bool RCP = false>
__device__ __forceinline__ bool project(const Proj &P, float x, float y, float z, uint32_t &pix, float &w)
{
    uint32_t ix, iy;
    const bool ok = project<RCP>(P, x, y, z, ix, iy, w);
    pix = iy * (uint32_t)P.W + ix;
    return ok;
}

// Glyph-priority render (VisGlyph): a point that is not a glyph point
// carries bit 31 in the high word of its key, so any glyph point reaching a
// pixel beats every non-glyph point there (depth bits never use bit 31: the
// kept depths are positive).
constexpr uint32_t kNotGlyph = 0x80000000u;

__device__ __forceinline__ uint32_t glyph_rank(const uint8_t *glyph, uint64_t i)
{
    return glyph ? (glyph[i] ? 0u : kNotGlyph) : 0u;
}

template <int VARIANT>
__device__ __forceinline__ void merge(unsigned long long *keys, uint32_t pix, float w, uint32_t idx, uint32_t rank = 0)
{
    const unsigned long long key = ((unsigned long long)(__float_as_uint(w) | rank) << 32) | idx;
    if (VARIANT == NARVIS_RENDER_EARLYZ) {
        if (key >= keys[pix]) return;
    }
    __hip_atomic_fetch_min(keys + pix, key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Chunk order.  Workgroups are handed to the XCDs round-robin, so blocks
// b = k, k + X, k + 2X, ... run on XCD k (X = xcds).  XCD k is given one
// contiguous stretch of chunks, which keeps the key lines that a coherent
// cloud touches inside that XCD's L2; within its stretch the XCD visits the
// chunks in a low-discrepancy order (index * stride mod per, stride coprime
// with per and near per / golden ratio), so that early in the frame the
// points already cover the whole image and the early depth test rejects most
// later points instead of letting them reach the atomic.
struct ChunkOrder {
    uint32_t xcds;
    uint32_t per;     // logical blocks per XCD (grid = xcds * per)
    uint32_t stride;  // coprime with per
};

__device__ __forceinline__ uint64_t logical_block(const ChunkOrder &o)
{
    const uint32_t b = blockIdx.x;
    const uint32_t k = b % o.xcds;
    const uint64_t j = b / o.xcds;
    return (uint64_t)k * o.per + (j * o.stride) % o.per;
}

template <int VARIANT>
__global__ __launch_bounds__(kBlock) void k_render_vec(const float *__restrict__ X, const float *__restrict__ Y,
                                                        const float *__restrict__ Z, uint64_t n, Proj P,
                                                        unsigned long long *__restrict__ keys, ChunkOrder order,
                                                        const uint8_t *__restrict__ glyph)
{
    const uint64_t nq = n >> 2;
    const uint64_t lb = logical_block(order);
    const uint64_t stride = (uint64_t)gridDim.x * kBlock * kQuadsPerThread;
    const uint32_t spread = (uint32_t)((lb * 2654435761ull) % (uint64_t)((uint32_t)P.W * (uint32_t)P.H));
    for (uint64_t base = lb * kBlock * kQuadsPerThread + threadIdx.x; base < nq; base += stride) {
        f32x4 xs[kQuadsPerThread], ys[kQuadsPerThread], zs[kQuadsPerThread];
#pragma unroll
        for (int k = 0; k < kQuadsPerThread; ++k) {
            const uint64_t q = base + (uint64_t)k * kBlock;
            if (q < nq) {
                xs[k] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(X) + q);
                ys[k] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(Y) + q);
                zs[k] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(Z) + q);
            }
        }
        // project all points of this thread first, then issue every early-z
        // read, and only then the atomics: an atomic may alias a later read,
        // so interleaving them would serialise one memory round trip per point
        constexpr int kPts = kQuadsPerThread * 4;
        uint32_t pix[kPts];
        unsigned long long key[kPts];
        bool hit[kPts];
#pragma unroll
        for (int k = 0; k < kQuadsPerThread; ++k) {
            const uint64_t q = base + (uint64_t)k * kBlock;
            const bool live = q < nq;
            const uint32_t i0 = (uint32_t)(q << 2);
            const float px[4] = {xs[k].x, xs[k].y, xs[k].z, xs[k].w};
            const float py[4] = {ys[k].x, ys[k].y, ys[k].z, ys[k].w};
            const float pz[4] = {zs[k].x, zs[k].y, zs[k].z, zs[k].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float w = 0.0f;
                uint32_t pp = 0;
                hit[k * 4 + j] = live && project(P, px[j], py[j], pz[j], pp, w);
                pix[k * 4 + j] = pp;
                const uint32_t rank = (live && glyph) ? glyph_rank(glyph, (q << 2) + j) : 0u;
                key[k * 4 + j] = ((unsigned long long)(__float_as_uint(w) | rank) << 32) | (i0 + (uint32_t)j);
            }
        }
        if (VARIANT == NARVIS_RENDER_EARLYZ) {
            // Branch-free reads: a lane whose point was culled reads the pixel
            // of the first live lane of its wave (the request merges with that
            // lane's), or a per-workgroup pixel when the whole wave is culled.
            // Conditional loads would each end in a wait on the memory counter.
            uint32_t addr[kPts];
#pragma unroll
            for (int t = 0; t < kPts; ++t) {
                const unsigned long long live = __ballot(hit[t]);
                const uint32_t lead = live ? (uint32_t)__builtin_ctzll(live) : 0u;
                const uint32_t lpix = live ? (uint32_t)__builtin_amdgcn_readlane((int)pix[t], (int)lead) : spread;
                addr[t] = hit[t] ? pix[t] : lpix;
            }
            unsigned long long cur[kPts];
#pragma unroll
            for (int t = 0; t < kPts; ++t) cur[t] = keys[addr[t]];
#pragma unroll
            for (int t = 0; t < kPts; ++t) hit[t] = hit[t] && key[t] < cur[t];
        }
#pragma unroll
        for (int t = 0; t < kPts; ++t)
            if (hit[t]) __hip_atomic_fetch_min(keys + pix[t], key[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the last n % 4 points
    if (blockIdx.x == 0 && threadIdx.x < (n & 3)) {
        const uint64_t i = (nq << 2) + threadIdx.x;
        uint32_t pix;
        float w;
        if (project(P, X[i], Y[i], Z[i], pix, w)) merge<VARIANT>(keys, pix, w, (uint32_t)i, glyph_rank(glyph, i));
    }
}

// LDS-binned render.  A workgroup folds the candidates of its chunk of
// kChunk points per pixel in LDS before touching the global key buffer:
//   insert -- every surviving point does a non-returning LDS 64-bit atomic
//             minimum of its key into slot (pixel mod kSlots) and records its
//             pixel in pixof[local index];
//   check  -- after a barrier each candidate looks at its slot: the slot's key
//             names the winning point, whose pixel is pixof[key index - first
//             index].  If that is another pixel, the candidate lost the slot to
//             a collision and takes the global early-z path itself;
//   flush  -- every occupied slot is one pixel's best candidate of the chunk:
//             early-z read of the global key, global atomic minimum if smaller.
// Each thread owns slots t, t + kBlock, ..., so a wave flushes 64 consecutive
// slots, i.e. runs of consecutive pixels of a row: its reads and atomics land
// on few cache lines (a gather pays per distinct address), and the global
// work per chunk is per touched pixel, not per point.
constexpr int kSlots = 2048;
constexpr int kChunk = kBlock * kQuadsPerThread * 4;
constexpr int kPts = kQuadsPerThread * 4;
constexpr int kPer = kSlots / kBlock;
constexpr uint32_t kNoPixel = 0xFFFFFFFFu;

// early-z reads for up to K candidates, issued together (an inactive lane reads
// the first active lane's address, so its request merges), then the atomics
template <int K>
__device__ __forceinline__ void global_merge(unsigned long long *__restrict__ keys, const uint32_t (&pix)[K],
                                             const unsigned long long (&key)[K], bool (&hit)[K], uint32_t spread)
{
    uint32_t addr[K];
    bool any[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        const unsigned long long live = __ballot(hit[t]);
        const uint32_t lead = live ? (uint32_t)__builtin_ctzll(live) : 0u;
        const uint32_t lpix = live ? (uint32_t)__builtin_amdgcn_readlane((int)pix[t], (int)lead) : spread;
        addr[t] = hit[t] ? pix[t] : lpix;
    }
    // a read that no lane of the wave needs is skipped (wave-uniform branch)
    unsigned long long cur[K];
#pragma unroll
    for (int t = 0; t < K; ++t) {
        any[t] = __ballot(hit[t]) != 0;
        cur[t] = 0;
    }
#pragma unroll
    for (int t = 0; t < K; ++t)
        if (any[t]) cur[t] = keys[addr[t]];
#pragma unroll
    for (int t = 0; t < K; ++t)
        if (hit[t] && key[t] < cur[t]) __hip_atomic_fetch_min(keys + pix[t], key[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Which chunks of kChunk points a launch renders: the multiples of `mul`,
// without those that are multiples of mul * excl when excl >= 2.  Virtual
// chunk v of the launch is real chunk mul v (excl = 0), or mul times the v-th
// integer that is not a multiple of excl.  `tail`: this launch also renders
// the last n % 4 points.
struct ChunkSel {
    uint32_t mul, excl;
    uint64_t nv;  // virtual chunks of this launch
    uint32_t tail;
};

__device__ __forceinline__ uint64_t real_chunk(const ChunkSel &c, uint64_t v)
{
    return (uint64_t)c.mul * (c.excl ? v + v / (c.excl - 1) + 1 : v);
}

// Screen tiles of 2^shift x 2^shift pixels, tiles_x per row, one depth bound
// per tile (the high 16 bits of the largest depth bits held by a pixel of the
// tile) and one per pixel (its depth bits), both taken by k_tile_bounds.
constexpr int kMaxTiles = 8192;

struct TileGrid {
    const uint16_t *bounds;
    const uint32_t *pixb;
    uint32_t shift, tiles_x, ntiles;
};

__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = fminf(v, __shfl_xor(v, d));
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = fmaxf(v, __shfl_xor(v, d));
    return v;
}

// Whole-batch cull of the layout render (every lane of the wave must call it
// with the same box; every lane returns the same answer, so a workgroup whose
// waves all call it stays uniform).  The eight corners of the batch's box are
// projected with the points' own arithmetic.  A point of the box has clip
// values within the corners' hull widened by the rounding of both
// evaluations (four rounded operations each: below 2^-21 of the row's sum of
// magnitudes S); the test widens by 2^-20 S.  Lane l takes corner (l & 31) >> 2
// and margin signs l & 3; min/max over the wave give the depth range and, when
// every depth is positive, the range of cx/w and cy/w (a ratio of affine
// functions takes its extremes at the hull's vertices; rounding is monotone),
// hence the screen rectangle.  True when no point of the box can be kept:
// its depth range misses [near, far], its rectangle misses the image, or
// (OCCL) its nearest depth exceeds the tile bound of every tile that the
// rectangle, one pixel wider on each side, touches.  A box without a finite
// point (+inf/-inf) is culled: non-finite points never pass the cull.
template <bool OCCL>
__device__ __forceinline__ bool batch_culled(const Proj &P, float4 lo, float4 hi, const uint16_t *tb, uint32_t shift,
                                             uint32_t tiles_x)
{
    if (!(lo.x <= hi.x)) return true;
    const uint32_t lane = threadIdx.x & 31, c = lane >> 2, sg = lane & 3;
    const float x = (c & 1) ? hi.x : lo.x, y = (c & 2) ? hi.y : lo.y, z = (c & 4) ? hi.z : lo.z;
    const float ax = fmaxf(fabsf(lo.x), fabsf(hi.x)), ay = fmaxf(fabsf(lo.y), fabsf(hi.y)),
                az = fmaxf(fabsf(lo.z), fabsf(hi.z));
    float cx = P.m00 * x;
    cx = cx + P.m01 * y;
    cx = cx + P.m02 * z;
    cx = cx + P.m03;
    float cy = P.m10 * x;
    cy = cy + P.m11 * y;
    cy = cy + P.m12 * z;
    cy = cy + P.m13;
    float w = P.m30 * x;
    w = w + P.m31 * y;
    w = w + P.m32 * z;
    w = w + P.m33;
    float sx = fabsf(P.m00) * ax;
    sx = sx + fabsf(P.m01) * ay;
    sx = sx + fabsf(P.m02) * az;
    sx = sx + fabsf(P.m03);
    float sy = fabsf(P.m10) * ax;
    sy = sy + fabsf(P.m11) * ay;
    sy = sy + fabsf(P.m12) * az;
    sy = sy + fabsf(P.m13);
    float sw = fabsf(P.m30) * ax;
    sw = sw + fabsf(P.m31) * ay;
    sw = sw + fabsf(P.m32) * az;
    sw = sw + fabsf(P.m33);
    const float mx = sx * 0x1p-20f, my = sy * 0x1p-20f, mw = sw * 0x1p-20f;
    const float wlo = wave_min(w - mw), whi = wave_max(w + mw);
    if (whi < P.near_f || wlo > P.far_f) return true;
    if (!(wlo > 0.0f)) return false;  // the box reaches behind the eye: no rectangle
    const float wv = (sg & 2) ? w + mw : w - mw;
    const float nx = ((sg & 1) ? cx + mx : cx - mx) / wv;
    const float ny = ((sg & 1) ? cy + my : cy - my) / wv;
    const float nxlo = wave_min(nx), nxhi = wave_max(nx), nylo = wave_min(ny), nyhi = wave_max(ny);
    float sxlo = nxlo * 0.5f;
    sxlo = sxlo + 0.5f;
    sxlo = sxlo * P.Wf;
    float sxhi = nxhi * 0.5f;
    sxhi = sxhi + 0.5f;
    sxhi = sxhi * P.Wf;
    float sylo = nyhi * 0.5f;
    sylo = 0.5f - sylo;
    sylo = sylo * P.Hf;
    float syhi = nylo * 0.5f;
    syhi = 0.5f - syhi;
    syhi = syhi * P.Hf;
    if (sxhi < 0.0f || sxlo >= P.Wf || syhi < 0.0f || sylo >= P.Hf) return true;
    if (!OCCL) return false;
    const uint32_t ix0 = (uint32_t)fmaxf(floorf(sxlo) - 1.0f, 0.0f);
    const uint32_t ix1 = (uint32_t)fminf(floorf(sxhi) + 1.0f, P.Wf - 1.0f);
    const uint32_t iy0 = (uint32_t)fmaxf(floorf(sylo) - 1.0f, 0.0f);
    const uint32_t iy1 = (uint32_t)fminf(floorf(syhi) + 1.0f, P.Hf - 1.0f);
    const uint32_t tx0 = ix0 >> shift, tx1 = ix1 >> shift, ty0 = iy0 >> shift, ty1 = iy1 >> shift;
    if (tx1 < tx0 || ty1 < ty0) return false;
    const uint32_t ntx = tx1 - tx0 + 1, nt = ntx * (ty1 - ty0 + 1);
    if (nt > 1024) return false;
    // kept points have depth >= max(lowest depth, near), positive: their bit
    // patterns order like the depths
    const uint32_t dlo = __float_as_uint(fmaxf(wlo, P.near_f)) >> 16;
    uint32_t m = 0;
    for (uint32_t t = threadIdx.x & 63; t < nt; t += 64) m = max(m, (uint32_t)tb[(ty0 + t / ntx) * tiles_x + tx0 + t % ntx]);
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, d));
    return dlo > m;
}

__device__ __forceinline__ void render_tail(const float *X, const float *Y, const float *Z, uint64_t n,
                                            const Proj &P, unsigned long long *keys, const ChunkSel &sel,
                                            const uint32_t *ix = nullptr, const uint8_t *glyph = nullptr)
{
    const uint64_t nq = n >> 2;
    if (sel.tail && blockIdx.x == 0 && threadIdx.x < (n & 3)) {
        const uint64_t i = (nq << 2) + threadIdx.x;
        uint32_t pix;
        float w;
        if (project(P, X[i], Y[i], Z[i], pix, w))
            merge<NARVIS_RENDER_EARLYZ>(keys, pix, w, ix ? ix[i] : (uint32_t)i, glyph_rank(glyph, i));
    }
}

// (4 waves per SIMD: the compiler keeps it within 128 registers)
// MODE 1 (layout): the points are in layout order; key indices come from the
// index stream, and a chunk (= one batch) outside the view volume is skipped
// whole.  The slot winner's pixel is then recorded by the winner itself (its
// key is unique) instead of being looked up from its position in the chunk.
// MODE 2 (glyph priority): the glyph mask, one byte per point, sets the rank
// bit of non-glyph points' keys.
template <bool RCP, int MODE>
__global__ __launch_bounds__(kBlock, 4) void k_render_lds(const float *__restrict__ X, const float *__restrict__ Y,
                                                        const float *__restrict__ Z, uint64_t n, Proj P,
                                                        unsigned long long *__restrict__ keys, ChunkOrder order,
                                                        ChunkSel sel, LayoutArgs lay)
{
    constexpr bool IX = MODE == 1, GLYPH = MODE == 2;
    __shared__ unsigned long long best[kSlots];
    __shared__ uint32_t pixof[kChunk];  // IX: pixel of each slot's winner
    for (int s = threadIdx.x; s < kSlots; s += kBlock) best[s] = NARVIS_KEY_EMPTY;
    const uint64_t nq = n >> 2;
    const uint64_t lb = logical_block(order);
    constexpr uint64_t kQuads = (uint64_t)kBlock * kQuadsPerThread;  // quads per chunk
    const uint32_t npx = (uint32_t)P.W * (uint32_t)P.H;
    const uint32_t spread = (uint32_t)((lb * 2654435761ull) % (uint64_t)npx);
    __syncthreads();
    // uniform trip count for the whole workgroup: the barriers below need it
    for (uint64_t v = lb; v < sel.nv; v += gridDim.x) {
        const uint64_t chunk = real_chunk(sel, v);
        const uint64_t start = chunk * kQuads;
        const uint32_t first = (uint32_t)(start << 2);  // index of the chunk's first point (mod 2^32)
        if (IX && batch_culled<false>(P, lay.box[2 * chunk], lay.box[2 * chunk + 1], nullptr, 0, 0)) continue;
        f32x4 xs[kQuadsPerThread], ys[kQuadsPerThread], zs[kQuadsPerThread];
        u32x4 is[kQuadsPerThread];
        uint32_t gq[kQuadsPerThread];
#pragma unroll
        for (int k = 0; k < kQuadsPerThread; ++k) {
            const uint64_t q = start + threadIdx.x + (uint64_t)k * kBlock;
            gq[k] = 0xFFFFFFFFu;
            if (q < nq) {
                xs[k] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(X) + q);
                ys[k] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(Y) + q);
                zs[k] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(Z) + q);
                if (IX) is[k] = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(lay.ix) + q);
                if (GLYPH) gq[k] = __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(lay.glyph) + q);
            }
        }
        uint32_t pix[kPts];
        unsigned long long key[kPts];
        bool hit[kPts];
#pragma unroll
        for (int k = 0; k < kQuadsPerThread; ++k) {
            const uint32_t lq = threadIdx.x + (uint32_t)k * kBlock;  // quad within the chunk
            const bool live = start + lq < nq;
            const float px[4] = {xs[k].x, xs[k].y, xs[k].z, xs[k].w};
            const float py[4] = {ys[k].x, ys[k].y, ys[k].z, ys[k].w};
            const float pz[4] = {zs[k].x, zs[k].y, zs[k].z, zs[k].w};
            uint32_t pi[4] = {first + lq * 4, first + lq * 4 + 1, first + lq * 4 + 2, first + lq * 4 + 3};
            if (IX) {
                pi[0] = is[k].x;
                pi[1] = is[k].y;
                pi[2] = is[k].z;
                pi[3] = is[k].w;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int t = k * 4 + j;
                float w = 0.0f;
                uint32_t pp = 0;
                hit[t] = project<RCP>(P, px[j], py[j], pz[j], pp, w) & live;
                pix[t] = pp;
                const uint32_t rank = (GLYPH && ((gq[k] >> (8 * j)) & 0xFFu) == 0u) ? kNotGlyph : 0u;
                key[t] = ((unsigned long long)(__float_as_uint(w) | rank) << 32) | pi[j];
                if (!IX) pixof[lq * 4 + j] = hit[t] ? pp : kNoPixel;
                if (hit[t]) atomicMin(&best[pp & (kSlots - 1)], key[t]);
            }
        }
        __syncthreads();
        // collision check: did my slot's winner come from my pixel?
        unsigned long long won[kPts];
#pragma unroll
        for (int t = 0; t < kPts; ++t) won[t] = best[pix[t] & (kSlots - 1)];
        if (IX) {
            // the winner (unique key) records its pixel for its slot
#pragma unroll
            for (int t = 0; t < kPts; ++t)
                if (hit[t] && won[t] == key[t]) pixof[pix[t] & (kSlots - 1)] = pix[t];
            __syncthreads();
#pragma unroll
            for (int t = 0; t < kPts; ++t) hit[t] = hit[t] && pixof[pix[t] & (kSlots - 1)] != pix[t];
        } else {
#pragma unroll
            for (int t = 0; t < kPts; ++t)
                hit[t] = hit[t] && pixof[((uint32_t)won[t] - first) & (kChunk - 1)] != pix[t];
        }
        // my slots' winners
        uint32_t fpix[kPer];
        unsigned long long fkey[kPer];
        bool fhit[kPer];
#pragma unroll
        for (int t = 0; t < kPer; ++t) {
            fkey[t] = best[threadIdx.x + t * kBlock];
            fhit[t] = fkey[t] != NARVIS_KEY_EMPTY;
            if (IX)
                fpix[t] = fhit[t] ? pixof[threadIdx.x + t * kBlock] : 0u;
            else
                fpix[t] = fhit[t] ? pixof[((uint32_t)fkey[t] - first) & (kChunk - 1)] : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < kPer; ++t) best[threadIdx.x + t * kBlock] = NARVIS_KEY_EMPTY;
        global_merge<kPer>(keys, fpix, fkey, fhit, spread);
        global_merge<kPts>(keys, pix, key, hit, spread);
        __syncthreads();
    }
    render_tail(X, Y, Z, n, P, keys, sel, lay.ix, lay.glyph);
}

// Key address with a 32-bit byte offset when the image has fewer than 2^29
// pixels (the load and atomic then take a scalar base and one offset register).
template <bool OFF32>
__device__ __forceinline__ unsigned long long *key_at(unsigned long long *keys, uint32_t pix)
{
    if (OFF32) return reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(keys) + (pix << 3));
    return keys + pix;
}

// quads per thread and workgroup size of the cull pass: one chunk of kChunk
// points per workgroup iteration
constexpr int kCullQpt = 2;
constexpr int kCullBlock = kChunk / 4 / kCullQpt;
constexpr int kCullPts = 4 * kCullQpt;

// Bounded render of the chunks `sel` picks, after some chunks have been
// rendered and k_tile_bounds has taken the bounds.  Keys only decrease, so a
// point deeper than its bound cannot win its pixel: each point is tested
// against its tile's bound (LDS), the survivors against their pixel's bound
// (a 32-bit global read; the 16 high bits would pass every point of a
// surface, whose depths at one pixel agree to a few ulps), and what is left
// goes to the atomic minimum.  No LDS table and no barrier in the loop: the
// waves stream independently.
// MODE 1 (layout): the points are in layout order (key indices from the
// index stream, read only for the points that reach the atomic), and a chunk
// (= one batch) whose box is outside the view volume or behind the tile
// bounds is skipped whole, before its points are loaded.  MODE 2 (glyph
// priority): the rank bit of non-glyph points takes part in every bound test
// and key, exactly like a depth bit above all others.
template <bool RCP, bool OFF32, int MODE>
__global__ __launch_bounds__(kCullBlock) void k_render_cull(const float *__restrict__ X, const float *__restrict__ Y,
                                                        const float *__restrict__ Z, uint64_t n, Proj P,
                                                        unsigned long long *__restrict__ keys, ChunkOrder order,
                                                        ChunkSel sel, TileGrid tg, LayoutArgs lay)
{
    constexpr bool IX = MODE == 1, GLYPH = MODE == 2;
    __shared__ uint16_t tb[kMaxTiles];
    for (uint32_t s = threadIdx.x; s < tg.ntiles; s += kCullBlock) tb[s] = tg.bounds[s];
    const uint64_t nq = n >> 2;
    const uint64_t lb = logical_block(order);
    constexpr uint64_t kQuads = (uint64_t)kCullBlock * kCullQpt;
    const uint32_t npx = (uint32_t)P.W * (uint32_t)P.H;
    const uint32_t spread = (uint32_t)((lb * 2654435761ull) % (uint64_t)npx);
    __syncthreads();
    f32x4 xs[kCullQpt], ys[kCullQpt], zs[kCullQpt];
    uint32_t gq[kCullQpt];
    // every quad index is clamped into the array so that each fetch issues
    // the same six loads (the extra quads are not live)
    auto fetch = [&](uint64_t v) {
        const uint64_t st = real_chunk(sel, v) * kQuads;
#pragma unroll
        for (int k = 0; k < kCullQpt; ++k) {
            uint64_t q = st + threadIdx.x + (uint64_t)k * kCullBlock;
            q = q < nq ? q : nq - 1;
            xs[k] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(X) + q);
            ys[k] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(Y) + q);
            zs[k] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(Z) + q);
            if (GLYPH) gq[k] = __builtin_nontemporal_load(reinterpret_cast<const uint32_t *>(lay.glyph) + q);
        }
    };
    // the first chunk at or after v (in steps of the grid) that is not culled
    // whole (wave-uniform; without a layout every chunk is rendered)
    auto visible = [&](uint64_t v) {
        if (IX) {
            while (v < sel.nv) {
                const uint64_t c = real_chunk(sel, v);
                if (!batch_culled<true>(P, lay.box[2 * c], lay.box[2 * c + 1], tb, tg.shift, tg.tiles_x)) break;
                v += gridDim.x;
            }
        }
        return v;
    };
    uint64_t v = visible(lb);
    if (v < sel.nv && nq > 0) fetch(v);
    while (v < sel.nv) {
        const uint64_t start = real_chunk(sel, v) * kQuads;
        const uint32_t first = (uint32_t)(start << 2);
        uint32_t pix[kCullPts];
        unsigned long long key[kCullPts];
        bool hit[kCullPts];
#pragma unroll
        for (int k = 0; k < kCullQpt; ++k) {
            const uint32_t lq = threadIdx.x + (uint32_t)k * kCullBlock;
            const bool live = start + lq < nq;
            const float px[4] = {xs[k].x, xs[k].y, xs[k].z, xs[k].w};
            const float py[4] = {ys[k].x, ys[k].y, ys[k].z, ys[k].w};
            const float pz[4] = {zs[k].x, zs[k].y, zs[k].z, zs[k].w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int t = k * 4 + j;
                float w = 0.0f;
                uint32_t ix = 0, iy = 0;
                bool h = project<RCP>(P, px[j], py[j], pz[j], ix, iy, w) & live;
                const uint32_t hw = __float_as_uint(w) | ((GLYPH && ((gq[k] >> (8 * j)) & 0xFFu) == 0u) ? kNotGlyph : 0u);
                const uint32_t tile = h ? __umul24(iy >> tg.shift, tg.tiles_x) + (ix >> tg.shift) : 0u;
                hit[t] = h & ((hw >> 16) <= (uint32_t)tb[tile]);
                pix[t] = __umul24(iy, (uint32_t)P.W) + ix;
                // IX: the low word holds the point's position until the atomic
                key[t] = ((unsigned long long)hw << 32) | (first + lq * 4 + (uint32_t)j);
            }
            // consecutive points on one pixel (a surface sampled finer than
            // the pixels): the last of a run carries the run's smallest key
            // (IX: only across different depths, where the index cannot matter)
#pragma unroll
            for (int j = 1; j < 4; ++j) {
                const int t = k * 4 + j;
                if (hit[t - 1] && hit[t] && pix[t - 1] == pix[t]) {
                    if (IX && (key[t - 1] >> 32) == (key[t] >> 32)) continue;
                    key[t] = key[t - 1] < key[t] ? key[t - 1] : key[t];
                    hit[t - 1] = false;
                }
            }
        }
        // the next chunk to render (its box test runs before the bound reads,
        // which would otherwise have to complete first)
        const uint64_t vn = visible(v + gridDim.x);
        // pixel bounds of the survivors (a lane without a survivor reads the
        // wave's shared pixel, so its request merges), then the atomics
        uint32_t pb[kCullPts];
#pragma unroll
        for (int t = 0; t < kCullPts; ++t) pb[t] = tg.pixb[hit[t] ? pix[t] : spread];
        // the next chunk's points are loaded while the bounds come back (both
        // load sequences have a fixed length, so the wait for the bounds
        // leaves the six point loads in flight)
        fetch(vn < sel.nv ? vn : v);
#pragma unroll
        for (int t = 0; t < kCullPts; ++t) hit[t] = hit[t] && (uint32_t)(key[t] >> 32) <= pb[t];
        if (IX) {
#pragma unroll
            for (int t = 0; t < kCullPts; ++t)
                if (hit[t]) key[t] = (key[t] & 0xFFFFFFFF00000000ull) | lay.ix[(uint32_t)key[t]];
        }
#pragma unroll
        for (int t = 0; t < kCullPts; ++t)
            if (hit[t])
                __hip_atomic_fetch_min(key_at<OFF32>(keys, pix[t]), key[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v = vn;
    }
    render_tail(X, Y, Z, n, P, keys, sel, lay.ix, lay.glyph);
}

// First level of a hinted bounded render: every pixel of an earlier key
// buffer (the previous frame of a viewer loop) names the point that won it;
// those points, rendered first, leave depths near the front of this frame
// too, so the bounds taken after the sample are tighter and fewer points of
// the later levels reach the atomics.  Any hint gives the exact result: the
// hinted points are points of this cloud and merge like any other (an empty
// key or an index >= n is skipped).
__global__ __launch_bounds__(kBlock) void k_hint_render(const unsigned long long *__restrict__ hint, uint32_t npx,
                                                        const float *__restrict__ X, const float *__restrict__ Y,
                                                        const float *__restrict__ Z, uint64_t n, Proj P,
                                                        unsigned long long *__restrict__ keys,
                                                        const uint8_t *__restrict__ glyph)
{
    const uint32_t q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= npx) return;
    const unsigned long long h = hint[q];
    const uint32_t i = (uint32_t)h;
    if (h == NARVIS_KEY_EMPTY || (uint64_t)i >= n) return;
    uint32_t pix;
    float w;
    if (project(P, X[i], Y[i], Z[i], pix, w)) merge<NARVIS_RENDER_EARLYZ>(keys, pix, w, i, glyph_rank(glyph, i));
}

// Depth bounds after the first levels: per pixel its depth bits, per screen
// tile the high 16 bits of the largest of those over the tile's pixels (an
// empty pixel counts as depth bits 0xFFFFFFFF, tile bound 0xFFFF, which culls
// nothing).  A point with bits(w) > the pixel bound, or (bits(w) >> 16) > the
// tile bound, is deeper than the key of its pixel.  One workgroup per tile.
__global__ __launch_bounds__(kBlock) void k_tile_bounds(const unsigned long long *__restrict__ keys, int32_t W,
                                                        int32_t H, uint32_t shift, uint32_t tiles_x,
                                                        uint16_t *__restrict__ bounds, uint32_t *__restrict__ pixb)
{
    __shared__ uint32_t red[kBlock / 64];
    const uint32_t t = blockIdx.x;
    const uint32_t x0 = (t % tiles_x) << shift, y0 = (t / tiles_x) << shift;
    const uint32_t side = 1u << shift;
    uint32_t m = 0;
    for (uint32_t i = threadIdx.x; i < side * side; i += kBlock) {
        const uint32_t x = x0 + (i & (side - 1)), y = y0 + (i >> shift);
        if (x < (uint32_t)W && y < (uint32_t)H) {
            const size_t p = (size_t)y * (uint32_t)W + x;
            const uint32_t d = (uint32_t)(keys[p] >> 32);
            pixb[p] = d;
            m = max(m, d);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kBlock / 64; ++k) m = max(m, red[k]);
        bounds[t] = (uint16_t)(m >> 16);
    }
}

template <int VARIANT>
__global__ __launch_bounds__(kBlock) void k_render_scalar(const float *__restrict__ X, const float *__restrict__ Y,
                                                           const float *__restrict__ Z, uint64_t n, Proj P,
                                                           unsigned long long *__restrict__ keys, ChunkOrder order,
                                                           const uint8_t *__restrict__ glyph)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = logical_block(order) * kBlock + threadIdx.x; i < n; i += stride) {
        uint32_t pix;
        float w;
        if (project(P, X[i], Y[i], Z[i], pix, w)) merge<VARIANT>(keys, pix, w, (uint32_t)i, glyph_rank(glyph, i));
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_empty(unsigned long long *__restrict__ keys, int64_t npx)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < npx) keys[i] = NARVIS_KEY_EMPTY;
}

__device__ __forceinline__ float half_to_float(uint32_t h)
{
    const uint32_t sign = (h & 0x8000u) << 16;
    const uint32_t e = (h >> 10) & 0x1Fu;
    const uint32_t m = h & 0x3FFu;
    if (e == 0) {
        // zero or subnormal: m * 2^-24 is exact in fp32
        const float v = (float)m * 5.9604644775390625e-8f;
        return __uint_as_float(__float_as_uint(v) | sign);
    }
    if (e == 31) return __uint_as_float(sign | 0x7F800000u | (m ? (0x00400000u | (m << 13)) : 0u));
    return __uint_as_float(sign | ((e + 112u) << 23) | (m << 13));
}

__device__ __forceinline__ float load_attr(const AttrArg &a, uint32_t i)
{
    const unsigned char *p = a.p + (size_t)i * (size_t)a.stride;
    switch (a.dtype) {
    case NARVIS_U8: return (float)(*p);
    case NARVIS_U16: return (float)(*reinterpret_cast<const uint16_t *>(p));
    case NARVIS_F16: return half_to_float(*reinterpret_cast<const uint16_t *>(p));
    default: return *reinterpret_cast<const float *>(p);
    }
}

struct ResolveArgs {
    const unsigned long long *keys;
    const float *X, *Y, *Z;
    float *depth, *attr, *rgb, *vel, *radius;
    const float *lut;
    int32_t lut_attr, vel_attr, rgb_mode, radius_attr;
    float lut_min, lut_inv, focal;
    int64_t npx;
    uint64_t n;
};

__global__ __launch_bounds__(kBlock) void k_resolve(ResolveArgs R, AttrPack A, Proj P)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= R.npx) return;
    const unsigned long long k = R.keys[p];
    // an index outside [0, n) can only come from a buffer this frame did not
    // render; it resolves as empty instead of reading out of bounds
    const bool empty = (k == NARVIS_KEY_EMPTY) || (uint64_t)(uint32_t)k >= R.n;
    const uint32_t i = (uint32_t)k;
    const float depth = __uint_as_float((uint32_t)(k >> 32) & ~kNotGlyph);
    if (R.depth) R.depth[p] = empty ? 0.0f : depth;
    // projected splat radius: the winner's world radius at its depth, in pixels
    if (R.radius) {
        float rp = 0.0f;
        if (!empty) {
            rp = load_attr(A.a[R.radius_attr], i) * R.focal;
            rp = rp / depth;
        }
        R.radius[p] = rp;
    }
    if (R.attr) {
        for (int c = 0; c < A.count; ++c) R.attr[c * R.npx + p] = empty ? 0.0f : load_attr(A.a[c], i);
    }
    if (R.rgb) {
        float r = 0.0f, g = 0.0f, b = 0.0f;
        if (!empty && R.rgb_mode == NARVIS_COLOR_RGB8) {
            const float s = 1.0f / 255.0f;
            r = load_attr(A.a[R.lut_attr], i) * s;
            g = load_attr(A.a[R.lut_attr + 1], i) * s;
            b = load_attr(A.a[R.lut_attr + 2], i) * s;
        } else if (!empty) {
            float t = load_attr(A.a[R.lut_attr], i) - R.lut_min;
            t = t * R.lut_inv;
            t = t * 256.0f;
            int q;
            if (!(t > 0.0f)) q = 0;
            else if (t >= 255.0f) q = 255;
            else q = (int)t;
            r = R.lut[q * 3 + 0];
            g = R.lut[q * 3 + 1];
            b = R.lut[q * 3 + 2];
        }
        R.rgb[p] = r;
        R.rgb[R.npx + p] = g;
        R.rgb[2 * R.npx + p] = b;
    }
    if (R.vel) {
        float o0 = 0.0f, o1 = 0.0f, o2 = 0.0f, o3 = 0.0f;
        if (!empty) {
            const float x = R.X[i], y = R.Y[i], z = R.Z[i];
            float cx = P.m00 * x; cx = cx + P.m01 * y; cx = cx + P.m02 * z; cx = cx + P.m03;
            float cy = P.m10 * x; cy = cy + P.m11 * y; cy = cy + P.m12 * z; cy = cy + P.m13;
            float w = P.m30 * x; w = w + P.m31 * y; w = w + P.m32 * z; w = w + P.m33;
            const float vx = load_attr(A.a[R.vel_attr], i);
            const float vy = load_attr(A.a[R.vel_attr + 1], i);
            const float vz = load_attr(A.a[R.vel_attr + 2], i);
            float dcx = P.m00 * vx; dcx = dcx + P.m01 * vy; dcx = dcx + P.m02 * vz;
            float dcy = P.m10 * vx; dcy = dcy + P.m11 * vy; dcy = dcy + P.m12 * vz;
            float dw = P.m30 * vx; dw = dw + P.m31 * vy; dw = dw + P.m32 * vz;
            const float ww = w * w;
            const float nxv = dcx * w - cx * dw;
            const float nyv = dcy * w - cy * dw;
            o0 = nxv / ww;
            o1 = nyv / ww;
            float m2 = o0 * o0;
            m2 = m2 + o1 * o1;
            o3 = sqrtf(m2);
            o2 = atan2f(o1, o0) / 3.14159265358979323846f;
        }
        R.vel[p] = o0;
        R.vel[R.npx + p] = o1;
        R.vel[2 * R.npx + p] = o2;
        R.vel[3 * R.npx + p] = o3;
    }
}

}  // namespace

Proj make_proj(const float vp[16], float near_f, float far_f, int32_t W, int32_t H)
{
    Proj P;
    P.m00 = vp[0]; P.m01 = vp[1]; P.m02 = vp[2]; P.m03 = vp[3];
    P.m10 = vp[4]; P.m11 = vp[5]; P.m12 = vp[6]; P.m13 = vp[7];
    P.m30 = vp[12]; P.m31 = vp[13]; P.m32 = vp[14]; P.m33 = vp[15];
    P.near_f = near_f;
    P.far_f = far_f;
    P.Wf = (float)W;
    P.Hf = (float)H;
    P.W = W;
    P.H = H;
    return P;
}

// Scratch of the allocation-free whole-frame call: the bounded render's tile
// and pixel bounds for images of up to NARVIS_STATIC_MAX_PIXELS pixels.  Each
// device holds its own copy from the library's load until the process ends.
// Host code never passes this name to a kernel (on the host it is only a
// stand-in): static_scratch() resolves the device address once per device.
static __device__ __align__(256) unsigned char scratch[NARVIS_STATIC_SCRATCH_BYTES];

hipError_t static_scratch(void **ptr)
{
    static std::mutex mu;
    static std::vector<void *> addr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_clear(uint64_t *keys, int64_t npx, hipStream_t s)
{
    const int64_t blocks = (npx + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_fill_empty, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                       reinterpret_cast<unsigned long long *>(keys), npx);
    return hipGetLastError();
}

namespace {

uint32_t gcd_u32(uint32_t a, uint32_t b)
{
    while (b) {
        const uint32_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// The integer nearest per / golden ratio that is coprime with per.
uint32_t coprime_stride(uint32_t per)
{
    if (per <= 2) return 1;
    uint32_t s = (uint32_t)((double)per * 0.6180339887498949 + 0.5);
    if (s < 1) s = 1;
    while (gcd_u32(s, per) != 1) ++s;
    return s % per ? s % per : 1;
}

}  // namespace

// Levels of the bounded render: the chunks that are multiples of 8 first
// (single-pass kernel), then all the others, culled against the tile bounds
// the first level left (more levels are supported: each later level is
// culled against the bounds of everything before it).
constexpr uint32_t kLevels[] = {8, 1};
constexpr int kNumLevels = sizeof(kLevels) / sizeof(kLevels[0]);

hipError_t launch_render(const float *x, const float *y, const float *z, uint64_t n, const Proj &P,
                         uint64_t *keys, int32_t variant, int32_t grid_blocks, uint16_t *bounds, const uint64_t *hint,
                         hipStream_t s, const LayoutArgs &lay)
{
    if (n == 0) return hipSuccess;
    const DeviceInfo dev = device_info();
    const uint32_t xcds = (uint32_t)dev.xcds;
    const bool vec = ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y) |
                       reinterpret_cast<uintptr_t>(z)) & 15u) == 0;
    const uint64_t per_block = vec ? (uint64_t)kBlock * kQuadsPerThread * 4 : (uint64_t)kBlock;
    // grid size as a multiple of the XCD count (keeps the block renumbering a
    // bijection), at most 2^22 workgroups (grid-stride loops cover the rest)
    auto grid_of = [&](uint64_t want) {
        uint64_t blocks = want < 1 ? 1 : want;
        if (blocks > (1u << 22)) blocks = 1u << 22;
        return (blocks + xcds - 1) / xcds * xcds;
    };
    auto order_of = [&](uint64_t blocks) {
        ChunkOrder order;
        order.xcds = xcds;
        order.per = (uint32_t)(blocks / xcds);
        order.stride = coprime_stride(order.per);
        return order;
    };
    uint64_t blocks = grid_of(grid_blocks > 0 ? (uint64_t)grid_blocks : (n + per_block - 1) / per_block);
    ChunkOrder order = order_of(blocks);
    auto *k = reinterpret_cast<unsigned long long *>(keys);
    if (variant == NARVIS_RENDER_AUTO) variant = vec ? NARVIS_RENDER_LDS : NARVIS_RENDER_EARLYZ;
    if (variant == NARVIS_RENDER_LDS && !vec) variant = NARVIS_RENDER_EARLYZ;
    // a layout is rendered by the LDS and cull kernels only (16-byte aligned
    // arrays; the C ABI checks this before any launch), and never with a
    // glyph mask; the LDS and cull kernels read the mask four bytes at a time
    if (lay.ix && (lay.glyph || !(vec && variant == NARVIS_RENDER_LDS && !(reinterpret_cast<uintptr_t>(lay.ix) & 15u))))
        return hipErrorInvalidValue;
    if (lay.glyph && vec && variant == NARVIS_RENDER_LDS && (reinterpret_cast<uintptr_t>(lay.glyph) & 3u))
        variant = NARVIS_RENDER_EARLYZ;
    if (vec && variant == NARVIS_RENDER_LDS) {
        // kept depths lie in [near_f, far_f]: the reciprocal path needs them in
        // the range where rcp_rn is exact
        const bool rcp = P.near_f >= 0x1p-124f && P.far_f < 0x1p125f;
        constexpr uint64_t kChunkQuads = (uint64_t)kBlock * kQuadsPerThread;
        const uint64_t nchunks = ((n >> 2) + kChunkQuads - 1) / kChunkQuads;
        const bool ix = lay.ix != nullptr;
        const int mode = ix ? 1 : (lay.glyph ? 2 : 0);
        auto lds_on = [&](const float *px, const float *py, const float *pz, uint64_t pn, const ChunkSel &sel,
                          uint64_t nblocks, const LayoutArgs &la) {
            const ChunkOrder o = order_of(nblocks);
            auto kern = rcp ? (mode == 1 ? k_render_lds<true, 1> : mode == 2 ? k_render_lds<true, 2> : k_render_lds<true, 0>)
                            : (mode == 1 ? k_render_lds<false, 1>
                                         : mode == 2 ? k_render_lds<false, 2> : k_render_lds<false, 0>);
            hipLaunchKernelGGL(kern, dim3((unsigned)nblocks), dim3(kBlock), 0, s, px, py, pz, pn, P, k, o, sel, la);
        };
        auto lds = [&](const ChunkSel &sel, uint64_t nblocks) { lds_on(x, y, z, n, sel, nblocks, lay); };
        // bounded render for at least two chunks (24-bit pixel arithmetic)
        if (bounds && n >= 4096 && P.W < (1 << 24) && P.H < (1 << 24)) {
            uint32_t *pixb = reinterpret_cast<uint32_t *>(bounds + kMaxTiles);
            TileGrid tg{bounds, pixb, 3u, 0u, 0u};
            while (true) {
                tg.tiles_x = ((uint32_t)P.W + (1u << tg.shift) - 1) >> tg.shift;
                tg.ntiles = tg.tiles_x * (((uint32_t)P.H + (1u << tg.shift) - 1) >> tg.shift);
                if (tg.ntiles <= (uint32_t)kMaxTiles) break;
                ++tg.shift;
            }
            auto ceil_div = [](uint64_t a, uint64_t b) { return (a + b - 1) / b; };
            if (hint && !ix) {
                const uint32_t npx = (uint32_t)P.W * (uint32_t)P.H;
                hipLaunchKernelGGL(k_hint_render, dim3((npx + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                                   reinterpret_cast<const unsigned long long *>(hint), npx, x, y, z, n, P, k,
                                   lay.glyph);
            }
            auto bounds_of_keys = [&]() {
                hipLaunchKernelGGL(k_tile_bounds, dim3(tg.ntiles), dim3(kBlock), 0, s, k, P.W, P.H, tg.shift,
                                   tg.tiles_x, bounds, pixb);
            };
            auto cull = [&](const ChunkSel &sel) {
                // a resident grid: each workgroup loads the bounds once
                const uint64_t resident = (uint64_t)dev.cus * (2048 / kCullBlock);
                const uint64_t nb = grid_of(grid_blocks > 0 ? (uint64_t)grid_blocks
                                                            : (sel.nv < resident ? sel.nv : resident));
                const ChunkOrder o = order_of(nb);
                const bool off32 = (uint64_t)P.W * (uint64_t)P.H < (1ull << 29);
                auto pick = [&](auto m) {
                    constexpr int M = decltype(m)::value;
                    return rcp ? (off32 ? k_render_cull<true, true, M> : k_render_cull<true, false, M>)
                               : (off32 ? k_render_cull<false, true, M> : k_render_cull<false, false, M>);
                };
                auto kern = mode == 1 ? pick(std::integral_constant<int, 1>{})
                                      : mode == 2 ? pick(std::integral_constant<int, 2>{})
                                                  : pick(std::integral_constant<int, 0>{});
                hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(kCullBlock), 0, s, x, y, z, n, P, k, o, sel, tg,
                                   lay);
            };
            if (ix && lay.sx) {
                // the layout's depth sample (every 8th point, spread over the
                // whole cloud) first, then every batch against its bounds (the
                // sampled points merge again, which changes nothing)
                const uint64_t ns_chunks = ((lay.ns >> 2) + kChunkQuads - 1) / kChunkQuads;
                LayoutArgs ls = lay;
                ls.ix = lay.six;
                ls.box = lay.sbox;
                const ChunkSel s0{1u, 0u, ns_chunks, 1u};
                lds_on(lay.sx, lay.sy, lay.sz, lay.ns, s0, grid_of(ns_chunks), ls);
                bounds_of_keys();
                cull(ChunkSel{1u, 0u, nchunks, 1u});
            } else {
                for (int lv = 0; lv < kNumLevels; ++lv) {
                    ChunkSel sel;
                    sel.mul = kLevels[lv];
                    sel.excl = lv ? kLevels[lv - 1] / kLevels[lv] : 0u;
                    sel.nv = ceil_div(nchunks, sel.mul) - (lv ? ceil_div(nchunks, kLevels[lv - 1]) : 0u);
                    sel.tail = lv == 0;
                    if (lv == 0) {
                        lds(sel, grid_of(sel.nv));
                    } else {
                        bounds_of_keys();
                        if (sel.nv == 0) continue;
                        cull(sel);
                    }
                }
            }
        } else {
            ChunkSel all{1u, 0u, nchunks, 1u};
            lds(all, blocks);
        }
    } else if (vec) {
        if (variant == NARVIS_RENDER_GLOBAL)
            hipLaunchKernelGGL(k_render_vec<NARVIS_RENDER_GLOBAL>, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                               x, y, z, n, P, k, order, lay.glyph);
        else
            hipLaunchKernelGGL(k_render_vec<NARVIS_RENDER_EARLYZ>, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                               x, y, z, n, P, k, order, lay.glyph);
    } else {
        if (variant == NARVIS_RENDER_GLOBAL)
            hipLaunchKernelGGL(k_render_scalar<NARVIS_RENDER_GLOBAL>, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                               x, y, z, n, P, k, order, lay.glyph);
        else
            hipLaunchKernelGGL(k_render_scalar<NARVIS_RENDER_EARLYZ>, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                               x, y, z, n, P, k, order, lay.glyph);
    }
    return hipGetLastError();
}

hipError_t launch_resolve(const float *x, const float *y, const float *z, uint64_t n, const Proj &P,
                          const AttrPack &attrs, const narvis_gbuffer &g, hipStream_t s)
{
    ResolveArgs R;
    R.n = n;
    R.keys = reinterpret_cast<const unsigned long long *>(g.keys);
    R.X = x;
    R.Y = y;
    R.Z = z;
    R.depth = g.depth;
    R.attr = g.attr;
    R.rgb = g.rgb;
    R.vel = g.vel2d;
    R.radius = g.radius;
    R.radius_attr = g.radius_attr;
    R.focal = g.radius_focal_px;
    R.lut = g.lut;
    R.lut_attr = g.lut_attr;
    R.vel_attr = g.vel_attr;
    R.rgb_mode = g.rgb_mode;
    R.lut_min = g.lut_min;
    R.lut_inv = g.lut_inv_range;
    R.npx = (int64_t)P.W * P.H;
    const int64_t blocks = (R.npx + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_resolve, dim3((unsigned)blocks), dim3(kBlock), 0, s, R, attrs, P);
    return hipGetLastError();
}

}  // namespace narvis

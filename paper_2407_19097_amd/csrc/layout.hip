// Spatial layout of a point cloud for the batch-culled render.
//
// Compute rasterization, which the multi-attribute rasterizer extends
// (Sec. 3.2), keeps the points sorted along a Morton (Z-order) curve in
// batches (Sec. 4.3 names its Morton-ordered data): a batch is then a compact
// piece of space, and one bounding box per batch lets the render skip whole
// batches outside the view volume or behind what is already drawn.  Built once
// per point cloud:
//   bbox    -- the box of the finite points (exact min/max, order-independent);
//   codes   -- per point a 30-bit Morton code of its cell in a 1024^3 grid over
//              that box (fp32 arithmetic, each operation rounded, no FMA), a
//              point with a non-finite coordinate gets 2^30;
//   sort    -- stable radix sort of (code, original index);
//   gather  -- the coordinates in sorted order and the original indices;
//   boxes   -- per batch of NARVIS_LAYOUT_BATCH sorted points the box of its
//              finite points (+inf/-inf when none).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

#pragma clang fp contract(off)

namespace narvis {

namespace {

constexpr int kT = 256;

// fp32 -> uint32 preserving order (-0 below +0; NaNs are never passed)
__device__ __forceinline__ uint32_t ordered(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float unordered(uint32_t o)
{
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

__device__ __forceinline__ bool finite3(float x, float y, float z)
{
    return __builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z);
}

__global__ __launch_bounds__(kT) void k_layout_init(uint32_t *bb, uint32_t *count, uint32_t n)
{
    if (threadIdx.x < 3) bb[threadIdx.x] = 0xFFFFFFFFu;
    else if (threadIdx.x < 6) bb[threadIdx.x] = 0u;
    else if (threadIdx.x == 6) *count = n;
}

// bb[0..2]: ordered minima of x, y, z; bb[3..5]: ordered maxima
__global__ __launch_bounds__(kT) void k_layout_bbox(const float *__restrict__ X, const float *__restrict__ Y,
                                                   const float *__restrict__ Z, uint64_t n, uint32_t *bb)
{
    __shared__ uint32_t red[6][kT / 64];
    uint32_t m[6] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0u, 0u, 0u};
    for (uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kT) {
        const float x = X[i], y = Y[i], z = Z[i];
        if (!finite3(x, y, z)) continue;
        const uint32_t o[3] = {ordered(x), ordered(y), ordered(z)};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            m[a] = min(m[a], o[a]);
            m[3 + a] = max(m[3 + a], o[a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) {
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) {
            const uint32_t v = (uint32_t)__shfl_xor((int)m[a], d);
            m[a] = a < 3 ? min(m[a], v) : max(m[a], v);
        }
        if ((threadIdx.x & 63) == 0) red[a][threadIdx.x >> 6] = m[a];
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int a = threadIdx.x;
        uint32_t v = red[a][0];
        for (int w = 1; w < kT / 64; ++w) v = a < 3 ? min(v, red[a][w]) : max(v, red[a][w]);
        if (a < 3) atomicMin(bb + a, v);
        else atomicMax(bb + a, v);
    }
}

// bit k of v (k < 10) to bit 3k
__device__ __forceinline__ uint32_t spread3(uint32_t v)
{
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < 10; ++k) r |= ((v >> k) & 1u) << (3 * k);
    return r;
}

__device__ __forceinline__ uint32_t cell(float a, float lo, float scale)
{
    float t = a - lo;
    t = t * scale;
    if (!(t > 0.0f)) return 0u;
    if (t >= 1023.0f) return 1023u;
    return (uint32_t)t;
}

__global__ __launch_bounds__(kT) void k_layout_codes(const float *__restrict__ X, const float *__restrict__ Y,
                                                    const float *__restrict__ Z, uint64_t n,
                                                    const uint32_t *__restrict__ bb, uint32_t *__restrict__ keys,
                                                    uint32_t *__restrict__ vals)
{
    const uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const float x = X[i], y = Y[i], z = Z[i];
    uint32_t code = 1u << 30;
    if (finite3(x, y, z)) {
        float lo[3], sc[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = unordered(bb[a]);
            const float ext = unordered(bb[3 + a]) - lo[a];
            sc[a] = ext > 0.0f ? 1024.0f / ext : 0.0f;
        }
        code = spread3(cell(x, lo[0], sc[0])) | (spread3(cell(y, lo[1], sc[1])) << 1) |
               (spread3(cell(z, lo[2], sc[2])) << 2);
    }
    keys[i] = code;
    vals[i] = (uint32_t)i;
}

// x, y, z of point i side by side at xyz[3 i], so that the gather below takes
// one cache line per point instead of three
__global__ __launch_bounds__(kT) void k_layout_interleave(const float *__restrict__ X, const float *__restrict__ Y,
                                                         const float *__restrict__ Z, uint64_t n,
                                                         float *__restrict__ xyz)
{
    const uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    xyz[3 * i] = X[i];
    xyz[3 * i + 1] = Y[i];
    xyz[3 * i + 2] = Z[i];
}

// ... and, when sx is given, the depth sample (every 8th point of the
// layout order) written on the way
__global__ __launch_bounds__(kT) void k_layout_gather_xyz(const uint32_t *__restrict__ order,
                                                         const float *__restrict__ xyz, uint64_t n,
                                                         float *__restrict__ xs, float *__restrict__ ys,
                                                         float *__restrict__ zs, uint32_t *__restrict__ ix,
                                                         float *__restrict__ sx, float *__restrict__ sy,
                                                         float *__restrict__ sz, uint32_t *__restrict__ six)
{
    const uint64_t j = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (j >= n) return;
    const uint32_t i = order[j];
    const bool ok = (uint64_t)i < n;  // always true for a permutation
    const float *p = xyz + 3 * (uint64_t)(ok ? i : 0u);
    const float x = ok ? p[0] : __builtin_nanf(""), y = ok ? p[1] : __builtin_nanf(""),
                z = ok ? p[2] : __builtin_nanf("");
    xs[j] = x;
    ys[j] = y;
    zs[j] = z;
    ix[j] = i;
    if (sx && (j & 7) == 0) {
        sx[j >> 3] = x;
        sy[j >> 3] = y;
        sz[j >> 3] = z;
        six[j >> 3] = i;
    }
}

__global__ __launch_bounds__(kT) void k_layout_gather(const uint32_t *__restrict__ order, const float *__restrict__ X,
                                                     const float *__restrict__ Y, const float *__restrict__ Z,
                                                     uint64_t n, float *__restrict__ xs, float *__restrict__ ys,
                                                     float *__restrict__ zs, uint32_t *__restrict__ ix)
{
    const uint64_t j = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (j >= n) return;
    const uint32_t i = order[j];
    const bool ok = (uint64_t)i < n;  // always true for a permutation
    xs[j] = ok ? X[i] : __builtin_nanf("");
    ys[j] = ok ? Y[i] : __builtin_nanf("");
    zs[j] = ok ? Z[i] : __builtin_nanf("");
    ix[j] = i;
}

// the depth sample: every 8th point of the layout order
__global__ __launch_bounds__(kT) void k_layout_sample(const float *__restrict__ xs, const float *__restrict__ ys,
                                                     const float *__restrict__ zs, const uint32_t *__restrict__ ix,
                                                     uint64_t ns, float *__restrict__ sx, float *__restrict__ sy,
                                                     float *__restrict__ sz, uint32_t *__restrict__ six)
{
    const uint64_t j = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (j >= ns) return;
    sx[j] = xs[8 * j];
    sy[j] = ys[8 * j];
    sz[j] = zs[8 * j];
    six[j] = ix[8 * j];
}

// one workgroup per batch: box of its finite points
__global__ __launch_bounds__(kT) void k_layout_boxes(const float *__restrict__ xs, const float *__restrict__ ys,
                                                    const float *__restrict__ zs, uint64_t n,
                                                    float4 *__restrict__ box)
{
    __shared__ float red[6][kT / 64];
    const uint64_t b = blockIdx.x;
    const uint64_t j0 = b * NARVIS_LAYOUT_BATCH;
    const uint64_t j1 = min(n, j0 + NARVIS_LAYOUT_BATCH);
    float m[6] = {__builtin_inff(), __builtin_inff(), __builtin_inff(), -__builtin_inff(), -__builtin_inff(),
                  -__builtin_inff()};
    for (uint64_t j = j0 + threadIdx.x; j < j1; j += kT) {
        const float x = xs[j], y = ys[j], z = zs[j];
        if (!finite3(x, y, z)) continue;
        m[0] = fminf(m[0], x);
        m[1] = fminf(m[1], y);
        m[2] = fminf(m[2], z);
        m[3] = fmaxf(m[3], x);
        m[4] = fmaxf(m[4], y);
        m[5] = fmaxf(m[5], z);
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) {
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) {
            const float v = __shfl_xor(m[a], d);
            m[a] = a < 3 ? fminf(m[a], v) : fmaxf(m[a], v);
        }
        if ((threadIdx.x & 63) == 0) red[a][threadIdx.x >> 6] = m[a];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float r[6];
        for (int a = 0; a < 6; ++a) {
            r[a] = red[a][0];
            for (int w = 1; w < kT / 64; ++w) r[a] = a < 3 ? fminf(r[a], red[a][w]) : fmaxf(r[a], red[a][w]);
        }
        box[2 * b] = make_float4(r[0], r[1], r[2], 0.0f);
        box[2 * b + 1] = make_float4(r[3], r[4], r[5], 0.0f);
    }
}

// ---------------------------------------------------------------------------
// World splat radius (Sec. 4.2): mean distance to the four nearest
// neighbours, on a hashed uniform grid.
//   cells  -- cube cells of edge c over the box of the finite points, chosen
//             on the host so that a point shares its cell with a few others
//             (mean occupancy measured with the hash table, c halved or
//             doubled until it lies in [1.5, 12]);
//   sort   -- (cell id, index) pairs sorted by cell (stable radix sort);
//   hash   -- cell id -> first position of the cell in the sorted pairs;
//   query  -- per point, rings of cells r = 1, 2, ... around its own; the
//             four smallest distances so far are final once the fourth is
//             below the distance any point outside the searched block can
//             have ((r - 1/2) c, less a relative 2^-20 for the rounding of
//             the cell coordinates and distances);
//   rest   -- a point not settled after four rings scans every point.
// ---------------------------------------------------------------------------

constexpr uint64_t kHashEmpty = 0xFFFFFFFFFFFFFFFFull;
constexpr uint64_t kNoCell = 0xFFFFFFFFFFFFFFFEull;  // sort key of a point with a non-finite coordinate
constexpr int kRings = 4;

struct Grid {
    float lo[3];
    float inv;          // cells per unit length, fp32(1 / cell)
    float cell;         // cell edge
    uint32_t g[3];      // cells per axis
    uint64_t hmask;     // hash slots - 1 (a power of two)
};

__device__ __forceinline__ uint32_t grid_coord(float a, float lo, float inv, uint32_t g)
{
    float t = a - lo;
    t = t * inv;
    if (!(t > 0.0f)) return 0u;
    if (!(t < (float)g)) return g - 1;
    return (uint32_t)t;
}

__device__ __forceinline__ uint64_t hash_slot(uint64_t k, uint64_t mask)
{
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return k & mask;
}

__global__ __launch_bounds__(kT) void k_hash_clear(unsigned long long *hkey, uint32_t *hval, uint64_t slots)
{
    const uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (i < slots) {
        hkey[i] = kHashEmpty;
        hval[i] = 0u;
    }
}

// insert (or find) key; returns its slot.  Linear probing; the table is at
// least twice the number of distinct keys, so a free slot always exists.
__device__ __forceinline__ uint64_t hash_insert(unsigned long long *hkey, uint64_t mask, uint64_t key)
{
    uint64_t s = hash_slot(key, mask);
    while (true) {
        const unsigned long long prev = atomicCAS(hkey + s, kHashEmpty, (unsigned long long)key);
        if (prev == kHashEmpty || prev == key) return s;
        s = (s + 1) & mask;
    }
}

__device__ __forceinline__ bool hash_find(const unsigned long long *hkey, uint64_t mask, uint64_t key, uint64_t &slot)
{
    uint64_t s = hash_slot(key, mask);
    while (true) {
        const unsigned long long k = hkey[s];
        if (k == key) {
            slot = s;
            return true;
        }
        if (k == kHashEmpty) return false;
        s = (s + 1) & mask;
    }
}

__device__ __forceinline__ uint64_t point_cell(const Grid &G, float x, float y, float z)
{
    if (!finite3(x, y, z)) return kNoCell;
    const uint32_t qx = grid_coord(x, G.lo[0], G.inv, G.g[0]);
    const uint32_t qy = grid_coord(y, G.lo[1], G.inv, G.g[1]);
    const uint32_t qz = grid_coord(z, G.lo[2], G.inv, G.g[2]);
    return ((uint64_t)qz * G.g[1] + qy) * G.g[0] + qx;
}

// number of points whose three coordinates are finite
__global__ __launch_bounds__(kT) void k_knn_finite(const float *__restrict__ X, const float *__restrict__ Y,
                                                   const float *__restrict__ Z, uint64_t n, unsigned long long *sum)
{
    unsigned long long c = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kT)
        c += finite3(X[i], Y[i], Z[i]) ? 1u : 0u;
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(sum, c);
}

// occupancy probe: count the points of every cell
__global__ __launch_bounds__(kT) void k_knn_count(const float *__restrict__ X, const float *__restrict__ Y,
                                                  const float *__restrict__ Z, uint64_t n, Grid G,
                                                  unsigned long long *hkey, uint32_t *hval)
{
    const uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const uint64_t c = point_cell(G, X[i], Y[i], Z[i]);
    if (c == kNoCell) return;
    atomicAdd(hval + hash_insert(hkey, G.hmask, c), 1u);
}

// sum over cells of count^2 (= sum over points of the points sharing their cell)
__global__ __launch_bounds__(kT) void k_knn_occupancy(const uint32_t *hval, uint64_t slots,
                                                      unsigned long long *sum)
{
    unsigned long long s = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x; i < slots; i += (uint64_t)gridDim.x * kT) {
        const unsigned long long c = hval[i];
        s += c * c;
    }
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(sum, s);
}

__global__ __launch_bounds__(kT) void k_knn_keys(const float *__restrict__ X, const float *__restrict__ Y,
                                                 const float *__restrict__ Z, uint64_t n, Grid G,
                                                 unsigned long long *keys, uint32_t *vals)
{
    const uint64_t i = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    keys[i] = point_cell(G, X[i], Y[i], Z[i]);
    vals[i] = (uint32_t)i;
}

// first position of every cell in the sorted pairs
__global__ __launch_bounds__(kT) void k_knn_starts(const unsigned long long *keys, uint64_t n, Grid G,
                                                   unsigned long long *hkey, uint32_t *hval)
{
    const uint64_t p = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (p >= n) return;
    const uint64_t k = keys[p];
    if (k == kNoCell) return;
    if (p == 0 || keys[p - 1] != k) hval[hash_insert(hkey, G.hmask, k)] = (uint32_t)p;
}

// the four smallest values seen so far, ascending (+inf when fewer)
struct Top4 {
    float d[4];
    __device__ __forceinline__ void init() { d[0] = d[1] = d[2] = d[3] = __builtin_inff(); }
    __device__ __forceinline__ void add(float v)
    {
        if (!(v < d[3])) return;
        d[3] = v;
        if (d[3] < d[2]) { const float t = d[2]; d[2] = d[3]; d[3] = t; }
        if (d[2] < d[1]) { const float t = d[1]; d[1] = d[2]; d[2] = t; }
        if (d[1] < d[0]) { const float t = d[0]; d[0] = d[1]; d[1] = t; }
    }
};

__device__ __forceinline__ float dist(float x0, float y0, float z0, float x1, float y1, float z1)
{
    const float dx = x1 - x0, dy = y1 - y0, dz = z1 - z0;
    float d2 = dx * dx;
    d2 = d2 + dy * dy;
    d2 = d2 + dz * dz;
    return sqrtf(d2);
}

// r = (((d1 + d2) + d3) + d4) * 0.25, or the mean of the m < 4 available
__device__ __forceinline__ float radius_of(const Top4 &t, uint64_t others)
{
    const int m = others < 4 ? (int)others : 4;
    if (m == 0) return 0.0f;
    float s = t.d[0];
    for (int k = 1; k < m; ++k) s = s + t.d[k];
    return m == 4 ? s * 0.25f : s / (float)m;
}

struct KnnArgs {
    const float *X, *Y, *Z;
    uint64_t n, finite;    // points, points with finite coordinates
    Grid G;
    const unsigned long long *keys;  // sorted cell ids
    const uint32_t *vals;            // original index of each sorted pair
    const unsigned long long *hkey;
    const uint32_t *hval;
    float *radius;
    uint32_t *unresolved;            // [0]: count, then the indices
    float settle;                    // (1 - 2^-20) * cell
};

// one thread per sorted position
__global__ __launch_bounds__(kT) void k_knn_query(KnnArgs A)
{
    const uint64_t p = (uint64_t)blockIdx.x * kT + threadIdx.x;
    if (p >= A.n) return;
    const uint32_t i = A.vals[p];
    const float x = A.X[i], y = A.Y[i], z = A.Z[i];
    if (A.keys[p] == kNoCell) {
        A.radius[i] = 0.0f;
        return;
    }
    const Grid &G = A.G;
    const int qx = (int)grid_coord(x, G.lo[0], G.inv, G.g[0]);
    const int qy = (int)grid_coord(y, G.lo[1], G.inv, G.g[1]);
    const int qz = (int)grid_coord(z, G.lo[2], G.inv, G.g[2]);
    Top4 t;
    t.init();
    const uint64_t others = A.finite - 1;
    for (int r = 0; r <= kRings; ++r) {
        for (int dz = -r; dz <= r; ++dz) {
            const int cz = qz + dz;
            if (cz < 0 || cz >= (int)G.g[2]) continue;
            for (int dy = -r; dy <= r; ++dy) {
                const int cy = qy + dy;
                if (cy < 0 || cy >= (int)G.g[1]) continue;
                for (int dx = -r; dx <= r; ++dx) {
                    if (max(max(abs(dx), abs(dy)), abs(dz)) != r) continue;  // the ring only
                    const int cx = qx + dx;
                    if (cx < 0 || cx >= (int)G.g[0]) continue;
                    const uint64_t id = ((uint64_t)cz * G.g[1] + cy) * G.g[0] + cx;
                    uint64_t slot;
                    if (!hash_find(A.hkey, G.hmask, id, slot)) continue;
                    for (uint64_t q = A.hval[slot]; q < A.n && A.keys[q] == id; ++q) {
                        const uint32_t j = A.vals[q];
                        if (j == i) continue;
                        t.add(dist(x, y, z, A.X[j], A.Y[j], A.Z[j]));
                    }
                }
            }
        }
        // every point outside the searched block is farther than (r + 1/2) cells
        // less the rounding slack: settled once the fourth distance is below
        if (r >= 1 && t.d[others < 4 ? (int)others - 1 : 3] < ((float)r - 0.5f) * A.settle) {
            A.radius[i] = radius_of(t, others);
            return;
        }
        if (others == 0) {
            A.radius[i] = 0.0f;
            return;
        }
    }
    const uint32_t slot = atomicAdd(A.unresolved, 1u);
    A.unresolved[1 + slot] = i;
}

// unresolved points: one workgroup each scans every point
__global__ __launch_bounds__(kT) void k_knn_brute(KnnArgs A)
{
    __shared__ float cand[kT * 4];
    const uint32_t count = A.unresolved[0];
    for (uint32_t u = blockIdx.x; u < count; u += gridDim.x) {
        const uint32_t i = A.unresolved[1 + u];
        const float x = A.X[i], y = A.Y[i], z = A.Z[i];
        Top4 t;
        t.init();
        for (uint64_t j = threadIdx.x; j < A.n; j += kT) {
            if (j == i) continue;
            const float a = A.X[j], b = A.Y[j], c = A.Z[j];
            if (!finite3(a, b, c)) continue;
            t.add(dist(x, y, z, a, b, c));
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) cand[threadIdx.x * 4 + k] = t.d[k];
        __syncthreads();
        if (threadIdx.x == 0) {
            Top4 all;
            all.init();
            for (int k = 0; k < kT * 4; ++k) all.add(cand[k]);
            A.radius[i] = radius_of(all, A.finite - 1);
        }
        __syncthreads();
    }
}

uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

}  // namespace

LayoutWorkspace layout_workspace(uint64_t n)
{
    LayoutWorkspace L{};
    uint64_t o = 0;
    L.off_bb = o; o = align256(o + 8 * 4);
    L.off_count = o; o = align256(o + 4);
    // va first: after the sort's four passes it holds the order, and ka, kb,
    // vb behind it form one free region of at least 12 n bytes for the
    // interleaved coordinates
    L.off_va = o; o = align256(o + n * 4);
    L.off_ka = o; o = align256(o + n * 4);
    L.off_kb = o; o = align256(o + n * 4);
    L.off_vb = o; o = align256(o + n * 4);
    L.off_hist = o; o = align256(o + radix_sort_hist_len(n) * 4);
    L.off_sums = o; o = align256(o + radix_sort_sums_len(n) * 4);
    L.bytes = o;
    return L;
}

hipError_t launch_layout(const float *x, const float *y, const float *z, uint64_t n, float *xs, float *ys, float *zs,
                         uint32_t *ix, float *box, float *sx, float *sy, float *sz, uint32_t *six, float *sbox,
                         void *ws, hipStream_t s)
{
    const LayoutWorkspace L = layout_workspace(n);
    char *base = static_cast<char *>(ws);
    auto *bb = reinterpret_cast<uint32_t *>(base + L.off_bb);
    auto *count = reinterpret_cast<uint32_t *>(base + L.off_count);
    auto *ka = reinterpret_cast<uint32_t *>(base + L.off_ka);
    auto *kb = reinterpret_cast<uint32_t *>(base + L.off_kb);
    auto *va = reinterpret_cast<uint32_t *>(base + L.off_va);
    auto *vb = reinterpret_cast<uint32_t *>(base + L.off_vb);
    auto *hist = reinterpret_cast<uint32_t *>(base + L.off_hist);
    auto *sums = reinterpret_cast<uint32_t *>(base + L.off_sums);
    hipLaunchKernelGGL(k_layout_init, dim3(1), dim3(kT), 0, s, bb, count, (uint32_t)n);
    if (n == 0) return hipGetLastError();
    const uint64_t blocks = (n + kT - 1) / kT;
    const uint64_t red_blocks = blocks < 4096 ? blocks : 4096;
    hipLaunchKernelGGL(k_layout_bbox, dim3((unsigned)red_blocks), dim3(kT), 0, s, x, y, z, n, bb);
    hipLaunchKernelGGL(k_layout_codes, dim3((unsigned)blocks), dim3(kT), 0, s, x, y, z, n, bb, ka, va);
    bool in_b = false;
    hipError_t e = launch_radix_sort32(ka, va, kb, vb, count, n, 31, hist, sums, s, &in_b);
    if (e != hipSuccess) return e;
    if (!in_b) {
        // the order is in va; ka, kb and vb are free
        auto *xyz = reinterpret_cast<float *>(ka);
        hipLaunchKernelGGL(k_layout_interleave, dim3((unsigned)blocks), dim3(kT), 0, s, x, y, z, n, xyz);
        hipLaunchKernelGGL(k_layout_gather_xyz, dim3((unsigned)blocks), dim3(kT), 0, s, va, xyz, n, xs, ys, zs, ix,
                           sx, sy, sz, six);
    } else {
        hipLaunchKernelGGL(k_layout_gather, dim3((unsigned)blocks), dim3(kT), 0, s, vb, x, y, z, n, xs, ys, zs, ix);
    }
    const uint64_t nb = (n + NARVIS_LAYOUT_BATCH - 1) / NARVIS_LAYOUT_BATCH;
    hipLaunchKernelGGL(k_layout_boxes, dim3((unsigned)nb), dim3(kT), 0, s, xs, ys, zs, n,
                       reinterpret_cast<float4 *>(box));
    if (sx) {
        const uint64_t ns = (n + 7) / 8;
        if (in_b)  // else written by the gather
            hipLaunchKernelGGL(k_layout_sample, dim3((unsigned)((ns + kT - 1) / kT)), dim3(kT), 0, s, xs, ys, zs, ix,
                               ns, sx, sy, sz, six);
        const uint64_t nsb = (ns + NARVIS_LAYOUT_BATCH - 1) / NARVIS_LAYOUT_BATCH;
        hipLaunchKernelGGL(k_layout_boxes, dim3((unsigned)nsb), dim3(kT), 0, s, sx, sy, sz, ns,
                           reinterpret_cast<float4 *>(sbox));
    }
    return hipGetLastError();
}


KnnWorkspace knn_workspace(uint64_t n)
{
    KnnWorkspace K{};
    uint64_t slots = 1024;
    while (slots < 2 * n) slots <<= 1;
    K.slots = slots;
    uint64_t o = 0;
    K.off_bb = o; o = align256(o + 8 * 4);
    K.off_count = o; o = align256(o + 4);
    K.off_sum = o; o = align256(o + 8);
    K.off_ka = o; o = align256(o + n * 8);
    K.off_kb = o; o = align256(o + n * 8);
    K.off_va = o; o = align256(o + n * 4);
    K.off_vb = o; o = align256(o + n * 4);
    K.off_hist = o; o = align256(o + radix_sort_hist_len(n) * 4);
    K.off_sums = o; o = align256(o + radix_sort_sums_len(n) * 4);
    K.off_hkey = o; o = align256(o + slots * 8);
    K.off_hval = o; o = align256(o + slots * 4);
    K.off_unres = o; o = align256(o + (n + 1) * 4);
    K.bytes = o;
    return K;
}

namespace {

float host_unordered(uint32_t o)
{
    const uint32_t u = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

}  // namespace

hipError_t launch_knn(const float *x, const float *y, const float *z, uint64_t n, float *radius, void *ws,
                      hipStream_t s, KnnStats *stats)
{
    const KnnWorkspace K = knn_workspace(n);
    char *base = static_cast<char *>(ws);
    auto *bb = reinterpret_cast<uint32_t *>(base + K.off_bb);
    auto *count = reinterpret_cast<uint32_t *>(base + K.off_count);
    auto *sum = reinterpret_cast<unsigned long long *>(base + K.off_sum);
    auto *ka = reinterpret_cast<unsigned long long *>(base + K.off_ka);
    auto *kb = reinterpret_cast<unsigned long long *>(base + K.off_kb);
    auto *va = reinterpret_cast<uint32_t *>(base + K.off_va);
    auto *vb = reinterpret_cast<uint32_t *>(base + K.off_vb);
    auto *hist = reinterpret_cast<uint32_t *>(base + K.off_hist);
    auto *sums = reinterpret_cast<uint32_t *>(base + K.off_sums);
    auto *hkey = reinterpret_cast<unsigned long long *>(base + K.off_hkey);
    auto *hval = reinterpret_cast<uint32_t *>(base + K.off_hval);
    auto *unres = reinterpret_cast<uint32_t *>(base + K.off_unres);
    if (n == 0) return hipSuccess;
    const uint64_t blocks = (n + kT - 1) / kT;
    const uint64_t hblocks = (K.slots + kT - 1) / kT;
    hipLaunchKernelGGL(k_layout_init, dim3(1), dim3(kT), 0, s, bb, count, (uint32_t)n);
    hipLaunchKernelGGL(k_layout_bbox, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(kT), 0, s, x, y, z, n, bb);
    // the box and the number of finite points decide the grid: read them back
    hipError_t e = hipMemsetAsync(sum, 0, 8, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_knn_finite, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(kT), 0, s, x, y, z, n, sum);
    uint32_t hbb[6];
    unsigned long long finite = 0;
    e = hipMemcpyAsync(hbb, bb, sizeof(hbb), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&finite, sum, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    Grid G{};
    double ext[3], emax = 0.0;
    for (int a = 0; a < 3; ++a) {
        G.lo[a] = host_unordered(hbb[a]);
        ext[a] = finite ? (double)host_unordered(hbb[3 + a]) - (double)G.lo[a] : 0.0;
        if (ext[a] > emax) emax = ext[a];
    }
    G.hmask = K.slots - 1;
    // cube cells: start from the volume per point (axes below 2^-10 of the
    // longest count as that long), then halve or double until a point shares
    // its cell with 1.5 to 12 points on average; at most 2^20 cells per axis
    double cell = 1.0;
    if (finite > 1 && emax > 0.0) {
        double vol = 1.0;
        for (int a = 0; a < 3; ++a) vol *= std::max(ext[a], emax / 1024.0);
        cell = std::cbrt(vol * 4.0 / (double)finite);
    }
    const double min_cell = emax > 0.0 ? emax / 1048576.0 : 1.0;
    auto set_cell = [&](double c) {
        c = std::max(c, min_cell);
        G.cell = (float)c;
        G.inv = 1.0f / G.cell;
        for (int a = 0; a < 3; ++a) {
            const double g = std::floor(ext[a] * (double)G.inv) + 1.0;
            G.g[a] = (uint32_t)std::min(g, 1048577.0);
        }
        return c;
    };
    cell = set_cell(cell);
    double occupancy = 0.0;
    int dir = 0;
    for (int it = 0; it < 24 && finite > 1 && emax > 0.0; ++it) {
        hipLaunchKernelGGL(k_hash_clear, dim3((unsigned)hblocks), dim3(kT), 0, s, hkey, hval, K.slots);
        hipLaunchKernelGGL(k_knn_count, dim3((unsigned)blocks), dim3(kT), 0, s, x, y, z, n, G, hkey, hval);
        e = hipMemsetAsync(sum, 0, 8, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_knn_occupancy, dim3((unsigned)(hblocks < 4096 ? hblocks : 4096)), dim3(kT), 0, s, hval,
                           K.slots, sum);
        unsigned long long sq = 0;
        e = hipMemcpyAsync(&sq, sum, 8, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        occupancy = (double)sq / (double)finite;
        if (occupancy > 12.0 && cell > min_cell && dir <= 0) {
            dir = -1;
            cell = set_cell(cell * 0.5);
        } else if (occupancy < 1.5 && dir >= 0) {
            dir = 1;
            cell = set_cell(cell * 2.0);
        } else {
            break;
        }
    }
    // cell-sorted pairs, then each cell's first position in the hash table
    hipLaunchKernelGGL(k_knn_keys, dim3((unsigned)blocks), dim3(kT), 0, s, x, y, z, n, G, ka, va);
    int bits = 1;
    while (bits < 64 && ((uint64_t)1 << bits) <= (uint64_t)G.g[0] * G.g[1] * G.g[2]) ++bits;
    bool in_b = false;
    e = launch_radix_sort(ka, va, kb, vb, count, n, 64, hist, sums, s, &in_b);
    if (e != hipSuccess) return e;
    const unsigned long long *keys = in_b ? kb : ka;
    const uint32_t *vals = in_b ? vb : va;
    hipLaunchKernelGGL(k_hash_clear, dim3((unsigned)hblocks), dim3(kT), 0, s, hkey, hval, K.slots);
    hipLaunchKernelGGL(k_knn_starts, dim3((unsigned)blocks), dim3(kT), 0, s, keys, n, G, hkey, hval);
    e = hipMemsetAsync(unres, 0, 4, s);
    if (e != hipSuccess) return e;
    KnnArgs A;
    A.X = x;
    A.Y = y;
    A.Z = z;
    A.n = n;
    A.finite = finite;
    A.G = G;
    A.keys = keys;
    A.vals = vals;
    A.hkey = hkey;
    A.hval = hval;
    A.radius = radius;
    A.unresolved = unres;
    A.settle = G.cell * (1.0f - 0x1p-20f);
    hipLaunchKernelGGL(k_knn_query, dim3((unsigned)blocks), dim3(kT), 0, s, A);
    hipLaunchKernelGGL(k_knn_brute, dim3(1024), dim3(kT), 0, s, A);
    if (stats) {
        stats->cell = G.cell;
        stats->occupancy = (float)occupancy;
        stats->finite = finite;
        e = hipMemcpyAsync(&stats->unresolved, unres, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
    }
    (void)bits;
    return hipGetLastError();
}

}  // namespace narvis

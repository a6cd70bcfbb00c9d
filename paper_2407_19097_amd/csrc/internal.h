// Internal interfaces between the C-ABI glue and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "narvis.h"

namespace narvis {

// Projection constants of one frame: the three used rows of M, the cull
// bounds and the image size (float and integer).
struct Proj {
    float m00, m01, m02, m03;
    float m10, m11, m12, m13;
    float m30, m31, m32, m33;
    float near_f, far_f;
    float Wf, Hf;
    int32_t W, H;
};

struct AttrArg {
    const unsigned char *p;
    int32_t dtype;
    int32_t stride;
};

struct AttrPack {
    AttrArg a[NARVIS_MAX_ATTRS];
    int32_t count;
};

Proj make_proj(const float vp[16], float near_f, float far_f, int32_t W, int32_t H);

// Per-device facts cached on first use.
struct DeviceInfo {
    int cus;
    int xcds;
};
DeviceInfo device_info();

// Workspace carve-up of the nearest-neighbour radius (size query and launcher).
struct KnnWorkspace {
    uint64_t slots;  // hash table slots (a power of two >= 2 n)
    uint64_t off_bb, off_count, off_sum, off_ka, off_kb, off_va, off_vb, off_hist, off_sums, off_hkey, off_hval,
        off_unres;
    uint64_t bytes;
};
struct KnnStats {
    float cell, occupancy;
    uint64_t finite;
    uint32_t unresolved;
};
KnnWorkspace knn_workspace(uint64_t n);
hipError_t launch_knn(const float *x, const float *y, const float *z, uint64_t n, float *radius, void *ws,
                      hipStream_t s, KnnStats *stats);

// Extra per-point streams of the render.  Layout: the points are in layout
// order, ix gives the original index of each point and box one box per batch
// of NARVIS_LAYOUT_BATCH points (two float4: minima, maxima); ix == nullptr:
// original order.  glyph: one byte per point (nonzero = glyph point) for the
// glyph-priority render, or nullptr.  A layout and a glyph mask are not
// combined.
struct LayoutArgs {
    const uint32_t *ix;
    const float4 *box;
    const uint8_t *glyph;
    // the layout's depth sample (every 8th point), or null
    const float *sx, *sy, *sz;
    const uint32_t *six;
    const float4 *sbox;
    uint64_t ns;
};

hipError_t launch_clear(uint64_t *keys, int64_t npx, hipStream_t s);
hipError_t launch_render(const float *x, const float *y, const float *z, uint64_t n, const Proj &P,
                         uint64_t *keys, int32_t variant, int32_t grid_blocks, uint16_t *bounds, const uint64_t *hint,
                         hipStream_t s, const LayoutArgs &lay = LayoutArgs{nullptr, nullptr, nullptr});
// Device address of this device's static scratch of
// NARVIS_STATIC_SCRATCH_BYTES bytes (resolved on the first call per device).
hipError_t static_scratch(void **ptr);
hipError_t launch_resolve(const float *x, const float *y, const float *z, uint64_t n, const Proj &P,
                          const AttrPack &attrs, const narvis_gbuffer &g, hipStream_t s);

struct SplatLayout {
    int32_t tiles_x, tiles_y;
    uint64_t cap, nblk, nsums;
    uint64_t off_ctr, off_col, off_wbits, off_cnt, off_ka, off_va, off_kb, off_vb, off_hist, off_sums, off_range,
        off_conic, off_ext, off_scnt, off_npts, off_brange, off_part, off_plan;
    uint64_t bytes;
    int key_bits;
};
SplatLayout splat_layout(uint64_t n, int32_t W, int32_t H, float sigma, bool aniso, uint64_t max_pairs);
hipError_t launch_splat(const float *x, const float *y, const float *z, uint64_t n, const Proj &P, const AttrPack &A,
                        const narvis_splat_params &prm, float *img, void *ws, hipStream_t s);
// projection only, then the exact number of (tile, point) pairs (64-bit sum; synchronises)
hipError_t launch_splat_count(const float *x, const float *y, const float *z, uint64_t n, const Proj &P,
                              const AttrPack &A, const narvis_splat_params &prm, void *ws, hipStream_t s,
                              uint64_t *pairs);

// Workspace carve-up of the layout build (shared by the size query and the
// launcher).
struct LayoutWorkspace {
    uint64_t off_bb, off_count, off_ka, off_kb, off_va, off_vb, off_hist, off_sums;
    uint64_t bytes;
};
LayoutWorkspace layout_workspace(uint64_t n);
hipError_t launch_layout(const float *x, const float *y, const float *z, uint64_t n, float *xs, float *ys, float *zs,
                         uint32_t *ix, float *box, float *sx, float *sy, float *sz, uint32_t *six, float *sbox,
                         void *ws, hipStream_t s);

// Stable LSD radix sort (ceil(key_bits / 8) passes of equal digit width, at
// most 8 bits) of the first min(*count, cap) (key,
// value) pairs by the low key_bits bits of the keys, ping-ponging between
// (ka, va) and (kb, vb); *in_b tells where the result ends.  hist and sums
// hold radix_sort_hist_len(cap) and radix_sort_sums_len(cap) uint32.
hipError_t launch_radix_sort(unsigned long long *ka, uint32_t *va, unsigned long long *kb, uint32_t *vb,
                             const uint32_t *count, uint64_t cap, int key_bits, uint32_t *hist, uint32_t *sums,
                             hipStream_t s, bool *in_b);
// the same with 32-bit keys
hipError_t launch_radix_sort32(uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb, const uint32_t *count,
                               uint64_t cap, int key_bits, uint32_t *hist, uint32_t *sums, hipStream_t s, bool *in_b);
uint64_t radix_sort_hist_len(uint64_t cap);
uint64_t radix_sort_sums_len(uint64_t cap);

}  // namespace narvis

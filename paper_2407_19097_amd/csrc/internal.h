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

hipError_t launch_clear(uint64_t *keys, int64_t npx, hipStream_t s);
hipError_t launch_render(const float *x, const float *y, const float *z, uint64_t n, const Proj &P,
                         uint64_t *keys, int32_t variant, int32_t grid_blocks, uint16_t *bounds, const uint64_t *hint,
                         hipStream_t s);
hipError_t launch_resolve(const float *x, const float *y, const float *z, uint64_t n, const Proj &P,
                          const AttrPack &attrs, const narvis_gbuffer &g, hipStream_t s);

struct SplatLayout {
    int32_t tiles_x, tiles_y;
    uint64_t cap, nblk, nsums;
    uint64_t off_ctr, off_col, off_wbits, off_cnt, off_ka, off_va, off_kb, off_vb, off_hist, off_sums, off_range;
    uint64_t bytes;
    int key_bits;
};
SplatLayout splat_layout(uint64_t n, int32_t W, int32_t H, float sigma);
hipError_t launch_splat(const float *x, const float *y, const float *z, uint64_t n, const Proj &P, const AttrPack &A,
                        const narvis_splat_params &prm, float *img, void *ws, hipStream_t s);

}  // namespace narvis

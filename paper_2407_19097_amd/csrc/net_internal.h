// Internal interfaces of the post-processing network.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace narvis {
namespace net {

// Convolution (implicit GEMM).  Input and output are NHWC bf16 slices;
// in_mask (optional) zeroes input elements whose mask element is not > 0
// (the ReLU derivative in the input-gradient pass).
struct ConvArgs {
    const __bf16 *in;
    int in_stride, in_off, Cin;        // Cin: multiple of 8
    // optional second input: channels [Cin1, Cin) come from in2 (a decoder
    // layer reads the upsampled tensor and the skip tensor without a concat)
    const __bf16 *in2;
    int in2_stride, in2_off, Cin1;     // Cin1: multiple of 8 (of 32 for the halo kernel)
    int up_in;                         // nonzero: `in` is at H/2 x W/2 and is 2x bilinear-upsampled on load
    const __bf16 *in_mask;
    int mask_stride, mask_off;
    const __bf16 *wt;                  // [Cout_pad][Kpad]
    int Kpad;                          // multiple of 32
    const float *bias;                 // [Cout_pad] or null
    int Cout, Cout_pad;                // Cout_pad: multiple of 16
    int B, H, W;
    int relu;
    __bf16 *out;                       // NHWC slice (when out_f32 is null)
    int out_stride, out_off;           // multiples of 4
    float *out_f32;                    // planar [B][Cout][H][W]
    // optional fused 1x1 head on the (bf16-rounded) output, 3 x Cout weights
    // (row stride head_kpad) and 3 biases, written planar fp32 [B][3][H][W]
    // instead of `out` (3x3 layers with 32 output channels only)
    const __bf16 *head_w;
    int head_kpad;
    const float *head_b;
    float *head_out;
    // optional fused 2x2 average pooling of the (bf16-rounded) output, NHWC
    // slice at H/2 x W/2 (halo kernel, H and W even)
    __bf16 *pool_out;
    int pool_stride, pool_off;         // multiples of 4
    // gated output (halo kernel, Cout_pad = Cout a multiple of 64): the
    // weights' rows are in gate order (gate_rows), and the layer writes
    // y = ELU(z_f) * sigmoid(z_g) with Cout / 2 channels instead of z
    int gate;
    // depth-to-space output (1x1 layers, Cout a multiple of 16): row
    // (2 a + b) C + c of pixel (i, j) of the H x W grid goes to channel c of
    // pixel (2 i + a, 2 j + b) of the 2H x 2W output (C = Cout / 4)
    int shuffle;
};

// Pooling / upsampling / gradient-sum kernels over channel slices (C multiple of 8).
struct SliceArgs {
    const __bf16 *in;
    int in_stride, in_off;
    const __bf16 *in2;
    int in2_stride, in2_off;
    __bf16 *out;
    int out_stride, out_off;
    int C, B, H, W;                    // H, W: the larger grid except for k_upsample2
};

struct WgradArgs {
    const __bf16 *dy;
    int dy_stride, dy_off;
    const __bf16 *mask;                // the layer's own output (ReLU derivative) or null
    int mask_stride, mask_off;
    const __bf16 *x;                   // the layer's input
    int x_stride, x_off;
    const __bf16 *x2;                  // optional second input: channels [xCin1, Cin)
    int x2_stride, x2_off, xCin1;
    int Cin, KS, Cout, Cout_pad, Kpad;
    int B, H, W;
    int splits;
    int64_t pix_per_split;             // multiple of 64
    float *part;                       // [splits][Cout_pad][Kpad]
    float *bpart;                      // [splits][Cout_pad]
};

hipError_t conv(const ConvArgs &a, int KS, hipStream_t s);
hipError_t conv_fp8(const ConvArgs &a, int KS, const uint8_t *wq, const float *sw, float sa, hipStream_t s);
hipError_t quant_weights(const float *master, int Cout, int Cin, int KS, int rows, int kpad, uint8_t *wq, float *sw,
                         hipStream_t s);
hipError_t absmax_bf16(const __bf16 *x, int64_t n, unsigned int *out, hipStream_t s);
hipError_t absdiff_max_f32(const float *a, const float *b, int64_t n, unsigned int *out, hipStream_t s);
hipError_t features(const float *in, __bf16 *out, int B, int H, int W, hipStream_t s);
hipError_t upsample2(const SliceArgs &a, hipStream_t s);
hipError_t upsample2_bwd(const SliceArgs &a, hipStream_t s);
hipError_t pool2_bwd_add(const SliceArgs &a, hipStream_t s);
hipError_t wgrad(const WgradArgs &a, float *dw, float *db, hipStream_t s);
hipError_t loss(const float *y, const float *t, int B, int H, int W, float lam, __bf16 *grad, float *partial,
                float *out, hipStream_t s);
// CinD: input channels of the device layouts (>= Cin, the rest zero; 0 = Cin)
hipError_t prep_weights(const float *master, int Cout, int Cin, int KS, __bf16 *fwd, int fwd_rows, int fwd_kpad,
                        __bf16 *bwd, int bwd_rows, int bwd_cin, int bwd_kpad, hipStream_t s, int CinD = 0);
hipError_t adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t s);
hipError_t grad_to_blob(const float *dw, int Kpad, int Cout, int Cin, int KS, float *blob, hipStream_t s,
                        int CinD = 0);
hipError_t copy_f32(const float *src, float *dst, int64_t n, hipStream_t s);
hipError_t zero_bf16(__bf16 *p, int64_t n, hipStream_t s);
// the paper's gated U-Net
hipError_t gate(const __bf16 *z, __bf16 *y, int y_stride, int y_off, int C, int64_t P, hipStream_t s);
hipError_t gate_bwd(const __bf16 *z, const __bf16 *dy, int dy_stride, int dy_off, __bf16 *dz, int C, int64_t P,
                    hipStream_t s);
hipError_t pool2(const SliceArgs &a, hipStream_t s);
hipError_t shuffle_down(const SliceArgs &a, hipStream_t s);
hipError_t features_pad(const float *in, __bf16 *out, int B, int H, int W, int Hp, int Wp, int oc, hipStream_t s);
hipError_t crop_planes(const float *src, float *dst, int BC, int H, int W, int Hp, int Wp, hipStream_t s);
hipError_t bias_phases(const float *b, int C, float *rows, hipStream_t s);
// rows of a gated layer's forward weights (and biases) in gate order: in each
// group of 32 device rows, 16 rows of z's first half, then the 16 matching
// rows of its second half
hipError_t gate_rows(const __bf16 *w, const float *b, int rows, int kpad, __bf16 *wg, float *bg, hipStream_t s);
hipError_t bias_grad_phases(const float *rows, int C, float *b, hipStream_t s);

}  // namespace net
}  // namespace narvis

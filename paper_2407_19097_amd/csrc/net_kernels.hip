// Kernels of the post-processing network (gfx950): implicit-GEMM convolution
// on MFMA (v_mfma_f32_16x16x32_bf16), pooling, bilinear upsampling, their
// backward passes, weight gradients, loss and Adam.
//
// Layouts.  Activations are NHWC bfloat16; a tensor may be a channel slice of
// a wider buffer (stride = channels per pixel of the buffer, off = first
// channel), which is how skip connections are concatenated without copies.
// Weights of a layer are a [Cout_pad][Kpad] bfloat16 matrix whose row holds
// the taps in (ky, kx, ci) order (K = taps * Cin, padded with zeros to a
// multiple of 32; rows padded to the output tile).
//
// MFMA operands (16x16x32, bf16, 64 lanes; lane l, g = l / 16, r = l % 16):
// A[m][k] is supplied by lane r + 16 g as its elements k = 8g .. 8g+7 of row
// m = r; B[k][n] likewise for column n = r; lane l receives D[4g + e][r],
// e = 0..3.  The convolution uses A = weights (m = output channel) and
// B = im2col^T (n = pixel), so each lane ends with 4 consecutive output
// channels of one pixel: one 8-byte store per fragment.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "net_internal.h"

#pragma clang fp contract(off)

namespace narvis {
namespace net {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kWaves = 4;

__device__ __forceinline__ bf16x8 zero8()
{
    bf16x8 z;
#pragma unroll
    for (int j = 0; j < 8; ++j) z[j] = (__bf16)0.0f;
    return z;
}

__device__ __forceinline__ bf16x8 load8(const __bf16 *p) { return *reinterpret_cast<const bf16x8 *>(p); }

// element (pixel q, channel c) of a convolution's input (one or two sources)
__device__ __forceinline__ const __bf16 *in_at(const ConvArgs &a, int64_t q, int c)
{
    if (a.in2 && c >= a.Cin1) return a.in2 + q * a.in2_stride + a.in2_off + (c - a.Cin1);
    return a.in + q * a.in_stride + a.in_off + c;
}

// ---------------------------------------------------------------------------
// convolution (forward and input-gradient)
// ---------------------------------------------------------------------------

// Convolution kernel (bf16 or FP8 operands).  Each wave computes FCO x 16
// output channels for FPX x 16 pixels; the next k-step's operands are loaded
// while the current MFMAs run.  A lane's group of 8 consecutive k values
// (one tap, 8 input channels) is tracked incrementally as (tap, ci).
template <bool FP8>
struct ConvOps;

template <>
struct ConvOps<false> {
    typedef bf16x8 A;
    typedef bf16x8 Bv;
    static __device__ __forceinline__ A load_a(const ConvArgs &a, const uint8_t *, int row, int kk)
    {
        return load8(a.wt + (int64_t)row * a.Kpad + kk);
    }
    static __device__ __forceinline__ Bv zero() { return zero8(); }
    static __device__ __forceinline__ Bv to_b(bf16x8 v, float) { return v; }
    static __device__ __forceinline__ f32x4 mfma(A x, Bv y, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
    }
};

template <>
struct ConvOps<true> {
    typedef long A;
    typedef long Bv;
    static __device__ __forceinline__ A load_a(const ConvArgs &a, const uint8_t *wq, int row, int kk)
    {
        return *reinterpret_cast<const long *>(wq + (int64_t)row * a.Kpad + kk);
    }
    static __device__ __forceinline__ Bv zero() { return 0; }
    static __device__ __forceinline__ Bv to_b(bf16x8 v, float inv_sa)
    {
        float t[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) t[j] = fminf(fmaxf((float)v[j] * inv_sa, -448.0f), 448.0f);
        int lo = __builtin_amdgcn_cvt_pk_fp8_f32(t[0], t[1], 0, false);
        lo = __builtin_amdgcn_cvt_pk_fp8_f32(t[2], t[3], lo, true);
        int hi = __builtin_amdgcn_cvt_pk_fp8_f32(t[4], t[5], 0, false);
        hi = __builtin_amdgcn_cvt_pk_fp8_f32(t[6], t[7], hi, true);
        return (long)(uint32_t)lo | ((long)(uint32_t)hi << 32);
    }
    static __device__ __forceinline__ f32x4 mfma(A x, Bv y, f32x4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(x, y, c, 0, 0, 0);
    }
};

template <int FCO, int FPX, int KS, bool FP8>
__global__ __launch_bounds__(64 * kWaves) void k_conv(ConvArgs a, const uint8_t *wq, const float *sw, float sa)
{
    typedef ConvOps<FP8> Ops;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    constexpr int TP = 16 * FPX;
    const int64_t P = (int64_t)a.B * a.H * a.W;
    const int64_t p0 = ((int64_t)blockIdx.x * kWaves + wave) * TP;
    const int co0 = blockIdx.y * 16 * FCO;
    if (p0 >= P) return;  // whole wave idle (no barriers in this kernel)
    const float inv_sa = FP8 ? 1.0f / sa : 1.0f;

    int bb[FPX], yy[FPX], xx[FPX];
    bool pv[FPX];
#pragma unroll
    for (int f = 0; f < FPX; ++f) {
        const int64_t p = p0 + 16 * f + r;
        pv[f] = p < P;
        const int64_t pc = pv[f] ? p : 0;
        const int64_t hw = (int64_t)a.H * a.W;
        bb[f] = (int)(pc / hw);
        const int64_t rem = pc - (int64_t)bb[f] * hw;
        yy[f] = (int)(rem / a.W);
        xx[f] = (int)(rem - (int64_t)yy[f] * a.W);
    }
    f32x4 acc[FCO][FPX];
#pragma unroll
    for (int i = 0; i < FCO; ++i)
#pragma unroll
        for (int f = 0; f < FPX; ++f) acc[i][f] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

    constexpr int T = KS * KS;
    auto load_step = [&](int kk, int tap, int ci, typename Ops::A (&A)[FCO], typename Ops::Bv (&Bv)[FPX]) {
#pragma unroll
        for (int i = 0; i < FCO; ++i) A[i] = Ops::load_a(a, wq, co0 + 16 * i + r, kk);
        const bool kvalid = tap < T;
        const int dy = KS == 3 ? tap / 3 - 1 : 0;
        const int dx = KS == 3 ? tap % 3 - 1 : 0;
#pragma unroll
        for (int f = 0; f < FPX; ++f) {
            const int y2 = yy[f] + dy, x2 = xx[f] + dx;
            const bool ok = kvalid && pv[f] && y2 >= 0 && y2 < a.H && x2 >= 0 && x2 < a.W;
            Bv[f] = Ops::zero();
            if (ok) {
                const int64_t q = ((int64_t)bb[f] * a.H + y2) * a.W + x2;
                bf16x8 v = load8(in_at(a, q, ci));
                if (a.in_mask) {
                    const bf16x8 m = load8(a.in_mask + q * a.mask_stride + a.mask_off + ci);
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        if (!((float)m[j] > 0.0f)) v[j] = (__bf16)0.0f;
                }
                Bv[f] = Ops::to_b(v, inv_sa);
            }
        }
    };
    int tap = (8 * g) / a.Cin;
    int ci = 8 * g - tap * a.Cin;
    typename Ops::A av[FCO], an[FCO];
    typename Ops::Bv bv[FPX], bn[FPX];
    load_step(8 * g, tap, ci, av, bv);
    for (int k0 = 0; k0 < a.Kpad; k0 += 32) {
        int ntap = tap, nci = ci + 32;
        while (nci >= a.Cin) {
            nci -= a.Cin;
            ++ntap;
        }
        const bool more = k0 + 32 < a.Kpad;
        if (more) load_step(k0 + 32 + 8 * g, ntap, nci, an, bn);
#pragma unroll
        for (int i = 0; i < FCO; ++i)
#pragma unroll
            for (int f = 0; f < FPX; ++f) acc[i][f] = Ops::mfma(av[i], bv[f], acc[i][f]);
        if (more) {
#pragma unroll
            for (int i = 0; i < FCO; ++i) av[i] = an[i];
#pragma unroll
            for (int f = 0; f < FPX; ++f) bv[f] = bn[f];
            tap = ntap;
            ci = nci;
        }
    }
    // epilogue: lane holds channels co0 + 16 i + 4 g + e of pixel p0 + 16 f + r
#pragma unroll
    for (int i = 0; i < FCO; ++i) {
        const int cb = co0 + 16 * i + 4 * g;
        float bias[4], scale[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            bias[e] = a.bias ? a.bias[cb + e] : 0.0f;
            scale[e] = FP8 ? sw[cb + e] * sa : 1.0f;
        }
#pragma unroll
        for (int f = 0; f < FPX; ++f) {
            if (!pv[f]) continue;
            const int64_t p = p0 + 16 * f + r;
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                v[e] = FP8 ? acc[i][f][e] * scale[e] + bias[e] : acc[i][f][e] + bias[e];
                if (a.relu) v[e] = fmaxf(v[e], 0.0f);
            }
            if (a.out_f32) {
                // planar fp32 [B][Cout][H][W]
                const int64_t hw = (int64_t)a.H * a.W;
                const int64_t b = p / hw, pix = p - b * hw;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (cb + e < a.Cout) a.out_f32[(b * a.Cout + cb + e) * hw + pix] = v[e];
            } else if (cb < a.Cout) {
                __bf16 *o = a.out + p * a.out_stride + a.out_off + cb;
                typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
                bf16x4 w4;
#pragma unroll
                for (int e = 0; e < 4; ++e) w4[e] = (__bf16)v[e];
                *reinterpret_cast<bf16x4 *>(o) = w4;
            }
        }
    }
}

// LDS-staged convolution for the large layers.  A workgroup (4 waves) owns a
// tile of TCO output channels x TPX pixels and walks K in chunks of 64: each
// chunk of weights (TCO x 64) and of the im2col input (TPX x 64, eight k per
// 16-byte piece: one tap, eight channels) is loaded with every lane reading 16
// consecutive bytes (a wave reads 1 KB over 8 cache lines instead of one
// line per lane), stored in LDS (double-buffered, rows padded against bank
// conflicts), and the MFMA operands are read back with 16-byte LDS reads.
// Each wave computes 32 output channels x 64 pixels (2 x 4 fragments).
constexpr int kKC = 64;           // K per LDS chunk

// LDS address (in elements) of 8-element piece p of row `row`.  bf16 rows are
// 128 bytes with the piece index XOR-swizzled by the row (conflict-free
// 16-byte reads down a fragment's 16 rows and conflict-free stores along a
// row); FP8 rows are 64 bytes padded to 72, which spreads 8-byte reads over
// the banks.
template <bool FP8>
__device__ __forceinline__ int lds_at(int row, int p)
{
    if constexpr (FP8) return row * 72 + 8 * p;
    else return row * 64 + 8 * (p ^ (row & 7));
}

template <int TCO, int TPX, int KS, bool FP8, bool MASK>
__global__ __launch_bounds__(256) void k_conv_lds(ConvArgs a, const uint8_t *wq, const float *sw, float sa)
{
    typedef typename std::conditional<FP8, uint8_t, __bf16>::type E;
    constexpr int RS = FP8 ? 72 : 64;                 // LDS row stride (elements)
    __shared__ __attribute__((aligned(16))) E la[2][TCO * RS];
    __shared__ __attribute__((aligned(16))) E lb[2][TPX * RS];
    constexpr int WCO = TCO / 32;                     // waves along output channels
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int wco = (wave % WCO) * 32, wpx = (wave / WCO) * 64;
    const int64_t P = (int64_t)a.B * a.H * a.W;
    const int64_t p0 = (int64_t)blockIdx.x * TPX;
    const int co0 = blockIdx.y * TCO;
    const float inv_sa = FP8 ? 1.0f / sa : 1.0f;
    constexpr int T = KS * KS;
    const int K = T * a.Cin;
    // staging roles: piece kc (8 k values) of rows t / 8 + 32 j
    const int kc = threadIdx.x & 7;
    constexpr int AJ = TCO / 32, BJ = TPX / 32;
    int bb[BJ], yy[BJ], xx[BJ];
    bool pv[BJ];
#pragma unroll
    for (int j = 0; j < BJ; ++j) {
        const int64_t p = p0 + (threadIdx.x >> 3) + 32 * j;
        pv[j] = p < P;
        const int64_t pc = pv[j] ? p : 0;
        const int64_t hw = (int64_t)a.H * a.W;
        bb[j] = (int)(pc / hw);
        const int64_t rem = pc - (int64_t)bb[j] * hw;
        yy[j] = (int)(rem / a.W);
        xx[j] = (int)(rem - (int64_t)yy[j] * a.W);
    }
    // registers holding the next chunk between its global load and its LDS
    // store; the ReLU mask and the FP8 conversion are applied at the store so
    // the loads stay in flight behind the MFMAs of the current chunk
    typedef typename std::conditional<FP8, long, bf16x8>::type Piece;
    Piece ra[AJ];
    bf16x8 rb[BJ];
    bf16x8 rm[MASK ? BJ : 1];
    int tap = (8 * kc) / a.Cin;
    int ci = 8 * kc - tap * a.Cin;
    auto gload = [&](int k0, int tp, int c) {
        const int kk = k0 + 8 * kc;
#pragma unroll
        for (int j = 0; j < AJ; ++j) {
            const int row = co0 + (threadIdx.x >> 3) + 32 * j;
            if constexpr (FP8) {
                ra[j] = kk < a.Kpad ? *reinterpret_cast<const long *>(wq + (int64_t)row * a.Kpad + kk) : 0;
            } else {
                ra[j] = kk < a.Kpad ? load8(a.wt + (int64_t)row * a.Kpad + kk) : zero8();
            }
        }
        const bool kvalid = tp < T && kk < K;
        const int dy = KS == 3 ? tp / 3 - 1 : 0, dx = KS == 3 ? tp % 3 - 1 : 0;
#pragma unroll
        for (int j = 0; j < BJ; ++j) {
            const int y2 = yy[j] + dy, x2 = xx[j] + dx;
            rb[j] = zero8();
            if (kvalid && pv[j] && y2 >= 0 && y2 < a.H && x2 >= 0 && x2 < a.W) {
                const int64_t q = ((int64_t)bb[j] * a.H + y2) * a.W + x2;
                rb[j] = load8(in_at(a, q, c));
                if constexpr (MASK) rm[j] = load8(a.in_mask + q * a.mask_stride + a.mask_off + c);
            }
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int j = 0; j < AJ; ++j)
            *reinterpret_cast<Piece *>(&la[buf][lds_at<FP8>((threadIdx.x >> 3) + 32 * j, kc)]) = ra[j];
#pragma unroll
        for (int j = 0; j < BJ; ++j) {
            bf16x8 v = rb[j];
            if constexpr (MASK) {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    if (!((float)rm[j][e] > 0.0f)) v[e] = (__bf16)0.0f;
            }
            if constexpr (FP8)
                *reinterpret_cast<long *>(&lb[buf][lds_at<FP8>((threadIdx.x >> 3) + 32 * j, kc)]) =
                    ConvOps<true>::to_b(v, inv_sa);
            else
                *reinterpret_cast<bf16x8 *>(&lb[buf][lds_at<FP8>((threadIdx.x >> 3) + 32 * j, kc)]) = v;
        }
    };
    f32x4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int f = 0; f < 4; ++f) acc[i][f] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int nchunks = (a.Kpad + kKC - 1) / kKC;
    gload(0, tap, ci);
    lstore(0);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        const bool more = c + 1 < nchunks;
        if (more) {
            ci += kKC;
            while (ci >= a.Cin) {
                ci -= a.Cin;
                ++tap;
            }
            gload((c + 1) * kKC, tap, ci);
        }
#pragma unroll
        for (int s = 0; s < kKC / 32; ++s) {
            typename ConvOps<FP8>::A av[2];
            typename ConvOps<FP8>::Bv bv[4];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                av[i] = *reinterpret_cast<const typename ConvOps<FP8>::A *>(&la[buf][lds_at<FP8>(wco + 16 * i + r, 4 * s + g)]);
#pragma unroll
            for (int f = 0; f < 4; ++f)
                bv[f] = *reinterpret_cast<const typename ConvOps<FP8>::Bv *>(&lb[buf][lds_at<FP8>(wpx + 16 * f + r, 4 * s + g)]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int f = 0; f < 4; ++f) acc[i][f] = ConvOps<FP8>::mfma(av[i], bv[f], acc[i][f]);
        }
        if (more) lstore(buf ^ 1);
        __syncthreads();
    }
    // epilogue: lane holds channels co0 + wco + 16 i + 4 g + e of pixel p0 + wpx + 16 f + r.
    // A bf16 output on 8-channel boundaries is staged through LDS (the input
    // tiles are no longer read) and written as 16-byte pieces, a pixel's TCO
    // channels contiguous, instead of 8 bytes per lane at pixel stride.
    constexpr int kOutPitch = TCO + 8;  // elements per staged pixel row (16-byte aligned rows)
    static_assert(sizeof(lb) >= (size_t)TPX * kOutPitch * 2, "the output tile fits in the input tile's LDS");
    const bool staged = !a.out_f32 && !(a.out_stride & 7) && !(a.out_off & 7) && !(a.Cout & 7) &&
                        (!a.shuffle || !((a.Cout >> 2) & 7));
    if (staged) {
        __bf16 *so = reinterpret_cast<__bf16 *>(&lb[0][0]);
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int cl = wco + 16 * i + 4 * g, cb = co0 + cl;
            float bias[4], scale[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                bias[e] = a.bias && cb + e < a.Cout_pad ? a.bias[cb + e] : 0.0f;
                scale[e] = FP8 ? sw[cb + e] * sa : 1.0f;
            }
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
                bf16x4 w4;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float v = FP8 ? acc[i][f][e] * scale[e] + bias[e] : acc[i][f][e] + bias[e];
                    if (a.relu) v = fmaxf(v, 0.0f);
                    w4[e] = (__bf16)v;
                }
                *reinterpret_cast<bf16x4 *>(&so[(wpx + 16 * f + r) * kOutPitch + cl]) = w4;
            }
        }
        __syncthreads();
        constexpr int PIECES = TCO / 8;
        for (int idx = threadIdx.x; idx < TPX * PIECES; idx += 256) {
            const int pr = idx / PIECES, pc = idx - pr * PIECES;
            const int64_t p = p0 + pr;
            const int cb = co0 + 8 * pc;
            if (p >= P || cb >= a.Cout) continue;
            int64_t q = p;
            int c = cb;
            if (a.shuffle) {  // depth-to-space, as below; the 8 channels share one phase
                const int C4 = a.Cout >> 2, ph = cb / C4;
                c = cb - ph * C4;
                const int64_t hw = (int64_t)a.H * a.W;
                const int64_t b = p / hw, rem = p - b * hw;
                const int64_t yi = rem / a.W, xj = rem - yi * a.W;
                q = (b * 2 * a.H + 2 * yi + (ph >> 1)) * (2 * (int64_t)a.W) + 2 * xj + (ph & 1);
            }
            *reinterpret_cast<uint4 *>(a.out + q * a.out_stride + a.out_off + c) =
                *reinterpret_cast<const uint4 *>(&so[pr * kOutPitch + 8 * pc]);
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int cb = co0 + wco + 16 * i + 4 * g;
        float bias[4], scale[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            bias[e] = a.bias ? a.bias[cb + e] : 0.0f;
            scale[e] = FP8 ? sw[cb + e] * sa : 1.0f;
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const int64_t p = p0 + wpx + 16 * f + r;
            if (p >= P) continue;
            float v[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                v[e] = FP8 ? acc[i][f][e] * scale[e] + bias[e] : acc[i][f][e] + bias[e];
                if (a.relu) v[e] = fmaxf(v[e], 0.0f);
            }
            if (a.out_f32) {
                const int64_t hw = (int64_t)a.H * a.W;
                const int64_t b = p / hw, pix = p - b * hw;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (cb + e < a.Cout) a.out_f32[(b * a.Cout + cb + e) * hw + pix] = v[e];
            } else if (cb < a.Cout) {
                int64_t q = p;
                int c = cb;
                if (a.shuffle) {
                    // depth-to-space: phase (2 sy + sx) of the 2x2 block (C = Cout / 4 a multiple of 4,
                    // so the lane's 4 channels share one phase)
                    const int C4 = a.Cout >> 2, ph = cb / C4;
                    c = cb - ph * C4;
                    const int64_t hw = (int64_t)a.H * a.W;
                    const int64_t b = p / hw, rem = p - b * hw;
                    const int64_t i = rem / a.W, j = rem - i * a.W;
                    q = (b * 2 * a.H + 2 * i + (ph >> 1)) * (2 * (int64_t)a.W) + 2 * j + (ph & 1);
                }
                __bf16 *o = a.out + q * a.out_stride + a.out_off + c;
                typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
                bf16x4 w4;
#pragma unroll
                for (int e = 0; e < 4; ++e) w4[e] = (__bf16)v[e];
                *reinterpret_cast<bf16x4 *>(o) = w4;
            }
        }
    }
}

// source index and weight of output o for a x2 bilinear upsample of n samples
// (half-pixel centres, clamped): out[o] = (1 - f) in[i0] + f in[i1]
__device__ __forceinline__ void up_src(int o, int n, int &i0, int &i1, float &f)
{
    float src = ((float)o + 0.5f) * 0.5f - 0.5f;
    src = fmaxf(src, 0.0f);
    i0 = min((int)src, n - 1);
    i1 = min(i0 + 1, n - 1);
    f = src - (float)i0;
}

// 8 channels of the 2x bilinear upsample of a [B][h][w] slice at output pixel
// (y, x) of the [B][2h][2w] grid (the same arithmetic as k_upsample2)
__device__ __forceinline__ bf16x8 upsample_piece(const __bf16 *in, int stride, int off, int b, int h, int w, int y,
                                                 int x, int c)
{
    int y0, y1, x0, x1;
    float fy, fx;
    up_src(y, h, y0, y1, fy);
    up_src(x, w, x0, x1, fx);
    const int64_t rb = (int64_t)b * h;
    const bf16x8 v00 = load8(in + ((rb + y0) * w + x0) * stride + off + c);
    const bf16x8 v01 = load8(in + ((rb + y0) * w + x1) * stride + off + c);
    const bf16x8 v10 = load8(in + ((rb + y1) * w + x0) * stride + off + c);
    const bf16x8 v11 = load8(in + ((rb + y1) * w + x1) * stride + off + c);
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const float top = (1.0f - fx) * (float)v00[j] + fx * (float)v01[j];
        const float bot = (1.0f - fx) * (float)v10[j] + fx * (float)v11[j];
        o[j] = (__bf16)((1.0f - fy) * top + fy * bot);
    }
    return o;
}

// Direct 3x3 convolution for layers with 32 output channels and Cin a
// multiple of 32 (the full-resolution layers).  A workgroup of 4 waves owns 4
// output rows x 64 pixels; for each group of 32 input channels it stages the
// 6 x 66 pixel halo tile in LDS once, and all nine taps read their B
// fragments from it at shifted positions (the im2col matrix is never formed).
// The group's weights (9 taps x 32 x 32) are staged in LDS beside the tile.
// Within a pixel's 64 bytes the four 16-byte pieces are XOR-swizzled by
// pixel bits 1-2, so eight lanes reading eight consecutive pixels at the same
// channel offset hit distinct banks, for every tap shift.
// the gated convolution's activation: ELU (alpha 1) times the logistic gate
__device__ __forceinline__ float elu1(float x) { return x > 0.0f ? x : expm1f(x); }
__device__ __forceinline__ float sigm(float x) { return 1.0f / (1.0f + expf(-x)); }

constexpr int kHaloRows = 4;   // output rows per workgroup of the first-layer kernel
constexpr int kHaloCols = 64;  // output pixels per row of a tile

__device__ __forceinline__ int halo_at(int p, int part) { return p * 32 + 8 * (part ^ ((p >> 1) & 3)); }

template <int CO, int ROWS, bool MASK, bool HEAD, bool UP, bool FP8, bool GATE = false>
__global__ __launch_bounds__(64 * ROWS * CO / 32, 4) void k_conv_halo(ConvArgs a, const uint8_t *wq, const float *sw,
                                                                      float sa)
{
    static_assert(!FP8 || (!MASK && !HEAD), "FP8 runs inference layers without the fused head");
    static_assert(!GATE || (!MASK && !HEAD && !UP && !FP8), "the gated output is an inference epilogue");
    static_assert(ROWS % 2 == 0 && (CO / 32) * (ROWS / 2) * 8 * 64 * 8 <= 9 * CO * 32 * (FP8 ? 1 : 2),
                  "room in the weights' LDS for the pooled rows");
    typedef ConvOps<FP8> Ops;
    // LDS holds bf16, or e4m3 for FP8 (activations converted on the way in)
    constexpr int EB = FP8 ? 1 : 2;
    typedef typename std::conditional<FP8, long, bf16x8>::type Piece;  // 8 channels
    const float inv_sa = FP8 ? 1.0f / sa : 1.0f;

    constexpr int NCH = CO / 32;                  // waves per output row (32 channels each)
    constexpr int NT = 64 * ROWS * NCH;           // threads
    constexpr int HR = ROWS + 2, HC = kHaloCols + 2;
    constexpr int NPIECE = HR * HC * 4;           // 16-byte pieces of the halo tile
    constexpr int SJ = (NPIECE + NT - 1) / NT;
    constexpr int NWPIECE = 9 * CO * 4;           // pieces of the weights (9 taps x CO x 32 ci)
    constexpr int WJ = (NWPIECE + NT - 1) / NT;
    // upsampled groups: the low-resolution source rows y0/2 - 1 .. y0/2 + ROWS/2
    // and columns x0/2 - 1 .. x0/2 + 32 cover every source the tile needs
    constexpr int SR = UP ? ROWS / 2 + 2 : 1, SC = UP ? kHaloCols / 2 + 2 : 1;
    constexpr int NLPIECE = SR * SC * 4;
    constexpr int LJ = (NLPIECE + NT - 1) / NT;
    __shared__ __attribute__((aligned(16))) uint8_t xs[HR * HC * 32 * EB];
    __shared__ __attribute__((aligned(16))) uint8_t ws[9 * CO * 32 * EB];   // row (tap * CO + co), 32 ci
    __shared__ __attribute__((aligned(16))) __bf16 lo[SR * SC * 32];
    // byte offset of the 8-channel piece `part` of LDS row p: 64-byte bf16
    // rows swizzled by row bits 1-2, 32-byte FP8 rows by row bits 2-3 (16
    // lanes reading 8 bytes from 16 consecutive rows hit distinct banks)
    auto at = [](int p, int part) {
        return FP8 ? p * 32 + 8 * (part ^ ((p >> 2) & 3)) : 2 * halo_at(p, part);
    };
    auto put = [&](uint8_t *base, int off, bf16x8 v) {
        if constexpr (FP8) *reinterpret_cast<long *>(base + off) = Ops::to_b(v, inv_sa);
        else *reinterpret_cast<bf16x8 *>(base + off) = v;
    };
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int wch = wave % NCH, wrow = wave / NCH;  // this wave: channels 32 wch.., output row wrow
    const int ctiles = a.Cout_pad / CO;
    const int x0 = blockIdx.x * kHaloCols, y0 = blockIdx.y * ROWS;
    const int b = blockIdx.z / ctiles, co0 = (blockIdx.z - b * ctiles) * CO;
    f32x4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int f = 0; f < 4; ++f) acc[i][f] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int nchunks = a.Cin / 32;
    for (int c = 0; c < nchunks; ++c) {
        // the group's source (uniform): `in`, or `in2` past Cin1
        const bool second = a.in2 && 32 * c >= a.Cin1;
        const __bf16 *src = second ? a.in2 : a.in;
        const int sstride = second ? a.in2_stride : a.in_stride;
        const int soff = second ? a.in2_off + 32 * c - a.Cin1 : a.in_off + 32 * c;
        Piece wv[WJ];
#pragma unroll
        for (int j = 0; j < WJ; ++j) {
            const int piece = threadIdx.x + NT * j;
            const int row = piece >> 2, part = piece & 3;   // row = tap * CO + co
            const int tap = row / CO, co = row - tap * CO;
            const int64_t k = (int64_t)(co0 + co) * a.Kpad + tap * a.Cin + 32 * c + 8 * part;
            if constexpr (FP8) wv[j] = piece < NWPIECE ? *reinterpret_cast<const long *>(wq + k) : 0;
            else wv[j] = piece < NWPIECE ? load8(a.wt + k) : zero8();
        }
        auto store_w = [&]() {
#pragma unroll
            for (int j = 0; j < WJ; ++j) {
                const int piece = threadIdx.x + NT * j;
                if (piece < NWPIECE) *reinterpret_cast<Piece *>(ws + at(piece >> 2, piece & 3)) = wv[j];
            }
        };
        if (UP && !second) {
            // upsampled group: stage the low-resolution source tile (rows and
            // columns clamped to the source image), then interpolate from LDS
            const int h = a.H / 2, w = a.W / 2;
            const int sy0 = y0 / 2 - 1, sx0 = x0 / 2 - 1;
            bf16x8 lv[LJ];
#pragma unroll
            for (int j = 0; j < LJ; ++j) {
                const int piece = threadIdx.x + NT * j;
                const int p = piece >> 2, part = piece & 3;
                const int ly = p / SC, lx = p - ly * SC;
                const int sy = min(max(sy0 + ly, 0), h - 1), sx = min(max(sx0 + lx, 0), w - 1);
                lv[j] = zero8();
                if (piece < NLPIECE)
                    lv[j] = load8(src + (((int64_t)b * h + sy) * w + sx) * sstride + soff + 8 * part);
            }
            if (c) __syncthreads();  // the previous group's taps are done with the tiles
            store_w();
#pragma unroll
            for (int j = 0; j < LJ; ++j) {
                const int piece = threadIdx.x + NT * j;
                if (piece < NLPIECE) *reinterpret_cast<bf16x8 *>(&lo[halo_at(piece >> 2, piece & 3)]) = lv[j];
            }
            __syncthreads();
#pragma unroll 1
            for (int piece = threadIdx.x; piece < NPIECE; piece += NT) {
                const int p = piece >> 2, part = piece & 3;
                const int hy = p / HC, hx = p - hy * HC;
                const int y = y0 - 1 + hy, x = x0 - 1 + hx;
                bf16x8 t = zero8();
                if (y >= 0 && y < a.H && x >= 0 && x < a.W) {
                    int iy0, iy1, ix0, ix1;
                    float fy, fx;
                    up_src(y, h, iy0, iy1, fy);
                    up_src(x, w, ix0, ix1, fx);
                    iy0 -= sy0, iy1 -= sy0, ix0 -= sx0, ix1 -= sx0;
                    const bf16x8 v00 = *reinterpret_cast<const bf16x8 *>(&lo[halo_at(iy0 * SC + ix0, part)]);
                    const bf16x8 v01 = *reinterpret_cast<const bf16x8 *>(&lo[halo_at(iy0 * SC + ix1, part)]);
                    const bf16x8 v10 = *reinterpret_cast<const bf16x8 *>(&lo[halo_at(iy1 * SC + ix0, part)]);
                    const bf16x8 v11 = *reinterpret_cast<const bf16x8 *>(&lo[halo_at(iy1 * SC + ix1, part)]);
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        const float top = (1.0f - fx) * (float)v00[j] + fx * (float)v01[j];
                        const float bot = (1.0f - fx) * (float)v10[j] + fx * (float)v11[j];
                        t[j] = (__bf16)((1.0f - fy) * top + fy * bot);
                    }
                }
                put(xs, at(p, part), t);
            }
        } else {
            bf16x8 v[SJ];
#pragma unroll
            for (int j = 0; j < SJ; ++j) {
                const int piece = threadIdx.x + NT * j;
                const int p = piece >> 2, part = piece & 3;
                const int hy = p / HC, hx = p - hy * HC;
                const int y = y0 - 1 + hy, x = x0 - 1 + hx;
                v[j] = zero8();
                if (piece < NPIECE && y >= 0 && y < a.H && x >= 0 && x < a.W) {
                    const int64_t q = ((int64_t)b * a.H + y) * a.W + x;
                    v[j] = load8(src + q * sstride + soff + 8 * part);
                    if constexpr (MASK) {
                        const bf16x8 m = load8(a.in_mask + q * a.mask_stride + a.mask_off + 32 * c + 8 * part);
#pragma unroll
                        for (int e = 0; e < 8; ++e)
                            if (!((float)m[e] > 0.0f)) v[j][e] = (__bf16)0.0f;
                    }
                }
            }
            if (c) __syncthreads();  // the previous group's taps are done with the tiles
            store_w();
#pragma unroll
            for (int j = 0; j < SJ; ++j) {
                const int piece = threadIdx.x + NT * j;
                if (piece < NPIECE) put(xs, at(piece >> 2, piece & 3), v[j]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap % 3;
            typename Ops::A av[2];
            typename Ops::Bv bv[4];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                av[i] = *reinterpret_cast<const typename Ops::A *>(ws + at(tap * CO + 32 * wch + 16 * i + r, g));
#pragma unroll
            for (int f = 0; f < 4; ++f)
                bv[f] = *reinterpret_cast<const typename Ops::Bv *>(xs + at((wrow + dy) * HC + 16 * f + r + dx, g));
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int f = 0; f < 4; ++f) acc[i][f] = Ops::mfma(av[i], bv[f], acc[i][f]);
        }
    }
    // lane holds channels co0 + 32 wch + 16 i + 4 g + e of pixel (y0 + wrow, x0 + 16 f + r)
    const int y = y0 + wrow;
    if constexpr (HEAD) {
        static_assert(CO == 32, "the fused head needs all 32 channels in one wave");
        // 1x1 head: each lane dots its 8 channels with the head rows, the four
        // lane groups (g) are summed with two butterfly shuffles, group 0 writes
        float hw[3][8], hb[3];
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            hb[o] = a.head_b[o];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) hw[o][4 * i + e] = (float)a.head_w[o * a.head_kpad + 16 * i + 4 * g + e];
        }
        float cbias[8];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) cbias[4 * i + e] = a.bias ? a.bias[16 * i + 4 * g + e] : 0.0f;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            float part[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    float t = acc[i][f][e] + cbias[4 * i + e];
                    if (a.relu) t = fmaxf(t, 0.0f);
                    t = (float)(__bf16)t;
#pragma unroll
                    for (int o = 0; o < 3; ++o) part[o] += t * hw[o][4 * i + e];
                }
#pragma unroll
            for (int o = 0; o < 3; ++o) {
                part[o] += __shfl_xor(part[o], 16);
                part[o] += __shfl_xor(part[o], 32);
            }
            const int x = x0 + 16 * f + r;
            if (g == 0 && y < a.H && x < a.W) {
                const int64_t hw_ = (int64_t)a.H * a.W, pix = (int64_t)y * a.W + x;
#pragma unroll
                for (int o = 0; o < 3; ++o) a.head_out[((int64_t)b * 3 + o) * hw_ + pix] = part[o] + hb[o];
            }
        }
        return;
    }
    // Fused 2x2 average pooling (pool_out): the odd row of each pair leaves
    // its rounded outputs in the weights' LDS, the even row adds them to its
    // own and its right neighbour's in the standalone kernel's order.  Every
    // wave reaches both barriers (the pooling flag is uniform).
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    const bool pool = a.pool_out != nullptr;
    bf16x4 *const pl = reinterpret_cast<bf16x4 *>(ws);  // [(wch, row pair, i, f)][lane]
    const int pslot = (wch * (ROWS / 2) + (wrow >> 1)) * 8;
    if (pool) __syncthreads();  // every wave is done with the tiles
    // GATE: device rows co0 + 32 wch + 4 g + e (acc[0]) and the same + 16
    // (acc[1]) are the two halves of output channel (co0 + 32 wch) / 2 + 4 g + e
    constexpr int NI = GATE ? 1 : 2;
    const int cout_lim = GATE ? a.Cout / 2 : a.Cout;
    auto out_base = [&](int i) { return GATE ? (co0 + 32 * wch) / 2 + 4 * g : co0 + 32 * wch + 16 * i + 4 * g; };
    bf16x4 own[NI][4];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int cb = out_base(i);
        const int rb = co0 + 32 * wch + 16 * i + 4 * g;
        float bias[4], scale[4], bias_g[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            bias[e] = a.bias ? a.bias[rb + e] : 0.0f;
            bias_g[e] = GATE && a.bias ? a.bias[rb + 16 + e] : 0.0f;
            scale[e] = FP8 ? sw[rb + e] * sa : 1.0f;  // FP8: dequantise (weight scale x activation scale)
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const int x = x0 + 16 * f + r;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                if constexpr (GATE) {
                    // z rounded to bf16 as the unfused layer stores it
                    const float zf = (float)(__bf16)(acc[0][f][e] + bias[e]);
                    const float zg = (float)(__bf16)(acc[1][f][e] + bias_g[e]);
                    own[i][f][e] = (__bf16)(elu1(zf) * sigm(zg));
                } else {
                    float t = FP8 ? acc[i][f][e] * scale[e] + bias[e] : acc[i][f][e] + bias[e];
                    if (a.relu) t = fmaxf(t, 0.0f);
                    own[i][f][e] = (__bf16)t;
                }
            }
            if (pool && (wrow & 1)) pl[(pslot + 4 * i + f) * 64 + lane] = own[i][f];
            if (y >= a.H || x >= a.W || cb >= cout_lim) continue;
            const int64_t p = ((int64_t)b * a.H + y) * a.W + x;
            *reinterpret_cast<bf16x4 *>(a.out + p * a.out_stride + a.out_off + cb) = own[i][f];
        }
    }
    if (!pool) return;
    __syncthreads();
    if (wrow & 1) return;
    const int Wo = a.W / 2;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int cb = out_base(i);
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            // the right neighbour's output (lane r ^ 1), as two 32-bit words
            typedef int int2v __attribute__((ext_vector_type(2)));
            int2v mine = __builtin_bit_cast(int2v, own[i][f]), theirs;
            theirs[0] = __shfl_xor(mine[0], 1);
            theirs[1] = __shfl_xor(mine[1], 1);
            const bf16x4 right = __builtin_bit_cast(bf16x4, theirs);
            const int x = x0 + 16 * f + r;
            if ((r & 1) || y >= a.H || x >= a.W || cb >= cout_lim) continue;
            const bf16x4 below = pl[(pslot + 4 * i + f) * 64 + lane];
            const bf16x4 below_right = pl[(pslot + 4 * i + f) * 64 + lane + 1];
            bf16x4 o;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float t = 0.0f;
                t = t + (float)own[i][f][e];
                t = t + (float)right[e];
                t = t + (float)below[e];
                t = t + (float)below_right[e];
                o[e] = (__bf16)(t * 0.25f);
            }
            const int64_t q = ((int64_t)b * (a.H / 2) + y / 2) * Wo + x / 2;
            *reinterpret_cast<bf16x4 *>(a.pool_out + q * a.pool_stride + a.pool_off + cb) = o;
        }
    }
}

// Direct 3x3 convolution of the 8-channel feature image (first layer, 32
// output channels).  A pixel is one 16-byte piece, so a K step of 32 covers
// four taps: lane group g of step s takes tap 4 s + g (K = 72 padded to 96).
// Tile as above: 4 output rows x 64 pixels per workgroup, the 6 x 66 halo
// tile and the 32 x 96 weight matrix staged in LDS (weight rows padded to 104
// elements so that 16-byte reads down 8 rows hit distinct banks).
__global__ __launch_bounds__(256) void k_conv_c8(ConvArgs a)
{
    constexpr int HR = kHaloRows + 2, HC = kHaloCols + 2;
    constexpr int NPIECE = HR * HC;
    constexpr int RSW = 104;
    __shared__ __attribute__((aligned(16))) __bf16 xs[NPIECE * 8];
    __shared__ __attribute__((aligned(16))) __bf16 ws[32 * RSW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int x0 = blockIdx.x * kHaloCols, y0 = blockIdx.y * kHaloRows, b = blockIdx.z;
    bf16x8 v[2], wv[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int p = threadIdx.x + 256 * j;
        const int hy = p / HC, hx = p - hy * HC;
        const int y = y0 - 1 + hy, x = x0 - 1 + hx;
        v[j] = zero8();
        if (p < NPIECE && y >= 0 && y < a.H && x >= 0 && x < a.W)
            v[j] = load8(a.in + (((int64_t)b * a.H + y) * a.W + x) * a.in_stride + a.in_off);
        const int row = p / 12, part = p - row * 12;
        wv[j] = zero8();
        if (p < 32 * 12) wv[j] = load8(a.wt + (int64_t)row * a.Kpad + 8 * part);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int p = threadIdx.x + 256 * j;
        if (p < NPIECE) *reinterpret_cast<bf16x8 *>(&xs[p * 8]) = v[j];
        const int row = p / 12, part = p - row * 12;
        if (p < 32 * 12) *reinterpret_cast<bf16x8 *>(&ws[row * RSW + 8 * part]) = wv[j];
    }
    __syncthreads();
    f32x4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int f = 0; f < 4; ++f) acc[i][f] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int st = 0; st < 3; ++st) {
        const int tap = 4 * st + g;
        const int dy = tap / 3, dx = tap % 3;
        bf16x8 av[2], bv[4];
#pragma unroll
        for (int i = 0; i < 2; ++i) av[i] = *reinterpret_cast<const bf16x8 *>(&ws[(16 * i + r) * RSW + 32 * st + 8 * g]);
#pragma unroll
        for (int f = 0; f < 4; ++f)
            bv[f] = tap < 9 ? *reinterpret_cast<const bf16x8 *>(&xs[((wave + dy) * HC + 16 * f + r + dx) * 8]) : zero8();
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int f = 0; f < 4; ++f)
                acc[i][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[f], acc[i][f], 0, 0, 0);
    }
    const int y = y0 + wave;
    if (y >= a.H) return;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int cb = 16 * i + 4 * g;
        float bias[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) bias[e] = a.bias ? a.bias[cb + e] : 0.0f;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const int x = x0 + 16 * f + r;
            if (x >= a.W || cb >= a.Cout) continue;
            const int64_t p = ((int64_t)b * a.H + y) * a.W + x;
            typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
            bf16x4 w4;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float t = acc[i][f][e] + bias[e];
                if (a.relu) t = fmaxf(t, 0.0f);
                w4[e] = (__bf16)t;
            }
            *reinterpret_cast<bf16x4 *>(a.out + p * a.out_stride + a.out_off + cb) = w4;
        }
    }
}

// ---------------------------------------------------------------------------
// features, pooling, upsampling
// ---------------------------------------------------------------------------

// planar fp32 G-buffer planes [B][8][H][W] (r, g, b, depth, v'x, v'y, theta, |v'|)
// -> NHWC bf16 [B*H*W][8]; depth becomes inverse depth (0 where empty)
__global__ __launch_bounds__(256) void k_features(const float *in, __bf16 *out, int64_t P, int64_t hw)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    const int64_t b = p / hw, pix = p - b * hw;
    const float *src = in + b * 8 * hw + pix;
    bf16x8 v;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        float x = src[c * hw];
        if (c == 3) x = x > 0.0f ? 1.0f / x : 0.0f;
        v[c] = (__bf16)x;
    }
    *reinterpret_cast<bf16x8 *>(out + p * 8) = v;
}

// Upsampling (and its adjoint, and the pooling adjoint below): blockIdx.y
// walks output rows (b, y) (uniform, so the row arithmetic is scalar), x and
// the 8-channel group come from the thread index within the row.  The 2x2
// average pooling itself is fused into the convolution that produces its
// input (k_conv_halo, pool_out).

// 2x bilinear upsample, in: [B][H][W] slice, out: [B][2H][2W] slice
__global__ __launch_bounds__(256) void k_upsample2(SliceArgs s)
{
    const int groups = s.C / 8;
    const int Ho = 2 * s.H, Wo = 2 * s.W;
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= Wo * groups) return;
    const int x = t / groups, c8 = t - x * groups;
    int x0, x1;
    float fx;
    up_src(x, s.W, x0, x1, fx);
    const int64_t rows = (int64_t)s.B * Ho;
    for (int64_t ro = blockIdx.y; ro < rows; ro += gridDim.y) {
        const int64_t b = ro / Ho;
        const int y = (int)(ro - b * Ho);
        int y0, y1;
        float fy;
        up_src(y, s.H, y0, y1, fy);
        const int64_t rb = b * s.H;
        const bf16x8 v00 = load8(s.in + ((rb + y0) * s.W + x0) * s.in_stride + s.in_off + c8 * 8);
        const bf16x8 v01 = load8(s.in + ((rb + y0) * s.W + x1) * s.in_stride + s.in_off + c8 * 8);
        const bf16x8 v10 = load8(s.in + ((rb + y1) * s.W + x0) * s.in_stride + s.in_off + c8 * 8);
        const bf16x8 v11 = load8(s.in + ((rb + y1) * s.W + x1) * s.in_stride + s.in_off + c8 * 8);
        bf16x8 o;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float top = (1.0f - fx) * (float)v00[j] + fx * (float)v01[j];
            const float bot = (1.0f - fx) * (float)v10[j] + fx * (float)v11[j];
            o[j] = (__bf16)((1.0f - fy) * top + fy * bot);
        }
        *reinterpret_cast<bf16x8 *>(s.out + (ro * Wo + x) * s.out_stride + s.out_off + c8 * 8) = o;
    }
}

// gradient of k_upsample2, gather form: in-grad [B][H][W] from out-grad [B][2H][2W]
// (s.in = out-grad slice at 2H x 2W, s.out = in-grad slice at H x W)
__global__ __launch_bounds__(256) void k_upsample2_bwd(SliceArgs s)
{
    const int groups = s.C / 8;
    const int Ho = 2 * s.H, Wo = 2 * s.W;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t total = (int64_t)s.B * s.H * s.W * groups;
    if (t >= total) return;
    const int c8 = (int)(t % groups);
    const int64_t pi = t / groups;
    const int64_t b = pi / ((int64_t)s.H * s.W);
    const int64_t rem = pi - b * s.H * s.W;
    const int i = (int)(rem / s.W), j = (int)(rem % s.W);
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int oy = max(0, 2 * i - 2); oy <= min(Ho - 1, 2 * i + 3); ++oy) {
        int y0, y1;
        float fy;
        up_src(oy, s.H, y0, y1, fy);
        const float wy = (y0 == i ? 1.0f - fy : 0.0f) + (y1 == i ? fy : 0.0f);
        if (wy == 0.0f) continue;
        for (int ox = max(0, 2 * j - 2); ox <= min(Wo - 1, 2 * j + 3); ++ox) {
            int x0, x1;
            float fx;
            up_src(ox, s.W, x0, x1, fx);
            const float wx = (x0 == j ? 1.0f - fx : 0.0f) + (x1 == j ? fx : 0.0f);
            if (wx == 0.0f) continue;
            const bf16x8 v = load8(s.in + ((b * Ho + oy) * Wo + ox) * s.in_stride + s.in_off + c8 * 8);
            const float w = wy * wx;
#pragma unroll
            for (int q = 0; q < 8; ++q) acc[q] = acc[q] + w * (float)v[q];
        }
    }
    bf16x8 o;
#pragma unroll
    for (int q = 0; q < 8; ++q) o[q] = (__bf16)acc[q];
    *reinterpret_cast<bf16x8 *>(s.out + pi * s.out_stride + s.out_off + c8 * 8) = o;
}

// out[p] = 0.25 * pooled_grad[p / 2] + skip_grad[p]  (gradient of a level's
// output that feeds both the next level's pooling and a decoder concat)
// s.in = pooled grad [B][H/2][W/2], s.in2 = skip grad slice [B][H][W], s.out [B][H][W]
__global__ __launch_bounds__(256) void k_pool2_bwd_add(SliceArgs s)
{
    const int groups = s.C / 8;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t total = (int64_t)s.B * s.H * s.W * groups;
    if (t >= total) return;
    const int c8 = (int)(t % groups);
    const int64_t p = t / groups;
    const int64_t b = p / ((int64_t)s.H * s.W);
    const int64_t rem = p - b * s.H * s.W;
    const int y = (int)(rem / s.W), x = (int)(rem % s.W);
    const int64_t q = (b * (s.H / 2) + y / 2) * (s.W / 2) + x / 2;
    const bf16x8 g = load8(s.in + q * s.in_stride + s.in_off + c8 * 8);
    const bf16x8 k = load8(s.in2 + p * s.in2_stride + s.in2_off + c8 * 8);
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = (__bf16)(0.25f * (float)g[j] + (float)k[j]);
    *reinterpret_cast<bf16x8 *>(s.out + p * s.out_stride + s.out_off + c8 * 8) = o;
}

// ---------------------------------------------------------------------------
// weight gradient: dW[co][k] = sum_p dy_eff[p][co] * im2col(x)[p][k],
// db[co] = sum_p dy_eff[p][co], dy_eff = dy * (mask > 0) where a mask is given.
// Workgroup: 64 output channels x 64 k-columns over a pixel range (split-K);
// chunks of 32 pixels are staged transposed in LDS so that every MFMA
// operand is 8 consecutive pixels of one row.
// ---------------------------------------------------------------------------

constexpr int kWgPix = 64;  // pixels per LDS chunk (two MFMA K steps)

// LDS rows of 64 pixels (128 bytes) for one channel / im2col column; the 16-byte
// octets of pixels are XOR-swizzled by row so that the transposing 8-byte
// stores (rows 8 group + j) and the 16-byte fragment reads (16 consecutive
// rows) spread over the banks.  Returns the element offset of pixel quad q.
__device__ __forceinline__ int wg_at(int row, int q)
{
    const int f = (row ^ (row >> 3)) & 7;
    return row * kWgPix + (((q >> 1) ^ f) << 3) + ((q & 1) << 2);
}

// dW tile of TCO output channels x TK im2col columns per workgroup (64 x 128,
// or 32 x 256 for layers with 32 output channels), over the pixel range of
// its split; wave (wm, wn) computes channels 32 wm.. x columns 64 wn.. (2 x 4
// fragments), the pixels being the MFMA's K.
template <int TCO>
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a)
{
    constexpr int TK = 8192 / TCO;        // 128 or 256 columns
    constexpr int NWM = TCO / 32;         // waves along the channels
    __shared__ __attribute__((aligned(16))) __bf16 sdy[TCO * kWgPix];   // [co][pixel]
    __shared__ __attribute__((aligned(16))) __bf16 sx[TK * kWgPix];     // [k][pixel]
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int wm = wave % NWM, wn = wave / NWM;
    const int co0 = blockIdx.y * TCO;
    const int k0 = blockIdx.x * TK;
    const int64_t P = (int64_t)a.B * a.H * a.W;
    const int64_t pbeg = (int64_t)blockIdx.z * a.pix_per_split;
    const int64_t pend = min(P, pbeg + a.pix_per_split);
    const int K = a.KS * a.KS * a.Cin;
    const int hw = a.H * a.W;  // B * H * W < 2^31
    // staging roles: dy by threads 0 .. 2 TCO - 1 (pixel quad, group of 8
    // channels), the im2col columns by all 256 threads, TK / 128 groups of 8
    // columns each (pixel quad, column group)
    constexpr int XG = TK / 128;
    const int qd = threadIdx.x / (TCO / 8), cg = threadIdx.x % (TCO / 8);
    const int qx = threadIdx.x >> 4;
    int kg[XG], ty[XG], tx[XG], xstride[XG];
    bool kin[XG];
    const __bf16 *xsrc[XG];
#pragma unroll
    for (int h = 0; h < XG; ++h) {
        kg[h] = (threadIdx.x & 15) + 16 * h;
        const int kk = k0 + kg[h] * 8;
        int tap = 0, ci = 0;
        ty[h] = tx[h] = 0;
        kin[h] = kk < K;
        if (kin[h]) {
            tap = kk / a.Cin;
            ci = kk - tap * a.Cin;
            ty[h] = a.KS == 3 ? tap / 3 - 1 : 0;
            tx[h] = a.KS == 3 ? tap % 3 - 1 : 0;
        }
        const bool second = a.x2 && ci >= a.xCin1;
        xsrc[h] = second ? a.x2 + a.x2_off + (ci - a.xCin1) : a.x + a.x_off + ci;
        xstride[h] = second ? a.x2_stride : a.x_stride;
    }
    f32x4 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int f = 0; f < 4; ++f) acc[i][f] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float bsum = 0.0f;
    // the chunk's loads land in registers (dy, its mask and the im2col
    // columns) and go to LDS at the top of the next iteration, so the loads of
    // chunk c + 1 are in flight during the MFMAs of chunk c
    bf16x8 dv[4], dm[4], xv[XG][4];
    auto gload = [&](int64_t pc) {
        if (threadIdx.x < 2 * TCO) {
            const int c = co0 + cg * 8;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t p = pc + 4 * qd + e;
                dv[e] = zero8();
                dm[e] = zero8();
                if (p < pend && c < a.Cout) {
                    dv[e] = load8(a.dy + p * a.dy_stride + a.dy_off + c);
                    if (a.mask) dm[e] = load8(a.mask + p * a.mask_stride + a.mask_off + c);
                }
            }
        }
#pragma unroll
        for (int h = 0; h < XG; ++h) {
            const int64_t p0 = pc + 4 * qx;
            int b = (int)(p0 / hw);
            const int rem = (int)(p0 - (int64_t)b * hw);
            int y = rem / a.W;
            int x = rem - y * a.W;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                xv[h][e] = zero8();
                const int y2 = y + ty[h], x2 = x + tx[h];
                if (kin[h] && p0 + e < pend && y2 >= 0 && y2 < a.H && x2 >= 0 && x2 < a.W)
                    xv[h][e] = load8(xsrc[h] + (((int64_t)b * a.H + y2) * a.W + x2) * xstride[h]);
                if (++x == a.W) {  // next pixel (W >= 8, so at most one wrap in a quad)
                    x = 0;
                    if (++y == a.H) {
                        y = 0;
                        ++b;
                    }
                }
            }
        }
    };
    auto lstore = [&]() {
        if (threadIdx.x < 2 * TCO) {
            if (a.mask) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        if (!((float)dm[e][j] > 0.0f)) dv[e][j] = (__bf16)0.0f;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j)
                *reinterpret_cast<bf16x4 *>(&sdy[wg_at(cg * 8 + j, qd)]) =
                    bf16x4{dv[0][j], dv[1][j], dv[2][j], dv[3][j]};
        }
#pragma unroll
        for (int h = 0; h < XG; ++h)
#pragma unroll
            for (int j = 0; j < 8; ++j)
                *reinterpret_cast<bf16x4 *>(&sx[wg_at(kg[h] * 8 + j, qx)]) =
                    bf16x4{xv[h][0][j], xv[h][1][j], xv[h][2][j], xv[h][3][j]};
    };
    if (pbeg < pend) gload(pbeg);
    for (int64_t pc = pbeg; pc < pend; pc += kWgPix) {
        lstore();
        __syncthreads();
        if (pc + kWgPix < pend) gload(pc + kWgPix);
#pragma unroll
        for (int st = 0; st < kWgPix / 32; ++st) {
            // fragment lane (g, r): row r of the fragment, pixels 32 st + 8 g .. + 7
            const int q = 8 * st + 2 * g;
            bf16x8 av[2], bv[4];
#pragma unroll
            for (int i = 0; i < 2; ++i) av[i] = *reinterpret_cast<const bf16x8 *>(&sdy[wg_at(32 * wm + 16 * i + r, q)]);
#pragma unroll
            for (int f = 0; f < 4; ++f) bv[f] = *reinterpret_cast<const bf16x8 *>(&sx[wg_at(64 * wn + 16 * f + r, q)]);
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int f = 0; f < 4; ++f)
                    acc[i][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[f], acc[i][f], 0, 0, 0);
        }
        if (blockIdx.x == 0 && threadIdx.x < TCO) {
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                const bf16x8 t = *reinterpret_cast<const bf16x8 *>(&sdy[threadIdx.x * kWgPix + 8 * o]);
#pragma unroll
                for (int j = 0; j < 8; ++j) bsum = bsum + (float)t[j];
            }
        }
        __syncthreads();
    }
    // partial results: part[split][co][k] (fp32), reduced in split order later
    float *out = a.part + (int64_t)blockIdx.z * a.Cout_pad * a.Kpad;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int f = 0; f < 4; ++f)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int co = co0 + 32 * wm + 16 * i + 4 * g + e;
                const int k = k0 + 64 * wn + 16 * f + r;
                if (co < a.Cout_pad && k < a.Kpad) out[(int64_t)co * a.Kpad + k] = acc[i][f][e];
            }
    if (blockIdx.x == 0 && threadIdx.x < TCO && co0 + threadIdx.x < a.Cout_pad)
        a.bpart[(int64_t)blockIdx.z * a.Cout_pad + co0 + threadIdx.x] = bsum;
}

// sum the split partials (deterministic): 16 lanes per output element, lane
// j summing splits j, j + 16, ... in order, then the 16 lane sums added in
// lane order; one workgroup covers 16 consecutive outputs (threads 16 j + o),
// so a wave reads 16 consecutive outputs of 4 splits at a time
constexpr int kRedLanes = 16;

__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *part, const float *bpart, int splits,
                                                      int64_t nw, int nb, float *dw, float *db)
{
    __shared__ float sw[256], sb[256];
    const int j = threadIdx.x / 16, o = threadIdx.x % 16;
    const int64_t i = (int64_t)blockIdx.x * 16 + o;
    float w = 0.0f, bsum = 0.0f;
    if (i < nw)
        for (int z = j; z < splits; z += kRedLanes) w = w + part[(int64_t)z * nw + i];
    if (i < nb)
        for (int z = j; z < splits; z += kRedLanes) bsum = bsum + bpart[(int64_t)z * nb + i];
    sw[threadIdx.x] = w;
    sb[threadIdx.x] = bsum;
    __syncthreads();
    if (j == 0) {
        float t = 0.0f, u = 0.0f;
        for (int k = 0; k < kRedLanes; ++k) {
            t = t + sw[16 * k + o];
            u = u + sb[16 * k + o];
        }
        if (i < nw) dw[i] = t;
        if (i < nb) db[i] = u;
    }
}

// ---------------------------------------------------------------------------
// loss: mean squared error + lam * (mean |horizontal diff| + mean |vertical diff|)
// y, t planar fp32 [B][3][H][W]; grad written as NHWC bf16 [B*H*W][8] (channels
// 3..7 zero) for the head's backward; per-block partial sums of the loss.
// ---------------------------------------------------------------------------

// The scales are computed on the host: c_all = 1/(3P), c_mse = 2/(3P),
// c_hx = lam/(3B H (W-1)) and c_hy = lam/(3B (H-1) W) (0 when that difference
// does not exist).
__global__ __launch_bounds__(256) void k_loss(const float *y, const float *t, int B, int H, int W, float c_all,
                                              float c_mse, float c_hx, float c_hy, __bf16 *grad, float *partial)
{
    __shared__ float red[256];
    const int64_t hw = (int64_t)H * W;
    const int64_t P = (int64_t)B * hw;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float l = 0.0f;
    bf16x8 go = zero8();
    if (p < P) {
        const int64_t b = p / hw, pix = p - b * hw;
        const int yy = (int)(pix / W), xx = (int)(pix % W);
        for (int c = 0; c < 3; ++c) {
            const float *yc = y + (b * 3 + c) * hw;
            const float d = yc[pix] - t[(b * 3 + c) * hw + pix];
            float gsum = c_mse * d;
            l = l + d * d * c_all;
            if (xx + 1 < W) {
                const float h = yc[pix + 1] - yc[pix];
                l = l + fabsf(h) * c_hx;
                gsum = gsum - c_hx * (h > 0.0f ? 1.0f : (h < 0.0f ? -1.0f : 0.0f));
            }
            if (xx > 0) {
                const float h = yc[pix] - yc[pix - 1];
                gsum = gsum + c_hx * (h > 0.0f ? 1.0f : (h < 0.0f ? -1.0f : 0.0f));
            }
            if (yy + 1 < H) {
                const float h = yc[pix + W] - yc[pix];
                l = l + fabsf(h) * c_hy;
                gsum = gsum - c_hy * (h > 0.0f ? 1.0f : (h < 0.0f ? -1.0f : 0.0f));
            }
            if (yy > 0) {
                const float h = yc[pix] - yc[pix - W];
                gsum = gsum + c_hy * (h > 0.0f ? 1.0f : (h < 0.0f ? -1.0f : 0.0f));
            }
            go[c] = (__bf16)gsum;
        }
        *reinterpret_cast<bf16x8 *>(grad + p * 8) = go;
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_sum(const float *partial, int64_t n, float *out)
{
    __shared__ float red[256];
    float s = 0.0f;
    for (int64_t i = threadIdx.x; i < n; i += 256) s = s + partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// ---------------------------------------------------------------------------
// parameters: fp32 master copies -> bf16 forward and input-gradient matrices
// ---------------------------------------------------------------------------

// master W in the blob's [Cout][Cin][k][k] order
// device layouts use CinD >= Cin input channels (the ones past Cin are zero)
__global__ __launch_bounds__(256) void k_prep_weights(const float *master, int Cout, int Cin, int CinD, int KS,
                                                      __bf16 *fwd, int fwd_rows, int fwd_kpad, __bf16 *bwd,
                                                      int bwd_rows, int bwd_cin, int bwd_kpad)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nf = (int64_t)fwd_rows * fwd_kpad;
    const int64_t nb = (int64_t)bwd_rows * bwd_kpad;
    const int T = KS * KS;
    if (i < nf) {
        const int co = (int)(i / fwd_kpad), k = (int)(i % fwd_kpad);
        float v = 0.0f;
        if (co < Cout && k < T * CinD) {
            const int tap = k / CinD, ci = k % CinD;
            if (ci < Cin) v = master[((int64_t)co * Cin + ci) * T + tap];
        }
        fwd[i] = (__bf16)v;
    }
    if (bwd && i < nb) {
        // input-gradient conv: in-channels = Cout (padded to bwd_cin), out-channels = Cin,
        // taps flipped: Wb[ci][tap'][co] = W[co][ci][T - 1 - tap']
        const int ci = (int)(i / bwd_kpad), k = (int)(i % bwd_kpad);
        float v = 0.0f;
        if (ci < Cin && k < T * bwd_cin) {
            const int tapb = k / bwd_cin, co = k % bwd_cin;
            if (co < Cout) v = master[((int64_t)co * Cin + ci) * T + (T - 1 - tapb)];
        }
        bwd[i] = (__bf16)v;
    }
}

// Adam on the fp32 master parameters (blob order) with gradients in blob order
__global__ __launch_bounds__(256) void k_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                                              float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1;
    const float vh = vi / c2;
    p[i] = p[i] - lr * mh / (sqrtf(vh) + eps);
}

// gradient matrix [Cout_pad][Kpad] in (tap, ci) order -> blob order [Cout][Cin][k][k]
__global__ __launch_bounds__(256) void k_grad_to_blob(const float *dw, int Kpad, int Cout, int Cin, int CinD, int KS,
                                                      float *blob)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int T = KS * KS;
    if (i >= (int64_t)Cout * Cin * T) return;
    const int tap = (int)(i % T);
    const int ci = (int)((i / T) % Cin);
    const int co = (int)(i / ((int64_t)T * Cin));
    blob[i] = dw[(int64_t)co * Kpad + tap * CinD + ci];
}

__global__ __launch_bounds__(256) void k_copy_f32(const float *src, float *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_zero_bf16(__bf16 *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = (__bf16)0.0f;
}

// ---------------------------------------------------------------------------
// FP8 (OCP e4m3, largest finite 448) inference: per-output-channel weight
// scales, one static activation scale per layer input, fp32 accumulation.
// y = (sum_k q_w[co][k] * q_x[p][k]) * s_w[co] * s_a + b[co]
// ---------------------------------------------------------------------------

__device__ __forceinline__ float clamp448(float v) { return fminf(fmaxf(v, -448.0f), 448.0f); }

// per output row: s_w = max |W[co][k]| / 448 (1 for an all-zero row), q = fp8(W / s_w)
__global__ __launch_bounds__(256) void k_quant_weights(const float *master, int Cout, int Cin, int KS, int rows,
                                                       int kpad, uint8_t *wq, float *sw)
{
    __shared__ float red[256];
    const int co = blockIdx.x;
    const int T = KS * KS;
    float m = 0.0f;
    for (int k = threadIdx.x; k < kpad; k += 256) {
        if (co < Cout && k < T * Cin) {
            const int tap = k / Cin, ci = k % Cin;
            m = fmaxf(m, fabsf(master[((int64_t)co * Cin + ci) * T + tap]));
        }
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s2]);
        __syncthreads();
    }
    const float mx = red[0];
    const float scale = mx > 0.0f ? mx / 448.0f : 1.0f;
    if (threadIdx.x == 0) sw[co] = scale;
    for (int k = threadIdx.x; k < kpad; k += 256) {
        float v = 0.0f;
        if (co < Cout && k < T * Cin) {
            const int tap = k / Cin, ci = k % Cin;
            v = clamp448(master[((int64_t)co * Cin + ci) * T + tap] / scale);
        }
        const int b = __builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false);
        wq[(int64_t)co * kpad + k] = (uint8_t)(b & 0xFF);
    }
}

// max |x| over a bf16 buffer (order-free: atomic max on the bit pattern of a
// non-negative float)
__global__ __launch_bounds__(256) void k_absmax_bf16(const __bf16 *x, int64_t n, unsigned int *out)
{
    __shared__ float red[256];
    float m = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float v = fabsf((float)x[i]);
        if (v == v) m = fmaxf(m, v);
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s2]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, __float_as_uint(red[0]));
}

unsigned nblocks(int64_t n, int per = 256) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <bool FP8>
static hipError_t launch_conv(const ConvArgs &a, int KS, const uint8_t *wq, const float *sw, float sa, hipStream_t s)
{
    const int64_t P = (int64_t)a.B * a.H * a.W;
    const int cop = a.Cout_pad;
    if (a.head_out && (FP8 || KS != 3 || cop != 32 || a.Cin % 32 != 0 || a.out_f32)) return hipErrorInvalidValue;
    if (a.in2 && (a.in_mask || a.Cin1 <= 0 || a.Cin1 >= a.Cin || a.Cin1 % 8 != 0)) return hipErrorInvalidValue;
    // the upsampling input is read by the halo kernel only
    if (a.up_in && (KS != 3 || !a.in2 || a.Cin1 % 32 != 0 || a.Cin % 32 != 0 || a.out_f32 || a.in_mask ||
                    a.H % 2 || a.W % 2))
        return hipErrorInvalidValue;
    const unsigned gx = (unsigned)((a.W + kHaloCols - 1) / kHaloCols);
    const unsigned gy = (unsigned)((a.H + kHaloRows - 1) / kHaloRows);
    // the fused pooling is the halo kernel's
    const bool halo_ok = KS == 3 && a.Cin % 32 == 0 && (!a.in2 || a.Cin1 % 32 == 0) && !a.out_f32 &&
                         (FP8 ? cop % 64 == 0 && !a.in_mask : cop % 32 == 0) &&
                         (int64_t)a.B * (cop % 64 ? cop / 32 : cop / 64) <= 65535;
    if (a.pool_out && (!halo_ok || a.head_out || a.H % 2 || a.W % 2 || a.pool_stride % 4 || a.pool_off % 4))
        return hipErrorInvalidValue;
    if (a.gate) {
        if (FP8 || !halo_ok || cop % 64 || a.Cout != cop || a.in_mask || a.up_in || a.head_out) return hipErrorInvalidValue;
        const dim3 grid(gx, (unsigned)((a.H + 3) / 4), (unsigned)(a.B * (cop / 64)));
        hipLaunchKernelGGL((k_conv_halo<64, 4, false, false, false, false, true>), grid, dim3(512), 0, s, a, wq, sw, sa);
        return hipGetLastError();
    }
    // first layer (8 input channels, 32 output channels)
    if (!FP8 && KS == 3 && cop == 32 && a.Cin == 8 && a.Kpad == 96 && !a.in_mask && !a.in2 && !a.out_f32) {
        hipLaunchKernelGGL(k_conv_c8, dim3(gx, gy, (unsigned)a.B), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    // 3x3 layers with Cin a multiple of 32: direct convolution from halo tiles
    // (32 output channels per 8 waves and 8 rows, or 64 per 8 waves and 4
    // rows; FP8 for the latter)
    const bool halo = halo_ok;
    if (halo && cop % 64) {
        // tiles of 32 output channels (cop = 32, or 96 for an input gradient)
        const dim3 grid(gx, (unsigned)((a.H + 7) / 8), (unsigned)(a.B * (cop / 32)));
        if (a.head_out) {
            if (a.in_mask || a.Cout != 32 || cop != 32 || a.up_in) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_conv_halo<32, 8, false, true, false, false>), grid, dim3(512), 0, s, a, wq, sw, sa);
        } else if (a.in_mask) {
            hipLaunchKernelGGL((k_conv_halo<32, 8, true, false, false, false>), grid, dim3(512), 0, s, a, wq, sw, sa);
        } else if (a.up_in) {
            hipLaunchKernelGGL((k_conv_halo<32, 8, false, false, true, false>), grid, dim3(512), 0, s, a, wq, sw, sa);
        } else {
            hipLaunchKernelGGL((k_conv_halo<32, 8, false, false, false, false>), grid, dim3(512), 0, s, a, wq, sw, sa);
        }
        return hipGetLastError();
    }
    if (a.head_out) return hipErrorInvalidValue;
    if (halo) {
        const dim3 grid(gx, (unsigned)((a.H + 3) / 4), (unsigned)(a.B * (cop / 64)));
        if (a.in_mask)
            hipLaunchKernelGGL((k_conv_halo<64, 4, true, false, false, false>), grid, dim3(512), 0, s, a, wq, sw, sa);
        else if (a.up_in)
            hipLaunchKernelGGL((k_conv_halo<64, 4, false, false, true, FP8>), grid, dim3(512), 0, s, a, wq, sw, sa);
        else
            hipLaunchKernelGGL((k_conv_halo<64, 4, false, false, false, FP8>), grid, dim3(512), 0, s, a, wq, sw, sa);
        return hipGetLastError();
    }
    if (a.up_in) return hipErrorInvalidValue;
    // 1x1 layers with 64 or more output channels (the U-Net's transposed
    // convolutions, optionally written depth-to-space): LDS-staged tiles
    const bool lds1 = !FP8 && KS == 1 && cop % 64 == 0 && !a.out_f32 && !a.in_mask;
    if (a.shuffle && (!lds1 || a.Cout != cop || a.Cout % 16)) return hipErrorInvalidValue;
    if (lds1) {
        dim3 grid(nblocks(P, 128), cop / 64);
        hipLaunchKernelGGL((k_conv_lds<64, 128, 1, false, false>), grid, dim3(256), 0, s, a, wq, sw, sa);
        return hipGetLastError();
    }
    // other 3x3 layers with 64 or more output channels (FP8, or Cin not a
    // multiple of 32): LDS-staged im2col tiles
    if (KS == 3 && cop % 64 == 0) {
        dim3 grid(nblocks(P, 128), cop / 64);
        if (a.in_mask)
            hipLaunchKernelGGL((k_conv_lds<64, 128, 3, FP8, true>), grid, dim3(256), 0, s, a, wq, sw, sa);
        else
            hipLaunchKernelGGL((k_conv_lds<64, 128, 3, FP8, false>), grid, dim3(256), 0, s, a, wq, sw, sa);
        return hipGetLastError();
    }
    // wave tile: FCO x 16 output channels by FPX x 16 pixels
    if (cop % 64 == 0) {
        dim3 grid(nblocks(P, 32 * kWaves), cop / 64);
        if (KS == 3) hipLaunchKernelGGL((k_conv<4, 2, 3, FP8>), grid, dim3(64 * kWaves), 0, s, a, wq, sw, sa);
        else hipLaunchKernelGGL((k_conv<4, 2, 1, FP8>), grid, dim3(64 * kWaves), 0, s, a, wq, sw, sa);
    } else if (cop % 32 == 0) {
        dim3 grid(nblocks(P, 64 * kWaves), cop / 32);
        if (KS == 3) hipLaunchKernelGGL((k_conv<2, 4, 3, FP8>), grid, dim3(64 * kWaves), 0, s, a, wq, sw, sa);
        else hipLaunchKernelGGL((k_conv<2, 4, 1, FP8>), grid, dim3(64 * kWaves), 0, s, a, wq, sw, sa);
    } else {
        dim3 grid(nblocks(P, 64 * kWaves), cop / 16);
        if (KS == 3) hipLaunchKernelGGL((k_conv<1, 4, 3, FP8>), grid, dim3(64 * kWaves), 0, s, a, wq, sw, sa);
        else hipLaunchKernelGGL((k_conv<1, 4, 1, FP8>), grid, dim3(64 * kWaves), 0, s, a, wq, sw, sa);
    }
    return hipGetLastError();
}

hipError_t conv(const ConvArgs &a, int KS, hipStream_t s) { return launch_conv<false>(a, KS, nullptr, nullptr, 1.0f, s); }

hipError_t conv_fp8(const ConvArgs &a, int KS, const uint8_t *wq, const float *sw, float sa, hipStream_t s)
{
    return launch_conv<true>(a, KS, wq, sw, sa, s);
}

hipError_t quant_weights(const float *master, int Cout, int Cin, int KS, int rows, int kpad, uint8_t *wq, float *sw,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_quant_weights, dim3((unsigned)rows), dim3(256), 0, s, master, Cout, Cin, KS, rows, kpad, wq, sw);
    return hipGetLastError();
}

// max |a - b| over two fp32 buffers (NaN counts as +inf: a calibration that
// produced one must not pass)
__global__ __launch_bounds__(256) void k_absdiff_max(const float *a, const float *b, int64_t n, unsigned int *out)
{
    __shared__ float red[256];
    float m = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float d = fabsf(a[i] - b[i]);
        m = fmaxf(m, d == d ? d : __builtin_inff());
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s2 = 128; s2 > 0; s2 >>= 1) {
        if (threadIdx.x < s2) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s2]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, __float_as_uint(red[0]));
}

hipError_t absdiff_max_f32(const float *a, const float *b, int64_t n, unsigned int *out, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(k_absdiff_max, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, s, a, b, n, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// kernels of the paper's gated U-Net
// ---------------------------------------------------------------------------

// y = ELU(z[:, :C]) * sigmoid(z[:, C:]), z dense [P][2C], y a slice
__global__ __launch_bounds__(256) void k_gate(const __bf16 *z, __bf16 *y, int y_stride, int y_off, int C, int64_t P)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= P * C) return;
    const int64_t p = t / C;
    const int c = (int)(t - p * C);
    const float f = (float)z[p * 2 * C + c], g = (float)z[p * 2 * C + C + c];
    y[p * y_stride + y_off + c] = (__bf16)(elu1(f) * sigm(g));
}

// dz = [dy sigmoid(g) ELU'(f), dy ELU(f) sigmoid(g) (1 - sigmoid(g))]
__global__ __launch_bounds__(256) void k_gate_bwd(const __bf16 *z, const __bf16 *dy, int dy_stride, int dy_off,
                                                  __bf16 *dz, int C, int64_t P)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= P * C) return;
    const int64_t p = t / C;
    const int c = (int)(t - p * C);
    const float f = (float)z[p * 2 * C + c], g = (float)z[p * 2 * C + C + c];
    const float d = (float)dy[p * dy_stride + dy_off + c];
    const float sg = sigm(g);
    const float de = f > 0.0f ? 1.0f : expf(f);
    dz[p * 2 * C + c] = (__bf16)(d * sg * de);
    dz[p * 2 * C + C + c] = (__bf16)(d * elu1(f) * sg * (1.0f - sg));
}

// 2x2 average pooling of a slice [B][H][W][C] -> [B][H/2][W/2][C] (C multiple of 8)
__global__ __launch_bounds__(256) void k_pool2(SliceArgs s)
{
    const int groups = s.C / 8;
    const int H2 = s.H / 2, W2 = s.W / 2;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)s.B * H2 * W2 * groups) return;
    const int c8 = (int)(t % groups);
    const int64_t q = t / groups;
    const int64_t b = q / ((int64_t)H2 * W2);
    const int64_t rem = q - b * H2 * W2;
    const int y = (int)(rem / W2), x = (int)(rem % W2);
    const int64_t p00 = (b * s.H + 2 * y) * s.W + 2 * x;
    const bf16x8 a0 = load8(s.in + p00 * s.in_stride + s.in_off + c8 * 8);
    const bf16x8 a1 = load8(s.in + (p00 + 1) * s.in_stride + s.in_off + c8 * 8);
    const bf16x8 a2 = load8(s.in + (p00 + s.W) * s.in_stride + s.in_off + c8 * 8);
    const bf16x8 a3 = load8(s.in + (p00 + s.W + 1) * s.in_stride + s.in_off + c8 * 8);
    bf16x8 o;
#pragma unroll
    for (int j = 0; j < 8; ++j) o[j] = (__bf16)(0.25f * (((float)a0[j] + (float)a1[j]) + ((float)a2[j] + (float)a3[j])));
    *reinterpret_cast<bf16x8 *>(s.out + q * s.out_stride + s.out_off + c8 * 8) = o;
}

// adjoint of the depth-to-space step of the transposed convolution (a 1x1
// convolution with 4C outputs, row (2a + b) C + c, written to
// out[2i + a][2j + b][c]): in a slice of the high grid, out [B][H][W][4C]
// with out[i][j][(2a + b) C + c] = in[2i + a][2j + b][c]; s.H, s.W: the low grid
__global__ __launch_bounds__(256) void k_shuffle_down(SliceArgs s)
{
    const int groups = s.C / 8;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)s.B * s.H * s.W * 4 * groups) return;
    const int c8 = (int)(t % groups);
    const int64_t r = t / groups;
    const int ph = (int)(r % 4);
    const int64_t q = r / 4;
    const int64_t b = q / ((int64_t)s.H * s.W);
    const int64_t rem = q - b * s.H * s.W;
    const int i = (int)(rem / s.W), j = (int)(rem % s.W);
    const int a = ph >> 1, bb = ph & 1;
    const int64_t o = (b * 2 * s.H + 2 * i + a) * (2 * s.W) + 2 * j + bb;
    *reinterpret_cast<bf16x8 *>(s.out + q * s.out_stride + s.out_off + ph * s.C + c8 * 8) =
        load8(s.in + o * s.in_stride + s.in_off + c8 * 8);
}

// bias of the 4C rows of a transposed convolution from its C biases, and the
// C bias gradients from the 4C row gradients
// network input of an H x W frame on the zero-padded Hp x Wp grid (padded
// pixels are empty pixels: every channel 0); out [B][Hp][Wp][oc], the 8
// input channels then oc - 8 zero channels (oc a multiple of 8)
__global__ __launch_bounds__(256) void k_features_pad(const float *in, __bf16 *out, int B, int H, int W, int Hp, int Wp,
                                                      int oc)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= (int64_t)B * Hp * Wp) return;
    const int64_t b = p / ((int64_t)Hp * Wp);
    const int64_t rem = p - b * Hp * Wp;
    const int y = (int)(rem / Wp), x = (int)(rem % Wp);
    bf16x8 v = zero8();
    if (y < H && x < W) {
        const int64_t hw = (int64_t)H * W;
        const float *src = in + b * 8 * hw + (int64_t)y * W + x;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            float f = src[c * hw];
            if (c == 3) f = f > 0.0f ? 1.0f / f : 0.0f;
            v[c] = (__bf16)f;
        }
    }
    *reinterpret_cast<bf16x8 *>(out + p * oc) = v;
    for (int c = 8; c < oc; c += 8) *reinterpret_cast<bf16x8 *>(out + p * oc + c) = zero8();
}

// planar [B][C][Hp][Wp] fp32 -> its top-left [B][C][H][W]
__global__ __launch_bounds__(256) void k_crop_planes(const float *src, float *dst, int BC, int H, int W, int Hp, int Wp)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)BC * H * W) return;
    const int64_t bc = t / ((int64_t)H * W);
    const int64_t rem = t - bc * H * W;
    const int y = (int)(rem / W), x = (int)(rem % W);
    dst[t] = src[(bc * Hp + y) * Wp + x];
}

__global__ __launch_bounds__(256) void k_bias_phases(const float *b, int C, float *rows)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < 4 * C) rows[i] = b[i % C];
}

__global__ __launch_bounds__(256) void k_bias_grad_phases(const float *rows, int C, float *b)
{
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c < C) b[c] = ((rows[c] + rows[C + c]) + rows[2 * C + c]) + rows[3 * C + c];
}

hipError_t gate(const __bf16 *z, __bf16 *y, int y_stride, int y_off, int C, int64_t P, hipStream_t s)
{
    hipLaunchKernelGGL(k_gate, dim3(nblocks(P * C)), dim3(256), 0, s, z, y, y_stride, y_off, C, P);
    return hipGetLastError();
}

hipError_t gate_bwd(const __bf16 *z, const __bf16 *dy, int dy_stride, int dy_off, __bf16 *dz, int C, int64_t P,
                    hipStream_t s)
{
    hipLaunchKernelGGL(k_gate_bwd, dim3(nblocks(P * C)), dim3(256), 0, s, z, dy, dy_stride, dy_off, dz, C, P);
    return hipGetLastError();
}

hipError_t pool2(const SliceArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_pool2, dim3(nblocks((int64_t)a.B * (a.H / 2) * (a.W / 2) * (a.C / 8))), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t shuffle_down(const SliceArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_shuffle_down, dim3(nblocks((int64_t)a.B * a.H * a.W * 4 * (a.C / 8))), dim3(256), 0, s, a);
    return hipGetLastError();
}

// wg row d = w row (first half of z: 16 q + t for t < 16, second half:
// rows / 2 + 16 q + t - 16), q = d / 32, t = d % 32
__global__ __launch_bounds__(256) void k_gate_rows(const __bf16 *w, const float *b, int rows, int kpad, __bf16 *wg,
                                                   float *bg)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= (int64_t)rows * kpad) return;
    const int d = (int)(i / kpad), k = (int)(i - (int64_t)d * kpad);
    const int q = d >> 5, t = d & 31;
    const int src = t < 16 ? 16 * q + t : rows / 2 + 16 * q + (t - 16);
    wg[i] = w[(int64_t)src * kpad + k];
    if (k == 0) bg[d] = b[src];
}

hipError_t gate_rows(const __bf16 *w, const float *b, int rows, int kpad, __bf16 *wg, float *bg, hipStream_t s)
{
    if (rows % 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gate_rows, dim3(nblocks((int64_t)rows * kpad)), dim3(256), 0, s, w, b, rows, kpad, wg, bg);
    return hipGetLastError();
}

hipError_t features_pad(const float *in, __bf16 *out, int B, int H, int W, int Hp, int Wp, int oc, hipStream_t s)
{
    if (oc < 8 || oc % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_features_pad, dim3(nblocks((int64_t)B * Hp * Wp)), dim3(256), 0, s, in, out, B, H, W, Hp, Wp,
                       oc);
    return hipGetLastError();
}

hipError_t crop_planes(const float *src, float *dst, int BC, int H, int W, int Hp, int Wp, hipStream_t s)
{
    hipLaunchKernelGGL(k_crop_planes, dim3(nblocks((int64_t)BC * H * W)), dim3(256), 0, s, src, dst, BC, H, W, Hp, Wp);
    return hipGetLastError();
}

hipError_t bias_phases(const float *b, int C, float *rows, hipStream_t s)
{
    hipLaunchKernelGGL(k_bias_phases, dim3((unsigned)((4 * C + 255) / 256)), dim3(256), 0, s, b, C, rows);
    return hipGetLastError();
}

hipError_t bias_grad_phases(const float *rows, int C, float *b, hipStream_t s)
{
    hipLaunchKernelGGL(k_bias_grad_phases, dim3((unsigned)((C + 255) / 256)), dim3(256), 0, s, rows, C, b);
    return hipGetLastError();
}

hipError_t absmax_bf16(const __bf16 *x, int64_t n, unsigned int *out, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(k_absmax_bf16, dim3((unsigned)(blocks > 0 ? blocks : 1)), dim3(256), 0, s, x, n, out);
    return hipGetLastError();
}

hipError_t features(const float *in, __bf16 *out, int B, int H, int W, hipStream_t s)
{
    const int64_t P = (int64_t)B * H * W;
    hipLaunchKernelGGL(k_features, dim3(nblocks(P)), dim3(256), 0, s, in, out, P, (int64_t)H * W);
    return hipGetLastError();
}

// grid for the row-walking kernels: x covers one row's (pixel, group) pairs
static dim3 row_grid(int64_t row_items, int64_t rows)
{
    return dim3(nblocks(row_items), (unsigned)std::min<int64_t>(rows, 65535));
}

hipError_t upsample2(const SliceArgs &a, hipStream_t s)
{
    if ((int64_t)a.B * a.H * a.W == 0) return hipSuccess;
    hipLaunchKernelGGL(k_upsample2, row_grid((int64_t)(2 * a.W) * (a.C / 8), (int64_t)a.B * 2 * a.H), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t upsample2_bwd(const SliceArgs &a, hipStream_t s)
{
    const int64_t n = (int64_t)a.B * a.H * a.W * (a.C / 8);
    hipLaunchKernelGGL(k_upsample2_bwd, dim3(nblocks(n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t pool2_bwd_add(const SliceArgs &a, hipStream_t s)
{
    const int64_t n = (int64_t)a.B * a.H * a.W * (a.C / 8);
    hipLaunchKernelGGL(k_pool2_bwd_add, dim3(nblocks(n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t wgrad(const WgradArgs &a, float *dw, float *db, hipStream_t s)
{
    if (a.Cout_pad <= 32) {
        dim3 grid((unsigned)((a.Kpad + 255) / 256), 1u, (unsigned)a.splits);
        hipLaunchKernelGGL(k_wgrad<32>, grid, dim3(256), 0, s, a);
    } else {
        dim3 grid((unsigned)((a.Kpad + 127) / 128), (unsigned)((a.Cout_pad + 63) / 64), (unsigned)a.splits);
        hipLaunchKernelGGL(k_wgrad<64>, grid, dim3(256), 0, s, a);
    }
    const int64_t nw = (int64_t)a.Cout_pad * a.Kpad;
    const int64_t nout = nw > a.Cout_pad ? nw : a.Cout_pad;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(nblocks(nout, 16)), dim3(256), 0, s, a.part, a.bpart, a.splits,
                       nw, a.Cout_pad, dw, db);
    return hipGetLastError();
}

hipError_t loss(const float *y, const float *t, int B, int H, int W, float lam, __bf16 *grad, float *partial,
                float *out, hipStream_t s)
{
    const int64_t P = (int64_t)B * H * W;
    const unsigned nb = nblocks(P);
    const double n_all = 3.0 * (double)P;
    const double n_hx = 3.0 * (double)B * H * (W - 1);
    const double n_hy = 3.0 * (double)B * (H - 1) * W;
    const float c_all = (float)(1.0 / n_all);
    const float c_mse = (float)(2.0 / n_all);
    const float c_hx = W > 1 ? (float)((double)lam / n_hx) : 0.0f;
    const float c_hy = H > 1 ? (float)((double)lam / n_hy) : 0.0f;
    hipLaunchKernelGGL(k_loss, dim3(nb), dim3(256), 0, s, y, t, B, H, W, c_all, c_mse, c_hx, c_hy, grad, partial);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, partial, (int64_t)nb, out);
    return hipGetLastError();
}

hipError_t prep_weights(const float *master, int Cout, int Cin, int KS, __bf16 *fwd, int fwd_rows, int fwd_kpad,
                        __bf16 *bwd, int bwd_rows, int bwd_cin, int bwd_kpad, hipStream_t s, int CinD)
{
    const int64_t nf = (int64_t)fwd_rows * fwd_kpad, nb = bwd ? (int64_t)bwd_rows * bwd_kpad : 0;
    hipLaunchKernelGGL(k_prep_weights, dim3(nblocks(nf > nb ? nf : nb)), dim3(256), 0, s, master, Cout, Cin,
                       CinD > 0 ? CinD : Cin, KS, fwd, fwd_rows, fwd_kpad, bwd, bwd_rows, bwd_cin, bwd_kpad);
    return hipGetLastError();
}

hipError_t adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3(nblocks(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t grad_to_blob(const float *dw, int Kpad, int Cout, int Cin, int KS, float *blob, hipStream_t s, int CinD)
{
    const int64_t n = (int64_t)Cout * Cin * KS * KS;
    hipLaunchKernelGGL(k_grad_to_blob, dim3(nblocks(n)), dim3(256), 0, s, dw, Kpad, Cout, Cin, CinD > 0 ? CinD : Cin,
                       KS, blob);
    return hipGetLastError();
}

hipError_t copy_f32(const float *src, float *dst, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_f32, dim3(nblocks(n)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t zero_bf16(__bf16 *p, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_bf16, dim3(nblocks(n)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace net
}  // namespace narvis

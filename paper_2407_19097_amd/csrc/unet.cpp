// The paper's own post-processing network (Sec. 3.3, Fig. 4): a gated U-Net
// with 1x1-convolution G-buffer descriptors injected at five scales.
//
//   descriptors  d_0 = conv1x1(x_0) (8 -> 8 channels, bias), d_l = avgpool2(d_{l-1});
//   encoder      level l = 0..4: z = conv3x3([x_l | d_l]) with 2 w_l outputs,
//                y_l = ELU(z[:w_l]) * sigmoid(z[w_l:]), x_{l+1} = avgpool2(y_l);
//   decoder      level l = 3..0: u = convT2x2 stride 2 (w_{l+1} -> w_l) of the
//                level above, z = conv3x3([u | y_l]), y'_l = gate(z);
//   head         conv1x1(w_0 -> 3), linear.
//
// Every convolution runs on the small network's matrix-core kernels (bf16
// operands, fp32 accumulation, NHWC activations); a concatenated input is
// read from two tensors.  The encoder's descriptor channels are carried in
// 32-channel tensors (8 channels and 24 zeros; level 0 holds the 8 input
// channels, the 8 descriptor channels and 16 zeros) so that every 3x3 layer
// reads whole 32-channel groups and runs on the direct halo-tile kernel; the
// device weights have zero columns there.  In inference the gate (and the
// encoder's pooling) is the convolution's epilogue, on weights whose rows are
// stored in gate order.  The transposed convolution is a 1x1 convolution
// with 4 w_l outputs (one block per output phase) followed by a depth-to-
// space copy.  Training: MSE + TV loss, backward through every layer with
// the same kernels (input gradients on flipped weights, weight gradients by
// split-K), Adam on fp32 master parameters.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "narvis.h"
#include "net_internal.h"

using namespace narvis;
using namespace narvis::net;

namespace {

constexpr int kLevels = 5;
constexpr int kUL = 15;  // desc, enc0..enc4, up3, dec3, up2, dec2, up1, dec1, up0, dec0, head
enum { U_DESC = 0, U_ENC0 = 1, U_HEAD = 14 };
int u_up(int l) { return 6 + 2 * (3 - l); }   // up3 = 6, up2 = 8, up1 = 10, up0 = 12
int u_dec(int l) { return 7 + 2 * (3 - l); }  // dec3 = 7, ..., dec0 = 13

enum { K_GATE3 = 0, K_TCONV = 1, K_CONV1 = 2 };

int round_up(int v, int m) { return (v + m - 1) / m * m; }
uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

struct ULayer {
    int kind, cin, cout, ks;       // the convolution's view (gate3: 2 w outputs; tconv: 4 w)
    int cind;                      // input channels of the device layouts (>= cin, the rest zero)
    int rows, kpad, bcin, brows, bkpad;
    int nbias;                     // biases in the blob (tconv: w, not 4 w)
    int64_t blob_w, blob_b;
    __bf16 *wf, *wb, *wg;          // wg: gate3 forward weights in gate order (inference)
    float *bias, *dw, *db, *bg;
};

bool widths_ok(const int32_t *w)
{
    if (!w) return false;
    for (int l = 0; l < kLevels; ++l)
        if (w[l] < 32 || w[l] > 4096 || w[l] % 32) return false;
    return true;
}

// device input channels of encoder level l: [x_l | d_l] with the 8
// descriptor channels in a 32-channel group (level 0: one 32-channel group
// holding the 8 input and the 8 descriptor channels)
int enc_cind(const int32_t *w, int l) { return l ? w[l - 1] + 32 : 32; }

void describe(const int32_t *w, ULayer *L)
{
    auto set = [](ULayer &l, int kind, int cin, int cind, int cout, int ks, int nbias) {
        l.kind = kind;
        l.cin = cin;
        l.cind = cind;
        l.cout = cout;
        l.ks = ks;
        l.nbias = nbias;
        l.rows = round_up(cout, 16);
        l.kpad = round_up(ks * ks * cind, 32);
        l.bcin = round_up(cout, 8);
        l.brows = round_up(cind, 16);
        l.bkpad = round_up(ks * ks * l.bcin, 32);
    };
    set(L[U_DESC], K_CONV1, 8, 8, 8, 1, 8);
    for (int l = 0; l < kLevels; ++l)
        set(L[U_ENC0 + l], K_GATE3, (l ? w[l - 1] : 8) + 8, enc_cind(w, l), 2 * w[l], 3, 2 * w[l]);
    for (int l = 3; l >= 0; --l) {
        set(L[u_up(l)], K_TCONV, w[l + 1], w[l + 1], 4 * w[l], 1, w[l]);
        set(L[u_dec(l)], K_GATE3, 2 * w[l], 2 * w[l], 2 * w[l], 3, 2 * w[l]);
    }
    set(L[U_HEAD], K_CONV1, w[0], w[0], 3, 1, 3);
    int64_t o = 0;
    for (int i = 0; i < kUL; ++i) {
        L[i].blob_w = o;
        o += (int64_t)L[i].cout * L[i].cin * L[i].ks * L[i].ks;
        L[i].blob_b = o;
        o += L[i].nbias;
    }
}

int64_t count_params(const int32_t *w)
{
    ULayer L[kUL];
    describe(w, L);
    return L[kUL - 1].blob_b + L[kUL - 1].nbias;
}

}  // namespace

struct narvis_unet {
    int device;
    int32_t w[kLevels];
    ULayer L[kUL];
    int64_t nparams;
    float *master, *grad, *m, *v;
    void *pool;
    int64_t step;
};

namespace {

// Workspace plan for B images of H x W, run on the grid padded to multiples
// of 16 (Hp x Wp).
struct UPlan {
    int B, H, W, Hp, Wp;
    int64_t P[kLevels];
    uint64_t x0, d[kLevels], dzero, dzero_end, x[kLevels], ez[kLevels], ey[kLevels], u[4], dz[4], dy[4];
    uint64_t out;
    uint64_t gy, g_dy[4], g_ey4, g_dz[4], g_dcat[4], g_tz[4], g_ey[4], g_ez[kLevels], g_ecat[kLevels], g_d[4];
    uint64_t part, bpart, lpart;
    uint64_t bytes;
};

int wgrad_splits(int rows, int kpad, int64_t P, int64_t *per)
{
    const int tiles = rows <= 32 ? (kpad + 255) / 256 : ((kpad + 127) / 128) * ((rows + 63) / 64);
    int64_t splits = std::min<int64_t>(1024, std::max<int64_t>(1, (2048 + tiles - 1) / tiles));
    int64_t pp = (P + splits - 1) / splits;
    pp = (pp + 63) / 64 * 64;
    *per = pp;
    return (int)((P + pp - 1) / pp);
}

int layer_level(int i)
{
    if (i == U_DESC || i == U_HEAD) return 0;
    if (i >= U_ENC0 && i < U_ENC0 + kLevels) return i - U_ENC0;
    for (int l = 0; l < 4; ++l) {
        if (i == u_up(l)) return l + 1;  // runs on the low grid
        if (i == u_dec(l)) return l;
    }
    return 0;
}

UPlan make_uplan(const narvis_unet *u, int B, int H, int W, bool train)
{
    UPlan p{};
    p.B = B;
    p.H = H;
    p.W = W;
    p.Hp = round_up(H, 16);
    p.Wp = round_up(W, 16);
    for (int l = 0; l < kLevels; ++l) p.P[l] = (int64_t)B * (p.Hp >> l) * (p.Wp >> l);
    const int32_t *w = u->w;
    uint64_t o = 0;
    auto bf = [&](int64_t px, int ch) {
        const uint64_t at = o;
        o = align256(o + (uint64_t)px * ch * 2);
        return at;
    };
    p.x0 = bf(p.P[0], 32);  // [input (8) | d_0 (8) | 0 (16)]
    p.dzero = o;
    for (int l = 1; l < kLevels; ++l) p.d[l] = bf(p.P[l], 32);  // [d_l (8) | 0 (24)]
    p.dzero_end = o;
    for (int l = 1; l < kLevels; ++l) p.x[l] = bf(p.P[l], w[l - 1]);
    for (int l = 0; l < kLevels; ++l) {
        p.ez[l] = bf(p.P[l], 2 * w[l]);
        p.ey[l] = bf(p.P[l], w[l]);
    }
    for (int l = 0; l < 4; ++l) {
        p.u[l] = bf(p.P[l], w[l]);
        p.dz[l] = bf(p.P[l], 2 * w[l]);
        p.dy[l] = bf(p.P[l], w[l]);
    }
    p.out = o;
    o = align256(o + (uint64_t)p.P[0] * 3 * 4);
    if (train) {
        p.gy = bf(p.P[0], 8);
        for (int l = 0; l < 4; ++l) {
            p.g_dy[l] = bf(p.P[l], w[l]);
            p.g_dz[l] = bf(p.P[l], 2 * w[l]);
            p.g_dcat[l] = bf(p.P[l], 2 * w[l]);
            p.g_tz[l] = bf(p.P[l + 1], 4 * w[l]);
            p.g_ey[l] = bf(p.P[l], w[l]);
            p.g_d[l] = bf(p.P[l], 8);
        }
        p.g_ey4 = bf(p.P[4], w[4]);
        for (int l = 0; l < kLevels; ++l) {
            p.g_ez[l] = bf(p.P[l], 2 * w[l]);
            p.g_ecat[l] = bf(p.P[l], enc_cind(w, l));
        }
        int64_t pf = 0, bfl = 0;
        for (int i = 0; i < kUL; ++i) {
            const ULayer &l = u->L[i];
            int64_t per;
            const int splits = wgrad_splits(l.rows, l.kpad, p.P[layer_level(i)], &per);
            pf = std::max<int64_t>(pf, (int64_t)splits * l.rows * l.kpad);
            bfl = std::max<int64_t>(bfl, (int64_t)splits * l.rows);
        }
        p.part = o;
        o = align256(o + (uint64_t)pf * 4);
        p.bpart = o;
        o = align256(o + (uint64_t)bfl * 4);
        p.lpart = o;
        o = align256(o + (uint64_t)((p.P[0] + 255) / 256 + 1) * 4);
    }
    p.bytes = o;
    return p;
}

#define TRY(x)                                  \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

struct UCtx {
    char *ws;
    __bf16 *b(uint64_t off) const { return reinterpret_cast<__bf16 *>(ws + off); }
};

ConvArgs uconv(const ULayer &l, const __bf16 *in, int in_stride, int cin1, const __bf16 *in2, int in2_stride,
               __bf16 *out, int B, int H, int W)
{
    ConvArgs a{};
    a.in = in;
    a.in_stride = in_stride;
    a.Cin = l.cind;
    if (in2) {
        a.in2 = in2;
        a.in2_stride = in2_stride;
        a.Cin1 = cin1;
    }
    a.wt = l.wf;
    a.Kpad = l.kpad;
    a.bias = l.bias;
    a.Cout = l.cout;
    a.Cout_pad = l.rows;
    a.B = B;
    a.H = H;
    a.W = W;
    a.out = out;
    a.out_stride = l.cout;
    return a;
}

SliceArgs uslice(const __bf16 *in, int is, int io, __bf16 *out, int os, int oo, int C, int B, int H, int W)
{
    SliceArgs s{};
    s.in = in;
    s.in_stride = is;
    s.in_off = io;
    s.out = out;
    s.out_stride = os;
    s.out_off = oo;
    s.C = C;
    s.B = B;
    s.H = H;
    s.W = W;
    return s;
}

// fused: inference (gates and encoder pooling in the convolutions'
// epilogues, z never stored); otherwise every z is kept for the backward pass
hipError_t uforward(const narvis_unet *u, const float *feat_planes, char *ws, const UPlan &p, float *img, bool fused,
                    hipStream_t s)
{
    UCtx c{ws};
    const int B = p.B;
    const int32_t *w = u->w;
    const ULayer *L = u->L;
    auto Hl = [&](int l) { return p.Hp >> l; };
    auto Wl = [&](int l) { return p.Wp >> l; };
    TRY(features_pad(feat_planes, c.b(p.x0), B, p.H, p.W, p.Hp, p.Wp, 32, s));
    // descriptors at five scales: d_0 into channels 8..15 of the level-0 input
    ConvArgs dc = uconv(L[U_DESC], c.b(p.x0), 32, 0, nullptr, 0, c.b(p.x0), B, p.Hp, p.Wp);
    dc.out_stride = 32;
    dc.out_off = 8;
    TRY(conv(dc, 1, s));
    TRY(zero_bf16(c.b(p.dzero), (int64_t)(p.dzero_end - p.dzero) / 2, s));
    TRY(pool2(uslice(c.b(p.x0), 32, 8, c.b(p.d[1]), 32, 0, 8, B, Hl(0), Wl(0)), s));
    for (int l = 2; l < kLevels; ++l)
        TRY(pool2(uslice(c.b(p.d[l - 1]), 32, 0, c.b(p.d[l]), 32, 0, 8, B, Hl(l - 1), Wl(l - 1)), s));
    // encoder
    for (int l = 0; l < kLevels; ++l) {
        const ULayer &ly = L[U_ENC0 + l];
        ConvArgs a = l ? uconv(ly, c.b(p.x[l]), w[l - 1], w[l - 1], c.b(p.d[l]), 32, c.b(p.ez[l]), B, Hl(l), Wl(l))
                       : uconv(ly, c.b(p.x0), 32, 0, nullptr, 0, c.b(p.ez[l]), B, Hl(l), Wl(l));
        if (fused) {
            a.gate = 1;
            a.wt = ly.wg;
            a.bias = ly.bg;
            a.out = c.b(p.ey[l]);
            a.out_stride = w[l];
            if (l + 1 < kLevels) {
                a.pool_out = c.b(p.x[l + 1]);
                a.pool_stride = w[l];
            }
            TRY(conv(a, 3, s));
            continue;
        }
        TRY(conv(a, 3, s));
        TRY(gate(c.b(p.ez[l]), c.b(p.ey[l]), w[l], 0, w[l], p.P[l], s));
        if (l + 1 < kLevels)
            TRY(pool2(uslice(c.b(p.ey[l]), w[l], 0, c.b(p.x[l + 1]), w[l], 0, w[l], B, Hl(l), Wl(l)), s));
    }
    // decoder
    const __bf16 *up_in = c.b(p.ey[4]);
    for (int l = 3; l >= 0; --l) {
        const ULayer &ly = L[u_dec(l)];
        // transposed convolution: 1x1 with 4 w_l outputs written depth-to-space
        ConvArgs t = uconv(L[u_up(l)], up_in, w[l + 1], 0, nullptr, 0, c.b(p.u[l]), B, Hl(l + 1), Wl(l + 1));
        t.shuffle = 1;
        t.out_stride = w[l];
        TRY(conv(t, 1, s));
        ConvArgs a = uconv(ly, c.b(p.u[l]), w[l], w[l], c.b(p.ey[l]), w[l], c.b(p.dz[l]), B, Hl(l), Wl(l));
        if (fused) {
            a.gate = 1;
            a.wt = ly.wg;
            a.bias = ly.bg;
            a.out = c.b(p.dy[l]);
            a.out_stride = w[l];
            TRY(conv(a, 3, s));
        } else {
            TRY(conv(a, 3, s));
            TRY(gate(c.b(p.dz[l]), c.b(p.dy[l]), w[l], 0, w[l], p.P[l], s));
        }
        up_in = c.b(p.dy[l]);
    }
    ConvArgs h = uconv(L[U_HEAD], c.b(p.dy[0]), w[0], 0, nullptr, 0, nullptr, B, p.Hp, p.Wp);
    const bool padded = p.Hp != p.H || p.Wp != p.W;
    h.out_f32 = padded ? reinterpret_cast<float *>(ws + p.out) : img;
    TRY(conv(h, 1, s));
    if (padded) TRY(crop_planes(h.out_f32, img, B * 3, p.H, p.W, p.Hp, p.Wp, s));
    return hipSuccess;
}

// weight gradient (and, when dx is given, input gradient) of one layer
hipError_t ulayer_backward(const ULayer &l, const __bf16 *dy, int dy_stride, const __bf16 *x, int x_stride,
                           const __bf16 *x2, int x2_stride, int xcin1, __bf16 *dx, int B, int H, int W,
                           const UPlan &p, char *ws, hipStream_t s)
{
    WgradArgs a{};
    a.dy = dy;
    a.dy_stride = dy_stride;
    a.x = x;
    a.x_stride = x_stride;
    a.x2 = x2;
    a.x2_stride = x2_stride;
    a.xCin1 = x2 ? xcin1 : 0;
    a.Cin = l.cind;
    a.KS = l.ks;
    a.Cout = l.cout;
    a.Cout_pad = l.rows;
    a.Kpad = l.kpad;
    a.B = B;
    a.H = H;
    a.W = W;
    const int64_t P = (int64_t)B * H * W;
    int64_t per;
    a.splits = wgrad_splits(l.rows, l.kpad, P, &per);
    a.pix_per_split = per;
    a.part = reinterpret_cast<float *>(ws + p.part);
    a.bpart = reinterpret_cast<float *>(ws + p.bpart);
    TRY(wgrad(a, l.dw, l.db, s));
    if (dx) {
        ConvArgs c{};
        c.in = dy;
        c.in_stride = dy_stride;
        c.Cin = l.bcin;
        c.wt = l.wb;
        c.Kpad = l.bkpad;
        c.Cout = l.cind;
        c.Cout_pad = l.brows;
        c.B = B;
        c.H = H;
        c.W = W;
        c.out = dx;
        c.out_stride = l.cind;
        TRY(conv(c, l.ks, s));
    }
    return hipSuccess;
}

hipError_t ubackward(const narvis_unet *u, char *ws, const UPlan &p, hipStream_t s)
{
    UCtx c{ws};
    const int B = p.B;
    const int32_t *w = u->w;
    const ULayer *L = u->L;
    auto Hl = [&](int l) { return p.Hp >> l; };
    auto Wl = [&](int l) { return p.Wp >> l; };
    // head: loss gradient [P][8] (3 channels used)
    TRY(ulayer_backward(L[U_HEAD], c.b(p.gy), 8, c.b(p.dy[0]), w[0], nullptr, 0, 0, c.b(p.g_dy[0]), B, p.Hp, p.Wp, p, ws,
                        s));
    // decoder, from level 0 back up
    for (int l = 0; l < 4; ++l) {
        TRY(gate_bwd(c.b(p.dz[l]), c.b(p.g_dy[l]), w[l], 0, c.b(p.g_dz[l]), w[l], p.P[l], s));
        TRY(ulayer_backward(L[u_dec(l)], c.b(p.g_dz[l]), 2 * w[l], c.b(p.u[l]), w[l], c.b(p.ey[l]), w[l], w[l],
                            c.b(p.g_dcat[l]), B, Hl(l), Wl(l), p, ws, s));
        TRY(shuffle_down(uslice(c.b(p.g_dcat[l]), 2 * w[l], 0, c.b(p.g_tz[l]), 4 * w[l], 0, w[l], B, Hl(l + 1),
                                Wl(l + 1)),
                         s));
        const __bf16 *up_in = l == 3 ? c.b(p.ey[4]) : c.b(p.dy[l + 1]);
        __bf16 *g_up_in = l == 3 ? c.b(p.g_ey4) : c.b(p.g_dy[l + 1]);
        TRY(ulayer_backward(L[u_up(l)], c.b(p.g_tz[l]), 4 * w[l], up_in, w[l + 1], nullptr, 0, 0, g_up_in, B,
                            Hl(l + 1), Wl(l + 1), p, ws, s));
    }
    // encoder, deepest first
    for (int l = kLevels - 1; l >= 0; --l) {
        const int cprev = l ? w[l - 1] : 8;
        const __bf16 *gy_l;
        if (l == kLevels - 1) {
            gy_l = c.b(p.g_ey4);
        } else {
            // pooled path from the level below + the skip part of the decoder's input gradient
            SliceArgs a = uslice(c.b(p.g_ecat[l + 1]), enc_cind(w, l + 1), 0, c.b(p.g_ey[l]), w[l], 0, w[l], B, Hl(l),
                                 Wl(l));
            a.in2 = c.b(p.g_dcat[l]);
            a.in2_stride = 2 * w[l];
            a.in2_off = w[l];
            TRY(pool2_bwd_add(a, s));
            gy_l = c.b(p.g_ey[l]);
        }
        TRY(gate_bwd(c.b(p.ez[l]), gy_l, w[l], 0, c.b(p.g_ez[l]), w[l], p.P[l], s));
        if (l)
            TRY(ulayer_backward(L[U_ENC0 + l], c.b(p.g_ez[l]), 2 * w[l], c.b(p.x[l]), cprev, c.b(p.d[l]), 32, cprev,
                                c.b(p.g_ecat[l]), B, Hl(l), Wl(l), p, ws, s));
        else
            TRY(ulayer_backward(L[U_ENC0], c.b(p.g_ez[0]), 2 * w[0], c.b(p.x0), 32, nullptr, 0, 0, c.b(p.g_ecat[0]), B,
                                Hl(0), Wl(0), p, ws, s));
    }
    // descriptors: d_l = pool^l(d_0), so the gradient of d_0 sums every scale's
    // (d_l sits after the cprev_l = w_{l-1} (level 0: 8) channels of x_l)
    for (int l = kLevels - 2; l >= 0; --l) {
        SliceArgs a = l == kLevels - 2 ? uslice(c.b(p.g_ecat[l + 1]), enc_cind(w, l + 1), w[l], c.b(p.g_d[l]), 8, 0, 8,
                                                B, Hl(l), Wl(l))
                                       : uslice(c.b(p.g_d[l + 1]), 8, 0, c.b(p.g_d[l]), 8, 0, 8, B, Hl(l), Wl(l));
        a.in2 = c.b(p.g_ecat[l]);
        a.in2_stride = enc_cind(w, l);
        a.in2_off = l ? w[l - 1] : 8;
        TRY(pool2_bwd_add(a, s));
    }
    TRY(ulayer_backward(L[U_DESC], c.b(p.g_d[0]), 8, c.b(p.x0), 32, nullptr, 0, 0, nullptr, B, p.Hp, p.Wp, p, ws, s));
    // gradient matrices -> blob order
    for (int i = 0; i < kUL; ++i) {
        const ULayer &l = L[i];
        TRY(grad_to_blob(l.dw, l.kpad, l.cout, l.cin, l.ks, u->grad + l.blob_w, s, l.cind));
        if (l.kind == K_TCONV)
            TRY(bias_grad_phases(l.db, l.nbias, u->grad + l.blob_b, s));
        else
            TRY(copy_f32(l.db, u->grad + l.blob_b, l.nbias, s));
    }
    return hipSuccess;
}

hipError_t urefresh(narvis_unet *u, hipStream_t s)
{
    for (int i = 0; i < kUL; ++i) {
        ULayer &l = u->L[i];
        TRY(prep_weights(u->master + l.blob_w, l.cout, l.cin, l.ks, l.wf, l.rows, l.kpad, l.wb, l.brows, l.bcin,
                         l.bkpad, s, l.cind));
        if (l.kind == K_TCONV)
            TRY(bias_phases(u->master + l.blob_b, l.nbias, l.bias, s));
        else
            TRY(copy_f32(u->master + l.blob_b, l.bias, l.nbias, s));
        if (l.kind == K_GATE3) TRY(gate_rows(l.wf, l.bias, l.rows, l.kpad, l.wg, l.bg, s));
    }
    return hipSuccess;
}

// any frame size for inference (run on the padded grid); training frames
// are whole multiples of 16
bool udims_ok(int B, int W, int H, bool train)
{
    if (B < 1 || W < 1 || H < 1 || W > 32768 || H > 32768) return false;
    if (train && (W % 16 || H % 16)) return false;
    return (int64_t)B * round_up(W, 16) * round_up(H, 16) < (int64_t(1) << 31);
}

narvis_status ust(hipError_t e) { return e == hipSuccess ? NARVIS_OK : NARVIS_ERR_DEVICE; }

// the handle's device must be the current one (its buffers live there)
bool u_on_device(const narvis_unet *u)
{
    int cur = -1;
    return hipGetDevice(&cur) == hipSuccess && cur == u->device;
}

narvis_status uloss_backward(narvis_unet *u, const float *feat, const float *target, int32_t B, int32_t W, int32_t H,
                             float lam_tv, float *loss_out, void *ws, size_t ws_bytes, hipStream_t s)
{
    if (!u || !feat || !target || !loss_out || !ws || !udims_ok(B, W, H, true) || !std::isfinite(lam_tv) ||
        lam_tv < 0)
        return NARVIS_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) || !u_on_device(u)) return NARVIS_ERR_INVALID_ARG;
    const UPlan p = make_uplan(u, B, H, W, true);
    if (ws_bytes < p.bytes) return NARVIS_ERR_WORKSPACE;
    char *base = static_cast<char *>(ws);
    float *y = reinterpret_cast<float *>(base + p.out);
    hipError_t e = uforward(u, feat, base, p, y, false, s);
    if (e == hipSuccess)
        e = loss(y, target, B, H, W, lam_tv, reinterpret_cast<__bf16 *>(base + p.gy),
                 reinterpret_cast<float *>(base + p.lpart), loss_out, s);
    if (e == hipSuccess) e = ubackward(u, base, p, s);
    return ust(e);
}

}  // namespace

extern "C" size_t narvis_unet_param_count(const int32_t widths[5])
{
    if (!widths_ok(widths)) return 0;
    return (size_t)count_params(widths);
}

extern "C" narvis_status narvis_unet_create(const int32_t widths[5], const float *host_blob, size_t count,
                                            narvis_unet **out)
{
    if (!widths_ok(widths) || !host_blob || !out || count != (size_t)count_params(widths)) return NARVIS_ERR_INVALID_ARG;
    for (size_t i = 0; i < count; ++i)
        if (!std::isfinite(host_blob[i])) return NARVIS_ERR_INVALID_ARG;
    narvis_unet *u = new narvis_unet();
    if (hipGetDevice(&u->device) != hipSuccess) {
        delete u;
        return NARVIS_ERR_DEVICE;
    }
    std::memcpy(u->w, widths, sizeof(u->w));
    describe(widths, u->L);
    u->nparams = count_params(widths);
    const uint64_t blob_bytes = align256((uint64_t)u->nparams * 4);
    uint64_t o = 4 * blob_bytes;
    std::vector<uint64_t> offs(kUL * 7);
    for (int i = 0; i < kUL; ++i) {
        const ULayer &l = u->L[i];
        const bool g = l.kind == K_GATE3;
        offs[i * 7 + 0] = o; o = align256(o + (uint64_t)l.rows * l.kpad * 2);
        offs[i * 7 + 1] = o; o = align256(o + (uint64_t)l.brows * l.bkpad * 2);
        offs[i * 7 + 2] = o; o = align256(o + (uint64_t)l.rows * 4);
        offs[i * 7 + 3] = o; o = align256(o + (uint64_t)l.rows * l.kpad * 4);
        offs[i * 7 + 4] = o; o = align256(o + (uint64_t)l.rows * 4);
        offs[i * 7 + 5] = o; o = align256(o + (g ? (uint64_t)l.rows * l.kpad * 2 : 0));
        offs[i * 7 + 6] = o; o = align256(o + (g ? (uint64_t)l.rows * 4 : 0));
    }
    if (hipMalloc(&u->pool, o) != hipSuccess) {
        delete u;
        return NARVIS_ERR_OUT_OF_MEMORY;
    }
    char *base = static_cast<char *>(u->pool);
    u->master = reinterpret_cast<float *>(base);
    u->grad = reinterpret_cast<float *>(base + blob_bytes);
    u->m = reinterpret_cast<float *>(base + 2 * blob_bytes);
    u->v = reinterpret_cast<float *>(base + 3 * blob_bytes);
    for (int i = 0; i < kUL; ++i) {
        ULayer &l = u->L[i];
        l.wf = reinterpret_cast<__bf16 *>(base + offs[i * 7 + 0]);
        l.wb = reinterpret_cast<__bf16 *>(base + offs[i * 7 + 1]);
        l.bias = reinterpret_cast<float *>(base + offs[i * 7 + 2]);
        l.dw = reinterpret_cast<float *>(base + offs[i * 7 + 3]);
        l.db = reinterpret_cast<float *>(base + offs[i * 7 + 4]);
        l.wg = l.kind == K_GATE3 ? reinterpret_cast<__bf16 *>(base + offs[i * 7 + 5]) : nullptr;
        l.bg = l.kind == K_GATE3 ? reinterpret_cast<float *>(base + offs[i * 7 + 6]) : nullptr;
    }
    hipError_t e = hipMemset(u->pool, 0, o);
    if (e == hipSuccess) e = hipMemcpy(u->master, host_blob, count * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = urefresh(u, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(u->pool);
        delete u;
        return NARVIS_ERR_DEVICE;
    }
    *out = u;
    return NARVIS_OK;
}

extern "C" void narvis_unet_destroy(narvis_unet *u)
{
    if (!u) return;
    // best effort: a destroy has no error to report
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(u->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(u->pool);
    (void)hipSetDevice(prev);
    delete u;
}

extern "C" narvis_status narvis_unet_read(const narvis_unet *u, float *host_blob, size_t count)
{
    if (!u || !host_blob || count != (size_t)u->nparams) return NARVIS_ERR_INVALID_ARG;
    if (hipDeviceSynchronize() != hipSuccess) return NARVIS_ERR_DEVICE;
    return ust(hipMemcpy(host_blob, u->master, count * 4, hipMemcpyDeviceToHost));
}

extern "C" size_t narvis_unet_workspace_size(const narvis_unet *u, int32_t B, int32_t W, int32_t H, int32_t train)
{
    if (!u || !udims_ok(B, W, H, train != 0)) return 0;
    return (size_t)make_uplan(u, B, H, W, train != 0).bytes;
}

extern "C" narvis_status narvis_unet_forward(const narvis_unet *u, const float *feat, int32_t B, int32_t W, int32_t H,
                                             float *img, void *ws, size_t ws_bytes, void *stream)
{
    if (!u || !feat || !img || !ws || !udims_ok(B, W, H, false) || !u_on_device(u)) return NARVIS_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) || (reinterpret_cast<uintptr_t>(feat) & 3u) ||
        (reinterpret_cast<uintptr_t>(img) & 3u))
        return NARVIS_ERR_INVALID_ARG;
    const UPlan p = make_uplan(u, B, H, W, false);
    if (ws_bytes < p.bytes) return NARVIS_ERR_WORKSPACE;
    return ust(uforward(u, feat, static_cast<char *>(ws), p, img, true, static_cast<hipStream_t>(stream)));
}

extern "C" narvis_status narvis_unet_gradients(narvis_unet *u, const float *feat, const float *target, int32_t B,
                                               int32_t W, int32_t H, float lam_tv, float *grad_out, float *loss_out,
                                               void *ws, size_t ws_bytes, void *stream)
{
    if (!grad_out) return NARVIS_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const narvis_status st = uloss_backward(u, feat, target, B, W, H, lam_tv, loss_out, ws, ws_bytes, s);
    if (st != NARVIS_OK) return st;
    return ust(copy_f32(u->grad, grad_out, u->nparams, s));
}

extern "C" narvis_status narvis_unet_train_step(narvis_unet *u, const float *feat, const float *target, int32_t B,
                                                int32_t W, int32_t H, float lr, float lam_tv, float *loss_out, void *ws,
                                                size_t ws_bytes, void *stream)
{
    if (!std::isfinite(lr) || lr <= 0.0f) return NARVIS_ERR_INVALID_ARG;
    hipStream_t s = static_cast<hipStream_t>(stream);
    narvis_status st = uloss_backward(u, feat, target, B, W, H, lam_tv, loss_out, ws, ws_bytes, s);
    if (st != NARVIS_OK) return st;
    u->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)u->step));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)u->step));
    hipError_t e = adam(u->master, u->grad, u->m, u->v, u->nparams, lr, b1, b2, 1e-8f, c1, c2, s);
    if (e == hipSuccess) e = urefresh(u, s);
    return ust(e);
}

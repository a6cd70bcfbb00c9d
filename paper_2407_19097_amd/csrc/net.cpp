// Host side of the post-processing network: layer table, weight handle,
// workspace plan and the forward / backward / Adam sequences.
//
// The network (a small U-shaped encoder-decoder, after the post-processor of
// Sec. 3.3): four levels of 32-64-128-256 channels with two 3x3 conv + ReLU
// each and 2x2 average pooling between levels; the decoder upsamples x2
// (bilinear), concatenates [upsampled, skip] and applies two 3x3 conv + ReLU;
// a 1x1 head maps 32 channels to RGB.  Training minimises mean squared error
// plus a small total-variation term (Eq. 1 without its perceptual term) with
// Adam.  Skip tensors are written straight into the channel slice of the
// decoder's concat buffer, so concatenation costs nothing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"
#include "narvis.h"
#include "net_internal.h"

using namespace narvis;
using namespace narvis::net;

namespace {

struct LayerDef {
    int cin, cout, ks, relu;
};

// forward order, identical to the parameter blob order
const LayerDef kLayers[] = {
    {8, 32, 3, 1},    {32, 32, 3, 1},    // e1a e1b
    {32, 64, 3, 1},   {64, 64, 3, 1},    // e2a e2b
    {64, 128, 3, 1},  {128, 128, 3, 1},  // e3a e3b
    {128, 256, 3, 1}, {256, 256, 3, 1},  // e4a e4b
    {384, 128, 3, 1}, {128, 128, 3, 1},  // d3a d3b
    {192, 64, 3, 1},  {64, 64, 3, 1},    // d2a d2b
    {96, 32, 3, 1},   {32, 32, 3, 1},    // d1a d1b
    {32, 3, 1, 0},                       // head
};
constexpr int kNumLayers = sizeof(kLayers) / sizeof(kLayers[0]);
enum { E1A, E1B, E2A, E2B, E3A, E3B, E4A, E4B, D3A, D3B, D2A, D2B, D1A, D1B, HEAD };

// resolution level a layer runs at (0 full, 1 half, 2 quarter, 3 eighth)
int layer_level(int l)
{
    static const int level[] = {0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0, 0};
    return level[l];
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }
uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

struct LayerBuf {
    int cin, cout, ks, relu;
    int rows, kpad;          // forward matrix
    int brows, bcin, bkpad;  // input-gradient matrix
    int64_t blob_w, blob_b;  // offsets (floats) in the parameter blob
    __bf16 *wf, *wb;
    float *bias;             // [rows]
    float *dw, *db;          // gradient matrix [rows][kpad] and [rows]
    uint8_t *wq;             // FP8 forward matrix [rows][kpad]
    float *sw;               // FP8 per-row weight scales [rows]
    float sa;                // FP8 activation scale of the layer input
};

}  // namespace

struct narvis_weights {
    int device;
    LayerBuf L[kNumLayers];
    int64_t nparams;
    float *master, *grad, *m, *v;
    void *pool;              // one device allocation for everything above
    unsigned int *amax;      // [kNumLayers] activation max-abs (calibration)
    int64_t step;
    bool fp8_ready;
    uint32_t fp8_mask;       // layers that run in FP8 (bit l = layer l), set by calibration
};

namespace {

int64_t param_count()
{
    int64_t n = 0;
    for (const LayerDef &d : kLayers) n += (int64_t)d.cout * d.cin * d.ks * d.ks + d.cout;
    return n;
}

// Split-K of a layer's weight gradient over the P pixels of a batch: enough
// splits for about 2048 workgroups (64 x 128 output tiles, 32 x 256 for
// layers with at most 32 output channels), at most 1024, each
// split a multiple of 64 pixels.  Returns the number of splits, *per the
// pixels per split.
int wgrad_splits(int rows, int kpad, int64_t P, int64_t *per)
{
    const int tiles = rows <= 32 ? (kpad + 255) / 256 : ((kpad + 127) / 128) * ((rows + 63) / 64);
    int64_t splits = std::min<int64_t>(1024, std::max<int64_t>(1, (2048 + tiles - 1) / tiles));
    int64_t pp = (P + splits - 1) / splits;
    pp = (pp + 63) / 64 * 64;
    *per = pp;
    return (int)((P + pp - 1) / pp);
}

// Workspace plan for a batch of B images of H x W (multiples of 8).
struct Plan {
    int B, H, W;
    int64_t P[4];  // pixels per level
    // sk*: encoder outputs kept for the skip connections; up*: upsampled decoder
    // inputs (a decoder layer reads [up | sk] as its input channels)
    uint64_t feat, e1a, sk1, pool1, e2a, sk2, pool2, e3a, sk3, pool3, e4a, e4b, up3, d3a, d3b, up2, d2a, d2b, up1, d1a,
        d1b;
    uint64_t out;  // fp32 planar [B][3][H][W] (training only)
    // training
    uint64_t gy, g_d1b, g_d1a, g_cat1, g_d2b, g_d2a, g_cat2, g_d3b, g_d3a, g_cat3, g_e4b, g_e4a, g_pool3, g_e3b,
        g_e3a, g_pool2, g_e2b, g_e2a, g_pool1, g_e1b, g_e1a;
    uint64_t part, bpart, lpart;
    int64_t part_floats, bpart_floats;
    uint64_t bytes;
};

Plan make_plan(int B, int H, int W, bool train)
{
    Plan p{};
    p.B = B;
    p.H = H;
    p.W = W;
    for (int l = 0; l < 4; ++l) p.P[l] = (int64_t)B * (H >> l) * (W >> l);
    uint64_t o = 0;
    auto bf = [&](int64_t px, int ch) {
        const uint64_t at = o;
        o = align256(o + (uint64_t)px * ch * 2);
        return at;
    };
    p.feat = bf(p.P[0], 8);
    p.e1a = bf(p.P[0], 32);
    p.sk1 = bf(p.P[0], 32);
    p.pool1 = bf(p.P[1], 32);
    p.e2a = bf(p.P[1], 64);
    p.sk2 = bf(p.P[1], 64);
    p.pool2 = bf(p.P[2], 64);
    p.e3a = bf(p.P[2], 128);
    p.sk3 = bf(p.P[2], 128);
    p.pool3 = bf(p.P[3], 128);
    p.e4a = bf(p.P[3], 256);
    p.e4b = bf(p.P[3], 256);
    p.up3 = bf(p.P[2], 256);
    p.d3a = bf(p.P[2], 128);
    p.d3b = bf(p.P[2], 128);
    p.up2 = bf(p.P[1], 128);
    p.d2a = bf(p.P[1], 64);
    p.d2b = bf(p.P[1], 64);
    p.up1 = bf(p.P[0], 64);
    p.d1a = bf(p.P[0], 32);
    p.d1b = bf(p.P[0], 32);
    if (train) {
        p.out = o;
        o = align256(o + (uint64_t)p.P[0] * 3 * 4);
        p.gy = bf(p.P[0], 8);
        p.g_d1b = bf(p.P[0], 32);
        p.g_d1a = bf(p.P[0], 32);
        p.g_cat1 = bf(p.P[0], 96);
        p.g_d2b = bf(p.P[1], 64);
        p.g_d2a = bf(p.P[1], 64);
        p.g_cat2 = bf(p.P[1], 192);
        p.g_d3b = bf(p.P[2], 128);
        p.g_d3a = bf(p.P[2], 128);
        p.g_cat3 = bf(p.P[2], 384);
        p.g_e4b = bf(p.P[3], 256);
        p.g_e4a = bf(p.P[3], 256);
        p.g_pool3 = bf(p.P[3], 128);
        p.g_e3b = bf(p.P[2], 128);
        p.g_e3a = bf(p.P[2], 128);
        p.g_pool2 = bf(p.P[2], 64);
        p.g_e2b = bf(p.P[1], 64);
        p.g_e2a = bf(p.P[1], 64);
        p.g_pool1 = bf(p.P[1], 32);
        p.g_e1b = bf(p.P[0], 32);
        p.g_e1a = bf(p.P[0], 32);
        // split-K partials for the weight gradients (the largest layer need)
        int64_t pf = 0, bfl = 0;
        for (int l = 0; l < kNumLayers; ++l) {
            const LayerDef &d = kLayers[l];
            const int rows = round_up(d.cout, 16), kpad = round_up(d.ks * d.ks * d.cin, 32);
            const int level = layer_level(l);
            int64_t per;
            const int splits = wgrad_splits(rows, kpad, p.P[level], &per);
            pf = std::max<int64_t>(pf, (int64_t)splits * rows * kpad);
            bfl = std::max<int64_t>(bfl, (int64_t)splits * rows);
        }
        p.part_floats = pf;
        p.bpart_floats = bfl;
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

struct Ctx {
    char *ws;
    const Plan &p;
    __bf16 *b(uint64_t off) const { return reinterpret_cast<__bf16 *>(ws + off); }
};

ConvArgs conv_args(const LayerBuf &l, const __bf16 *in, int in_stride, int in_off, __bf16 *out, int out_stride,
                   int out_off, int B, int H, int W)
{
    ConvArgs a{};
    a.in = in;
    a.in_stride = in_stride;
    a.in_off = in_off;
    a.Cin = l.cin;
    a.wt = l.wf;
    a.Kpad = l.kpad;
    a.bias = l.bias;
    a.Cout = l.cout;
    a.Cout_pad = l.rows;
    a.B = B;
    a.H = H;
    a.W = W;
    a.relu = l.relu;
    a.out = out;
    a.out_stride = out_stride;
    a.out_off = out_off;
    return a;
}

// a decoder layer's input: channels [0, cin1) from a.in, the rest from `skip`
ConvArgs with_skip(ConvArgs a, const __bf16 *skip, int skip_stride, int cin1)
{
    a.in2 = skip;
    a.in2_stride = skip_stride;
    a.in2_off = 0;
    a.Cin1 = cin1;
    return a;
}

// The layer also writes the 2x2 average pool of its output (stride = Cout).
ConvArgs with_pool(ConvArgs a, __bf16 *pooled)
{
    a.pool_out = pooled;
    a.pool_stride = a.Cout;
    a.pool_off = 0;
    return a;
}

SliceArgs slice(const __bf16 *in, int is, int io, __bf16 *out, int os, int oo, int C, int B, int H, int W)
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

#define TRY(x)                                  \
    do {                                        \
        hipError_t e_ = (x);                    \
        if (e_ != hipSuccess) return e_;        \
    } while (0)

// Forward pass; the head writes fp32 planar [B][3][H][W] to `img`.
// Under FP8 the layers of w->fp8_mask run in FP8, the others in bfloat16.
// Candidates are the ten layers below full resolution (the matrix-core
// bound part); the full-resolution layers (bandwidth bound, and closest to the
// raw features and to the output image) and the head always stay in bfloat16.
bool fp8_candidate(int layer) { return layer >= E2A && layer <= D2B; }

hipError_t run_conv(const narvis_weights *w, int layer, const ConvArgs &a, bool fp8, hipStream_t s)
{
    const LayerBuf &l = w->L[layer];
    return (fp8 && ((w->fp8_mask >> layer) & 1u)) ? conv_fp8(a, l.ks, l.wq, l.sw, l.sa, s) : conv(a, l.ks, s);
}

hipError_t forward(const narvis_weights *w, const float *feat_planes, char *ws, const Plan &p, float *img, hipStream_t s,
                   bool fp8, bool keep_acts)
{
    Ctx c{ws, p};
    const int B = p.B, H = p.H, W = p.W;
    const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
    const LayerBuf *L = w->L;
    TRY(features(feat_planes, c.b(p.feat), B, H, W, s));
    TRY(run_conv(w, E1A, conv_args(L[E1A], c.b(p.feat), 8, 0, c.b(p.e1a), 32, 0, B, H, W), fp8, s));
    // the second layer of each encoder level also writes the pooled input of
    // the next level
    TRY(run_conv(w, E1B, with_pool(conv_args(L[E1B], c.b(p.e1a), 32, 0, c.b(p.sk1), 32, 0, B, H, W), c.b(p.pool1)),
                 fp8, s));
    TRY(run_conv(w, E2A, conv_args(L[E2A], c.b(p.pool1), 32, 0, c.b(p.e2a), 64, 0, B, H1, W1), fp8, s));
    TRY(run_conv(w, E2B, with_pool(conv_args(L[E2B], c.b(p.e2a), 64, 0, c.b(p.sk2), 64, 0, B, H1, W1), c.b(p.pool2)),
                 fp8, s));
    TRY(run_conv(w, E3A, conv_args(L[E3A], c.b(p.pool2), 64, 0, c.b(p.e3a), 128, 0, B, H2, W2), fp8, s));
    TRY(run_conv(w, E3B,
                 with_pool(conv_args(L[E3B], c.b(p.e3a), 128, 0, c.b(p.sk3), 128, 0, B, H2, W2), c.b(p.pool3)), fp8, s));
    TRY(run_conv(w, E4A, conv_args(L[E4A], c.b(p.pool3), 128, 0, c.b(p.e4a), 256, 0, B, H3, W3), fp8, s));
    TRY(run_conv(w, E4B, conv_args(L[E4B], c.b(p.e4a), 256, 0, c.b(p.e4b), 256, 0, B, H3, W3), fp8, s));
    // A decoder layer's input is [2x upsample of the layer below | skip].  In
    // inference the upsample is done while the layer stages its input;
    // training materialises it (the backward pass reads it).
    const bool fuse_up = !keep_acts;
    if (fuse_up) {
        ConvArgs a = with_skip(conv_args(L[D3A], c.b(p.e4b), 256, 0, c.b(p.d3a), 128, 0, B, H2, W2), c.b(p.sk3), 128, 256);
        a.up_in = 1;
        TRY(run_conv(w, D3A, a, fp8, s));
    } else {
        TRY(upsample2(slice(c.b(p.e4b), 256, 0, c.b(p.up3), 256, 0, 256, B, H3, W3), s));
        TRY(run_conv(w, D3A, with_skip(conv_args(L[D3A], c.b(p.up3), 256, 0, c.b(p.d3a), 128, 0, B, H2, W2), c.b(p.sk3), 128, 256),
                     fp8, s));
    }
    TRY(run_conv(w, D3B, conv_args(L[D3B], c.b(p.d3a), 128, 0, c.b(p.d3b), 128, 0, B, H2, W2), fp8, s));
    if (fuse_up) {
        ConvArgs a = with_skip(conv_args(L[D2A], c.b(p.d3b), 128, 0, c.b(p.d2a), 64, 0, B, H1, W1), c.b(p.sk2), 64, 128);
        a.up_in = 1;
        TRY(run_conv(w, D2A, a, fp8, s));
    } else {
        TRY(upsample2(slice(c.b(p.d3b), 128, 0, c.b(p.up2), 128, 0, 128, B, H2, W2), s));
        TRY(run_conv(w, D2A, with_skip(conv_args(L[D2A], c.b(p.up2), 128, 0, c.b(p.d2a), 64, 0, B, H1, W1), c.b(p.sk2), 64, 128),
                     fp8, s));
    }
    TRY(run_conv(w, D2B, conv_args(L[D2B], c.b(p.d2a), 64, 0, c.b(p.d2b), 64, 0, B, H1, W1), fp8, s));
    if (!fuse_up) {
        TRY(upsample2(slice(c.b(p.d2b), 64, 0, c.b(p.up1), 64, 0, 64, B, H1, W1), s));
        TRY(run_conv(w, D1A, with_skip(conv_args(L[D1A], c.b(p.up1), 64, 0, c.b(p.d1a), 32, 0, B, H, W), c.b(p.sk1), 32, 64),
                     fp8, s));
    } else {
        ConvArgs a = with_skip(conv_args(L[D1A], c.b(p.d2b), 64, 0, c.b(p.d1a), 32, 0, B, H, W), c.b(p.sk1), 32, 64);
        a.up_in = 1;
        TRY(run_conv(w, D1A, a, fp8, s));
    }
    if (keep_acts) {
        // training: the last layer's output is kept for the backward pass
        TRY(run_conv(w, D1B, conv_args(L[D1B], c.b(p.d1a), 32, 0, c.b(p.d1b), 32, 0, B, H, W), fp8, s));
        ConvArgs head = conv_args(L[HEAD], c.b(p.d1b), 32, 0, nullptr, 0, 0, B, H, W);
        head.out_f32 = img;
        TRY(run_conv(w, HEAD, head, fp8, s));
    } else {
        // inference: the 1x1 head is applied in the last layer's epilogue
        ConvArgs a = conv_args(L[D1B], c.b(p.d1a), 32, 0, nullptr, 0, 0, B, H, W);
        a.head_w = L[HEAD].wf;
        a.head_kpad = L[HEAD].kpad;
        a.head_b = L[HEAD].bias;
        a.head_out = img;
        TRY(run_conv(w, D1B, a, fp8, s));
    }
    return hipSuccess;
}

// Backward of one conv layer: weight gradient into l.dw / l.db and, when dx is
// given, the input gradient.  dy is masked by the layer's own output (ReLU).
hipError_t layer_backward(const LayerBuf &l, const __bf16 *dy, int dy_stride, int dy_off, const __bf16 *own,
                          int own_stride, int own_off, const __bf16 *x, int x_stride, int x_off, __bf16 *dx,
                          int dx_stride, int dx_off, int B, int H, int W, const Plan &p, char *ws, hipStream_t s,
                          const __bf16 *x2 = nullptr, int x2_stride = 0, int xcin1 = 0)
{
    const __bf16 *mask = l.relu ? own : nullptr;
    WgradArgs a{};
    a.dy = dy;
    a.dy_stride = dy_stride;
    a.dy_off = dy_off;
    a.mask = mask;
    a.mask_stride = own_stride;
    a.mask_off = own_off;
    a.x = x;
    a.x_stride = x_stride;
    a.x_off = x_off;
    a.x2 = x2;
    a.x2_stride = x2_stride;
    a.x2_off = 0;
    a.xCin1 = xcin1;
    a.Cin = l.cin;
    a.KS = l.ks;
    a.Cout = l.cout;
    a.Cout_pad = l.rows;
    a.Kpad = l.kpad;
    a.B = B;
    a.H = H;
    a.W = W;
    const int64_t P = (int64_t)B * H * W;
    int64_t per;
    const int splits = wgrad_splits(l.rows, l.kpad, P, &per);
    a.splits = splits;
    a.pix_per_split = per;
    a.part = reinterpret_cast<float *>(ws + p.part);
    a.bpart = reinterpret_cast<float *>(ws + p.bpart);
    TRY(wgrad(a, l.dw, l.db, s));
    if (dx) {
        ConvArgs c{};
        c.in = dy;
        c.in_stride = dy_stride;
        c.in_off = dy_off;
        c.Cin = l.bcin;
        c.in_mask = mask;
        c.mask_stride = own_stride;
        c.mask_off = own_off;
        c.wt = l.wb;
        c.Kpad = l.bkpad;
        c.bias = nullptr;
        c.Cout = l.cin;
        c.Cout_pad = l.brows;
        c.B = B;
        c.H = H;
        c.W = W;
        c.relu = 0;
        c.out = dx;
        c.out_stride = dx_stride;
        c.out_off = dx_off;
        TRY(conv(c, l.ks, s));
    }
    return hipSuccess;
}

hipError_t backward(const narvis_weights *w, char *ws, const Plan &p, hipStream_t s)
{
    Ctx c{ws, p};
    const int B = p.B, H = p.H, W = p.W;
    const int H1 = H / 2, W1 = W / 2, H2 = H / 4, W2 = W / 4, H3 = H / 8, W3 = W / 8;
    const LayerBuf *L = w->L;
    // head (1x1, linear): dy = loss gradient [P][8]
    TRY(layer_backward(L[HEAD], c.b(p.gy), 8, 0, nullptr, 0, 0, c.b(p.d1b), 32, 0, c.b(p.g_d1b), 32, 0, B, H, W, p, ws, s));
    TRY(layer_backward(L[D1B], c.b(p.g_d1b), 32, 0, c.b(p.d1b), 32, 0, c.b(p.d1a), 32, 0, c.b(p.g_d1a), 32, 0, B, H, W, p, ws, s));
    TRY(layer_backward(L[D1A], c.b(p.g_d1a), 32, 0, c.b(p.d1a), 32, 0, c.b(p.up1), 64, 0, c.b(p.g_cat1), 96, 0, B, H, W, p, ws, s,
                       c.b(p.sk1), 32, 64));
    TRY(upsample2_bwd(slice(c.b(p.g_cat1), 96, 0, c.b(p.g_d2b), 64, 0, 64, B, H1, W1), s));
    TRY(layer_backward(L[D2B], c.b(p.g_d2b), 64, 0, c.b(p.d2b), 64, 0, c.b(p.d2a), 64, 0, c.b(p.g_d2a), 64, 0, B, H1, W1, p, ws, s));
    TRY(layer_backward(L[D2A], c.b(p.g_d2a), 64, 0, c.b(p.d2a), 64, 0, c.b(p.up2), 128, 0, c.b(p.g_cat2), 192, 0, B, H1, W1, p, ws,
                       s, c.b(p.sk2), 64, 128));
    TRY(upsample2_bwd(slice(c.b(p.g_cat2), 192, 0, c.b(p.g_d3b), 128, 0, 128, B, H2, W2), s));
    TRY(layer_backward(L[D3B], c.b(p.g_d3b), 128, 0, c.b(p.d3b), 128, 0, c.b(p.d3a), 128, 0, c.b(p.g_d3a), 128, 0, B, H2, W2, p, ws, s));
    TRY(layer_backward(L[D3A], c.b(p.g_d3a), 128, 0, c.b(p.d3a), 128, 0, c.b(p.up3), 256, 0, c.b(p.g_cat3), 384, 0, B, H2, W2, p,
                       ws, s, c.b(p.sk3), 128, 256));
    TRY(upsample2_bwd(slice(c.b(p.g_cat3), 384, 0, c.b(p.g_e4b), 256, 0, 256, B, H3, W3), s));
    TRY(layer_backward(L[E4B], c.b(p.g_e4b), 256, 0, c.b(p.e4b), 256, 0, c.b(p.e4a), 256, 0, c.b(p.g_e4a), 256, 0, B, H3, W3, p, ws, s));
    TRY(layer_backward(L[E4A], c.b(p.g_e4a), 256, 0, c.b(p.e4a), 256, 0, c.b(p.pool3), 128, 0, c.b(p.g_pool3), 128, 0, B, H3, W3, p, ws, s));
    {
        SliceArgs a = slice(c.b(p.g_pool3), 128, 0, c.b(p.g_e3b), 128, 0, 128, B, H2, W2);
        a.in2 = c.b(p.g_cat3);
        a.in2_stride = 384;
        a.in2_off = 256;
        TRY(pool2_bwd_add(a, s));
    }
    TRY(layer_backward(L[E3B], c.b(p.g_e3b), 128, 0, c.b(p.sk3), 128, 0, c.b(p.e3a), 128, 0, c.b(p.g_e3a), 128, 0, B, H2, W2, p, ws, s));
    TRY(layer_backward(L[E3A], c.b(p.g_e3a), 128, 0, c.b(p.e3a), 128, 0, c.b(p.pool2), 64, 0, c.b(p.g_pool2), 64, 0, B, H2, W2, p, ws, s));
    {
        SliceArgs a = slice(c.b(p.g_pool2), 64, 0, c.b(p.g_e2b), 64, 0, 64, B, H1, W1);
        a.in2 = c.b(p.g_cat2);
        a.in2_stride = 192;
        a.in2_off = 128;
        TRY(pool2_bwd_add(a, s));
    }
    TRY(layer_backward(L[E2B], c.b(p.g_e2b), 64, 0, c.b(p.sk2), 64, 0, c.b(p.e2a), 64, 0, c.b(p.g_e2a), 64, 0, B, H1, W1, p, ws, s));
    TRY(layer_backward(L[E2A], c.b(p.g_e2a), 64, 0, c.b(p.e2a), 64, 0, c.b(p.pool1), 32, 0, c.b(p.g_pool1), 32, 0, B, H1, W1, p, ws, s));
    {
        SliceArgs a = slice(c.b(p.g_pool1), 32, 0, c.b(p.g_e1b), 32, 0, 32, B, H, W);
        a.in2 = c.b(p.g_cat1);
        a.in2_stride = 96;
        a.in2_off = 64;
        TRY(pool2_bwd_add(a, s));
    }
    TRY(layer_backward(L[E1B], c.b(p.g_e1b), 32, 0, c.b(p.sk1), 32, 0, c.b(p.e1a), 32, 0, c.b(p.g_e1a), 32, 0, B, H, W, p, ws, s));
    TRY(layer_backward(L[E1A], c.b(p.g_e1a), 32, 0, c.b(p.e1a), 32, 0, c.b(p.feat), 8, 0, nullptr, 0, 0, B, H, W, p, ws, s));
    // gradient matrices -> blob order
    for (int i = 0; i < kNumLayers; ++i) {
        const LayerBuf &l = L[i];
        TRY(grad_to_blob(l.dw, l.kpad, l.cout, l.cin, l.ks, w->grad + l.blob_w, s));
        TRY(copy_f32(l.db, w->grad + l.blob_b, l.cout, s));
    }
    return hipSuccess;
}

hipError_t refresh(narvis_weights *w, hipStream_t s)
{
    for (int i = 0; i < kNumLayers; ++i) {
        LayerBuf &l = w->L[i];
        TRY(prep_weights(w->master + l.blob_w, l.cout, l.cin, l.ks, l.wf, l.rows, l.kpad, l.wb, l.brows, l.bcin, l.bkpad, s));
        TRY(copy_f32(w->master + l.blob_b, l.bias, l.cout, s));
    }
    return hipSuccess;
}

bool dims_ok(int B, int W, int H)
{
    return B >= 1 && W >= 8 && H >= 8 && W <= 32768 && H <= 32768 && W % 8 == 0 && H % 8 == 0 &&
           (int64_t)B * W * H < (int64_t(1) << 31);
}

narvis_status st(hipError_t e) { return e == hipSuccess ? NARVIS_OK : NARVIS_ERR_DEVICE; }

// the handle's device must be the current one (its buffers live there)
bool on_device(int dev)
{
    int cur = -1;
    return hipGetDevice(&cur) == hipSuccess && cur == dev;
}

}  // namespace

extern "C" size_t narvis_net_param_count(void) { return (size_t)param_count(); }

extern "C" narvis_status narvis_weights_create(const float *host_blob, size_t count, narvis_weights **out)
{
    if (!host_blob || !out || count != (size_t)param_count()) return NARVIS_ERR_INVALID_ARG;
    for (size_t i = 0; i < count; ++i)
        if (!std::isfinite(host_blob[i])) return NARVIS_ERR_INVALID_ARG;
    narvis_weights *w = new narvis_weights();
    if (hipGetDevice(&w->device) != hipSuccess) {
        delete w;
        return NARVIS_ERR_DEVICE;
    }
    w->nparams = param_count();
    // carve one allocation: master, grad, m, v (fp32 blob each), then per layer
    uint64_t o = 0;
    const uint64_t blob_bytes = align256((uint64_t)w->nparams * 4);
    o = 4 * blob_bytes;
    int64_t boff = 0;
    std::vector<uint64_t> offs(kNumLayers * 7);
    for (int i = 0; i < kNumLayers; ++i) {
        const LayerDef &d = kLayers[i];
        LayerBuf &l = w->L[i];
        l.cin = d.cin;
        l.cout = d.cout;
        l.ks = d.ks;
        l.relu = d.relu;
        l.rows = round_up(d.cout, 16);
        l.kpad = round_up(d.ks * d.ks * d.cin, 32);
        l.bcin = round_up(d.cout, 8);
        l.brows = round_up(d.cin, 16);
        l.bkpad = round_up(d.ks * d.ks * l.bcin, 32);
        l.blob_w = boff;
        boff += (int64_t)d.cout * d.cin * d.ks * d.ks;
        l.blob_b = boff;
        boff += d.cout;
        offs[i * 7 + 0] = o; o = align256(o + (uint64_t)l.rows * l.kpad * 2);
        offs[i * 7 + 1] = o; o = align256(o + (uint64_t)l.brows * l.bkpad * 2);
        offs[i * 7 + 2] = o; o = align256(o + (uint64_t)l.rows * 4);
        offs[i * 7 + 3] = o; o = align256(o + (uint64_t)l.rows * l.kpad * 4);
        offs[i * 7 + 4] = o; o = align256(o + (uint64_t)l.rows * 4);
        offs[i * 7 + 5] = o; o = align256(o + (uint64_t)l.rows * l.kpad);
        offs[i * 7 + 6] = o; o = align256(o + (uint64_t)l.rows * 4);
        l.sa = 1.0f;
    }
    const uint64_t off_amax = o;
    o = align256(o + kNumLayers * 4);
    if (hipMalloc(&w->pool, o) != hipSuccess) {
        delete w;
        return NARVIS_ERR_OUT_OF_MEMORY;
    }
    char *base = static_cast<char *>(w->pool);
    w->master = reinterpret_cast<float *>(base);
    w->grad = reinterpret_cast<float *>(base + blob_bytes);
    w->m = reinterpret_cast<float *>(base + 2 * blob_bytes);
    w->v = reinterpret_cast<float *>(base + 3 * blob_bytes);
    for (int i = 0; i < kNumLayers; ++i) {
        LayerBuf &l = w->L[i];
        l.wf = reinterpret_cast<__bf16 *>(base + offs[i * 7 + 0]);
        l.wb = reinterpret_cast<__bf16 *>(base + offs[i * 7 + 1]);
        l.bias = reinterpret_cast<float *>(base + offs[i * 7 + 2]);
        l.dw = reinterpret_cast<float *>(base + offs[i * 7 + 3]);
        l.db = reinterpret_cast<float *>(base + offs[i * 7 + 4]);
        l.wq = reinterpret_cast<uint8_t *>(base + offs[i * 7 + 5]);
        l.sw = reinterpret_cast<float *>(base + offs[i * 7 + 6]);
    }
    w->amax = reinterpret_cast<unsigned int *>(base + off_amax);
    w->fp8_ready = false;
    w->fp8_mask = 0;
    hipError_t e = hipMemset(w->pool, 0, o);
    if (e == hipSuccess) e = hipMemcpy(w->master, host_blob, count * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = refresh(w, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(w->pool);
        delete w;
        return NARVIS_ERR_DEVICE;
    }
    w->step = 0;
    *out = w;
    return NARVIS_OK;
}

extern "C" void narvis_weights_destroy(narvis_weights *w)
{
    if (!w) return;
    // best effort: a destroy has no error to report
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(w->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(w->pool);
    (void)hipSetDevice(cur);
    delete w;
}

extern "C" narvis_status narvis_weights_read(const narvis_weights *w, float *host_blob, size_t count)
{
    if (!w || !host_blob || count != (size_t)w->nparams) return NARVIS_ERR_INVALID_ARG;
    if (hipDeviceSynchronize() != hipSuccess) return NARVIS_ERR_DEVICE;
    return st(hipMemcpy(host_blob, w->master, count * 4, hipMemcpyDeviceToHost));
}

extern "C" size_t narvis_postprocess_workspace_size(int32_t B, int32_t W, int32_t H)
{
    if (!dims_ok(B, W, H)) return 0;
    return (size_t)make_plan(B, H, W, false).bytes;
}

extern "C" narvis_status narvis_postprocess(const narvis_weights *w, const float *feat, int32_t B, int32_t W, int32_t H,
                                            float *img, int32_t precision, void *ws, size_t ws_bytes, void *stream)
{
    if (!w || !feat || !img || !ws || !dims_ok(B, W, H) || !on_device(w->device)) return NARVIS_ERR_INVALID_ARG;
    if (precision != NARVIS_PRECISION_BF16 && precision != NARVIS_PRECISION_FP8) return NARVIS_ERR_INVALID_ARG;
    if (precision == NARVIS_PRECISION_FP8 && !w->fp8_ready) return NARVIS_ERR_UNSUPPORTED;
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) || (reinterpret_cast<uintptr_t>(feat) & 3u) ||
        (reinterpret_cast<uintptr_t>(img) & 3u))
        return NARVIS_ERR_INVALID_ARG;
    const Plan p = make_plan(B, H, W, false);
    if (ws_bytes < p.bytes) return NARVIS_ERR_WORKSPACE;
    return st(forward(w, feat, static_cast<char *>(ws), p, img, static_cast<hipStream_t>(stream),
                      precision == NARVIS_PRECISION_FP8, false));
}

extern "C" size_t narvis_train_workspace_size(int32_t B, int32_t W, int32_t H)
{
    if (!dims_ok(B, W, H)) return 0;
    return (size_t)make_plan(B, H, W, true).bytes;
}

namespace {

narvis_status train_common(narvis_weights *w, const float *feat, const float *target, int32_t B, int32_t W, int32_t H,
                           float lam_tv, float *loss_out, void *ws, size_t ws_bytes, hipStream_t s, Plan &p)
{
    if (!w || !feat || !target || !loss_out || !ws || !dims_ok(B, W, H) || !std::isfinite(lam_tv) || lam_tv < 0)
        return NARVIS_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(ws) & 255u) || !on_device(w->device)) return NARVIS_ERR_INVALID_ARG;
    p = make_plan(B, H, W, true);
    if (ws_bytes < p.bytes) return NARVIS_ERR_WORKSPACE;
    char *base = static_cast<char *>(ws);
    float *y = reinterpret_cast<float *>(base + p.out);
    hipError_t e = forward(w, feat, base, p, y, s, false, true);
    if (e == hipSuccess) {
        e = zero_bf16(reinterpret_cast<__bf16 *>(base + p.gy), p.P[0] * 8, s);
    }
    if (e == hipSuccess)
        e = loss(y, target, B, H, W, lam_tv, reinterpret_cast<__bf16 *>(base + p.gy),
                 reinterpret_cast<float *>(base + p.lpart), loss_out, s);
    if (e == hipSuccess) e = backward(w, base, p, s);
    return st(e);
}

}  // namespace

extern "C" narvis_status narvis_train_gradients(narvis_weights *w, const float *feat, const float *target, int32_t B,
                                                int32_t W, int32_t H, float lam_tv, float *grad_out, float *loss_out,
                                                void *ws, size_t ws_bytes, void *stream)
{
    if (!grad_out) return NARVIS_ERR_INVALID_ARG;
    Plan p;
    hipStream_t s = static_cast<hipStream_t>(stream);
    narvis_status r = train_common(w, feat, target, B, W, H, lam_tv, loss_out, ws, ws_bytes, s, p);
    if (r != NARVIS_OK) return r;
    return st(copy_f32(w->grad, grad_out, w->nparams, s));
}

extern "C" narvis_status narvis_train_step(narvis_weights *w, const float *feat, const float *target, int32_t B,
                                           int32_t W, int32_t H, float lr, float lam_tv, float *loss_out, void *ws,
                                           size_t ws_bytes, void *stream)
{
    if (!(lr > 0.0f) || !std::isfinite(lr)) return NARVIS_ERR_INVALID_ARG;
    Plan p;
    hipStream_t s = static_cast<hipStream_t>(stream);
    narvis_status r = train_common(w, feat, target, B, W, H, lam_tv, loss_out, ws, ws_bytes, s, p);
    if (r != NARVIS_OK) return r;
    w->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)w->step));
    const float c2 = (float)(1.0 - std::pow(0.999, (double)w->step));
    hipError_t e = adam(w->master, w->grad, w->m, w->v, w->nparams, lr, b1, b2, 1e-8f, c1, c2, s);
    if (e == hipSuccess) e = refresh(w, s);
    w->fp8_ready = false;  // the FP8 copies describe the old parameters
    return st(e);
}

namespace {

// Named tensors of the training workspace: {name, plan member, level,
// channels}; level -1 marks the fp32 planar output.
struct NamedTensor {
    const char *name;
    uint64_t Plan::*off;
    int level, ch;
};

const NamedTensor kTensors[] = {
    {"feat", &Plan::feat, 0, 8},      {"e1a", &Plan::e1a, 0, 32},       {"sk1", &Plan::sk1, 0, 32},
    {"pool1", &Plan::pool1, 1, 32},   {"e2a", &Plan::e2a, 1, 64},       {"sk2", &Plan::sk2, 1, 64},
    {"pool2", &Plan::pool2, 2, 64},   {"e3a", &Plan::e3a, 2, 128},      {"sk3", &Plan::sk3, 2, 128},
    {"pool3", &Plan::pool3, 3, 128},  {"e4a", &Plan::e4a, 3, 256},      {"e4b", &Plan::e4b, 3, 256},
    {"up3", &Plan::up3, 2, 256},      {"d3a", &Plan::d3a, 2, 128},      {"d3b", &Plan::d3b, 2, 128},
    {"up2", &Plan::up2, 1, 128},      {"d2a", &Plan::d2a, 1, 64},       {"d2b", &Plan::d2b, 1, 64},
    {"up1", &Plan::up1, 0, 64},       {"d1a", &Plan::d1a, 0, 32},       {"d1b", &Plan::d1b, 0, 32},
    {"out", &Plan::out, -1, 3},       {"gy", &Plan::gy, 0, 8},          {"g_d1b", &Plan::g_d1b, 0, 32},
    {"g_d1a", &Plan::g_d1a, 0, 32},   {"g_cat1", &Plan::g_cat1, 0, 96}, {"g_d2b", &Plan::g_d2b, 1, 64},
    {"g_d2a", &Plan::g_d2a, 1, 64},   {"g_cat2", &Plan::g_cat2, 1, 192}, {"g_d3b", &Plan::g_d3b, 2, 128},
    {"g_d3a", &Plan::g_d3a, 2, 128},  {"g_cat3", &Plan::g_cat3, 2, 384}, {"g_e4b", &Plan::g_e4b, 3, 256},
    {"g_e4a", &Plan::g_e4a, 3, 256},  {"g_pool3", &Plan::g_pool3, 3, 128}, {"g_e3b", &Plan::g_e3b, 2, 128},
    {"g_e3a", &Plan::g_e3a, 2, 128},  {"g_pool2", &Plan::g_pool2, 2, 64}, {"g_e2b", &Plan::g_e2b, 1, 64},
    {"g_e2a", &Plan::g_e2a, 1, 64},   {"g_pool1", &Plan::g_pool1, 1, 32}, {"g_e1b", &Plan::g_e1b, 0, 32},
    {"g_e1a", &Plan::g_e1a, 0, 32},
};

}  // namespace

extern "C" narvis_status narvis_train_tensor(int32_t B, int32_t W, int32_t H, const char *name, size_t *offset,
                                             int32_t *channels, int32_t *height, int32_t *width, int32_t *dtype)
{
    if (!name || !offset || !channels || !height || !width || !dtype || !dims_ok(B, W, H))
        return NARVIS_ERR_INVALID_ARG;
    const Plan p = make_plan(B, H, W, true);
    for (const NamedTensor &t : kTensors) {
        if (std::strcmp(t.name, name) != 0) continue;
        const int lv = t.level < 0 ? 0 : t.level;
        *offset = (size_t)(p.*(t.off));
        *channels = t.ch;
        *height = H >> lv;
        *width = W >> lv;
        *dtype = t.level < 0 ? 1 : 0;
        return NARVIS_OK;
    }
    return NARVIS_ERR_INVALID_ARG;
}

// Largest max-abs change of the image that the FP8 layers may make on the
// calibration batch (images in [0, 1]).
constexpr float kFp8Budget = 0.025f;

extern "C" narvis_status narvis_weights_calibrate_fp8(narvis_weights *w, const float *feat, int32_t B, int32_t W,
                                                      int32_t H, void *ws, size_t ws_bytes, void *stream)
{
    if (!w || !feat || !ws || !dims_ok(B, W, H) || (reinterpret_cast<uintptr_t>(ws) & 255u) || !on_device(w->device))
        return NARVIS_ERR_INVALID_ARG;
    const Plan p = make_plan(B, H, W, true);
    if (ws_bytes < p.bytes) return NARVIS_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);
    hipError_t e = forward(w, feat, base, p, reinterpret_cast<float *>(base + p.out), s, false, true);
    // input tensor of every layer, in layer order
    // (a decoder layer's input is two tensors: the upsampled one and the skip)
    const struct { uint64_t off; int64_t px; int ch; uint64_t off2; int ch2; } in[kNumLayers] = {
        {p.feat, p.P[0], 8, 0, 0},     {p.e1a, p.P[0], 32, 0, 0},    {p.pool1, p.P[1], 32, 0, 0},
        {p.e2a, p.P[1], 64, 0, 0},     {p.pool2, p.P[2], 64, 0, 0},  {p.e3a, p.P[2], 128, 0, 0},
        {p.pool3, p.P[3], 128, 0, 0},  {p.e4a, p.P[3], 256, 0, 0},   {p.up3, p.P[2], 256, p.sk3, 128},
        {p.d3a, p.P[2], 128, 0, 0},    {p.up2, p.P[1], 128, p.sk2, 64}, {p.d2a, p.P[1], 64, 0, 0},
        {p.up1, p.P[0], 64, p.sk1, 32}, {p.d1a, p.P[0], 32, 0, 0},    {p.d1b, p.P[0], 32, 0, 0}};
    if (e == hipSuccess) e = hipMemsetAsync(w->amax, 0, kNumLayers * 4, s);
    for (int i = 0; i < kNumLayers && e == hipSuccess; ++i) {
        e = absmax_bf16(reinterpret_cast<const __bf16 *>(base + in[i].off), in[i].px * in[i].ch, w->amax + i, s);
        if (e == hipSuccess && in[i].ch2)
            e = absmax_bf16(reinterpret_cast<const __bf16 *>(base + in[i].off2), in[i].px * in[i].ch2, w->amax + i, s);
    }
    unsigned int host[kNumLayers];
    if (e == hipSuccess) e = hipMemcpyAsync(host, w->amax, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return NARVIS_ERR_DEVICE;
    for (int i = 0; i < kNumLayers && e == hipSuccess; ++i) {
        LayerBuf &l = w->L[i];
        float m;
        std::memcpy(&m, &host[i], 4);
        l.sa = (m > 0.0f && std::isfinite(m)) ? m / 448.0f : 1.0f;
        e = quant_weights(w->master + l.blob_w, l.cout, l.cin, l.ks, l.rows, l.kpad, l.wq, l.sw, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return NARVIS_ERR_DEVICE;
    // Which layers run in FP8: e4m3 keeps three significand bits, and how
    // much a layer's rounding moves the image depends on the trained weights
    // downstream of it.  On the calibration batch, with the bfloat16 forward
    // as reference (in the gradient region g_cat1, unused by a forward), take
    // each candidate alone in FP8 and measure max |image - reference|; then
    // add the candidates in ascending order of that error while the error of
    // the whole set stays within kFp8Budget.
    const int64_t nimg = (int64_t)B * 3 * H * W;
    float *ref = reinterpret_cast<float *>(base + p.g_cat1);
    float *out = reinterpret_cast<float *>(base + p.out);
    e = forward(w, feat, base, p, ref, s, false, false);
    auto image_error = [&](uint32_t mask, float *err) {
        w->fp8_mask = mask;
        hipError_t r = forward(w, feat, base, p, out, s, true, false);
        if (r == hipSuccess) r = hipMemsetAsync(w->amax, 0, 4, s);
        if (r == hipSuccess) r = absdiff_max_f32(out, ref, nimg, w->amax, s);
        unsigned int bits = 0;
        if (r == hipSuccess) r = hipMemcpyAsync(&bits, w->amax, 4, hipMemcpyDeviceToHost, s);
        if (r == hipSuccess) r = hipStreamSynchronize(s);
        std::memcpy(err, &bits, 4);
        return r;
    };
    std::vector<std::pair<float, int>> solo;
    for (int i = 0; i < kNumLayers && e == hipSuccess; ++i) {
        if (!fp8_candidate(i)) continue;
        float err = 0.0f;
        e = image_error(1u << i, &err);
        solo.push_back({err, i});
    }
    std::stable_sort(solo.begin(), solo.end(),
                     [](const std::pair<float, int> &a, const std::pair<float, int> &b) { return a.first < b.first; });
    uint32_t mask = 0;
    for (size_t k = 0; k < solo.size() && e == hipSuccess; ++k) {
        float err = 0.0f;
        e = image_error(mask | (1u << solo[k].second), &err);
        if (err <= kFp8Budget) mask |= 1u << solo[k].second;
    }
    w->fp8_mask = mask;
    if (e != hipSuccess) return NARVIS_ERR_DEVICE;
    w->fp8_ready = true;
    return NARVIS_OK;
}

extern "C" narvis_status narvis_weights_fp8_layers(const narvis_weights *w, uint32_t *mask)
{
    if (!w || !mask) return NARVIS_ERR_INVALID_ARG;
    if (!w->fp8_ready) return NARVIS_ERR_UNSUPPORTED;
    *mask = w->fp8_mask;
    return NARVIS_OK;
}

// Host orchestration of the warm-start network: a 4-level 2-D U-Net (base channels c,
// 2c, 4c, 8c; two 3x3 conv + ReLU per level, 2x2 max pooling, 2x2 stride-2 transposed
// convolutions up, skip concatenation, 1x1 head, residual output), trained with MSE and Adam
// on FP32 master weights. Every layer runs in the BF16 MFMA / element-wise kernels of
// nn_kernels.hip and nn_misc.hip; this file only lays out buffers and sequences launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "eitomo.h"
#include "nn_internal.h"

using namespace eit::nn;

namespace eit {
int nn_fail(int code, const char* msg);   // api.cpp (thread-local error message)
}

namespace {

#define NN_TRY(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return eit::nn_fail(EIT_ERR_DEVICE, hipGetErrorString(e_));   \
    } while (0)

struct Layer {
    int kind;          // 0 conv3x3 + ReLU, 1 transposed conv 2x2, 2 head 1x1
    int cin, cout;
    size_t w, b;       // FP32 offsets of weights and bias in the parameter vector
    size_t wt;         // BF16 offset of the transposed copy (conv / up-conv)
};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

}  // namespace

struct eit_unet {
    int base;
    std::vector<Layer> L;     // a1 b1 a2 b2 a3 b3 a4 b4 up3 d3a d3b up2 d2a d2b up1 d1a d1b head
    size_t n_params;
};

namespace {

enum { A1, B1, A2, B2, A3, B3, A4, B4, UP3, D3A, D3B, UP2, D2A, D2B, UP1, D1A, D1B, HEAD, NLAYERS };

constexpr int kInC = 8;   // the 2 input channels padded to 8 (16-byte channel groups)

// Workspace carve-up for a batch of nb images of h x w.
struct Acts {
    Tensor X0, E1a, CAT1, P1, E2a, CAT2, P2, E3a, CAT3, P3, E4a, E4b, D3a, D3b, D2a, D2b, D1a, D1b;
};

struct WsLayout {
    size_t wbf, wtb;                  // BF16 weight copies (forward layout, transposed layout)
    size_t acts, grads;               // activation and activation-gradient arenas (BF16)
    size_t out, dout;                 // FP32 network output and its gradient
    size_t part, mpart, sums;         // split-K partials, loss partials, channel-sum partials
    size_t end;
    size_t act_elems;
    size_t part_elems;
};

struct Shape { int H, W, C; };

std::vector<std::pair<const char*, Shape>> act_shapes(int c, int h, int w) {
    return {{"X0", {h, w, kInC}},          {"E1a", {h, w, c}},
            {"CAT1", {h, w, 2 * c}},       {"P1", {h / 2, w / 2, c}},
            {"E2a", {h / 2, w / 2, 2 * c}}, {"CAT2", {h / 2, w / 2, 4 * c}},
            {"P2", {h / 4, w / 4, 2 * c}}, {"E3a", {h / 4, w / 4, 4 * c}},
            {"CAT3", {h / 4, w / 4, 8 * c}}, {"P3", {h / 8, w / 8, 4 * c}},
            {"E4a", {h / 8, w / 8, 8 * c}}, {"E4b", {h / 8, w / 8, 8 * c}},
            {"D3a", {h / 4, w / 4, 4 * c}}, {"D3b", {h / 4, w / 4, 4 * c}},
            {"D2a", {h / 2, w / 2, 2 * c}}, {"D2b", {h / 2, w / 2, 2 * c}},
            {"D1a", {h, w, c}},            {"D1b", {h, w, c}}};
}

// pixel slabs of the weight-gradient GEMMs: about 1024 pixels each (16 steps of 64), at
// most 256, so that even the 32-channel layers launch several blocks per CU
int wgrad_splits(size_t pixels) {
    long s = (long)(pixels / 1024);
    return (int)std::max(1L, std::min(256L, s));
}

WsLayout layout(const eit_unet* u, int nb, int h, int w, bool train) {
    WsLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.wbf = take(sizeof(bf16) * u->n_params);
    L.wtb = take(sizeof(bf16) * u->n_params);
    size_t ae = 0;
    for (auto& s : act_shapes(u->base, h, w)) ae += align256((size_t)nb * s.second.H * s.second.W * s.second.C);
    L.act_elems = ae;
    L.acts = take(sizeof(bf16) * ae);
    L.grads = train ? take(sizeof(bf16) * ae) : 0;
    const size_t img = (size_t)nb * 2 * h * w;
    L.out = take(sizeof(float) * img);
    L.dout = train ? take(sizeof(float) * img) : 0;
    size_t pe = 0;
    if (train) {
        for (int i = 0; i < NLAYERS; ++i) {
            const Layer& l = u->L[i];
            int hh = h, ww = w;      // resolution of the layer's input pixels
            if (i >= A2 && i <= B2) { hh = h / 2; ww = w / 2; }
            if (i >= A3 && i <= B3) { hh = h / 4; ww = w / 4; }
            if (i >= A4 && i <= UP3) { hh = h / 8; ww = w / 8; }
            if (i >= D3A && i <= UP2) { hh = h / 4; ww = w / 4; }
            if (i >= D2A && i <= UP1) { hh = h / 2; ww = w / 2; }
            const size_t pix = (size_t)nb * hh * ww;
            const size_t mn = l.kind == 0 ? (size_t)l.cout * 9 * l.cin + l.cout : (size_t)4 * l.cout * (l.cin + 1);
            const size_t parts = l.kind == 0 ? (size_t)conv_wgrad_parts(nb, hh, ww, l.cin, l.cout, wgrad_splits(pix))
                                             : (size_t)wgrad_splits_used((int)pix, wgrad_splits(pix));
            if (l.kind != 2) pe = std::max(pe, mn * parts);
        }
    }
    L.part_elems = pe;
    L.part = take(sizeof(float) * std::max<size_t>(pe, 1));
    L.mpart = take(sizeof(double) * kSumBlocks);
    L.sums = take(sizeof(float) * kSumBlocks * (size_t)(2 * 8 * u->base + 2));
    L.end = off;
    return L;
}

Acts carve(const eit_unet* u, char* base, size_t off, int nb, int h, int w) {
    Acts A;
    Tensor* slots[] = {&A.X0, &A.E1a, &A.CAT1, &A.P1, &A.E2a, &A.CAT2, &A.P2, &A.E3a, &A.CAT3,
                       &A.P3, &A.E4a, &A.E4b, &A.D3a, &A.D3b, &A.D2a, &A.D2b, &A.D1a, &A.D1b};
    size_t o = 0;
    int i = 0;
    for (auto& s : act_shapes(u->base, h, w)) {
        Tensor& t = *slots[i++];
        t.p = (bf16*)(base + off) + o;
        t.B = nb; t.H = s.second.H; t.W = s.second.W; t.C = s.second.C; t.cs = t.C; t.coff = 0;
        o += align256((size_t)nb * t.H * t.W * t.C);
    }
    return A;
}

Tensor view(const Tensor& t, int coff, int C) {
    Tensor v = t;
    v.coff = t.coff + coff;
    v.C = C;
    return v;
}

struct Ctx {
    const eit_unet* u;
    const float* prm;       // FP32 master parameters
    const bf16* wf;         // BF16 forward-layout weights (same offsets as prm)
    const bf16* wt;         // BF16 transposed weights
    hipStream_t s;
};

// Forward pass; activations stay in A for the backward pass.
int forward(const Ctx& c, const Acts& A, const float* x, float* out, int nb, int h, int w) {
    const auto& L = c.u->L;
    const int C = c.u->base;
    auto conv = [&](int li, const Tensor& in, const Tensor& o) -> int {
        NN_TRY(conv_fwd(in, c.wf + L[li].w, c.prm + L[li].b, 1, o, 3, c.s));
        return EIT_OK;
    };
    auto up = [&](int li, const Tensor& in, const Tensor& o) -> int {
        NN_TRY(upconv_fwd(in, c.wf + L[li].w, c.prm + L[li].b, o, c.s));
        return EIT_OK;
    };
    int rc;
    NN_TRY(pack_input(x, nb, h, w, A.X0, c.s));
    const Tensor S1 = view(A.CAT1, C, C), S2 = view(A.CAT2, 2 * C, 2 * C), S3 = view(A.CAT3, 4 * C, 4 * C);
    if ((rc = conv(A1, A.X0, A.E1a)) || (rc = conv(B1, A.E1a, S1))) return rc;
    NN_TRY(maxpool_fwd(S1, A.P1, c.s));
    if ((rc = conv(A2, A.P1, A.E2a)) || (rc = conv(B2, A.E2a, S2))) return rc;
    NN_TRY(maxpool_fwd(S2, A.P2, c.s));
    if ((rc = conv(A3, A.P2, A.E3a)) || (rc = conv(B3, A.E3a, S3))) return rc;
    NN_TRY(maxpool_fwd(S3, A.P3, c.s));
    if ((rc = conv(A4, A.P3, A.E4a)) || (rc = conv(B4, A.E4a, A.E4b))) return rc;
    if ((rc = up(UP3, A.E4b, view(A.CAT3, 0, 4 * C)))) return rc;
    if ((rc = conv(D3A, A.CAT3, A.D3a)) || (rc = conv(D3B, A.D3a, A.D3b))) return rc;
    if ((rc = up(UP2, A.D3b, view(A.CAT2, 0, 2 * C)))) return rc;
    if ((rc = conv(D2A, A.CAT2, A.D2a)) || (rc = conv(D2B, A.D2a, A.D2b))) return rc;
    if ((rc = up(UP1, A.D2b, view(A.CAT1, 0, C)))) return rc;
    if ((rc = conv(D1A, A.CAT1, A.D1a)) || (rc = conv(D1B, A.D1a, A.D1b))) return rc;
    NN_TRY(head_fwd(A.D1b, c.prm + L[HEAD].w, c.prm + L[HEAD].b, x, out, nb, h, w, c.s));
    return EIT_OK;
}

// Backward pass from dout (FP32 gradient of the output) into grad (FP32, parameter layout).
int backward(const Ctx& c, const Acts& A, const Acts& G, const float* dout, float* grad, float* part,
             float* sums, int nb, int h, int w) {
    const auto& L = c.u->L;
    const int C = c.u->base;
    const hipStream_t s = c.s;
    // conv layer li with input X and incoming gradient dY, already multiplied by the ReLU
    // derivative of the layer's output by whichever kernel produced it (a data gradient's
    // epilogue, the pooling backward or the head's backward); writes dW, db and, if dX is
    // given, the input gradient, masked by X > 0 when mask_dx (X the post-ReLU output of
    // the layer before, whose backward consumes dX directly)
    auto conv_b = [&](int li, const Tensor& X, const Tensor& dY, const Tensor* dX, bool mask_dx) -> int {
        const size_t pix = (size_t)X.B * X.H * X.W;
        const int sp = wgrad_splits(pix);
        // weight and bias partials; one reduction writes both (the bias directly follows the
        // weights in the parameter layout)
        NN_TRY(conv_wgrad(X, dY, part, sp, 3, s));
        NN_TRY(splitk_reduce(part, conv_wgrad_parts(X.B, X.H, X.W, X.C, dY.C, sp),
                             L[li].cout * 9 * L[li].cin + L[li].cout, grad + L[li].w, s));
        if (dX) NN_TRY(conv_dgrad(dY, c.wt + L[li].wt, *dX, 3, s, mask_dx ? &X : nullptr));
        return EIT_OK;
    };
    // transposed conv li: input X (half size, the post-ReLU output of the layer before),
    // output-gradient view gY, writes dX masked by X > 0
    auto up_b = [&](int li, const Tensor& X, const Tensor& gY, const Tensor& dX) -> int {
        const size_t pix = (size_t)X.B * X.H * X.W;
        const int sp = wgrad_splits(pix);
        NN_TRY(upconv_wgrad(X, gY, part, sp, s));
        const int parts = wgrad_splits_used((int)pix, sp);
        const size_t nw = (size_t)4 * L[li].cout * L[li].cin, ld = nw + 4 * L[li].cout;
        NN_TRY(splitk_reduce(part, parts, (int)nw, grad + L[li].w, s, ld));
        // bias: the 4 Co row sums reduced over the slabs (into the scratch sums), then over d
        NN_TRY(splitk_reduce(part + nw, parts, 4 * L[li].cout, sums, s, ld));
        NN_TRY(fold_sums(sums, 1, 0, L[li].cout, 4, grad + L[li].b, s));
        NN_TRY(upconv_dgrad(gY, c.wt + L[li].wt, dX, s, &X));
        return EIT_OK;
    };
    int rc;
    // head: dD1b = (W^T dout) masked by D1b > 0, head dW/db
    NN_TRY(head_bwd(A.D1b, c.prm + L[HEAD].w, dout, nb, h, w, grad + L[HEAD].w, grad + L[HEAD].b,
                    sums, kSumBlocks, G.D1b, s));
    // D1b's gradient leaves head_bwd masked. A block's first conv (input: a concatenation,
    // a pooled map or the packed input) writes its input gradient unmasked: the up-conv half
    // of a concatenation has no ReLU, and the skip half and the pooled maps are masked by the
    // pooling backward, after the pooled gradient has been added.
    if ((rc = conv_b(D1B, A.D1a, G.D1b, &G.D1a, true))) return rc;
    if ((rc = conv_b(D1A, A.CAT1, G.D1a, &G.CAT1, false))) return rc;
    if ((rc = up_b(UP1, A.D2b, view(G.CAT1, 0, C), G.D2b))) return rc;
    if ((rc = conv_b(D2B, A.D2a, G.D2b, &G.D2a, true))) return rc;
    if ((rc = conv_b(D2A, A.CAT2, G.D2a, &G.CAT2, false))) return rc;
    if ((rc = up_b(UP2, A.D3b, view(G.CAT2, 0, 2 * C), G.D3b))) return rc;
    if ((rc = conv_b(D3B, A.D3a, G.D3b, &G.D3a, true))) return rc;
    if ((rc = conv_b(D3A, A.CAT3, G.D3a, &G.CAT3, false))) return rc;
    if ((rc = up_b(UP3, A.E4b, view(G.CAT3, 0, 4 * C), G.E4b))) return rc;
    if ((rc = conv_b(B4, A.E4a, G.E4b, &G.E4a, true))) return rc;
    if ((rc = conv_b(A4, A.P3, G.E4a, &G.P3, false))) return rc;
    const Tensor S1 = view(A.CAT1, C, C), S2 = view(A.CAT2, 2 * C, 2 * C), S3 = view(A.CAT3, 4 * C, 4 * C);
    const Tensor dS1 = view(G.CAT1, C, C), dS2 = view(G.CAT2, 2 * C, 2 * C), dS3 = view(G.CAT3, 4 * C, 4 * C);
    NN_TRY(maxpool_bwd_add(S3, A.P3, G.P3, dS3, s));          // skip gradient + pooled gradient
    if ((rc = conv_b(B3, A.E3a, dS3, &G.E3a, true))) return rc;
    if ((rc = conv_b(A3, A.P2, G.E3a, &G.P2, false))) return rc;
    NN_TRY(maxpool_bwd_add(S2, A.P2, G.P2, dS2, s));
    if ((rc = conv_b(B2, A.E2a, dS2, &G.E2a, true))) return rc;
    if ((rc = conv_b(A2, A.P1, G.E2a, &G.P1, false))) return rc;
    NN_TRY(maxpool_bwd_add(S1, A.P1, G.P1, dS1, s));
    if ((rc = conv_b(B1, A.E1a, dS1, &G.E1a, true))) return rc;
    if ((rc = conv_b(A1, A.X0, G.E1a, nullptr, false))) return rc;
    return EIT_OK;
}

int prepare_weights(const eit_unet* u, const float* prm, bf16* wf, bf16* wt, hipStream_t s) {
    NN_TRY(to_bf16(prm, wf, u->n_params, s));
    OtiTable tab{};
    for (const Layer& l : u->L) {
        if (l.kind != 0 && l.kind != 1) continue;
        const int j = tab.n++;
        tab.O[j] = l.cout;
        tab.T[j] = l.kind == 0 ? 9 : 4;
        tab.I[j] = l.cin;
        tab.src[j] = l.w;
        tab.dst[j] = l.wt;
        tab.begin[j + 1] = tab.begin[j] + (size_t)tab.O[j] * tab.T[j] * tab.I[j];
    }
    NN_TRY(transpose_oti(tab, prm, wt, s));
    return EIT_OK;
}

int check_dims(const eit_unet* u, int nb, int h, int w) {
    if (!u) return eit::nn_fail(EIT_ERR_INVALID_ARG, "network is NULL");
    if (nb < 1 || h < 8 || w < 8 || h % 8 || w % 8)
        return eit::nn_fail(EIT_ERR_SHAPE, "batch >= 1 and image sides multiples of 8 (>= 8) required");
    if ((size_t)nb * h * w * 16 * u->base > ((size_t)1 << 31))
        return eit::nn_fail(EIT_ERR_SHAPE, "activation tensor exceeds 2^31 elements");
    return EIT_OK;
}

}  // namespace

extern "C" int eit_unet_create(int32_t base, eit_unet** out) {
    if (!out) return eit::nn_fail(EIT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (base < 8 || base > 64 || (base & (base - 1)))
        return eit::nn_fail(EIT_ERR_INVALID_ARG, "base channels must be a power of two in [8, 64]");
    eit_unet* u = new eit_unet();
    u->base = base;
    const int c = base;
    struct Def { int kind, cin, cout; };
    const Def defs[NLAYERS] = {{0, kInC, c},      {0, c, c},          {0, c, 2 * c},      {0, 2 * c, 2 * c},
                               {0, 2 * c, 4 * c}, {0, 4 * c, 4 * c},  {0, 4 * c, 8 * c},  {0, 8 * c, 8 * c},
                               {1, 8 * c, 4 * c}, {0, 8 * c, 4 * c},  {0, 4 * c, 4 * c},  {1, 4 * c, 2 * c},
                               {0, 4 * c, 2 * c}, {0, 2 * c, 2 * c},  {1, 2 * c, c},      {0, 2 * c, c},
                               {0, c, c},         {2, c, 2}};
    size_t off = 0;
    for (const Def& d : defs) {
        Layer l{};
        l.kind = d.kind; l.cin = d.cin; l.cout = d.cout;
        const size_t nw = d.kind == 0 ? (size_t)d.cout * 9 * d.cin
                          : d.kind == 1 ? (size_t)4 * d.cout * d.cin : (size_t)d.cout * d.cin;
        l.w = off;
        l.wt = off;                      // transposed copy uses the same offset in its buffer
        l.b = off + nw;                  // bias directly after the weights
        off += nw + d.cout;
        u->L.push_back(l);
    }
    u->n_params = off;
    *out = u;
    return EIT_OK;
}

extern "C" void eit_unet_destroy(eit_unet* u) { delete u; }

extern "C" int64_t eit_unet_param_count(const eit_unet* u) { return u ? (int64_t)u->n_params : 0; }

extern "C" int eit_unet_layers(const eit_unet* u, eit_unet_layer* out, int32_t cap) {
    if (!u) return 0;
    const int n = (int)u->L.size();
    for (int i = 0; i < n && i < cap && out; ++i) {
        out[i].kind = u->L[i].kind;
        out[i].cin = u->L[i].cin;
        out[i].cout = u->L[i].cout;
        out[i].w_off = (int64_t)u->L[i].w;
        out[i].b_off = (int64_t)u->L[i].b;
    }
    return n;
}

extern "C" size_t eit_unet_workspace_bytes(const eit_unet* u, int32_t nb, int32_t h, int32_t w,
                                           int32_t train) {
    if (!u || check_dims(u, nb, h, w)) return 0;
    return layout(u, nb, h, w, train != 0).end;
}

extern "C" int eit_unet_forward(const eit_unet* u, const float* params, const float* x, float* y,
                                int32_t nb, int32_t h, int32_t w, void* ws, size_t ws_bytes,
                                void* stream) {
    if (int rc = check_dims(u, nb, h, w)) return rc;
    if (!params || !x || !y || !ws) return eit::nn_fail(EIT_ERR_INVALID_ARG, "NULL argument");
    const WsLayout W = layout(u, nb, h, w, false);
    if (ws_bytes < W.end) return eit::nn_fail(EIT_ERR_NOMEM, "workspace too small");
    char* base = (char*)ws;
    hipStream_t s = (hipStream_t)stream;
    bf16* wf = (bf16*)(base + W.wbf);
    bf16* wt = (bf16*)(base + W.wtb);
    if (int rc = prepare_weights(u, params, wf, wt, s)) return rc;
    const Acts A = carve(u, base, W.acts, nb, h, w);
    Ctx c{u, params, wf, wt, s};
    if (int rc = forward(c, A, x, y, nb, h, w)) return rc;
    return EIT_OK;
}

extern "C" int eit_unet_train_step(const eit_unet* u, float* params, float* adam_m, float* adam_v,
                                   float* grad, int32_t step, double lr, const float* x,
                                   const float* target, int32_t nb, int32_t h, int32_t w,
                                   double* loss, void* ws, size_t ws_bytes, void* stream) {
    if (int rc = check_dims(u, nb, h, w)) return rc;
    if (!params || !grad || !x || !target || !loss || !ws)
        return eit::nn_fail(EIT_ERR_INVALID_ARG, "NULL argument");
    if (step > 0 && (!adam_m || !adam_v)) return eit::nn_fail(EIT_ERR_INVALID_ARG, "Adam moments are NULL");
    if (!(lr >= 0.0) || !std::isfinite(lr)) return eit::nn_fail(EIT_ERR_INVALID_ARG, "lr must be finite and >= 0");
    const WsLayout W = layout(u, nb, h, w, true);
    if (ws_bytes < W.end) return eit::nn_fail(EIT_ERR_NOMEM, "workspace too small");
    char* base = (char*)ws;
    hipStream_t s = (hipStream_t)stream;
    bf16* wf = (bf16*)(base + W.wbf);
    bf16* wt = (bf16*)(base + W.wtb);
    if (int rc = prepare_weights(u, params, wf, wt, s)) return rc;
    const Acts A = carve(u, base, W.acts, nb, h, w);
    const Acts G = carve(u, base, W.grads, nb, h, w);
    // every gradient tensor is written by a data-gradient GEMM before anything accumulates
    // into it (max-pool backward adds onto the skip gradients), so the arena needs no clearing
    float* out = (float*)(base + W.out);
    float* dout = (float*)(base + W.dout);
    Ctx c{u, params, wf, wt, s};
    if (int rc = forward(c, A, x, out, nb, h, w)) return rc;
    const size_t n = (size_t)nb * 2 * h * w;
    NN_TRY(mse_loss(out, target, n, (double*)(base + W.mpart), kSumBlocks, loss, dout, s));
    if (int rc = backward(c, A, G, dout, grad, (float*)(base + W.part), (float*)(base + W.sums), nb, h, w))
        return rc;
    if (step > 0) {
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, step)));
        const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, step)));
        NN_TRY(adam(params, adam_m, adam_v, grad, u->n_params, (float)lr, b1, b2, eps, c1, c2, s));
    }
    return EIT_OK;
}

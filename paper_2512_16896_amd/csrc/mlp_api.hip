// mlp_api.hip -- C ABI of the learned proposal's network: init, forward,
// backward (gradients into caller buffers) and one AdamW training step.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"
#include "scn.h"

namespace {

int check_net(const scn_mlp* n, bool train) {
    if (!n) return scn_fail(SCN_E_INVALID_ARG, "null network");
    for (int l = 0; l <= SCN_MLP_LAYERS; ++l)
        if (n->dims[l] <= 0) return scn_fail(SCN_E_INVALID_ARG, "dims[%d] must be > 0", l);
    for (int l = 0; l < SCN_MLP_LAYERS; ++l) {
        if (n->dims[l] % 32) return scn_fail(SCN_E_INVALID_ARG, "dims[%d] must be a multiple of 32", l);
        if (!n->w[l] || !n->b[l] || !n->wb[l] || !n->wt[l])
            return scn_fail(SCN_E_INVALID_ARG, "layer %d tensors missing", l);
        if (train && (!n->m_w[l] || !n->v_w[l] || !n->m_b[l] || !n->v_b[l]))
            return scn_fail(SCN_E_INVALID_ARG, "layer %d AdamW moments missing", l);
    }
    return SCN_OK;
}

int max_hidden(const scn_mlp* n) {
    int h = 0;
    for (int l = 1; l < SCN_MLP_LAYERS; ++l) h = n->dims[l] > h ? n->dims[l] : h;
    return h;
}

using scn::align256;

// Bump allocator over the caller's workspace.
struct Arena {
    char* base;
    size_t off;
    template <typename T>
    T* take(size_t count) {
        T* p = (T*)(base + off);
        off += align256(count * sizeof(T));
        return p;
    }
};

// Forward pass; activations of layers 1..3 (BF16, [M][dims[l]]) go to act[1..3],
// the FP32 logits to `logits`.
int forward(const scn_mlp* n, const uint16_t* x, int M, uint16_t* const* act, float* logits,
            hipStream_t st, const int32_t* m_dev = nullptr) {
    const void* in = x;
    for (int l = 0; l < SCN_MLP_LAYERS; ++l) {
        const int K = n->dims[l], N = n->dims[l + 1];
        const bool last = l == SCN_MLP_LAYERS - 1;
        SCN_HIP(scn::launch_gemm(M, N, K, in, K, n->wb[l], K, n->b[l], !last,
                                 last ? logits : nullptr, last ? nullptr : act[l + 1], N, st,
                                 m_dev));
        in = act[l + 1];
    }
    return SCN_OK;
}

// Backward pass into gw / gb (FP32, caller layout) and *loss, with its
// buffers in `ws` (ws_mlp_backward_bytes).
int backward(const scn_mlp* n, const uint16_t* x, int M, const int32_t* bins, const float* tgt,
             int L, float* const* gw, float* const* gb, float* loss, void* ws, hipStream_t st) {
    const int H = max_hidden(n), NO = n->dims[SCN_MLP_LAYERS];
    int maxdim = NO;
    for (int l = 0; l <= SCN_MLP_LAYERS; ++l) maxdim = n->dims[l] > maxdim ? n->dims[l] : maxdim;
    Arena a{(char*)ws, 0};
    uint16_t* act[SCN_MLP_LAYERS] = {nullptr};
    for (int l = 1; l < SCN_MLP_LAYERS; ++l) act[l] = a.take<uint16_t>((size_t)M * H);
    float* logits = a.take<float>((size_t)M * NO);
    float* dz32 = a.take<float>((size_t)M * NO);
    uint16_t* dzb = a.take<uint16_t>((size_t)M * NO);
    uint16_t* dyt = a.take<uint16_t>((size_t)maxdim * M);
    uint16_t* int_ = a.take<uint16_t>((size_t)maxdim * M);
    float* da = a.take<float>((size_t)M * H);
    uint16_t* dp = a.take<uint16_t>((size_t)M * H);

    if (int r = forward(n, x, M, act, logits, st)) return r;
    SCN_HIP(scn::launch_fill_f32(dz32, (size_t)M * NO, 0.f, st));
    SCN_HIP(scn::launch_fill_f32(loss, 1, 0.f, st));
    SCN_HIP(scn::launch_bce(M, NO, L, logits, bins, tgt, 1.f / (float)((size_t)M * L), dz32,
                            loss, st));
    SCN_HIP(scn::launch_f32_to_bf16(M * NO, dz32, dzb, st));

    // dY of the current layer: BF16 [M][dims[l+1]]
    const uint16_t* dy = dzb;
    for (int l = SCN_MLP_LAYERS - 1; l >= 0; --l) {
        const int K = n->dims[l], N = n->dims[l + 1];
        const void* in = l == 0 ? (const void*)x : (const void*)act[l];
        // dW = dY^T X  (reduction over the M states)
        SCN_HIP(scn::launch_transpose_bf16(M, N, dy, N, dyt, M, st));
        SCN_HIP(scn::launch_transpose_bf16(M, K, in, K, int_, M, st));
        SCN_HIP(scn::launch_gemm(N, K, M, dyt, M, int_, M, nullptr, false, gw[l], nullptr, K, st));
        // db = column sums of dY (the last layer from the FP32 gradient)
        if (l == SCN_MLP_LAYERS - 1)
            SCN_HIP(scn::launch_colsum_f32(M, N, dz32, gb[l], st));
        else
            SCN_HIP(scn::launch_colsum_bf16(M, N, dy, gb[l], st));
        if (l == 0) break;
        // dX = dY W, then through the ReLU of layer l's input
        SCN_HIP(scn::launch_gemm(M, K, N, dy, N, n->wt[l], N, nullptr, false, da, nullptr, K, st));
        SCN_HIP(scn::launch_relu_bwd(M * K, da, act[l], dp, st));
        dy = dp;
    }
    return SCN_OK;
}

int max_dim(const scn_mlp* n) {
    int m = 0;
    for (int l = 0; l <= SCN_MLP_LAYERS; ++l) m = n->dims[l] > m ? n->dims[l] : m;
    return m;
}

size_t grad_bytes(const scn_mlp* n) {
    size_t b = 0;
    for (int l = 0; l < SCN_MLP_LAYERS; ++l)
        b += align256((size_t)n->dims[l + 1] * n->dims[l] * 4) + align256((size_t)n->dims[l + 1] * 4);
    return b;
}

}  // namespace

size_t scn::ws_mlp_forward_bytes(const scn_mlp* n, int rows) {
    return rows > 0 ? 3 * align256((size_t)rows * max_hidden(n) * 2) : 0;
}

size_t scn::ws_mlp_backward_bytes(const scn_mlp* n, int rows) {
    if (rows <= 0) return 0;
    const size_t M = (size_t)rows, H = (size_t)max_hidden(n), NO = (size_t)n->dims[SCN_MLP_LAYERS];
    const size_t D = (size_t)max_dim(n);
    return 3 * align256(M * H * 2) + 2 * align256(M * NO * 4) + align256(M * NO * 2) +
           2 * align256(D * M * 2) + align256(M * H * 4) + align256(M * H * 2);
}

size_t scn::ws_mlp_train_bytes(const scn_mlp* n, int rows) {
    return rows > 0 ? ws_mlp_backward_bytes(n, rows) + grad_bytes(n) : 0;
}

int scn_mlp_forward_ws(const scn_mlp* n, const uint16_t* x, int M, float* logits, void* act_ws,
                       hipStream_t st, const int32_t* m_dev) {
    if (M <= 0) return SCN_OK;
    Arena a{(char*)act_ws, 0};
    uint16_t* act[SCN_MLP_LAYERS] = {nullptr};
    for (int l = 1; l < SCN_MLP_LAYERS; ++l) act[l] = a.take<uint16_t>((size_t)M * max_hidden(n));
    return forward(n, x, M, act, logits, st, m_dev);
}

extern "C" {

int scn_mlp_init(scn_ctx* c, scn_mlp* n, uint64_t seed, scn_stream stream) {
    if (int r = scn_check_ctx(c)) return r;
    if (int r = check_net(n, false)) return r;
    const hipStream_t st = (hipStream_t)stream;
    for (int l = 0; l < SCN_MLP_LAYERS; ++l) {
        const int rows = n->dims[l + 1], cols = n->dims[l];
        SCN_HIP(scn::launch_init_layer(rows, cols, seed, l, n->w[l], n->wb[l], n->wt[l], st));
        SCN_HIP(scn::launch_fill_f32(n->b[l], rows, 0.f, st));
        if (n->m_w[l]) SCN_HIP(scn::launch_fill_f32(n->m_w[l], (size_t)rows * cols, 0.f, st));
        if (n->v_w[l]) SCN_HIP(scn::launch_fill_f32(n->v_w[l], (size_t)rows * cols, 0.f, st));
        if (n->m_b[l]) SCN_HIP(scn::launch_fill_f32(n->m_b[l], rows, 0.f, st));
        if (n->v_b[l]) SCN_HIP(scn::launch_fill_f32(n->v_b[l], rows, 0.f, st));
    }
    n->step = 0;
    return SCN_OK;
}

int scn_mlp_forward(scn_ctx* c, const scn_mlp* n, const uint16_t* x, int32_t M, float* logits,
                    scn_stream stream) {
    if (int r = scn_check_ctx(c)) return r;
    if (int r = check_net(n, false)) return r;
    if (M < 0) return scn_fail(SCN_E_INVALID_ARG, "M must be >= 0");
    if (M == 0) return SCN_OK;
    if (!x || !logits) return scn_fail(SCN_E_INVALID_ARG, "x and logits required");
    void* ws;
    if (int r = scn_workspace(c, scn::ws_mlp_forward_bytes(n, M), &ws)) return r;
    return scn_mlp_forward_ws(n, x, M, logits, ws, (hipStream_t)stream);
}

int scn_mlp_backward(scn_ctx* c, const scn_mlp* n, const uint16_t* x, int32_t M,
                     const int32_t* bins, const float* tgt, int32_t L, float* const* gw,
                     float* const* gb, float* loss, scn_stream stream) {
    if (int r = scn_check_ctx(c)) return r;
    if (int r = check_net(n, false)) return r;
    if (M <= 0 || M % 32) return scn_fail(SCN_E_INVALID_ARG, "M must be a positive multiple of 32");
    if (L <= 0) return scn_fail(SCN_E_INVALID_ARG, "L must be > 0");
    if (!x || !bins || !tgt || !gw || !gb || !loss)
        return scn_fail(SCN_E_INVALID_ARG, "x, labels, gradients and loss required");
    for (int l = 0; l < SCN_MLP_LAYERS; ++l)
        if (!gw[l] || !gb[l]) return scn_fail(SCN_E_INVALID_ARG, "gradient buffer %d missing", l);
    void* ws;
    if (int r = scn_workspace(c, scn::ws_mlp_backward_bytes(n, M), &ws)) return r;
    return backward(n, x, M, bins, tgt, L, gw, gb, loss, ws, (hipStream_t)stream);
}

int scn_mlp_train_step(scn_ctx* c, scn_mlp* n, const uint16_t* x, int32_t M, const int32_t* bins,
                       const float* tgt, int32_t L, const scn_adamw* opt, float* loss,
                       scn_stream stream) {
    if (int r = scn_check_ctx(c)) return r;
    if (int r = check_net(n, true)) return r;
    if (!opt || !(opt->lr > 0.f) || !(opt->beta1 >= 0.f && opt->beta1 < 1.f) ||
        !(opt->beta2 >= 0.f && opt->beta2 < 1.f) || !(opt->eps > 0.f) || !(opt->weight_decay >= 0.f))
        return scn_fail(SCN_E_INVALID_ARG, "bad AdamW parameters");
    if (M <= 0 || M % 32) return scn_fail(SCN_E_INVALID_ARG, "M must be a positive multiple of 32");
    if (L <= 0 || !x || !bins || !tgt || !loss)
        return scn_fail(SCN_E_INVALID_ARG, "x, labels and loss required");
    const hipStream_t st = (hipStream_t)stream;
    // the backward pass takes the front of the workspace, the gradients the
    // block after it
    const size_t bw = scn::ws_mlp_backward_bytes(n, M);
    void* ws;
    if (int r = scn_workspace(c, scn::ws_mlp_train_bytes(n, M), &ws)) return r;
    Arena g{(char*)ws + bw, 0};
    float* gw[SCN_MLP_LAYERS];
    float* gb[SCN_MLP_LAYERS];
    for (int l = 0; l < SCN_MLP_LAYERS; ++l) {
        gw[l] = g.take<float>((size_t)n->dims[l + 1] * n->dims[l]);
        gb[l] = g.take<float>((size_t)n->dims[l + 1]);
    }
    if (int r = backward(n, x, M, bins, tgt, L, gw, gb, loss, ws, st)) return r;
    const double t = (double)(n->step + 1);
    const float c1 = (float)(1.0 - std::pow((double)opt->beta1, t));
    const float c2 = (float)(1.0 - std::pow((double)opt->beta2, t));
    for (int l = 0; l < SCN_MLP_LAYERS; ++l) {
        const int rows = n->dims[l + 1], cols = n->dims[l];
        SCN_HIP(scn::launch_adamw(rows, cols, n->w[l], gw[l], n->m_w[l], n->v_w[l], n->wb[l],
                                  n->wt[l], opt->lr, opt->beta1, opt->beta2, opt->eps,
                                  opt->weight_decay, c1, c2, st));
        // biases: no decay, no BF16 copy
        SCN_HIP(scn::launch_adamw(1, rows, n->b[l], gb[l], n->m_b[l], n->v_b[l], nullptr, nullptr,
                                  opt->lr, opt->beta1, opt->beta2, opt->eps, 0.f, c1, c2, st));
    }
    n->step += 1;
    return SCN_OK;
}

}  // extern "C"

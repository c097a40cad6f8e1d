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

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Bump allocator over the context workspace.
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
            hipStream_t st) {
    const void* in = x;
    for (int l = 0; l < SCN_MLP_LAYERS; ++l) {
        const int K = n->dims[l], N = n->dims[l + 1];
        const bool last = l == SCN_MLP_LAYERS - 1;
        SCN_HIP(scn::launch_gemm(M, N, K, in, K, n->wb[l], K, n->b[l], !last,
                                 last ? logits : nullptr, last ? nullptr : act[l + 1], N, st));
        in = act[l + 1];
    }
    return SCN_OK;
}

// Backward pass into gw / gb (FP32, caller layout) and *loss.
int backward(scn_ctx* c, const scn_mlp* n, const uint16_t* x, int M, const int32_t* bins,
             const float* tgt, int L, float* const* gw, float* const* gb, float* loss,
             hipStream_t st) {
    const int H = max_hidden(n), NO = n->dims[SCN_MLP_LAYERS];
    int maxdim = NO;
    for (int l = 0; l <= SCN_MLP_LAYERS; ++l) maxdim = n->dims[l] > maxdim ? n->dims[l] : maxdim;
    const size_t need = 3 * align256((size_t)M * H * 2) + 2 * align256((size_t)M * NO * 4) +
                        align256((size_t)M * NO * 2) + 2 * align256((size_t)maxdim * M * 2) +
                        align256((size_t)M * H * 4) + align256((size_t)M * H * 2) + 256;
    void* ws;
    if (int r = scn_workspace(c, need, &ws)) return r;
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

}  // namespace

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
    const int H = max_hidden(n);
    void* ws;
    if (int r = scn_workspace(c, 3 * align256((size_t)M * H * 2) + 256, &ws)) return r;
    Arena a{(char*)ws, 0};
    uint16_t* act[SCN_MLP_LAYERS] = {nullptr};
    for (int l = 1; l < SCN_MLP_LAYERS; ++l) act[l] = a.take<uint16_t>((size_t)M * H);
    return forward(n, x, M, act, logits, (hipStream_t)stream);
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
    return backward(c, n, x, M, bins, tgt, L, gw, gb, loss, (hipStream_t)stream);
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
    // gradient buffers live in a second region after the backward workspace:
    // grow the workspace to hold both, backward's part first.
    size_t grad_floats = 0;
    for (int l = 0; l < SCN_MLP_LAYERS; ++l)
        grad_floats += (size_t)n->dims[l + 1] * n->dims[l] + n->dims[l + 1];
    // The backward pass takes the front of the workspace; keep the gradients
    // in a separately sized block at its end.
    const int H = max_hidden(n), NO = n->dims[SCN_MLP_LAYERS];
    int maxdim = NO;
    for (int l = 0; l <= SCN_MLP_LAYERS; ++l) maxdim = n->dims[l] > maxdim ? n->dims[l] : maxdim;
    const size_t bw = 3 * align256((size_t)M * H * 2) + 2 * align256((size_t)M * NO * 4) +
                      align256((size_t)M * NO * 2) + 2 * align256((size_t)maxdim * M * 2) +
                      align256((size_t)M * H * 4) + align256((size_t)M * H * 2) + 256;
    const size_t gbytes = align256(grad_floats * 4) + SCN_MLP_LAYERS * 256;
    void* ws;
    if (int r = scn_workspace(c, bw + gbytes, &ws)) return r;
    Arena g{(char*)ws + bw, 0};
    float* gw[SCN_MLP_LAYERS];
    float* gb[SCN_MLP_LAYERS];
    for (int l = 0; l < SCN_MLP_LAYERS; ++l) {
        gw[l] = g.take<float>((size_t)n->dims[l + 1] * n->dims[l]);
        gb[l] = g.take<float>((size_t)n->dims[l + 1]);
    }
    if (int r = backward(c, n, x, M, bins, tgt, L, gw, gb, loss, st)) return r;
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

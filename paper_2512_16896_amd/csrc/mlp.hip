// mlp.hip -- the learned pose proposal's network on CDNA4 matrix cores.
//
// A 4-layer perceptron (inputs -> 512 -> 512 -> 512 -> 4096 pose-bin logits,
// ReLU) with BF16 weights and activations on v_mfma_f32_16x16x32_bf16 and FP32
// accumulation, its backward pass (BF16 dgrad / wgrad GEMMs, FP32 bias and
// ReLU backward), binary cross-entropy on the labelled bins, and AdamW with
// FP32 master weights that refreshes the BF16 copies (W and W^T).
//
// Every GEMM is C[M x N] = A[M x K] * B[N x K]^T with both operands
// K-contiguous (row-major, leading dimensions lda / ldb), so each lane feeds
// the matrix core 8 consecutive BF16 values per operand; the backward pass
// gets its other orientations from explicit transposes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"
#include "internal.h"

namespace scn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(__bf16 v) { return (float)v; }
__device__ __forceinline__ __bf16 f2bf(float v) { return (__bf16)v; }   // round to nearest even

// ---------------------------------------------------------------------------
// GEMM.  Workgroup tile BM x BN (128 x 128 or 64 x 64), 4 waves in a 2 x 2
// grid, each wave (BM/2) x (BN/2) of MFMA 16x16x32 tiles; K in steps of 32.
// Both operand tiles of a step (BM x 32 and BN x 32 BF16) are staged in LDS,
// double-buffered: the global loads of step k+1 are in flight while the waves
// run step k's MFMAs from LDS, one barrier per step.  LDS rows are padded to
// 40 BF16 (80 B) so the 16 rows a fragment read touches fall in distinct
// banks.  Fragment layout (v_mfma_f32_16x16x32_bf16): lane l supplies row
// l % 16 of a 16-row fragment, 8 BF16 at column 8 (l / 16) of the K step; the
// result for lane l is rows 4 (l / 16) .. +3 of column l % 16.  Rows / columns
// past M / N are clamped on load and skipped on store.  K % 32 == 0.  With
// m_dev, the row count is min(M, *m_dev), read on the device: the grid covers
// M rows and the workgroups past the live rows leave at once (compacted
// batches whose size only the device knows).  Every output element sums its K
// products in the same order whatever the tile shape or row count.
constexpr int kLdsRow = 40;

template <int BM, int BN, bool kBias, bool kRelu>
__global__ __launch_bounds__(256) void k_gemm(int M, const int32_t* __restrict__ m_dev, int N,
                                             int K, const __bf16* __restrict__ A, int lda,
                                             const __bf16* __restrict__ B, int ldb,
                                             const float* __restrict__ bias, float* __restrict__ C32,
                                             __bf16* __restrict__ C16, int ldc) {
    constexpr int FM = BM / 32, FN = BN / 32;       // 16 x 16 fragments per wave
    constexpr int LA = BM / 64, LB = BN / 64;       // 16-B global loads per thread
    __shared__ __attribute__((aligned(16))) __bf16 As[2][BM * kLdsRow];
    __shared__ __attribute__((aligned(16))) __bf16 Bs[2][BN * kLdsRow];
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    // XCD-aware tile order.  The chip deals workgroup L (in launch order) to
    // XCD L % 8, each XCD with its own L2.  With a multiple of 8 row blocks,
    // XCD x takes row blocks x, x + 8, x + 16, ... with all their column
    // tiles, so a row block's A panel is fetched into one L2 and reused by its
    // column tiles there, and the live row blocks of a short (device-counted)
    // batch still spread over all XCDs.  Which workgroup computes a tile does
    // not change its result.
    int tm = blockIdx.y, tn = blockIdx.x;
    if ((gridDim.y & 7) == 0) {
        const int L = blockIdx.y * gridDim.x + blockIdx.x, slot = L >> 3;
        tm = (L & 7) + 8 * (slot / (int)gridDim.x);
        tn = slot % (int)gridDim.x;
    }
    const int bm = tm * BM, bn = tn * BN;
    if (m_dev) M = min(M, *m_dev);
    if (bm >= M) return;   // the whole workgroup, before any barrier
    const int r = lane & 15, kq = (lane >> 4) * 8;
    const int wm = (wave >> 1) * (BM / 2), wn = (wave & 1) * (BN / 2);

    // global source and LDS destination of this thread's chunks
    const __bf16* ga[LA];
    const __bf16* gb[LB];
    int la[LA], lb[LB];
#pragma unroll
    for (int i = 0; i < LA; ++i) {
        const int c = t + 256 * i, row = c >> 2, col = (c & 3) * 8;
        ga[i] = A + (size_t)min(bm + row, M - 1) * lda + col;
        la[i] = row * kLdsRow + col;
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
        const int c = t + 256 * i, row = c >> 2, col = (c & 3) * 8;
        gb[i] = B + (size_t)min(bn + row, N - 1) * ldb + col;
        lb[i] = row * kLdsRow + col;
    }
    bf16x8 ra[LA], rb[LB];
#pragma unroll
    for (int i = 0; i < LA; ++i) ra[i] = *(const bf16x8*)ga[i];
#pragma unroll
    for (int i = 0; i < LB; ++i) rb[i] = *(const bf16x8*)gb[i];
#pragma unroll
    for (int i = 0; i < LA; ++i) *(bf16x8*)&As[0][la[i]] = ra[i];
#pragma unroll
    for (int i = 0; i < LB; ++i) *(bf16x8*)&Bs[0][lb[i]] = rb[i];
    __syncthreads();

    f32x4 acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    int cur = 0;
    for (int k = 32; k <= K; k += 32) {
        const bool more = k < K;
        if (more) {   // next step's operands, in flight during this step's MFMAs
#pragma unroll
            for (int i = 0; i < LA; ++i) ra[i] = *(const bf16x8*)(ga[i] + k);
#pragma unroll
            for (int i = 0; i < LB; ++i) rb[i] = *(const bf16x8*)(gb[i] + k);
        }
        bf16x8 fa[FM], fb[FN];
#pragma unroll
        for (int i = 0; i < FM; ++i) fa[i] = *(const bf16x8*)&As[cur][(wm + 16 * i + r) * kLdsRow + kq];
#pragma unroll
        for (int j = 0; j < FN; ++j) fb[j] = *(const bf16x8*)&Bs[cur][(wn + 16 * j + r) * kLdsRow + kq];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        if (more) {
            // the other buffer was last read in the previous step, before the
            // barrier that ended it
#pragma unroll
            for (int i = 0; i < LA; ++i) *(bf16x8*)&As[cur ^ 1][la[i]] = ra[i];
#pragma unroll
            for (int i = 0; i < LB; ++i) *(bf16x8*)&Bs[cur ^ 1][lb[i]] = rb[i];
        }
        __syncthreads();
        cur ^= 1;
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        const int n = bn + wn + 16 * j + r;
        if (n >= N) continue;
        const float bv = kBias ? bias[n] : 0.f;
#pragma unroll
        for (int i = 0; i < FM; ++i) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = bm + wm + 16 * i + (lane >> 4) * 4 + e;
                if (m >= M) continue;
                float v = acc[i][j][e] + bv;
                if (kRelu) v = fmaxf(v, 0.f);
                if (C32) C32[(size_t)m * ldc + n] = v;
                if (C16) C16[(size_t)m * ldc + n] = f2bf(v);
            }
        }
    }
}

template <int BM, int BN>
static void launch_gemm_tile(int M, const int32_t* m_dev, int N, int K, const __bf16* a, int lda,
                             const __bf16* b, int ldb, const float* bias, bool relu, float* C32,
                             __bf16* c16, int ldc, hipStream_t st) {
    dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM), block(256);
    if (bias && relu)
        hipLaunchKernelGGL((k_gemm<BM, BN, true, true>), grid, block, 0, st, M, m_dev, N, K, a, lda, b, ldb, bias, C32, c16, ldc);
    else if (bias)
        hipLaunchKernelGGL((k_gemm<BM, BN, true, false>), grid, block, 0, st, M, m_dev, N, K, a, lda, b, ldb, bias, C32, c16, ldc);
    else if (relu)
        hipLaunchKernelGGL((k_gemm<BM, BN, false, true>), grid, block, 0, st, M, m_dev, N, K, a, lda, b, ldb, bias, C32, c16, ldc);
    else
        hipLaunchKernelGGL((k_gemm<BM, BN, false, false>), grid, block, 0, st, M, m_dev, N, K, a, lda, b, ldb, bias, C32, c16, ldc);
}

hipError_t launch_gemm(int M, int N, int K, const void* A, int lda, const void* B, int ldb,
                       const float* bias, bool relu, float* C32, void* C16, int ldc,
                       hipStream_t st, const int32_t* m_dev) {
    if (M <= 0 || N <= 0) return hipSuccess;
    if (K <= 0 || K % 32 || lda % 8 || ldb % 8) return hipErrorInvalidValue;
    auto a = (const __bf16*)A;
    auto b = (const __bf16*)B;
    auto c16 = (__bf16*)C16;
    // the large tile only when it still gives every compute unit a workgroup
    const long long big = (long long)((N + 127) / 128) * ((M + 127) / 128);
    if (big >= 256)
        launch_gemm_tile<128, 128>(M, m_dev, N, K, a, lda, b, ldb, bias, relu, C32, c16, ldc, st);
    else
        launch_gemm_tile<64, 64>(M, m_dev, N, K, a, lda, b, ldb, bias, relu, C32, c16, ldc, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// out[c][r] = in[r][c] for a rows x cols BF16 matrix (32 x 32 tiles via LDS).
__global__ __launch_bounds__(256) void k_transpose_bf16(int rows, int cols,
                                                       const __bf16* __restrict__ in, int ldi,
                                                       __bf16* __restrict__ out, int ldo) {
    __shared__ __bf16 tile[32][34];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int y = ty; y < 32; y += 8) {
        const int r = r0 + y, c = c0 + tx;
        if (r < rows && c < cols) tile[y][tx] = in[(size_t)r * ldi + c];
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        const int c = c0 + y, r = r0 + tx;
        if (r < rows && c < cols) out[(size_t)c * ldo + r] = tile[tx][y];
    }
}

hipError_t launch_transpose_bf16(int rows, int cols, const void* in, int ldi, void* out, int ldo,
                                 hipStream_t st) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_transpose_bf16, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(256), 0, st,
                       rows, cols, (const __bf16*)in, ldi, (__bf16*)out, ldo);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP32 -> BF16 conversion of a matrix (optionally with a column offset/pad).
__global__ void k_f32_to_bf16(int n, const float* __restrict__ in, __bf16* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f2bf(in[i]);
}

hipError_t launch_f32_to_bf16(int n, const float* in, void* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_f32_to_bf16, dim3((n + 255) / 256), dim3(256), 0, st, n, in, (__bf16*)out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Binary cross-entropy on labelled bins.  labels: bins [M][L] (int32, -1 =
// none) and targets [M][L] (0 / 1).  Writes the dense gradient of the mean loss
// w.r.t. the logits as BF16 (zeros elsewhere; the caller zeroes dz first) and
// adds sum(loss) / count to *loss.  Duplicate bins in a row accumulate.
__global__ void k_bce(int M, int N, int L, const float* __restrict__ z, const int32_t* __restrict__ bins,
                      const float* __restrict__ tgt, float inv_count, float* __restrict__ dz32,
                      float* __restrict__ loss) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float l = 0.f;
    if (i < M * L) {
        const int m = i / L;
        const int b = bins[i];
        if (b >= 0 && b < N) {
            const float zz = z[(size_t)m * N + b];
            const float t = tgt[i];
            // softplus(z) - t z, stable form
            l = fmaxf(zz, 0.f) - zz * t + log1pf(expf(-fabsf(zz)));
            const float g = (1.f / (1.f + expf(-zz)) - t) * inv_count;
            atomicAdd(dz32 + (size_t)m * N + b, g);
        }
    }
    // wave reduction of the loss, one atomic per wave
    for (int o = 32; o >= 1; o >>= 1) l += __shfl_xor(l, o, 64);
    if ((threadIdx.x & 63) == 0 && l != 0.f) atomicAdd(loss, l * inv_count);
}

hipError_t launch_bce(int M, int N, int L, const float* z, const int32_t* bins, const float* tgt,
                      float inv_count, float* dz32, float* loss, hipStream_t st) {
    const int n = M * L;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bce, dim3((n + 255) / 256), dim3(256), 0, st, M, N, L, z, bins, tgt,
                       inv_count, dz32, loss);
    return hipGetLastError();
}

// dP = dA (FP32) * [act > 0] as BF16 (ReLU backward; act is the BF16 output).
__global__ void k_relu_bwd(int n, const float* __restrict__ da, const __bf16* __restrict__ act,
                           __bf16* __restrict__ dp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dp[i] = f2bf(bf2f(act[i]) > 0.f ? da[i] : 0.f);
}

hipError_t launch_relu_bwd(int n, const float* da, const void* act, void* dp, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_relu_bwd, dim3((n + 255) / 256), dim3(256), 0, st, n, da,
                       (const __bf16*)act, (__bf16*)dp);
    return hipGetLastError();
}

// db[n] = sum_m d[m][n] (BF16 or FP32 rows).
template <typename T>
__global__ __launch_bounds__(256) void k_colsum(int M, int N, const T* __restrict__ d,
                                                float* __restrict__ db) {
    // 32 columns per workgroup, 8 row groups: thread (g, c) sums rows g, g+8, ...
    // of column c, then the 8 partial sums are added in LDS (fixed order)
    __shared__ float part[8][32];
    const int c = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int n = blockIdx.x * 32 + c;
    float s = 0.f;
    if (n < N)
        for (int m = g; m < M; m += 8) s += (float)d[(size_t)m * N + n];
    part[g][c] = s;
    __syncthreads();
    if (g == 0 && n < N) {
        float t = 0.f;
        for (int q = 0; q < 8; ++q) t += part[q][c];
        db[n] = t;
    }
}

hipError_t launch_colsum_bf16(int M, int N, const void* d, float* db, hipStream_t st) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_colsum<__bf16>), dim3((N + 31) / 32), dim3(256), 0, st, M, N,
                       (const __bf16*)d, db);
    return hipGetLastError();
}

hipError_t launch_colsum_f32(int M, int N, const float* d, float* db, hipStream_t st) {
    if (N <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_colsum<float>), dim3((N + 31) / 32), dim3(256), 0, st, M, N, d, db);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// AdamW (decoupled weight decay) on FP32 master weights [rows][cols]; refreshes
// the BF16 copy (same layout) and, when wt != nullptr, its transpose.
__global__ void k_adamw(int rows, int cols, float* __restrict__ w, const float* __restrict__ g,
                        float* __restrict__ m1, float* __restrict__ m2, __bf16* __restrict__ wb,
                        __bf16* __restrict__ wt, float lr, float b1, float b2, float eps, float wd,
                        float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * cols) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float v = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    const float mh = a / c1, vh = v / c2;
    const float nw = w[i] - lr * (mh / (sqrtf(vh) + eps) + wd * w[i]);
    w[i] = nw;
    const __bf16 q = f2bf(nw);
    if (wb) wb[i] = q;
    if (wt) {
        const int r = i / cols, c = i - r * cols;
        wt[(size_t)c * rows + r] = q;
    }
}

hipError_t launch_adamw(int rows, int cols, float* w, const float* g, float* m1, float* m2,
                        void* wb, void* wt, float lr, float b1, float b2, float eps, float wd,
                        float c1, float c2, hipStream_t st) {
    const int n = rows * cols;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adamw, dim3((n + 255) / 256), dim3(256), 0, st, rows, cols, w, g, m1, m2,
                       (__bf16*)wb, (__bf16*)wt, lr, b1, b2, eps, wd, c1, c2);
    return hipGetLastError();
}

// Kaiming-uniform weights (bound sqrt(6 / fan_in)) from Philox4x32-10 with
// counter (element, layer, 0x4D4C50, 0); biases zero.  Writes FP32 master,
// BF16 copy and BF16 transpose.
__global__ void k_init_layer(int rows, int cols, uint64_t seed, int layer, float* __restrict__ w,
                             __bf16* __restrict__ wb, __bf16* __restrict__ wt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * cols) return;
    const U4 r = philox10(U4{(uint32_t)i, (uint32_t)layer, 0x4D4C50u, 0u}, (uint32_t)seed,
                          (uint32_t)(seed >> 32));
    const float bound = sqrtf(6.f / (float)cols);
    const float v = bound * signed_unit(r.a);
    w[i] = v;
    const __bf16 q = f2bf(v);
    wb[i] = q;
    const int rr = i / cols, c = i - rr * cols;
    wt[(size_t)c * rows + rr] = q;
}

hipError_t launch_init_layer(int rows, int cols, uint64_t seed, int layer, float* w, void* wb,
                             void* wt, hipStream_t st) {
    const int n = rows * cols;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_layer, dim3((n + 255) / 256), dim3(256), 0, st, rows, cols, seed,
                       layer, w, (__bf16*)wb, (__bf16*)wt);
    return hipGetLastError();
}

__global__ void k_fill_f32(float* p, size_t n, float v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace scn

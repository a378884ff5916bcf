// Learned warm start: a small MLP predicting per-unit utilisations, trained
// and evaluated on the GPU with hand-written BF16 MFMA kernels (gfx950).
//
// Network: x[32] -> relu(x W1 + b1)[256] -> relu(h1 W2 + b2)[256]
//          -> sigmoid(h2 . w3 + b3) = predicted busy probability of a unit.
// Weights are kept in FP32 (master copy, Adam state) and cast to BF16 for
// the matrix products; products accumulate in FP32 on the matrix cores.
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace hqmlp {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// round-to-nearest-even FP32 -> BF16 (NaN kept quiet)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// C[M x N] (FP32) = op(A)[M x K] * op(B)[K x N] (+ C if accumulate), BF16 operands.
// op(A) = A (row-major M x K, leading dim lda) or, if TA, A^T for A stored
// K x M; op(B) = B (K x N) or, if TB, B^T for B stored N x K.  One wave per
// 32 x 32 output tile, v_mfma_f32_32x32x8_bf16 over K in steps of 8.
// Requires M % 32 == 0, N % 32 == 0, K % 8 == 0 (checked by the host).
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_bf16(const uint16_t* __restrict__ A, const uint16_t* __restrict__ B,
                                                 float* __restrict__ C, int M, int N, int K, int lda, int ldb,
                                                 int ldc, int accumulate) {
    const int lane = threadIdx.x & 63;
    const int wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int tiles_n = N >> 5;
    const int tm = wave / tiles_n, tn = wave % tiles_n;
    if (tm >= (M >> 5)) return;
    const int m0 = tm << 5, n0 = tn << 5;
    const int i = lane & 31, kk = (lane >> 5) << 2;
    f32x16 acc;
    for (int e = 0; e < 16; ++e) acc[e] = 0.0f;
    for (int k0 = 0; k0 < K; k0 += 8) {
        bf16x4 a, b;
        for (int e = 0; e < 4; ++e) {
            const int k = k0 + kk + e;
            a[e] = (short)(TA ? A[(size_t)k * lda + (m0 + i)] : A[(size_t)(m0 + i) * lda + k]);
            b[e] = (short)(TB ? B[(size_t)(n0 + i) * ldb + k] : B[(size_t)k * ldb + (n0 + i)]);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
    // D layout: element e of lane l holds row (e % 4) + 8 (e / 4) + 4 (l / 32), column l % 32
    for (int e = 0; e < 16; ++e) {
        const int row = (e & 3) + ((e >> 2) << 3) + ((lane >> 5) << 2);
        float* c = C + (size_t)(m0 + row) * ldc + (n0 + i);
        *c = accumulate ? *c + acc[e] : acc[e];
    }
}

// h = relu(z + bias) for a [rows x 256] block; writes BF16 copy for the next product.
__global__ void bias_relu(const float* __restrict__ z, const float* __restrict__ bias, float* __restrict__ pre,
                          uint16_t* __restrict__ hb, int rows, int cols) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * cols) return;
    const float v = z[idx] + bias[idx % cols];
    pre[idx] = v;
    hb[idx] = f2bf(v > 0.0f ? v : 0.0f);
}

// Output unit: y = sigmoid(h2 . w3 + b3) per row (BF16 h2, FP32 w3); with
// targets, also the MSE loss terms and dL/dz for rows < valid.
__global__ void head_forward(const uint16_t* __restrict__ h2, const float* __restrict__ w3, const float* __restrict__ b3,
                             const float* __restrict__ target, float* __restrict__ y, float* __restrict__ dz,
                             float* __restrict__ loss_terms, int rows, int valid, int cols) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    float z = b3[0];
    for (int c = 0; c < cols; ++c) z += bf2f(h2[(size_t)r * cols + c]) * w3[c];
    const float s = 1.0f / (1.0f + __expf(-z));
    y[r] = s;
    if (target) {
        const float d = (r < valid) ? (s - target[r]) : 0.0f;
        loss_terms[r] = d * d;
        dz[r] = (r < valid) ? 2.0f * d / (float)valid * s * (1.0f - s) : 0.0f;
    }
}

// dw3[c] = sum_r h2[r][c] dz[r]; db3 = sum_r dz[r] (one block per column group).
__global__ void head_backward(const uint16_t* __restrict__ h2, const float* __restrict__ dz, float* __restrict__ dw3,
                              float* __restrict__ db3, int rows, int cols) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < cols) {
        float s = 0.0f;
        for (int r = 0; r < rows; ++r) s += bf2f(h2[(size_t)r * cols + c]) * dz[r];
        dw3[c] = s;
    }
    if (c == 0) {
        float s = 0.0f;
        for (int r = 0; r < rows; ++r) s += dz[r];
        db3[0] = s;
    }
}

// dh2[r][c] = dz[r] w3[c] [pre2 > 0], as BF16 operand.
__global__ void head_to_hidden(const float* __restrict__ dz, const float* __restrict__ w3,
                               const float* __restrict__ pre, uint16_t* __restrict__ dhb, float* __restrict__ dh,
                               int rows, int cols) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * cols) return;
    const int r = idx / cols, c = idx % cols;
    const float v = pre[idx] > 0.0f ? dz[r] * w3[c] : 0.0f;
    dh[idx] = v;
    dhb[idx] = f2bf(v);
}

// g = g_in [pre > 0] -> FP32 and BF16 copies.
__global__ void relu_backward(const float* __restrict__ gin, const float* __restrict__ pre, float* __restrict__ g,
                              uint16_t* __restrict__ gb, int n) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const float v = pre[idx] > 0.0f ? gin[idx] : 0.0f;
    g[idx] = v;
    gb[idx] = f2bf(v);
}

// db[c] = sum_r g[r][c]
__global__ void col_sum(const float* __restrict__ g, float* __restrict__ db, int rows, int cols) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.0f;
    for (int r = 0; r < rows; ++r) s += g[(size_t)r * cols + c];
    db[c] = s;
}

// Adam on the FP32 master parameters, then the BF16 copy of the matrices.
__global__ void adam_step(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                          float* __restrict__ m2, uint16_t* __restrict__ pb, int n, float lr, float b1, float b2,
                          float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.0f - b1) * gi;
    const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = v;
    const float w = p[i] - lr * (a / c1) / (sqrtf(v / c2) + eps);
    p[i] = w;
    if (pb) pb[i] = f2bf(w);
}

__global__ void to_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = f2bf(src[i]);
}

}  // namespace hqmlp

namespace hqk {

using namespace hqmlp;

static inline dim3 g1(int n) { return dim3((n + 255) / 256); }

hipError_t mlp_gemm(bool ta, bool tb, const uint16_t* A, const uint16_t* B, float* C, int M, int N, int K, int lda,
                    int ldb, int ldc, bool accumulate, hipStream_t s) {
    if (M % 32 || N % 32 || K % 8 || M <= 0 || N <= 0 || K <= 0) return hipErrorInvalidValue;
    const int waves = (M / 32) * (N / 32);
    const dim3 grid((waves + 3) / 4), block(256);
    const int acc = accumulate ? 1 : 0;
    if (!ta && !tb)
        hipLaunchKernelGGL((gemm_bf16<false, false>), grid, block, 0, s, A, B, C, M, N, K, lda, ldb, ldc, acc);
    else if (ta && !tb)
        hipLaunchKernelGGL((gemm_bf16<true, false>), grid, block, 0, s, A, B, C, M, N, K, lda, ldb, ldc, acc);
    else if (!ta && tb)
        hipLaunchKernelGGL((gemm_bf16<false, true>), grid, block, 0, s, A, B, C, M, N, K, lda, ldb, ldc, acc);
    else
        hipLaunchKernelGGL((gemm_bf16<true, true>), grid, block, 0, s, A, B, C, M, N, K, lda, ldb, ldc, acc);
    return hipGetLastError();
}

hipError_t mlp_bias_relu(const float* z, const float* bias, float* pre, uint16_t* hb, int rows, int cols,
                         hipStream_t s) {
    hipLaunchKernelGGL(bias_relu, g1(rows * cols), dim3(256), 0, s, z, bias, pre, hb, rows, cols);
    return hipGetLastError();
}

hipError_t mlp_head_forward(const uint16_t* h2, const float* w3, const float* b3, const float* target, float* y,
                            float* dz, float* loss_terms, int rows, int valid, int cols, hipStream_t s) {
    hipLaunchKernelGGL(head_forward, g1(rows), dim3(256), 0, s, h2, w3, b3, target, y, dz, loss_terms, rows, valid,
                       cols);
    return hipGetLastError();
}

hipError_t mlp_head_backward(const uint16_t* h2, const float* dz, float* dw3, float* db3, int rows, int cols,
                             hipStream_t s) {
    hipLaunchKernelGGL(head_backward, g1(cols), dim3(256), 0, s, h2, dz, dw3, db3, rows, cols);
    return hipGetLastError();
}

hipError_t mlp_head_to_hidden(const float* dz, const float* w3, const float* pre, uint16_t* dhb, float* dh, int rows,
                              int cols, hipStream_t s) {
    hipLaunchKernelGGL(head_to_hidden, g1(rows * cols), dim3(256), 0, s, dz, w3, pre, dhb, dh, rows, cols);
    return hipGetLastError();
}

hipError_t mlp_relu_backward(const float* gin, const float* pre, float* g, uint16_t* gb, int n, hipStream_t s) {
    hipLaunchKernelGGL(relu_backward, g1(n), dim3(256), 0, s, gin, pre, g, gb, n);
    return hipGetLastError();
}

hipError_t mlp_col_sum(const float* g, float* db, int rows, int cols, hipStream_t s) {
    hipLaunchKernelGGL(col_sum, g1(cols), dim3(256), 0, s, g, db, rows, cols);
    return hipGetLastError();
}

hipError_t mlp_adam(float* p, const float* g, float* m1, float* m2, uint16_t* pb, int n, float lr, float b1,
                    float b2, float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(adam_step, g1(n), dim3(256), 0, s, p, g, m1, m2, pb, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t mlp_to_bf16(const float* src, uint16_t* dst, int n, hipStream_t s) {
    hipLaunchKernelGGL(to_bf16, g1(n), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

}  // namespace hqk

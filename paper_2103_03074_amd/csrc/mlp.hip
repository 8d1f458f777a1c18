// Learned step-time model: a 3-layer perceptron d_in -> H -> H -> 1 with ReLU,
// trained on measured step times (log milliseconds) with mean squared error
// and Adam.  Everything runs in these kernels in FP32: a tiled GEMM with
// optional bias / ReLU / ReLU-mask epilogues (forward and both backward
// products), column sums for the bias gradients, and the Adam update.  All
// reductions run in a fixed order (no atomics), so training is repeatable.
//
// Parameters are one flat FP32 array: W1 (d_in x H, row-major), b1 (H),
// W2 (H x H), b2 (H), W3 (H x 1), b3 (1).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <random>
#include <string>
#include <vector>

#include "mlp.hpp"

namespace tn {

namespace {

constexpr int TS = 16;   // GEMM tile

// C[M x N] = op(A) op(B) (+ bias[N]) with op(X) = X or X^T;
// epi 0: plain, 1: ReLU, 2: multiply by mask (Zmask > 0).
__global__ void __launch_bounds__(256) k_gemm(const float* A, const float* B, float* C, int M, int N, int K,
                                              int lda, int ldb, int ldc, int ta, int tb, const float* bias,
                                              int epi, const float* Zmask, int ldz) {
    __shared__ float As[TS][TS + 1], Bs[TS][TS + 1];
    const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
    const int row = blockIdx.y * TS + ty, col = blockIdx.x * TS + tx;
    float acc = 0.f;
    for (int k0 = 0; k0 < K; k0 += TS) {
        const int ka = k0 + tx, kb = k0 + ty;
        const int ar = blockIdx.y * TS + ty;
        As[ty][tx] = (ar < M && ka < K) ? (ta ? A[(size_t)ka * lda + ar] : A[(size_t)ar * lda + ka]) : 0.f;
        Bs[ty][tx] = (kb < K && col < N) ? (tb ? B[(size_t)col * ldb + kb] : B[(size_t)kb * ldb + col]) : 0.f;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < TS; ++k) acc = fmaf(As[ty][k], Bs[k][tx], acc);
        __syncthreads();
    }
    if (row < M && col < N) {
        if (bias) acc += bias[col];
        if (epi == 1) acc = fmaxf(acc, 0.f);
        if (epi == 2) acc = Zmask[(size_t)row * ldz + col] > 0.f ? acc : 0.f;
        C[(size_t)row * ldc + col] = acc;
    }
}

// out[j] = sum_i X[i * ld + j] for i < rows (fixed order)
__global__ void __launch_bounds__(256) k_colsum(const float* X, float* out, int rows, int cols, int ld) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= cols) return;
    float s = 0.f;
    for (int i = 0; i < rows; ++i) s += X[(size_t)i * ld + j];
    out[j] = s;
}

// dY = 2 (y - t) / B, and per-block partial sums of (y - t)^2
__global__ void __launch_bounds__(256) k_loss_grad(const float* y, const float* t, float* dy, int n, float* part) {
    __shared__ float sh[256];
    const int i = blockIdx.x * 256 + threadIdx.x;
    float e = 0.f;
    if (i < n) {
        const float d = y[i] - t[i];
        dy[i] = 2.f * d / (float)n;
        e = d * d;
    }
    sh[threadIdx.x] = e;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Adam (Kingma & Ba) with bias correction.
__global__ void __launch_bounds__(256) k_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1,
                                              float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t gemm(hipStream_t s, const float* A, const float* B, float* C, int M, int N, int K, int lda, int ldb,
                int ldc, int ta, int tb, const float* bias, int epi, const float* Z = nullptr, int ldz = 0) {
    dim3 grid((N + TS - 1) / TS, (M + TS - 1) / TS);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, s, A, B, C, M, N, K, lda, ldb, ldc, ta, tb, bias, epi, Z, ldz);
    return hipGetLastError();
}

}  // namespace

void step_features(int m, int n, int k, int b, int kernel, int esize, float* f) {
    f[0] = m / 32.f;
    f[1] = n / 32.f;
    f[2] = k / 32.f;
    f[3] = b / 16.f;
    f[4] = (m + n + b) / 32.f;
    f[5] = (m + k + b) / 32.f;
    f[6] = (n + k + b) / 32.f;
    f[7] = (m + n + k + b) / 48.f;
    const double bytes = esize * (std::exp2((double)(m + k + b)) + std::exp2((double)(n + k + b)) +
                                  std::exp2((double)(m + n + b)));
    f[8] = (float)(std::log2(bytes) / 40.0);
    f[9] = (kernel == 1 || kernel == 4 || kernel == 5) ? 1.f : 0.f;   // MFMA classes
    f[10] = kernel == 0 ? 1.f : 0.f;
    f[11] = kernel == 2 ? 1.f : 0.f;
}

int64_t Mlp::n_params() const { return (int64_t)d_in * H + H + (int64_t)H * H + H + H + 1; }

std::string Mlp::create(int d_in_, int hidden, uint64_t seed) {
    d_in = d_in_;
    H = hidden;
    const int64_t n = n_params();
    std::vector<float> h(n, 0.f);
    std::mt19937_64 rng(seed);
    auto fill = [&](int64_t off, int fan_in, int64_t cnt) {
        std::normal_distribution<float> nd(0.f, std::sqrt(2.f / (float)fan_in));
        for (int64_t i = 0; i < cnt; ++i) h[off + i] = nd(rng);
    };
    fill(o_w1(), d_in, (int64_t)d_in * H);
    fill(o_w2(), H, (int64_t)H * H);
    fill(o_w3(), H, H);
    if (hipMalloc(&params, sizeof(float) * n) != hipSuccess || hipMalloc(&grads, sizeof(float) * n) != hipSuccess ||
        hipMalloc(&m1, sizeof(float) * n) != hipSuccess || hipMalloc(&m2, sizeof(float) * n) != hipSuccess)
        return "hipMalloc failed";
    if (hipMemcpy(params, h.data(), sizeof(float) * n, hipMemcpyHostToDevice) != hipSuccess) return "upload failed";
    if (hipMemset(m1, 0, sizeof(float) * n) != hipSuccess || hipMemset(m2, 0, sizeof(float) * n) != hipSuccess)
        return "hipMemset failed";
    step = 0;
    return "";
}

std::string Mlp::ensure_batch(int B) {
    if (B <= cap) return "";
    release_batch();
    const size_t per = (size_t)B;
    if (hipMalloc(&z1, sizeof(float) * per * H) != hipSuccess || hipMalloc(&h1, sizeof(float) * per * H) != hipSuccess ||
        hipMalloc(&z2, sizeof(float) * per * H) != hipSuccess || hipMalloc(&h2, sizeof(float) * per * H) != hipSuccess ||
        hipMalloc(&dz2, sizeof(float) * per * H) != hipSuccess || hipMalloc(&dz1, sizeof(float) * per * H) != hipSuccess ||
        hipMalloc(&y, sizeof(float) * per) != hipSuccess || hipMalloc(&dy, sizeof(float) * per) != hipSuccess ||
        hipMalloc(&part, sizeof(float) * (per / 256 + 2)) != hipSuccess)
        return "hipMalloc failed";
    cap = B;
    return "";
}

void Mlp::release_batch() {
    for (float** p : {&z1, &h1, &z2, &h2, &dz2, &dz1, &y, &dy, &part})
        if (*p) {
            (void)hipFree(*p);
            *p = nullptr;
        }
    cap = 0;
}

void Mlp::release() {
    release_batch();
    for (float** p : {&params, &grads, &m1, &m2})
        if (*p) {
            (void)hipFree(*p);
            *p = nullptr;
        }
}

#define TN_CK(x)                                                                       \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) return std::string(#x) + ": " + hipGetErrorString(e_); \
    } while (0)

std::string Mlp::forward(const float* x, int B, float* out, hipStream_t s) {
    std::string e = ensure_batch(B);
    if (!e.empty()) return e;
    float* P = params;
    TN_CK(gemm(s, x, P + o_w1(), z1, B, H, d_in, d_in, H, H, 0, 0, P + o_b1(), 0));
    TN_CK(gemm(s, x, P + o_w1(), h1, B, H, d_in, d_in, H, H, 0, 0, P + o_b1(), 1));
    TN_CK(gemm(s, h1, P + o_w2(), z2, B, H, H, H, H, H, 0, 0, P + o_b2(), 0));
    TN_CK(gemm(s, h1, P + o_w2(), h2, B, H, H, H, H, H, 0, 0, P + o_b2(), 1));
    TN_CK(gemm(s, h2, P + o_w3(), out ? out : y, B, 1, H, H, 1, 1, 0, 0, P + o_b3(), 0));
    return "";
}

std::string Mlp::gradient(const float* x, const float* t, int B, float* loss, hipStream_t s) {
    std::string e = forward(x, B, y, s);
    if (!e.empty()) return e;
    float* P = params;
    float* G = grads;
    const int nb = (B + 255) / 256;
    hipLaunchKernelGGL(k_loss_grad, dim3(nb), dim3(256), 0, s, y, t, dy, B, part);
    TN_CK(hipGetLastError());
    // layer 3: dW3 = h2^T dy, db3 = sum dy, dz2 = (dy W3^T) * (z2 > 0)
    TN_CK(gemm(s, h2, dy, G + o_w3(), H, 1, B, H, 1, 1, 1, 0, nullptr, 0));
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, s, dy, G + o_b3(), B, 1, 1);
    TN_CK(hipGetLastError());
    TN_CK(gemm(s, dy, P + o_w3(), dz2, B, H, 1, 1, 1, H, 0, 1, nullptr, 2, z2, H));
    // layer 2
    TN_CK(gemm(s, h1, dz2, G + o_w2(), H, H, B, H, H, H, 1, 0, nullptr, 0));
    hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, s, dz2, G + o_b2(), B, H, H);
    TN_CK(hipGetLastError());
    TN_CK(gemm(s, dz2, P + o_w2(), dz1, B, H, H, H, H, H, 0, 1, nullptr, 2, z1, H));
    // layer 1
    TN_CK(gemm(s, x, dz1, G + o_w1(), d_in, H, B, d_in, H, H, 1, 0, nullptr, 0));
    hipLaunchKernelGGL(k_colsum, dim3((H + 255) / 256), dim3(256), 0, s, dz1, G + o_b1(), B, H, H);
    TN_CK(hipGetLastError());
    if (loss) {
        std::vector<float> hp(nb);
        TN_CK(hipMemcpyAsync(hp.data(), part, sizeof(float) * nb, hipMemcpyDeviceToHost, s));
        TN_CK(hipStreamSynchronize(s));
        double tot = 0;
        for (float v : hp) tot += v;
        *loss = (float)(tot / B);
    }
    return "";
}

std::string Mlp::adam(float lr, hipStream_t s) {
    ++step;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
    const int n = (int)n_params();
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, s, params, grads, m1, m2, n, lr, b1, b2, eps, c1,
                       c2);
    TN_CK(hipGetLastError());
    return "";
}

}  // namespace tn

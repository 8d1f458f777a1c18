// Learned step-time model (device side).  See mlp.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace tn {

struct Mlp {
    int d_in = 0, H = 0;
    float* params = nullptr;   // flat: W1, b1, W2, b2, W3, b3
    float* grads = nullptr;
    float* m1 = nullptr;       // Adam moments
    float* m2 = nullptr;
    int step = 0;
    int cap = 0;               // batch capacity of the activation buffers
    float *z1 = nullptr, *h1 = nullptr, *z2 = nullptr, *h2 = nullptr, *dz2 = nullptr, *dz1 = nullptr;
    float *y = nullptr, *dy = nullptr, *part = nullptr;
    // training support of the features (fallback to the FLOP model outside it)
    std::string support;

    int64_t n_params() const;
    int64_t o_w1() const { return 0; }
    int64_t o_b1() const { return (int64_t)d_in * H; }
    int64_t o_w2() const { return o_b1() + H; }
    int64_t o_b2() const { return o_w2() + (int64_t)H * H; }
    int64_t o_w3() const { return o_b2() + H; }
    int64_t o_b3() const { return o_w3() + H; }

    std::string create(int d_in, int hidden, uint64_t seed);
    std::string ensure_batch(int B);
    std::string forward(const float* x, int B, float* out, hipStream_t s);
    std::string gradient(const float* x, const float* t, int B, float* loss, hipStream_t s);
    std::string adam(float lr, hipStream_t s);
    void release_batch();
    void release();
};

// Step features for the model: shape logs, operand/output logs, log work,
// log bytes, kernel class one-hot.
constexpr int kFeatures = 12;
void step_features(int m, int n, int k, int b, int kernel, int esize, float* out);

}  // namespace tn

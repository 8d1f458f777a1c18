// Mixing the most probable computed bitstrings with random ones (section
// "Discussions", footnote on the correlation of the samples: the k bitstrings
// of highest probability in the computed subspace are mixed with a large
// number of random bitstrings, so that the set is barely correlated while its
// XEB stays positive).
//
// The k largest probabilities P = |A|^2 are found by a radix select on the
// bit patterns of the float64 probabilities (non-negative doubles order like
// their unsigned bit patterns): eight passes of 8-bit digit histograms,
// most significant digit first, each over the elements whose decided digits
// match.  Ties at the threshold go to the lowest indices.  A deterministic
// compaction (per-block counts, block offsets, in-block scans) writes the
// selected indices in increasing index order as whole n-bit strings (closed
// qubits at s1), and the selected probabilities are summed per block in a
// fixed order.  The random part is caller-supplied 64-bit words masked to n
// bits.
#include "mix.hpp"

#include <algorithm>
#include <vector>

namespace tn {

namespace {

constexpr int kThreads = 256;
constexpr int kPer = 4;                      // elements per thread
constexpr int kBlockElems = kThreads * kPer;

// Probability as the oracle forms it: both squares rounded, then the sum
// (no fused multiply-add), so both sides compare the same doubles.
__device__ __forceinline__ uint64_t prob_key(double2 a) {
    const double p = __dadd_rn(__dmul_rn(a.x, a.x), __dmul_rn(a.y, a.y));
    return (uint64_t)__double_as_longlong(p);
}

__device__ __forceinline__ bool prefix_match(uint64_t key, uint64_t prefix, int decided) {
    return decided == 0 || (key >> (64 - decided)) == (prefix >> (64 - decided));
}

__global__ void __launch_bounds__(kThreads) k_zero_u32(uint32_t* p, int n) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void __launch_bounds__(kThreads) k_topk_hist(const double2* amps, uint64_t n, uint64_t prefix,
                                                        int decided, uint32_t* hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0u;
    __syncthreads();
    const int shift = 56 - decided;
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kThreads) {
        const uint64_t key = prob_key(amps[i]);
        if (prefix_match(key, prefix, decided)) atomicAdd(&h[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    const uint32_t c = h[threadIdx.x];
    if (c) atomicAdd(&hist[threadIdx.x], c);
}

// Exclusive scan over the block of one 0/1 flag per element (kPer per
// thread, thread t holds elements kPer t ..); returns the thread's prefix and
// the block total.
__device__ int block_excl_scan(int mine, int* sh, int& total) {
    const int t = threadIdx.x;
    sh[t] = mine;
    __syncthreads();
    for (int d = 1; d < kThreads; d <<= 1) {
        const int v = t >= d ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    total = sh[kThreads - 1];
    const int excl = t > 0 ? sh[t - 1] : 0;
    __syncthreads();
    return excl;
}

// Per block of kBlockElems elements: how many keys exceed the threshold and
// how many equal it.
__global__ void __launch_bounds__(kThreads) k_topk_count(const double2* amps, uint64_t n, uint64_t thr,
                                                         uint32_t* gt, uint32_t* eq) {
    __shared__ int sh[kThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kBlockElems + (uint64_t)threadIdx.x * kPer;
    int g = 0, e = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        if (base + j >= n) break;
        const uint64_t key = prob_key(amps[base + j]);
        g += key > thr;
        e += key == thr;
    }
    int tg, te;
    (void)block_excl_scan(g, sh, tg);
    (void)block_excl_scan(e, sh, te);
    if (threadIdx.x == 0) {
        gt[blockIdx.x] = (uint32_t)tg;
        eq[blockIdx.x] = (uint32_t)te;
    }
}

// Writes the selected elements of each block at out[block_off[b] + rank]
// (rank in index order) as whole bitstrings, and the block's sum of their
// probabilities (tree reduction in a fixed order).
__global__ void __launch_bounds__(kThreads) k_topk_scatter(const double2* amps, uint64_t n, uint64_t thr,
                                                           const uint64_t* block_off, const uint32_t* eq_take,
                                                           MixBits mb, uint64_t* out, double* block_sum) {
    __shared__ int sh[kThreads];
    __shared__ double sd[kThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kBlockElems + (uint64_t)threadIdx.x * kPer;
    uint64_t key[kPer];
    double p[kPer];
    int e = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        key[j] = 0;
        p[j] = 0.0;
        if (base + j < n) {
            const double2 a = amps[base + j];
            key[j] = prob_key(a);
            p[j] = __longlong_as_double((long long)key[j]);
            e += key[j] == thr;
        }
    }
    int te;
    int er = block_excl_scan(e, sh, te);   // rank among the block's threshold ties
    const int take = (int)eq_take[blockIdx.x];
    bool sel[kPer];
    int s = 0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        sel[j] = false;
        if (base + j >= n) continue;
        if (key[j] > thr) sel[j] = true;
        else if (key[j] == thr) sel[j] = er++ < take;
        s += sel[j];
    }
    int ts;
    int pos = block_excl_scan(s, sh, ts);
    double mine = 0.0;
#pragma unroll
    for (int j = 0; j < kPer; ++j) {
        if (!sel[j]) continue;
        const uint64_t s2 = base + j;
        uint64_t v = mb.base;
        for (int q = 0; q < mb.n_open; ++q) v |= ((s2 >> (mb.n_open - 1 - q)) & 1ull) << mb.pos[q];
        out[block_off[blockIdx.x] + (uint64_t)pos++] = v;
        mine += p[j];
    }
    sd[threadIdx.x] = mine;
    __syncthreads();
    for (int d = kThreads / 2; d > 0; d >>= 1) {
        if (threadIdx.x < d) sd[threadIdx.x] += sd[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) block_sum[blockIdx.x] = sd[0];
}

__global__ void __launch_bounds__(kThreads) k_random_strings(const uint64_t* words, uint64_t n, uint64_t mask,
                                                             uint64_t* out) {
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kThreads)
        out[i] = words[i] & mask;
}

uint64_t n_blocks(uint64_t n) { return (n + kBlockElems - 1) / kBlockElems; }

struct Ws {
    uint32_t* hist;
    uint32_t* gt;
    uint32_t* eq;
    uint32_t* eq_take;
    uint64_t* off;
    double* sums;
};

Ws carve(void* ws, uint64_t blocks) {
    unsigned char* p = static_cast<unsigned char*>(ws);
    Ws w;
    w.sums = reinterpret_cast<double*>(p);
    p += 8 * blocks;
    w.off = reinterpret_cast<uint64_t*>(p);
    p += 8 * blocks;
    w.hist = reinterpret_cast<uint32_t*>(p);
    p += 4 * 256;
    w.gt = reinterpret_cast<uint32_t*>(p);
    p += 4 * blocks;
    w.eq = reinterpret_cast<uint32_t*>(p);
    p += 4 * blocks;
    w.eq_take = reinterpret_cast<uint32_t*>(p);
    return w;
}

}  // namespace

uint64_t mix_workspace_bytes(uint64_t n) {
    const uint64_t b = n_blocks(n);
    return 8 * b + 8 * b + 4 * 256 + 4 * b * 3;
}

std::string mix_topk(const double* d_amps, uint64_t n, uint64_t k, const MixBits& mb, const uint64_t* d_words,
                     uint64_t n_random, int n_qubits, uint64_t* d_out, void* ws, hipStream_t s, double& p_top) {
    p_top = 0.0;
    const uint64_t blocks = n_blocks(n);
    Ws w = carve(ws, blocks);
    const double2* amps = reinterpret_cast<const double2*>(d_amps);
    hipError_t e = hipSuccess;
    auto fail = [&](const char* what) { return std::string(what) + ": " + hipGetErrorString(e); };
    if (k > 0) {
        // radix select of the k-th largest key
        uint64_t prefix = 0, k_rem = k;
        const unsigned hist_grid = (unsigned)std::min<uint64_t>(std::max<uint64_t>(1, (n + kThreads - 1) / kThreads),
                                                                 2048);
        for (int decided = 0; decided < 64; decided += 8) {
            hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(kThreads), 0, s, w.hist, 256);
            hipLaunchKernelGGL(k_topk_hist, dim3(hist_grid), dim3(kThreads), 0, s, amps, n, prefix, decided, w.hist);
            uint32_t h[256];
            if ((e = hipGetLastError()) != hipSuccess ||
                (e = hipMemcpyAsync(h, w.hist, sizeof(h), hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return fail("top-k histogram");
            int dg = 255;
            for (; dg > 0; --dg) {
                if ((uint64_t)h[dg] >= k_rem) break;
                k_rem -= h[dg];
            }
            prefix |= (uint64_t)dg << (56 - decided);
        }
        // k_rem keys equal to the threshold are taken, lowest indices first
        hipLaunchKernelGGL(k_topk_count, dim3((unsigned)blocks), dim3(kThreads), 0, s, amps, n, prefix, w.gt, w.eq);
        std::vector<uint32_t> gt(blocks), eq(blocks), take(blocks);
        std::vector<uint64_t> off(blocks);
        if ((e = hipGetLastError()) != hipSuccess ||
            (e = hipMemcpyAsync(gt.data(), w.gt, 4 * blocks, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipMemcpyAsync(eq.data(), w.eq, 4 * blocks, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return fail("top-k counts");
        uint64_t run = 0, eq_left = k_rem;
        for (uint64_t b = 0; b < blocks; ++b) {
            take[b] = (uint32_t)std::min<uint64_t>(eq[b], eq_left);
            eq_left -= take[b];
            off[b] = run;
            run += gt[b] + take[b];
        }
        if (run != k || eq_left != 0) return "top-k selection inconsistent";
        std::vector<double> sums(blocks);
        if ((e = hipMemcpyAsync(w.eq_take, take.data(), 4 * blocks, hipMemcpyHostToDevice, s)) != hipSuccess ||
            (e = hipMemcpyAsync(w.off, off.data(), 8 * blocks, hipMemcpyHostToDevice, s)) != hipSuccess)
            return fail("top-k offsets");
        hipLaunchKernelGGL(k_topk_scatter, dim3((unsigned)blocks), dim3(kThreads), 0, s, amps, n, prefix, w.off,
                           w.eq_take, mb, d_out, w.sums);
        if ((e = hipGetLastError()) != hipSuccess ||
            (e = hipMemcpyAsync(sums.data(), w.sums, 8 * blocks, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return fail("top-k scatter");
        for (uint64_t b = 0; b < blocks; ++b) p_top += sums[b];
    }
    if (n_random > 0) {
        const uint64_t mask = n_qubits >= 64 ? ~0ull : ((1ull << n_qubits) - 1);
        const unsigned g = (unsigned)std::min<uint64_t>((n_random + kThreads - 1) / kThreads, 1u << 16);
        hipLaunchKernelGGL(k_random_strings, dim3(g), dim3(kThreads), 0, s, d_words, n_random, mask, d_out + k);
        if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(s)) != hipSuccess)
            return fail("random strings");
    }
    return "";
}

}  // namespace tn

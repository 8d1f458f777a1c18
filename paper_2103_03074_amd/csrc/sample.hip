// Sampling open-qubit bitstrings s2 from the conditional distribution
// P(s2 | s1) = |A[s2]|^2 / sum |A|^2 (appendix C; the conclusion notes that
// the method can sample from this distribution).  Inverse transform: the
// float64 inclusive prefix sum of |A|^2 in index order is built by a
// three-pass block scan (per-block scans, a scan of the block sums, then the
// block offsets added), and each caller-supplied uniform u picks the smallest
// index j with cdf[j] > u * cdf[L - 1] by binary search.  Every sum is taken
// in a fixed order, so results are bitwise repeatable.
#include "sample.hpp"

#include <algorithm>
#include <mutex>

namespace tn {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;                          // elements per thread
constexpr int kScanBlock = kScanThreads * kScanPer;  // elements per block

// Inclusive scan of a block's kScanBlock values held kScanPer per thread
// (thread t holds elements kScanPer t .. kScanPer t + kScanPer - 1); returns
// the exclusive prefix of thread t's first element and writes the block sum.
__device__ double block_exclusive_prefix(double mine, double* sh, double& total) {
    const int t = threadIdx.x;
    sh[t] = mine;
    __syncthreads();
    // Hillis-Steele over the per-thread sums (fixed order of additions)
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const double v = t >= d ? sh[t - d] : 0.0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    total = sh[kScanThreads - 1];
    const double excl = t > 0 ? sh[t - 1] : 0.0;
    __syncthreads();
    return excl;
}

// Pass 1 on the amplitudes: cdf[i] = block-local inclusive prefix of |A|^2,
// sums[b] = the block's total.
__global__ void __launch_bounds__(kScanThreads) k_prob_scan(const double2* amps, uint64_t n, double* cdf,
                                                            double* sums) {
    __shared__ double sh[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)threadIdx.x * kScanPer;
    double v[kScanPer];
    double run = 0.0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        double p = 0.0;
        if (base + i < n) {
            const double2 a = amps[base + i];
            p = a.x * a.x + a.y * a.y;
        }
        run += p;
        v[i] = run;
    }
    double total;
    const double excl = block_exclusive_prefix(run, sh, total);
#pragma unroll
    for (int i = 0; i < kScanPer; ++i)
        if (base + i < n) cdf[base + i] = excl + v[i];
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Same on a float64 array in place (the block sums of the level below).
__global__ void __launch_bounds__(kScanThreads) k_scan(double* x, uint64_t n, double* sums) {
    __shared__ double sh[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + (uint64_t)threadIdx.x * kScanPer;
    double v[kScanPer];
    double run = 0.0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        run += base + i < n ? x[base + i] : 0.0;
        v[i] = run;
    }
    double total;
    const double excl = block_exclusive_prefix(run, sh, total);
#pragma unroll
    for (int i = 0; i < kScanPer; ++i)
        if (base + i < n) x[base + i] = excl + v[i];
    if (sums && threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Pass 3: x[i] += (inclusive scan of the block sums)[block(i) - 1].
__global__ void __launch_bounds__(kScanThreads) k_add_offsets(double* x, uint64_t n, const double* scanned_sums) {
    const uint64_t blk = blockIdx.x;
    if (blk == 0) return;
    const double off = scanned_sums[blk - 1];
    const uint64_t base = blk * kScanBlock + (uint64_t)threadIdx.x * kScanPer;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i)
        if (base + i < n) x[base + i] += off;
}

__global__ void __launch_bounds__(256) k_search(const double* cdf, uint64_t n, const double* u, uint64_t n_samples,
                                                uint64_t* out) {
    const double total = cdf[n - 1];
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n_samples; i += (uint64_t)gridDim.x * 256) {
        const double target = u[i] * total;
        uint64_t lo = 0, hi = n - 1;   // smallest j with cdf[j] > target, clamped to n - 1
        while (lo < hi) {
            const uint64_t mid = lo + (hi - lo) / 2;
            if (cdf[mid] > target) hi = mid;
            else lo = mid + 1;
        }
        out[i] = lo;
    }
}

uint64_t blocks_for(uint64_t n) { return (n + kScanBlock - 1) / kScanBlock; }

}  // namespace

uint64_t sample_workspace_elems(uint64_t n) {
    uint64_t total = n;
    for (uint64_t m = blocks_for(n); ; m = blocks_for(m)) {
        total += m;
        if (m <= 1) break;
    }
    return total;
}

namespace {

constexpr uint64_t static_elems(uint64_t n) {
    uint64_t total = n;
    for (uint64_t m = (n + kScanBlock - 1) / kScanBlock; ; m = (m + kScanBlock - 1) / kScanBlock) {
        total += m;
        if (m <= 1) break;
    }
    return total;
}

// Workspace of the allocation-free entry point: 2^20 probabilities and their
// scan levels (8.0 MiB), one copy per GPU, held until the process ends.
// Host code never uses this name as an address: each device's address comes
// from hipGetSymbolAddress.
__device__ __align__(256) double scratch[static_elems(1ull << kStaticSampleMaxOpen)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hipError_t launch_sample_static(const double* amps, uint64_t n, const double* u, uint64_t n_samples, uint64_t* out,
                                hipStream_t s) {
    if (n == 0 || n > (1ull << kStaticSampleMaxOpen)) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    double* ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {   // once per device, with that device current
            void* ptr = nullptr;
            e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess) return e;
            g_scratch_ptr[dev] = static_cast<double*>(ptr);
        }
        ws = g_scratch_ptr[dev];
    }
    return launch_sample(amps, n, u, n_samples, out, ws, s);
}

hipError_t launch_sample(const double* amps, uint64_t n, const double* u, uint64_t n_samples, uint64_t* out,
                         double* ws, hipStream_t s) {
    if (n == 0) return hipErrorInvalidValue;
    // level 0: the cdf itself; level l + 1: the block sums of level l (each
    // level is 2^10 times shorter, so 8 levels cover n < 2^70; no host
    // allocation)
    constexpr int kMaxLevels = 8;
    double* lv_ptr[kMaxLevels];
    uint64_t lv_len[kMaxLevels];
    int n_lv = 0;
    double* p = ws;
    lv_ptr[n_lv] = p;
    lv_len[n_lv++] = n;
    p += n;
    for (uint64_t m = blocks_for(n); ; m = blocks_for(m)) {
        if (n_lv == kMaxLevels) return hipErrorInvalidValue;
        lv_ptr[n_lv] = p;
        lv_len[n_lv++] = m;
        p += m;
        if (m <= 1) break;
    }
    hipLaunchKernelGGL(k_prob_scan, dim3((unsigned)blocks_for(n)), dim3(kScanThreads), 0, s,
                       reinterpret_cast<const double2*>(amps), n, lv_ptr[0], lv_ptr[1]);
    hipError_t e = hipGetLastError();
    for (int l = 1; e == hipSuccess && l + 1 < n_lv; ++l) {
        hipLaunchKernelGGL(k_scan, dim3((unsigned)blocks_for(lv_len[l])), dim3(kScanThreads), 0, s, lv_ptr[l],
                           lv_len[l], lv_ptr[l + 1]);
        e = hipGetLastError();
    }
    for (int l = n_lv - 1; e == hipSuccess && l-- > 0;) {
        if (lv_len[l] <= (uint64_t)kScanBlock) continue;   // one block: nothing to add
        hipLaunchKernelGGL(k_add_offsets, dim3((unsigned)blocks_for(lv_len[l])), dim3(kScanThreads), 0, s,
                           lv_ptr[l], lv_len[l], lv_ptr[l + 1]);
        e = hipGetLastError();
    }
    if (e != hipSuccess || n_samples == 0) return e;
    const uint64_t sb = std::min<uint64_t>((n_samples + 255) / 256, 1u << 20);   // grid-stride beyond that
    hipLaunchKernelGGL(k_search, dim3((unsigned)sb), dim3(256), 0, s, lv_ptr[0], n, u, n_samples, out);
    return hipGetLastError();
}

}  // namespace tn

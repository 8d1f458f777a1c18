// Step kernels for gfx950 (CDNA4).
//
// One pairwise contraction step of the sliced network (appendix A, Fig. 3:
// cost 2^(nA + nB + nAB) for bond dimension 2) is
//     C[b, m, n] = sum_k A[k, b, m] * B[k, b, n]
// over complex numbers.  The planner lays every operand out as
// [K | batch | M] (resp. N) from the most to the least significant address
// bit, so A and B tiles are plain strided rows, and C goes to whatever
// address bits its consumer wants: the output tile is staged in LDS and
// written back in C-address order, which is where the index permutation of
// each step happens (no separate permute pass).
//
// Kernels:
//  k_valu        streaming VALU tile kernel (big-times-small steps, any shape)
//  k_splitk_red  sum of split-K partial tiles in fixed order
//  k_mfma_c64    complex GEMM on FP32 MFMA (v_mfma_f32_16x16x4f32): each
//                complex product is 4 real products; B is expanded on the fly
//                into the 2x2 real block [[re, im], [-im, re]]
//  k_slice_sum   float64 sum over the batch legs of the root into the
//                accumulator (fixed order, no atomics)
//  k_xeb_*       float64 block partials of sum P, sum P^2, max, min
#include "kernels.hpp"

#include <type_traits>

namespace tn {

namespace {

__device__ __forceinline__ float2 cfma(float2 acc, float2 a, float2 b) {
    acc.x = fmaf(a.x, b.x, acc.x);
    acc.x = fmaf(-a.y, b.y, acc.x);
    acc.y = fmaf(a.x, b.y, acc.y);
    acc.y = fmaf(a.y, b.x, acc.y);
    return acc;
}
__device__ __forceinline__ double2 cfma(double2 acc, double2 a, double2 b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}
template <typename T> __device__ __forceinline__ T czero();
template <> __device__ __forceinline__ float2 czero<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ __forceinline__ double2 czero<double2>() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// Scatter the bits [lo, hi) of x to the address bits pos[lo..hi).
__device__ __forceinline__ uint64_t deposit(uint64_t x, const uint8_t* pos, int lo, int hi) {
    uint64_t r = 0;
    for (int i = lo; i < hi; ++i) r |= ((x >> i) & 1ull) << pos[i];
    return r;
}

__device__ __forceinline__ float cabsmax(float2 v) { return fmaxf(fabsf(v.x), fabsf(v.y)); }
__device__ __forceinline__ float cabsmax(double2 v) { return (float)fmax(fabs(v.x), fabs(v.y)); }

// Largest |re|, |im| of a tile into *slot (the bit pattern of a non-negative
// float orders like an unsigned integer).  Reduced over the block first; the
// single vector atomic is skipped when the slot already holds a larger value,
// so a large grid does not serialise on one address.  All threads of the
// block must call it.
__device__ __forceinline__ void tile_max_atomic(float v, float* slot) {
    __shared__ float wmax[16];
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    if ((threadIdx.x & 63) == 0) wmax[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < nw; ++i) v = fmaxf(v, wmax[i]);
        unsigned int* p = reinterpret_cast<unsigned int*>(slot);
        const unsigned int u = __float_as_uint(v);
        if (u > __atomic_load_n(p, __ATOMIC_RELAXED)) atomicMax(p, u);
    }
}

__device__ __forceinline__ uint64_t slice_offset(const uint64_t* d_slice, int n, const uint8_t* bit,
                                                 const uint8_t* pos) {
    if (n == 0) return 0;
    const uint64_t sl = *d_slice;
    uint64_t off = 0;
    for (int i = 0; i < n; ++i) off += ((sl >> bit[i]) & 1ull) << pos[i];
    return off;
}

struct TileIndex {
    uint64_t m0, n0, beta, split;
};

__device__ __forceinline__ TileIndex tile_index(const GemmArgs& g) {
    const uint64_t nblk = (uint64_t)gridDim.x * gridDim.y;   // one block per tile (a power of two)
    const uint64_t bid = blockIdx.x + (uint64_t)blockIdx.y * gridDim.x;
    // Workgroups go round-robin to the 8 XCDs, each with its own L2: XCD x
    // takes the contiguous logical range [x, x + 1) * nblk / 8, and N tiles
    // vary fastest, so the blocks sharing one A row block run back to back on
    // one L2 and A is fetched from HBM about once.
    uint64_t t = (nblk & 7) == 0 ? (bid & 7) * (nblk >> 3) + (bid >> 3) : bid;
    const int mtb = g.m_log - g.tm, ntb = g.n_log - g.tn;
    TileIndex ti;
    ti.n0 = (t & ((1ull << ntb) - 1)) << g.tn;
    t >>= ntb;
    ti.m0 = (t & ((1ull << mtb) - 1)) << g.tm;
    t >>= mtb;
    ti.beta = t & ((1ull << g.b_log) - 1);
    t >>= g.b_log;
    ti.split = t;
    return ti;
}

// Decode tile element x (enumerated in C-address order) into its logical
// (m, n) position in the tile and its address offset.
__device__ __forceinline__ uint64_t decode_ep(const GemmArgs& g, int x, int& ml, int& nl) {
    uint64_t off = 0;
    ml = 0;
    nl = 0;
    for (int i = 0; i < g.ep_n; ++i) {
        const int bit = (x >> i) & 1;
        off |= (uint64_t)bit << g.ep_pos[i];
        const int s = g.ep_src[i];
        if (s < 32) ml |= bit << s;
        else nl |= bit << (s - 32);
    }
    return off;
}

}  // namespace

// ------------------------------------------------------------------ VALU

template <typename T, int R>
__global__ void __launch_bounds__(256) k_valu(GemmArgs g) {
    extern __shared__ unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int TM = 1 << g.tm, TN = 1 << g.tn, TK = 1 << g.tk;
    T* As = sm;
    T* Bs = sm + (TK << g.tm);
    const TileIndex ti = tile_index(g);
    const uint64_t sAk = 1ull << (g.m_log + g.b_log), sBk = 1ull << (g.n_log + g.b_log);
    const T* A = reinterpret_cast<const T*>(g.A) + slice_offset(g.d_slice, g.sa_n, g.sa_bit, g.sa_pos) +
                 (ti.beta << g.m_log) + ti.m0;
    const T* B = reinterpret_cast<const T*>(g.B) + slice_offset(g.d_slice, g.sb_n, g.sb_bit, g.sb_pos) +
                 (ti.beta << g.n_log) + ti.n0;
    const int kc_log = g.k_log - g.split_log;
    const uint64_t kb = ti.split << kc_log;
    const uint64_t kn = 1ull << kc_log;
    const int tid = threadIdx.x;
    const int ntile = 1 << (g.tm + g.tn);
    T acc[R];
#pragma unroll
    for (int j = 0; j < R; ++j) acc[j] = czero<T>();
    for (uint64_t k0 = 0; k0 < kn; k0 += TK) {
        for (int e = tid; e < (TK << g.tm); e += 256) {
            const int kk = e >> g.tm, mm = e & (TM - 1);
            As[e] = A[(kb + k0 + kk) * sAk + mm];
        }
        for (int e = tid; e < (TK << g.tn); e += 256) {
            const int kk = e >> g.tn, nn = e & (TN - 1);
            Bs[e] = B[(kb + k0 + kk) * sBk + nn];
        }
        __syncthreads();
        for (int kk = 0; kk < TK; ++kk) {
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const int o = tid + 256 * j;
                if (o < ntile) {
                    const int ml = o & (TM - 1), nl = o >> g.tm;
                    acc[j] = cfma(acc[j], As[(kk << g.tm) + ml], Bs[(kk << g.tn) + nl]);
                }
            }
        }
        __syncthreads();
    }
    if (g.split_log > 0) {
        T* P = reinterpret_cast<T*>(g.scratch);
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const int o = tid + 256 * j;
            if (o < ntile) {
                const int ml = o & (TM - 1), nl = o >> g.tm;
                const uint64_t idx =
                    ((((ti.split << g.b_log) | ti.beta) << g.n_log | (ti.n0 + nl)) << g.m_log) | (ti.m0 + ml);
                P[idx] = acc[j];
            }
        }
        return;
    }
    if (g.cmax) {
        float mx = 0.f;
#pragma unroll
        for (int j = 0; j < R; ++j)
            if (tid + 256 * j < ntile) mx = fmaxf(mx, cabsmax(acc[j]));
        tile_max_atomic(mx, g.cmax);
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
        const int o = tid + 256 * j;
        if (o < ntile) sm[o] = acc[j];
    }
    __syncthreads();
    const uint64_t cbase = deposit(ti.m0, g.cpm, g.tm, g.m_log) + deposit(ti.n0, g.cpn, g.tn, g.n_log) +
                           deposit(ti.beta, g.cpb, 0, g.b_log);
    T* C = reinterpret_cast<T*>(g.C) + cbase;
    for (int x = tid; x < ntile; x += 256) {
        int ml, nl;
        const uint64_t off = decode_ep(g, x, ml, nl);
        C[off] = sm[ml + (nl << g.tm)];
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_splitk_red(GemmArgs g) {
    const int lt = g.m_log + g.n_log + g.b_log;
    const uint64_t total = 1ull << lt;
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    const T* P = reinterpret_cast<const T*>(g.scratch);
    T s = czero<T>();
    if (i < total)
        for (uint64_t sp = 0; sp < (1ull << g.split_log); ++sp) s = cadd(s, P[(sp << lt) + i]);
    if (g.cmax) tile_max_atomic(cabsmax(s), g.cmax);
    if (i >= total) return;
    const uint64_t m = i & ((1ull << g.m_log) - 1);
    const uint64_t n = (i >> g.m_log) & ((1ull << g.n_log) - 1);
    const uint64_t be = i >> (g.m_log + g.n_log);
    const uint64_t off = deposit(m, g.cpm, 0, g.m_log) + deposit(n, g.cpn, 0, g.n_log) + deposit(be, g.cpb, 0, g.b_log);
    reinterpret_cast<T*>(g.C)[off] = s;
}

// ------------------------------------------------------------- streaming

// Big-times-small steps: K and N at most 16 (K*N <= 64), M large.  Each
// thread owns V = 2 consecutive m (complex64: one 16-byte load per k), issues
// all K loads before any arithmetic, reads B through uniform (scalar-cached)
// loads, and stores its N x V outputs straight to their bit-scattered C
// addresses; lines written partially by one lane are completed by its
// neighbours and merged in L2 before they reach HBM.
constexpr int kStreamKN = 64;

template <typename T, int V>
__global__ void __launch_bounds__(256) k_stream(GemmArgs g) {
    using VT = typename std::conditional<V == 2, float4, T>::type;   // V consecutive complex values
    const int K = 1 << g.k_log, N = 1 << g.n_log;
    const uint64_t beta = blockIdx.y;
    const uint64_t m0 = ((uint64_t)blockIdx.x * 256 + threadIdx.x) * V;
    const uint64_t sAk = 1ull << (g.m_log + g.b_log), sBk = 1ull << (g.n_log + g.b_log);
    const T* A = reinterpret_cast<const T*>(g.A) + slice_offset(g.d_slice, g.sa_n, g.sa_bit, g.sa_pos) +
                 (beta << g.m_log);
    const T* B = reinterpret_cast<const T*>(g.B) + slice_offset(g.d_slice, g.sb_n, g.sb_bit, g.sb_pos) +
                 (beta << g.n_log);
    const bool live = m0 < (1ull << g.m_log);
    T a[16][V];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k < K && live) {
            const VT v = *reinterpret_cast<const VT*>(A + (uint64_t)k * sAk + m0);
            if constexpr (V == 2) {
                a[k][0] = T{v.x, v.y};
                a[k][1] = T{v.z, v.w};
            } else {
                a[k][0] = v;
            }
        }
    }
    float mx = 0.f;
    if (live) {
        const uint64_t cm0 = deposit(m0, g.cpm, 0, g.m_log) + deposit(beta, g.cpb, 0, g.b_log);
        const uint64_t cm1 = V == 2 ? cm0 + (1ull << g.cpm[0]) : 0;   // m0 is even: m0 + 1 sets bit 0
        T* C = reinterpret_cast<T*>(g.C);
        for (int n = 0; n < N; ++n) {
            T acc[V];
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] = czero<T>();
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                if (k < K) {
                    const T b = B[(uint64_t)k * sBk + n];
#pragma unroll
                    for (int v = 0; v < V; ++v) acc[v] = cfma(acc[v], a[k][v], b);
                }
            }
            const uint64_t cn = deposit((uint64_t)n, g.cpn, 0, g.n_log);
            if constexpr (V == 2) {
                if (g.cpm[0] == 0) {   // the two m values are adjacent in C: one 16-byte store
                    *reinterpret_cast<float4*>(C + cm0 + cn) = float4{acc[0].x, acc[0].y, acc[1].x, acc[1].y};
                } else {
                    C[cm0 + cn] = acc[0];
                    C[cm1 + cn] = acc[1];
                }
            } else {
                C[cm0 + cn] = acc[0];
            }
#pragma unroll
            for (int v = 0; v < V; ++v) mx = fmaxf(mx, cabsmax(acc[v]));
        }
    }
    if (g.cmax) tile_max_atomic(mx, g.cmax);
}

// ------------------------------------------------------------------ MFMA

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaSmemFloats = 8192;   // LDS budget of a staging pass (32 KiB)

// Epilogue decode restricted to one staging pass: the tile rows are staged
// RP = 2^rp_log at a time; element f of pass p takes its pass-selecting m bits
// (logical m bits >= rp_log) from p and its remaining tile bits, in C-address
// order, from f.  Returns the address offset; ml is relative to the pass.
__device__ __forceinline__ uint64_t decode_pass(const GemmArgs& g, int rp_log, int p, int f, int& ml, int& nl) {
    uint64_t off = 0;
    ml = 0;
    nl = 0;
    int j = 0;
    for (int i = 0; i < g.ep_n; ++i) {
        const int s = g.ep_src[i];
        int bit;
        if (s < 32 && s >= rp_log) {
            bit = (p >> (s - rp_log)) & 1;
        } else {
            bit = (f >> j) & 1;
            ++j;
            if (s < 32) ml |= bit << s;
            else nl |= bit << (s - 32);
        }
        off |= (uint64_t)bit << g.ep_pos[i];
    }
    return off;
}

// Stage a register tile through LDS pass by pass and write it in C-address
// order.  put(i, j, v) writes accumulator value v of tile row i, real column
// j; the caller provides the register walk as a lambda.
template <int TM, int TNR, int RP, typename Walk>
__device__ __forceinline__ void store_tile(const GemmArgs& g, float* fs, float2* C, Walk walk) {
    constexpr int TN = TNR / 2;
    constexpr int rp_log = __builtin_ctz(RP);
    const float2* Cs = reinterpret_cast<const float2*>(fs);
    for (int p0 = 0; p0 < TM; p0 += RP) {
        walk([&](int i, int j, float v) {
            if (i >= p0 && i < p0 + RP) fs[(i - p0) * TNR + j] = v;
        });
        __syncthreads();
        for (int f = threadIdx.x; f < RP * TN; f += 256) {
            int ml, nl;
            const uint64_t off = decode_pass(g, rp_log, p0 >> rp_log, f, ml, nl);
            C[off] = Cs[ml * TN + nl];
        }
        __syncthreads();
    }
}

template <int TM, int TNR, int AB>
struct MfmaLds {
    static constexpr int PASS = (TM * TNR <= kMfmaSmemFloats) ? TM * TNR : AB;   // floats of one staging pass
    static constexpr int RP0 = PASS / TNR;
    static constexpr int RP = RP0 >= TM ? TM : (1 << (31 - __builtin_clz(RP0)));  // rows per pass (power of 2)
    static constexpr int FLOATS = AB > RP * TNR ? AB : RP * TNR;
};

// Complex GEMM on FP32 MFMA (v_mfma_f32_16x16x4f32), 4 real products per
// complex product: A' = [Re A | Im A] interleaved is read as stored, B is
// expanded to its 2x2 real block [[re, im], [-im, re]] while the fragment is
// built.  K runs in chunks of 16 complex (8 MFMA k-steps, fully unrolled);
// a shorter K is zero-filled.  The next chunk is loaded into registers while
// the current one is multiplied.
template <int WM, int WN, int WAVES_M, int WAVES_N>
__global__ void __launch_bounds__(256) k_mfma_c64(GemmArgs g) {
    constexpr int TM = WAVES_M * WM * 16;   // complex rows
    constexpr int TNR = WAVES_N * WN * 16;  // real columns
    constexpr int TN = TNR / 2;             // complex columns
    constexpr int TK = 16;
    constexpr int AB = TK * (TM + TN) * 2;  // floats of the A and B chunk tiles
    using L = MfmaLds<TM, TNR, AB>;
    __shared__ __attribute__((aligned(16))) float smem[L::FLOATS];
    float2* As = reinterpret_cast<float2*>(smem);
    float2* Bs = As + TK * TM;
    const TileIndex ti = tile_index(g);
    const uint64_t sAk = 1ull << (g.m_log + g.b_log), sBk = 1ull << (g.n_log + g.b_log);
    const float2* A = reinterpret_cast<const float2*>(g.A) + slice_offset(g.d_slice, g.sa_n, g.sa_bit, g.sa_pos) +
                      (ti.beta << g.m_log) + ti.m0;
    const float2* B = reinterpret_cast<const float2*>(g.B) + slice_offset(g.d_slice, g.sb_n, g.sb_bit, g.sb_pos) +
                      (ti.beta << g.n_log) + ti.n0;
    const uint64_t K = 1ull << g.k_log;
    const int TKe = K < (uint64_t)TK ? (int)K : TK;
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63;
    const int wm = w % WAVES_M, wn = w / WAVES_M;
    const int lr = lane & 15, lq = lane >> 4;
    const int kc_off = lq >> 1, comp = lq & 1;
    floatx4 acc[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    constexpr int PA = (TK * (TM / 2) + 255) / 256, PB = (TK * (TN / 2) + 255) / 256;
    float4 ra[PA], rb[PB];
    auto load_chunk = [&](uint64_t k0) {
#pragma unroll
        for (int i = 0; i < PA; ++i) {
            const int e = tid + 256 * i, kk = e / (TM / 2), mm = 2 * (e % (TM / 2));
            ra[i] = (e < TK * (TM / 2) && kk < TKe) ? *reinterpret_cast<const float4*>(A + (k0 + kk) * sAk + mm)
                                                   : float4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int e = tid + 256 * i, kk = e / (TN / 2), nn = 2 * (e % (TN / 2));
            rb[i] = (e < TK * (TN / 2) && kk < TKe) ? *reinterpret_cast<const float4*>(B + (k0 + kk) * sBk + nn)
                                                   : float4{0.f, 0.f, 0.f, 0.f};
        }
    };
    load_chunk(0);
    for (uint64_t k0 = 0; k0 < K; k0 += TK) {
#pragma unroll
        for (int i = 0; i < PA; ++i) {
            const int e = tid + 256 * i;
            if (e < TK * (TM / 2)) *reinterpret_cast<float4*>(As + 2 * e) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int e = tid + 256 * i;
            if (e < TK * (TN / 2)) *reinterpret_cast<float4*>(Bs + 2 * e) = rb[i];
        }
        __syncthreads();
        if (k0 + TK < K) load_chunk(k0 + TK);
#pragma unroll
        for (int kk = 0; kk < TK; kk += 2) {
            const int kc = kk + kc_off;
            float a[WM], b[WN];
#pragma unroll
            for (int bm = 0; bm < WM; ++bm) {
                const float2 v = As[kc * TM + (wm * WM + bm) * 16 + lr];
                a[bm] = comp ? v.y : v.x;
            }
#pragma unroll
            for (int bn = 0; bn < WN; ++bn) {
                const int jr = (wn * WN + bn) * 16 + lr;
                const float2 v = Bs[kc * TN + (jr >> 1)];
                b[bn] = (jr & 1) == 0 ? (comp == 0 ? v.x : -v.y) : (comp == 0 ? v.y : v.x);
            }
#pragma unroll
            for (int bm = 0; bm < WM; ++bm)
#pragma unroll
                for (int bn = 0; bn < WN; ++bn)
                    acc[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[bm], b[bn], acc[bm][bn], 0, 0, 0);
        }
        __syncthreads();
    }
    if (g.cmax) {
        float mx = 0.f;
#pragma unroll
        for (int bm = 0; bm < WM; ++bm)
#pragma unroll
            for (int bn = 0; bn < WN; ++bn)
#pragma unroll
                for (int r = 0; r < 4; ++r) mx = fmaxf(mx, fabsf(acc[bm][bn][r]));
        tile_max_atomic(mx, g.cmax);
    }
    const uint64_t cbase = deposit(ti.m0, g.cpm, g.tm, g.m_log) + deposit(ti.n0, g.cpn, g.tn, g.n_log) +
                           deposit(ti.beta, g.cpb, 0, g.b_log);
    store_tile<TM, TNR, L::RP>(g, smem, reinterpret_cast<float2*>(g.C) + cbase, [&](auto put) {
#pragma unroll
        for (int bm = 0; bm < WM; ++bm)
#pragma unroll
            for (int bn = 0; bn < WN; ++bn)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    put((wm * WM + bm) * 16 + 4 * lq + r, (wn * WN + bn) * 16 + lr, acc[bm][bn][r]);
    });
}

// ------------------------------------------------------- skinny MFMA

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef float floatv2 __attribute__((ext_vector_type(2)));

// The three high tile bits of the slab epilogues (taken from the unrolled
// store index j): address bit and LDS source offset of each (cs: LDS row
// stride in complex elements), read once instead of once per stored element.
struct EpHigh {
    uint64_t pos[3];
    int src[3];
    __device__ __forceinline__ uint64_t off(int j) const {
        return ((j & 1) ? pos[0] : 0) | ((j & 2) ? pos[1] : 0) | ((j & 4) ? pos[2] : 0);
    }
    __device__ __forceinline__ int from(int j) const {
        return ((j & 1) ? src[0] : 0) + ((j & 2) ? src[1] : 0) + ((j & 4) ? src[2] : 0);
    }
};

__device__ __forceinline__ EpHigh ep_high(const GemmArgs& g, int first, int cs) {
    EpHigh e;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const int i = first + b;
        const bool on = i < g.ep_n;
        const int sb = g.ep_src[i];
        e.pos[b] = on ? 1ull << g.ep_pos[i] : 0;
        e.src[b] = on ? (sb < 32 ? cs << sb : 1 << (sb - 32)) : 0;
    }
    return e;
}

// Big-times-small steps with N = 16..64 and K = 2..64 complex (the steps that
// dominate once small branches are merged, appendix B): HBM-bound, so A is
// streamed from global memory straight into MFMA operands and read once.
//
// v_mfma_f32_32x32x2f32 takes two real k per instruction.  Lane l holds row
// r = l & 31 of A for real k index h = l >> 5, and one 8-byte load per lane
// fetches the complex A[k0 + h][m0 + r]: its real parts feed one MFMA and its
// imaginary parts a second one, against the matching rows of the 2x2 real
// expansion of B:
//     re A:  [Re B, Im B]  (real columns 2n, 2n+1)
//     im A:  [-Im B, Re B]
// B (K x N complex) sits in LDS for the whole block; the output column j of a
// 32-column MFMA block is complex column j >> 1, component j & 1.  Each wave
// owns 32 rows of C at a time; every 16-column slab is staged in LDS (rows
// padded to 17 complex) and written in C-address order with the decode split
// into a per-lane part and a per-iteration part (the decode is additive over
// bits).  The block walks 128-row tiles of one batch entry with a grid
// stride; the A fragments of the next tile are loaded while the current one
// is multiplied.
template <int KT, int NB>
__global__ void __launch_bounds__(256) k_skinny(GemmArgs g) {
    constexpr int N = 16 * NB;
    constexpr int KP = KT / 2;              // complex k pairs
    constexpr int CS = 17;                  // staged row stride (complex)
    __shared__ __attribute__((aligned(16))) float2 Bs[KT * N];
    __shared__ __attribute__((aligned(16))) float2 Cs[4][32 * CS];
    const uint64_t beta = blockIdx.y;
    const uint64_t sAk = 1ull << (g.m_log + g.b_log), sBk = 1ull << (g.n_log + g.b_log);
    const float2* A = reinterpret_cast<const float2*>(g.A) + slice_offset(g.d_slice, g.sa_n, g.sa_bit, g.sa_pos) +
                      (beta << g.m_log);
    const float2* B = reinterpret_cast<const float2*>(g.B) + slice_offset(g.d_slice, g.sb_n, g.sb_bit, g.sb_pos) +
                      (beta << g.n_log);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int r = lane & 31, h = lane >> 5;
    for (int e = tid; e < KT * N; e += 256) Bs[e] = B[(uint64_t)(e / N) * sBk + (e % N)];
    // per-lane part of the epilogue decode (tile bits 0..5 of the C-order index)
    uint64_t off_lo = 0;
    int src_lo = 0;
    for (int i = 0; i < 6 && i < g.ep_n; ++i)
        if ((lane >> i) & 1) {
            off_lo |= 1ull << g.ep_pos[i];
            const int sb = g.ep_src[i];
            src_lo += sb < 32 ? CS << sb : 1 << (sb - 32);
        }
    const EpHigh eh = ep_high(g, 6, CS);
    __syncthreads();
    const uint64_t tiles = 1ull << (g.m_log - 7);
    uint64_t t = blockIdx.x;
    float2 a[KP], an[KP];
    auto load = [&](float2* dst, uint64_t tt) {
        const float2* src = A + tt * 128 + w * 32 + r + (uint64_t)h * sAk;
#pragma unroll
        for (int p = 0; p < KP; ++p) {   // A is read once: non-temporal (streaming) loads
            const floatv2 t = __builtin_nontemporal_load(reinterpret_cast<const floatv2*>(src + (uint64_t)(2 * p) * sAk));
            dst[p] = float2{t.x, t.y};
        }
    };
    if (t < tiles) load(a, t);
    float mx = 0.f;
    float2* C = reinterpret_cast<float2*>(g.C);
    float* cs = reinterpret_cast<float*>(Cs[w]);
    for (; t < tiles; t += gridDim.x) {
        if (t + gridDim.x < tiles) load(an, t + gridDim.x);
        floatx16 acc[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
            for (int v = 0; v < 16; ++v) acc[nb][v] = 0.f;
#pragma unroll
        for (int p = 0; p < KP; ++p) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const float2 b = Bs[(2 * p + h) * N + nb * 16 + (r >> 1)];
                const float b_re = (r & 1) ? b.y : b.x;
                const float b_im = (r & 1) ? b.x : -b.y;
                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].x, b_re, acc[nb], 0, 0, 0);
                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].y, b_im, acc[nb], 0, 0, 0);
            }
        }
        const uint64_t m0 = t * 128 + w * 32;
        const uint64_t cbase = deposit(m0, g.cpm, 5, g.m_log) + deposit(beta, g.cpb, 0, g.b_log);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int row = 8 * (v >> 2) + 4 * h + (v & 3);
                cs[row * (2 * CS) + r] = acc[nb][v];
                mx = fmaxf(mx, fabsf(acc[nb][v]));
            }
            __syncthreads();
            const uint64_t cb = cbase + deposit((uint64_t)nb << 4, g.cpn, 4, g.n_log);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const uint64_t off_hi = eh.off(j);
                const int src_hi = eh.from(j);
                C[cb + (off_lo | off_hi)] = Cs[w][src_lo + src_hi];
            }
            __syncthreads();
        }
#pragma unroll
        for (int p = 0; p < KP; ++p) a[p] = an[p];
    }
    if (g.cmax) tile_max_atomic(mx, g.cmax);
}

// ------------------------------------------------------------ panel MFMA

// Dense steps on the 32x32x2 FP32 MFMA with the operand scheme of k_skinny:
// a block owns 128 rows (4 waves x 32) and 16 NB complex columns; K runs in
// chunks of KC complex.  Each wave streams its A rows from global memory
// straight into MFMA operands (the next chunk is loaded while the current
// one is multiplied), the B chunk is staged in LDS through registers, and
// the 128 x 16 output slabs are staged in LDS and written in C-address order
// (tile bits m0..m6, n0..n3 in the epilogue decode).  Tiles are visited in
// the XCD-aware order of tile_index (tm = 7, tn = 4 + log2 NB).
template <int KC, int NB, bool NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KC == 16 ? (NB >= 4 ? 3 : 4) : 1)))
k_panel(GemmArgs g) {
    constexpr int N = 16 * NB;
    constexpr int KP = KC / 2;
    constexpr int CS = 17;
    constexpr int PBN = KC * N / 256;       // B chunk elements per thread
    // the B chunks and the output slabs share one LDS buffer (the epilogue
    // starts with a barrier after the last chunk), for more blocks per CU
    constexpr int SMEM = KC * N > 128 * CS ? KC * N : 128 * CS;
    __shared__ __attribute__((aligned(16))) float2 smem[SMEM];
    float2* const Bs = smem;
    float2* const Cs = smem;
    const TileIndex ti = tile_index(g);
    const uint64_t sAk = 1ull << (g.m_log + g.b_log), sBk = 1ull << (g.n_log + g.b_log);
    const float2* A = reinterpret_cast<const float2*>(g.A) + slice_offset(g.d_slice, g.sa_n, g.sa_bit, g.sa_pos) +
                      (ti.beta << g.m_log) + ti.m0;
    const float2* B = reinterpret_cast<const float2*>(g.B) + slice_offset(g.d_slice, g.sb_n, g.sb_bit, g.sb_pos) +
                      (ti.beta << g.n_log) + ti.n0;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int r = lane & 31, h = lane >> 5;
    const uint64_t K = 1ull << g.k_log;
    float2 a[KP], an[KP], bb[PBN];
    // NT: A is streamed with non-temporal loads (it is read by few N tiles)
    auto load_a = [&](float2* dst, uint64_t k0) {
        const float2* src = A + w * 32 + r + (k0 + h) * sAk;
#pragma unroll
        for (int p = 0; p < KP; ++p) {
            if constexpr (NT) {
                const floatv2 t = __builtin_nontemporal_load(reinterpret_cast<const floatv2*>(src + (uint64_t)(2 * p) * sAk));
                dst[p] = make_float2(t.x, t.y);
            } else {
                dst[p] = src[(uint64_t)(2 * p) * sAk];
            }
        }
    };
    auto load_b = [&](uint64_t k0) {
#pragma unroll
        for (int i = 0; i < PBN; ++i) {
            const int e = tid + 256 * i;
            bb[i] = B[(k0 + e / N) * sBk + (e % N)];
        }
    };
    floatx16 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[nb][v] = 0.f;
    // B before A: the wait for the B chunk (in-order load counter) then
    // leaves the A loads of the same chunk in flight
    load_b(0);
    load_a(a, 0);
    for (uint64_t k0 = 0; k0 < K; k0 += KC) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PBN; ++i) Bs[tid + 256 * i] = bb[i];
        __syncthreads();
        if (k0 + KC < K) {
            load_b(k0 + KC);
            load_a(an, k0 + KC);
        }
#pragma unroll
        for (int p = 0; p < KP; ++p) {
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const float2 b = Bs[(2 * p + h) * N + nb * 16 + (r >> 1)];
                const float b_re = (r & 1) ? b.y : b.x;
                const float b_im = (r & 1) ? b.x : -b.y;
                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].x, b_re, acc[nb], 0, 0, 0);
                acc[nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].y, b_im, acc[nb], 0, 0, 0);
            }
        }
#pragma unroll
        for (int p = 0; p < KP; ++p) a[p] = an[p];
    }
    // epilogue: tile bits m0..m6, n0..n3 (ep arrays for tm = 7, tn = 4)
    uint64_t off_lo = 0;
    int src_lo = 0;
    for (int i = 0; i < 8; ++i)
        if ((tid >> i) & 1) {
            off_lo |= 1ull << g.ep_pos[i];
            const int sb = g.ep_src[i];
            src_lo += sb < 32 ? CS << sb : 1 << (sb - 32);
        }
    const EpHigh eh = ep_high(g, 8, CS);
    float mx = 0.f;
    const uint64_t cbase = deposit(ti.m0, g.cpm, 7, g.m_log) + deposit(ti.beta, g.cpb, 0, g.b_log);
    float* cs = reinterpret_cast<float*>(Cs);
    float2* C = reinterpret_cast<float2*>(g.C);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        __syncthreads();
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int row = w * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
            cs[row * (2 * CS) + r] = acc[nb][v];
            mx = fmaxf(mx, fabsf(acc[nb][v]));
        }
        __syncthreads();
        const uint64_t cb = cbase + deposit(ti.n0 + ((uint64_t)nb << 4), g.cpn, 4, g.n_log);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint64_t off_hi = eh.off(j);
            const int src_hi = eh.from(j);
            C[cb + (off_lo | off_hi)] = Cs[src_lo + src_hi];
        }
    }
    if (g.cmax) tile_max_atomic(mx, g.cmax);
}

// Complex GEMM on FP32 MFMA with three real products per complex
// multiply-add instead of four (Gauss's form: T1 = (Re A + Im A) Re B,
// T2 = Re A (Im B - Re B), T3 = Im A (Re B + Im B); Re C = T1 - T3,
// Im C = T1 + T2), otherwise as k_panel: 128 rows and 16 NB complex columns
// per block, A streamed from HBM into MFMA operands, B chunks in LDS.  Each
// 32x32x2 MFMA covers 32 complex columns (lane r supplies column r), so a
// K pair costs 3 MFMAs per 32 columns instead of 4.  The rounding error of
// each output is bounded by the same products' magnitudes as the four-term
// form, up to a factor of about two.
template <int KC, int NB, bool NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KC == 16 ? (NB >= 4 ? 3 : 4) : 1)))
k_panel3(GemmArgs g) {
    constexpr int N = 16 * NB;
    constexpr int NT3 = N / 32;             // 32-column MFMA tiles
    constexpr int KP = KC / 2;
    constexpr int CS = 17;
    constexpr int PBN = KC * N / 256;
    // the B chunks and the two output slabs of a 32-column tile share LDS
    constexpr int SMEM = KC * N > 256 * CS ? KC * N : 256 * CS;
    __shared__ __attribute__((aligned(16))) float2 smem[SMEM];
    float2* const Bs = smem;
    float2* const Cs = smem;
    const TileIndex ti = tile_index(g);
    const uint64_t sAk = 1ull << (g.m_log + g.b_log), sBk = 1ull << (g.n_log + g.b_log);
    const float2* A = reinterpret_cast<const float2*>(g.A) + slice_offset(g.d_slice, g.sa_n, g.sa_bit, g.sa_pos) +
                      (ti.beta << g.m_log) + ti.m0;
    const float2* B = reinterpret_cast<const float2*>(g.B) + slice_offset(g.d_slice, g.sb_n, g.sb_bit, g.sb_pos) +
                      (ti.beta << g.n_log) + ti.n0;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int r = lane & 31, h = lane >> 5;
    const uint64_t K = 1ull << g.k_log;
    float2 a[KP], an[KP], bb[PBN];
    auto load_a = [&](float2* dst, uint64_t k0) {
        const float2* src = A + w * 32 + r + (k0 + h) * sAk;
#pragma unroll
        for (int p = 0; p < KP; ++p) {
            if constexpr (NT) {
                const floatv2 t = __builtin_nontemporal_load(reinterpret_cast<const floatv2*>(src + (uint64_t)(2 * p) * sAk));
                dst[p] = make_float2(t.x, t.y);
            } else {
                dst[p] = src[(uint64_t)(2 * p) * sAk];
            }
        }
    };
    auto load_b = [&](uint64_t k0) {
#pragma unroll
        for (int i = 0; i < PBN; ++i) {
            const int e = tid + 256 * i;
            bb[i] = B[(k0 + e / N) * sBk + (e % N)];
        }
    };
    floatx16 t1[NT3], t2[NT3], t3[NT3];
#pragma unroll
    for (int j = 0; j < NT3; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) t1[j][v] = t2[j][v] = t3[j][v] = 0.f;
    load_b(0);   // B first: see k_panel
    load_a(a, 0);
    for (uint64_t k0 = 0; k0 < K; k0 += KC) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PBN; ++i) Bs[tid + 256 * i] = bb[i];
        __syncthreads();
        if (k0 + KC < K) {
            load_b(k0 + KC);
            load_a(an, k0 + KC);
        }
#pragma unroll
        for (int p = 0; p < KP; ++p) {
            const float a1 = a[p].x + a[p].y;
#pragma unroll
            for (int j = 0; j < NT3; ++j) {
                const float2 b = Bs[(2 * p + h) * N + j * 32 + r];
                t1[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b.x, t1[j], 0, 0, 0);
                t2[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].x, b.y - b.x, t2[j], 0, 0, 0);
                t3[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[p].y, b.x + b.y, t3[j], 0, 0, 0);
            }
        }
#pragma unroll
        for (int p = 0; p < KP; ++p) a[p] = an[p];
    }
    // epilogue: 16-column slabs (tile bits m0..m6, n0..n3); the lanes holding
    // a slab's columns stage it
    uint64_t off_lo = 0;
    int src_lo = 0;
    for (int i = 0; i < 8; ++i)
        if ((tid >> i) & 1) {
            off_lo |= 1ull << g.ep_pos[i];
            const int sb = g.ep_src[i];
            src_lo += sb < 32 ? CS << sb : 1 << (sb - 32);
        }
    const EpHigh eh = ep_high(g, 8, CS);
    float mx = 0.f;
    const uint64_t cbase = deposit(ti.m0, g.cpm, 7, g.m_log) + deposit(ti.beta, g.cpb, 0, g.b_log);
    float2* C = reinterpret_cast<float2*>(g.C);
#pragma unroll
    for (int j = 0; j < NT3; ++j) {
        // both 16-column slabs of the tile at once: lane column r goes to
        // slab r >> 4
        __syncthreads();
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int row = w * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
            const float2 c = make_float2(t1[j][v] - t3[j][v], t1[j][v] + t2[j][v]);
            Cs[(r >> 4) * 128 * CS + row * CS + (r & 15)] = c;
            mx = fmaxf(mx, fmaxf(fabsf(c.x), fabsf(c.y)));
        }
        __syncthreads();
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            const uint64_t cb = cbase + deposit(ti.n0 + ((uint64_t)(2 * j + hf) << 4), g.cpn, 4, g.n_log);
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) {
                const uint64_t off_hi = eh.off(jj);
                const int src_hi = eh.from(jj);
                C[cb + (off_lo | off_hi)] = Cs[hf * 128 * CS + src_lo + src_hi];
            }
        }
    }
    if (g.cmax) tile_max_atomic(mx, g.cmax);
}

typedef __attribute__((address_space(3))) void* lds_void_ptr;

// k_panel3 with the A chunks staged in LDS by direct global-to-LDS loads
// (global_load_lds_dwordx4: each wave instruction moves one k row of the
// block's 128 rows, 1 KB, without passing through registers), double
// buffered in two separate LDS arrays so the compiler orders each read only
// after the loads into its own buffer; the next chunk's A and B loads are in
// flight while the current chunk is multiplied.  K chunks of 16.  The two
// A buffers double as the epilogue's slab buffers (128 rows x 17 complex).
template <int NB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NB >= 4 ? 3 : 4)))
k_panel3d(GemmArgs g) {
    constexpr int KC = 16, N = 16 * NB, NT3 = N / 32, KP = KC / 2, CS = 17, PBN = KC * N / 256;
    constexpr int AS = 128 * CS;             // a stage holds KC x 128 complex (and a slab when staging C)
    __shared__ __attribute__((aligned(16))) float2 As0[AS];
    __shared__ __attribute__((aligned(16))) float2 As1[AS];
    __shared__ __attribute__((aligned(16))) float2 Bs[KC * N];
    const TileIndex ti = tile_index(g);
    const uint64_t sAk = 1ull << (g.m_log + g.b_log), sBk = 1ull << (g.n_log + g.b_log);
    const float2* A = reinterpret_cast<const float2*>(g.A) + slice_offset(g.d_slice, g.sa_n, g.sa_bit, g.sa_pos) +
                      (ti.beta << g.m_log) + ti.m0;
    const float2* B = reinterpret_cast<const float2*>(g.B) + slice_offset(g.d_slice, g.sb_n, g.sb_bit, g.sb_pos) +
                      (ti.beta << g.n_log) + ti.n0;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int r = lane & 31, h = lane >> 5;
    const uint64_t K = 1ull << g.k_log;
    // wave w moves k rows 4w .. 4w+3 of a chunk; lane l the rows 2l, 2l+1
    auto load_a = [&](float2* stage, uint64_t k0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int kk = 4 * w + i;
            __builtin_amdgcn_global_load_lds(static_cast<const void*>(A + (k0 + kk) * sAk + 2 * lane),
                                             (lds_void_ptr)(stage + kk * 128), 16, 0, 0);
        }
    };
    float2 bb[PBN];
    auto load_b = [&](uint64_t k0) {
#pragma unroll
        for (int i = 0; i < PBN; ++i) {
            const int e = tid + 256 * i;
            bb[i] = B[(k0 + e / N) * sBk + (e % N)];
        }
    };
    floatx16 t1[NT3], t2[NT3], t3[NT3];
#pragma unroll
    for (int j = 0; j < NT3; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) t1[j][v] = t2[j][v] = t3[j][v] = 0.f;
    // Workgroup barrier after this wave's LDS stores have completed, without
    // the wait for all outstanding global loads that __syncthreads() implies
    // (it would also wait for the next chunk's loads, already in flight)
    auto lds_barrier = [] { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); };
    auto chunk = [&](const float2* cur, float2* nxt, uint64_t k0) {
        lds_barrier();   // the previous chunk's readers of Bs and of nxt are done
#pragma unroll
        for (int i = 0; i < PBN; ++i) Bs[tid + 256 * i] = bb[i];
        if (k0 + KC < K) {
            load_a(nxt, k0 + KC);
            load_b(k0 + KC);
            // this wave's loads of the current chunk have landed (loads
            // complete in order); the barrier makes every wave's visible
            asm volatile("s_waitcnt vmcnt(%0)" ::"n"(4 + PBN) : "memory");
        } else {
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        }
        lds_barrier();
#pragma unroll
        for (int p = 0; p < KP; ++p) {
            const float2 a = cur[(2 * p + h) * 128 + w * 32 + r];
            const float a1 = a.x + a.y;
#pragma unroll
            for (int j = 0; j < NT3; ++j) {
                const float2 b = Bs[(2 * p + h) * N + j * 32 + r];
                t1[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b.x, t1[j], 0, 0, 0);
                t2[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.x, b.y - b.x, t2[j], 0, 0, 0);
                t3[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a.y, b.x + b.y, t3[j], 0, 0, 0);
            }
        }
    };
    load_a(As0, 0);
    load_b(0);
    for (uint64_t k0 = 0; k0 < K; k0 += 2 * KC) {
        chunk(As0, As1, k0);
        if (k0 + KC < K) chunk(As1, As0, k0 + KC);
    }
    // epilogue: both 16-column slabs of a 32-column tile at once, slab hf in
    // the A buffer hf
    uint64_t off_lo = 0;
    int src_lo = 0;
    for (int i = 0; i < 8; ++i)
        if ((tid >> i) & 1) {
            off_lo |= 1ull << g.ep_pos[i];
            const int sb = g.ep_src[i];
            src_lo += sb < 32 ? CS << sb : 1 << (sb - 32);
        }
    const EpHigh eh = ep_high(g, 8, CS);
    float mx = 0.f;
    const uint64_t cbase = deposit(ti.m0, g.cpm, 7, g.m_log) + deposit(ti.beta, g.cpb, 0, g.b_log);
    float2* C = reinterpret_cast<float2*>(g.C);
#pragma unroll
    for (int j = 0; j < NT3; ++j) {
        __syncthreads();
        float2* slab = (r >> 4) ? As1 : As0;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int row = w * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
            const float2 c = make_float2(t1[j][v] - t3[j][v], t1[j][v] + t2[j][v]);
            slab[row * CS + (r & 15)] = c;
            mx = fmaxf(mx, fmaxf(fabsf(c.x), fabsf(c.y)));
        }
        __syncthreads();
#pragma unroll
        for (int hf = 0; hf < 2; ++hf) {
            const float2* src = hf ? As1 : As0;
            const uint64_t cb = cbase + deposit(ti.n0 + ((uint64_t)(2 * j + hf) << 4), g.cpn, 4, g.n_log);
#pragma unroll
            for (int jj = 0; jj < 8; ++jj) C[cb + (off_lo | eh.off(jj))] = src[src_lo + eh.from(jj)];
        }
    }
    if (g.cmax) tile_max_atomic(mx, g.cmax);
}

// ------------------------------------------------- low-precision MFMA

constexpr int kRowPad = 36;   // words per staged row: 32 k + 4 (bank spread, 16-byte aligned)

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

typedef __fp16 half2v __attribute__((ext_vector_type(2)));

// Pack two reals (re in the low half) after scaling by s.  FP16 uses the
// packed round-toward-zero conversion; in split mode the remainder
// x - hi is exact in FP32, so the rounding of hi is carried by lo
// (stored scaled by 2^11 so it stays normal in FP16).
template <int MODE>
__device__ __forceinline__ void split_pack(float2 v, float s, uint32_t& hi, uint32_t& lo) {
    if constexpr (MODE == LP_BF16) {
        const __bf16 r = (__bf16)(v.x * s), i = (__bf16)(v.y * s);
        hi = (uint32_t)__builtin_bit_cast(uint16_t, r) | ((uint32_t)__builtin_bit_cast(uint16_t, i) << 16);
        lo = 0;
    } else {
        const float xr = v.x * s, xi = v.y * s;
        const half2v h = __builtin_amdgcn_cvt_pkrtz(xr, xi);
        hi = __builtin_bit_cast(uint32_t, h);
        if constexpr (MODE == LP_SPLIT_FP16) {
            const half2v l = __builtin_amdgcn_cvt_pkrtz((xr - (float)h.x) * 2048.f, (xi - (float)h.y) * 2048.f);
            lo = __builtin_bit_cast(uint32_t, l);
        } else {
            lo = 0;
        }
    }
}

// B column of the real expansion: even real column (re part of C) takes
// (re, -im) pairs, odd real column (im part) takes (im, re) pairs.
__device__ __forceinline__ uint32_t bexp(uint32_t w, int odd) {
    return odd ? ((w >> 16) | (w << 16)) : (w ^ 0x80000000u);
}

// Split for the panels: v is scaled by s, which in split mode carries an
// extra 2^11, so hi = fp16(x) is 2^11 times the FP16 head of the operand and
// lo = fp16(x - hi) its remainder at the same scale (x - hi is exact in
// FP32).  The products hi_a hi_b + hi_a lo_b + lo_a hi_b then carry 2^22.
template <int MODE>
__device__ __forceinline__ void split_pack11(float2 v, float s, uint32_t& hi, uint32_t& lo) {
    if constexpr (MODE == LP_SPLIT_FP16) {
        const float xr = v.x * s, xi = v.y * s;
        const half2v h = __builtin_amdgcn_cvt_pkrtz(xr, xi);
        hi = __builtin_bit_cast(uint32_t, h);
        lo = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(xr - (float)h.x, xi - (float)h.y));
    } else {
        split_pack<MODE>(v, s, hi, lo);
    }
}

__device__ __forceinline__ int scale_exp(const float* mx) {
    const float m = mx ? *mx : 0.f;
    return m > 0.f ? ilogbf(m) + 1 : 0;   // m * 2^-e in [0.5, 1)
}

// Complex GEMM on FP16 / BF16 MFMA (v_mfma_f32_16x16x32_{f16,bf16}) with
// FP32 accumulation.  Operands are scaled by a power of two taken from the
// producers' max (exact, so nothing underflows FP16) and split into hi/lo
// FP16 pairs: x = hi + 2^-11 lo, product = hi*hi + 2^-11 (hi*lo + lo*hi)
// (split mode; the single-term modes use hi only).  The complex product is
// 4 real products as in the FP32 kernel: A' = [Re A | Im A] interleaved (one
// packed (re, im) word per complex k), B' = [[re, im], [-im, re]] (real
// column 2n holds (re, -im) words, column 2n+1 (im, re)).  Both are staged in
// LDS k-fastest, one row per m or real column, padded to 36 words, so a
// lane's eight k-slots (four words) are one 16-byte read.
template <int WM, int WN, int WAVES_M, int WAVES_N, int MODE>
__global__ void __launch_bounds__(256) k_mfma_lp(GemmArgs g) {
    constexpr int TM = WAVES_M * WM * 16;
    constexpr int TNR = WAVES_N * WN * 16;
    constexpr int TN = TNR / 2;
    constexpr int TK = 32;                  // complex k per chunk = two MFMA k-steps (32 real each)
    constexpr bool SPLIT = MODE == LP_SPLIT_FP16;
    constexpr int PLANES = SPLIT ? 2 : 1;
    constexpr int AB_WORDS = PLANES * (TM + TNR) * kRowPad;
    using L = MfmaLds<TM, TNR, AB_WORDS>;
    __shared__ __attribute__((aligned(16))) uint32_t smem[L::FLOATS];
    uint32_t* Ahi = smem;                               // [TM][kRowPad]
    uint32_t* Alo = Ahi + TM * kRowPad;
    uint32_t* Bhi = smem + PLANES * TM * kRowPad;       // [TNR][kRowPad]
    uint32_t* Blo = Bhi + TNR * kRowPad;
    const TileIndex ti = tile_index(g);
    const uint64_t sAk = 1ull << (g.m_log + g.b_log), sBk = 1ull << (g.n_log + g.b_log);
    const float2* A = reinterpret_cast<const float2*>(g.A) + slice_offset(g.d_slice, g.sa_n, g.sa_bit, g.sa_pos) +
                      (ti.beta << g.m_log) + ti.m0;
    const float2* B = reinterpret_cast<const float2*>(g.B) + slice_offset(g.d_slice, g.sb_n, g.sb_bit, g.sb_pos) +
                      (ti.beta << g.n_log) + ti.n0;
    const int ea = scale_exp(g.amax), eb = scale_exp(g.bmax);
    const float sa = ldexpf(1.f, -ea), sb = ldexpf(1.f, -eb);
    const uint64_t K = 1ull << g.k_log;
    const int TKe = K < (uint64_t)TK ? (int)K : TK;
    const int tid = threadIdx.x;
    const int w = tid >> 6, lane = tid & 63;
    const int wm = w % WAVES_M, wn = w / WAVES_M;
    const int lr = lane & 15, lg = lane >> 4;
    floatx4 acc[WM][WN], accx[SPLIT ? WM : 1][SPLIT ? WN : 1];
#pragma unroll
    for (int i = 0; i < WM; ++i)
#pragma unroll
        for (int j = 0; j < WN; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    if constexpr (SPLIT) {
#pragma unroll
        for (int i = 0; i < (SPLIT ? WM : 1); ++i)
#pragma unroll
            for (int j = 0; j < (SPLIT ? WN : 1); ++j) accx[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    constexpr int PA = (TK * TM + 255) / 256, PB = (TK * TN + 255) / 256;
    float2 ra[PA], rb[PB];
    auto load_chunk = [&](uint64_t k0) {
#pragma unroll
        for (int i = 0; i < PA; ++i) {
            const int e = tid + 256 * i, kk = e / TM, mm = e % TM;
            ra[i] = (e < TK * TM && kk < TKe) ? A[(k0 + kk) * sAk + mm] : float2{0.f, 0.f};
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int e = tid + 256 * i, kk = e / TN, nn = e % TN;
            rb[i] = (e < TK * TN && kk < TKe) ? B[(k0 + kk) * sBk + nn] : float2{0.f, 0.f};
        }
    };
    load_chunk(0);
    for (uint64_t k0 = 0; k0 < K; k0 += TK) {
#pragma unroll
        for (int i = 0; i < PA; ++i) {
            const int e = tid + 256 * i;
            if (e < TK * TM) {
                const int kk = e / TM, mm = e % TM;
                uint32_t hi, lo;
                split_pack<MODE>(ra[i], sa, hi, lo);
                Ahi[mm * kRowPad + kk] = hi;
                if constexpr (SPLIT) Alo[mm * kRowPad + kk] = lo;
            }
        }
#pragma unroll
        for (int i = 0; i < PB; ++i) {
            const int e = tid + 256 * i;
            if (e < TK * TN) {
                const int kk = e / TN, nn = e % TN;
                uint32_t hi, lo;
                split_pack<MODE>(rb[i], sb, hi, lo);
                Bhi[(2 * nn) * kRowPad + kk] = bexp(hi, 0);
                Bhi[(2 * nn + 1) * kRowPad + kk] = bexp(hi, 1);
                if constexpr (SPLIT) {
                    Blo[(2 * nn) * kRowPad + kk] = bexp(lo, 0);
                    Blo[(2 * nn + 1) * kRowPad + kk] = bexp(lo, 1);
                }
            }
        }
        __syncthreads();
        if (k0 + TK < K) load_chunk(k0 + TK);
#pragma unroll
        for (int ks = 0; ks < TK; ks += 16) {
            uint4 ah[WM], al[SPLIT ? WM : 1], bh[WN], bl[SPLIT ? WN : 1];
#pragma unroll
            for (int bm = 0; bm < WM; ++bm) {
                const int o = ((wm * WM + bm) * 16 + lr) * kRowPad + ks + 4 * lg;
                ah[bm] = *reinterpret_cast<const uint4*>(Ahi + o);
                if constexpr (SPLIT) al[bm] = *reinterpret_cast<const uint4*>(Alo + o);
            }
#pragma unroll
            for (int bn = 0; bn < WN; ++bn) {
                const int o = ((wn * WN + bn) * 16 + lr) * kRowPad + ks + 4 * lg;
                bh[bn] = *reinterpret_cast<const uint4*>(Bhi + o);
                if constexpr (SPLIT) bl[bn] = *reinterpret_cast<const uint4*>(Blo + o);
            }
#pragma unroll
            for (int bm = 0; bm < WM; ++bm)
#pragma unroll
                for (int bn = 0; bn < WN; ++bn) {
                    if constexpr (MODE == LP_BF16) {
                        acc[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            __builtin_bit_cast(bf16x8, ah[bm]), __builtin_bit_cast(bf16x8, bh[bn]), acc[bm][bn], 0,
                            0, 0);
                    } else {
                        acc[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                            __builtin_bit_cast(half8, ah[bm]), __builtin_bit_cast(half8, bh[bn]), acc[bm][bn], 0, 0,
                            0);
                        if constexpr (SPLIT) {
                            accx[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                                __builtin_bit_cast(half8, ah[bm]), __builtin_bit_cast(half8, bl[bn]), accx[bm][bn],
                                0, 0, 0);
                            accx[bm][bn] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                                __builtin_bit_cast(half8, al[bm]), __builtin_bit_cast(half8, bh[bn]), accx[bm][bn],
                                0, 0, 0);
                        }
                    }
                }
        }
        __syncthreads();
    }
    // undo the scaling exactly and fold in the cross terms
    const float sc = ldexpf(1.f, ea + eb);
    float mx = 0.f;
#pragma unroll
    for (int bm = 0; bm < WM; ++bm)
#pragma unroll
        for (int bn = 0; bn < WN; ++bn)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                float v = acc[bm][bn][r];
                if constexpr (SPLIT) v = fmaf(accx[bm][bn][r], 1.f / 2048.f, v);
                v *= sc;
                acc[bm][bn][r] = v;
                mx = fmaxf(mx, fabsf(v));
            }
    if (g.cmax) tile_max_atomic(mx, g.cmax);
    const uint64_t cbase = deposit(ti.m0, g.cpm, g.tm, g.m_log) + deposit(ti.n0, g.cpn, g.tn, g.n_log) +
                           deposit(ti.beta, g.cpb, 0, g.b_log);
    store_tile<TM, TNR, L::RP>(g, reinterpret_cast<float*>(smem), reinterpret_cast<float2*>(g.C) + cbase,
                               [&](auto put) {
#pragma unroll
        for (int bm = 0; bm < WM; ++bm)
#pragma unroll
            for (int bn = 0; bn < WN; ++bn)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    put((wm * WM + bm) * 16 + 4 * lg + r, (wn * WN + bn) * 16 + lr, acc[bm][bn][r]);
    });
}

// Mixed-precision form of k_panel (v_mfma_f32_32x32x16_{f16,bf16}): lane
// (r, h) supplies eight halves = four packed (re, im) words of complex k
// 4 h .. 4 h + 3 of an 8-k step, for row r; B' words are staged in LDS k-fastest
// (rows of real columns: (re, -im) for column 2n, (im, re) for 2n+1).  Split
// mode keeps one accumulator for 2^22 a b = hi_a hi_b + hi_a lo_b + lo_a hi_b
// with both operands split at 2^11 (split_pack11; |x| < 2^11 after scaling,
// well inside FP16); the result is acc * 2^(ea+eb-22).
template <int KC, int NB, int MODE, bool PRE, bool NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NB >= 8 ? 2 : (NB == 2 ? (KC == 16 ? 4 : 3) : (KC == 16 ? 3 : 1)))))
k_panel_lp(GemmArgs g) {
    constexpr int N = 16 * NB;
    constexpr int NR = 2 * N;
    constexpr bool SPLIT = MODE == LP_SPLIT_FP16;
    constexpr int PL = SPLIT ? 2 : 1;
    constexpr int RS = KC + 4;
    constexpr int CS = 17;
    constexpr int PBN = KC * N / 256;
    constexpr int NS = KC / 8;               // MFMA steps (8 complex k) per chunk
    // B' planes and the output slabs share one LDS buffer (the epilogue
    // starts with a barrier after the last chunk), for more blocks per CU
    constexpr int BW_WORDS = PL * NR * RS, CS_WORDS = 2 * 128 * CS;
    __shared__ __attribute__((aligned(16))) uint32_t smem[BW_WORDS > CS_WORDS ? BW_WORDS : CS_WORDS];
    uint32_t* const Bw[2] = {smem, smem + (PL - 1) * NR * RS};
    float2* const Cs = reinterpret_cast<float2*>(smem);
    const TileIndex ti = tile_index(g);
    const uint64_t sAk = 1ull << (g.m_log + g.b_log), sBk = 1ull << (g.n_log + g.b_log);
    const float2* A = reinterpret_cast<const float2*>(g.A) + slice_offset(g.d_slice, g.sa_n, g.sa_bit, g.sa_pos) +
                      (ti.beta << g.m_log) + ti.m0;
    const float2* B = reinterpret_cast<const float2*>(g.B) + slice_offset(g.d_slice, g.sb_n, g.sb_bit, g.sb_pos) +
                      (ti.beta << g.n_log) + ti.n0;
    const int ea = scale_exp(g.amax), eb = scale_exp(g.bmax);
    const float sa = ldexpf(1.f, -ea + (SPLIT ? 11 : 0)), sb = ldexpf(1.f, -eb + (SPLIT ? 11 : 0));
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int r = lane & 31, h = lane >> 5;
    const uint64_t K = 1ull << g.k_log;
    // A: NS steps of 8 complex k per chunk; lane (r, h) holds complex k
    // 4 h .. 4 h + 3 of each step for row r.  Without PRE they are loaded as
    // complex64 and split here; with PRE they arrive split, as 16-byte groups
    // of four k per row (planes g.A / g.a_lo, layout [K/4][batch, M][4]).
    float2 av[PRE ? 1 : NS][4], an[PRE ? 1 : NS][4], bb[PBN];
    uint4 ph[PRE ? NS : 1][PL], pn[PRE ? NS : 1][PL];
    const uint64_t rowA = (ti.beta << g.m_log) + ti.m0 + w * 32 + r;
    auto load_a = [&](float2 (&dst)[PRE ? 1 : NS][4], uint4 (&pdst)[PRE ? NS : 1][PL], uint64_t k0) {
        if constexpr (PRE) {
            const uint4* hp = reinterpret_cast<const uint4*>(g.A);
            const uint4* lp = reinterpret_cast<const uint4*>(g.a_lo);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const uint64_t q = ((k0 >> 2) + 2 * s + h) * sAk + rowA;
                pdst[s][0] = hp[q];
                if constexpr (SPLIT) pdst[s][PL - 1] = lp[q];
            }
        } else {
            const float2* src = A + w * 32 + r + (k0 + 4 * h) * sAk;
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if constexpr (NT) {   // non-temporal: A is read by few N tiles
                        const floatv2 t = __builtin_nontemporal_load(
                            reinterpret_cast<const floatv2*>(src + (uint64_t)(8 * s + i) * sAk));
                        dst[s][i] = make_float2(t.x, t.y);
                    } else {
                        dst[s][i] = src[(uint64_t)(8 * s + i) * sAk];
                    }
                }
        }
    };
    // B chunk element of thread slot i: each wave instruction covers 4
    // consecutive columns by 16 k, so the word stores into the k-fastest
    // rows below (row stride KC + 4 words) fall into 32 distinct banks per
    // half-wave (a column-fastest walk would put 8 lanes on each bank)
    auto b_elem = [&](int i, int& kk, int& nn) {
        constexpr int KQ = KC / 16;
        const int l = tid & 63, q = (tid >> 6) + 4 * i;
        kk = (l >> 2) + 16 * (q % KQ);
        nn = (l & 3) + 4 * (q / KQ);
    };
    auto load_b = [&](uint64_t k0) {
#pragma unroll
        for (int i = 0; i < PBN; ++i) {
            int kk, nn;
            b_elem(i, kk, nn);
            bb[i] = B[(k0 + kk) * sBk + nn];
        }
    };
    floatx16 acc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[nb][v] = 0.f;
    load_b(0);   // B first: see k_panel
    load_a(av, ph, 0);
    for (uint64_t k0 = 0; k0 < K; k0 += KC) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < PBN; ++i) {
            int kk, nn;
            b_elem(i, kk, nn);
            uint32_t hi, lo;
            split_pack11<MODE>(bb[i], sb, hi, lo);
            Bw[0][(2 * nn) * RS + kk] = bexp(hi, 0);
            Bw[0][(2 * nn + 1) * RS + kk] = bexp(hi, 1);
            if constexpr (SPLIT) {
                Bw[PL - 1][(2 * nn) * RS + kk] = bexp(lo, 0);
                Bw[PL - 1][(2 * nn + 1) * RS + kk] = bexp(lo, 1);
            }
        }
        __syncthreads();
        if (k0 + KC < K) {
            load_b(k0 + KC);
            load_a(an, pn, k0 + KC);
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            uint4 ah, al;
            if constexpr (PRE) {
                ah = ph[s][0];
                al = ph[s][PL - 1];
            } else {
                uint32_t hw[4], lw[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) split_pack11<MODE>(av[s][i], sa, hw[i], lw[i]);
                ah = uint4{hw[0], hw[1], hw[2], hw[3]};
                al = uint4{lw[0], lw[1], lw[2], lw[3]};
            }
            const half8 ah8 = __builtin_bit_cast(half8, ah), al8 = __builtin_bit_cast(half8, al);
            // G accumulation chains at a time with their B' fragments read
            // together: each chain's next MFMA is G issues later, and one
            // LDS wait covers the group's reads
            constexpr int G = NB >= 8 ? 4 : 2;
#pragma unroll
            for (int nb = 0; nb < NB; nb += G) {
                half8 bh[G], bl[SPLIT ? G : 1];
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    const int o = ((nb + q) * 32 + r) * RS + 8 * s + 4 * h;
                    bh[q] = __builtin_bit_cast(half8, *reinterpret_cast<const uint4*>(&Bw[0][o]));
                    if constexpr (SPLIT) bl[q] = __builtin_bit_cast(half8, *reinterpret_cast<const uint4*>(&Bw[PL - 1][o]));
                }
                if constexpr (MODE == LP_BF16) {
                    const bf16x8 ab = __builtin_bit_cast(bf16x8, ah);
#pragma unroll
                    for (int q = 0; q < G; ++q)
                        acc[nb + q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ab, __builtin_bit_cast(bf16x8, bh[q]),
                                                                              acc[nb + q], 0, 0, 0);
                } else {
                    if constexpr (SPLIT) {
#pragma unroll
                        for (int q = 0; q < G; ++q)
                            acc[nb + q] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah8, bl[q], acc[nb + q], 0, 0, 0);
#pragma unroll
                        for (int q = 0; q < G; ++q)
                            acc[nb + q] = __builtin_amdgcn_mfma_f32_32x32x16_f16(al8, bh[q], acc[nb + q], 0, 0, 0);
                    }
#pragma unroll
                    for (int q = 0; q < G; ++q)
                        acc[nb + q] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah8, bh[q], acc[nb + q], 0, 0, 0);
                }
            }
        }
        if constexpr (PRE) {
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int p = 0; p < PL; ++p) ph[s][p] = pn[s][p];
        } else {
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int i = 0; i < 4; ++i) av[s][i] = an[s][i];
        }
    }
    const float sc = ldexpf(1.f, ea + eb - (SPLIT ? 22 : 0));
    uint64_t off_lo = 0;
    int src_lo = 0;
    for (int i = 0; i < 8; ++i)
        if ((tid >> i) & 1) {
            off_lo |= 1ull << g.ep_pos[i];
            const int sbt = g.ep_src[i];
            src_lo += sbt < 32 ? CS << sbt : 1 << (sbt - 32);
        }
    const EpHigh eh = ep_high(g, 8, CS);
    float mx = 0.f;
    const uint64_t cbase = deposit(ti.m0, g.cpm, 7, g.m_log) + deposit(ti.beta, g.cpb, 0, g.b_log);
    float* cs = reinterpret_cast<float*>(Cs);
    float2* C = reinterpret_cast<float2*>(g.C);
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
        __syncthreads();
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const float x = acc[nb][v] * sc;
            const int row = w * 32 + 8 * (v >> 2) + 4 * h + (v & 3);
            cs[row * (2 * CS) + r] = x;
            mx = fmaxf(mx, fabsf(x));
        }
        __syncthreads();
        const uint64_t cb = cbase + deposit(ti.n0 + ((uint64_t)nb << 4), g.cpn, 4, g.n_log);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const uint64_t off_hi = eh.off(j);
            const int src_hi = eh.from(j);
            C[cb + (off_lo | off_hi)] = Cs[src_lo + src_hi];
        }
    }
    if (g.cmax) tile_max_atomic(mx, g.cmax);
}

// Split a complex64 A operand ([K | batch | M], scaled by 2^-e from the
// producer's max) into word planes laid out [K/4][batch, M][4]: the four k of
// one row that a lane of k_panel_lp needs are one 16-byte load.
template <int MODE>
__global__ void __launch_bounds__(256) k_lp_convert_a(GemmArgs g, uint32_t* hi, uint32_t* lo) {
    const float2* A = reinterpret_cast<const float2*>(g.A) + slice_offset(g.d_slice, g.sa_n, g.sa_bit, g.sa_pos);
    const uint64_t rows = 1ull << (g.m_log + g.b_log);
    const uint64_t n = rows << (g.k_log - 2);
    const float sc = ldexpf(1.f, -scale_exp(g.amax) + (MODE == LP_SPLIT_FP16 ? 11 : 0));
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x; t < n; t += stride) {
        const uint64_t q = t / rows, row = t % rows;
        uint32_t h[4], l[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) split_pack11<MODE>(A[(4 * q + i) * rows + row], sc, h[i], l[i]);
        reinterpret_cast<uint4*>(hi)[t] = uint4{h[0], h[1], h[2], h[3]};
        if constexpr (MODE == LP_SPLIT_FP16) reinterpret_cast<uint4*>(lo)[t] = uint4{l[0], l[1], l[2], l[3]};
    }
}

__global__ void __launch_bounds__(256) k_fill(float* p, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

// ------------------------------------------------------------ slice sum

struct RootSel {
    const uint64_t* d_slice;
    int n;
    uint8_t bit[8], pos[8];
};

template <typename T>
__global__ void __launch_bounds__(256) k_slice_sum(const T* root, double2* acc, int res_log,
                                                   const uint32_t* mask, uint64_t b0, uint64_t b1, RootSel rs) {
    root += slice_offset(rs.d_slice, rs.n, rs.bit, rs.pos);
    const uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= (1ull << res_log)) return;
    double sx = 0.0, sy = 0.0;
    for (uint64_t be = b0; be < b1; ++be) {
        if (mask && !((mask[be >> 5] >> (be & 31)) & 1u)) continue;
        const T v = root[(be << res_log) + r];
        sx += (double)v.x;
        sy += (double)v.y;
    }
    double2 a = acc[r];
    a.x += sx;
    a.y += sy;
    acc[r] = a;
}

// Graph replay state: the only device writes are vector stores from lane 0.
__global__ void k_group_set(GroupState* st, uint64_t first) {
    if (threadIdx.x == 0) {
        GroupState v;
        v.next_group = first;
        v.slice_base = 0;
        st[threadIdx.x] = v;
    }
}

__global__ void k_group_begin(GroupState* st, int batch_log2) {
    if (threadIdx.x == 0) {
        GroupState v = st[threadIdx.x];
        v.slice_base = v.next_group << batch_log2;
        v.next_group += 1;
        st[threadIdx.x] = v;
    }
}

__global__ void __launch_bounds__(256) k_copy(const double* src, double* dst, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ------------------------------------------------------------------ XEB

__global__ void __launch_bounds__(256) k_xeb_partials(const double2* amps, uint64_t n, double w, double* part) {
    __shared__ double s1[256], s2[256], smax[256], smin[256];
    double a = 0, b = 0, mx = 0, mn = 1e300;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
        const double2 v = amps[i];
        const double p = w * (v.x * v.x + v.y * v.y);
        a += p;
        b += p * p;
        mx = fmax(mx, p);
        mn = fmin(mn, p);
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    smax[threadIdx.x] = mx;
    smin[threadIdx.x] = mn;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            s1[threadIdx.x] += s1[threadIdx.x + h];
            s2[threadIdx.x] += s2[threadIdx.x + h];
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + h]);
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[4 * blockIdx.x + 0] = s1[0];
        part[4 * blockIdx.x + 1] = s2[0];
        part[4 * blockIdx.x + 2] = smax[0];
        part[4 * blockIdx.x + 3] = smin[0];
    }
}

// sum of the conditional probabilities P / P(s1) (appendix C)
__global__ void __launch_bounds__(256) k_xeb_cond(const double2* amps, uint64_t n, double w, double inv_sum,
                                                  double* part) {
    __shared__ double s1[256];
    double a = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256) {
        const double2 v = amps[i];
        a += (w * (v.x * v.x + v.y * v.y)) * inv_sum;
    }
    s1[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s1[threadIdx.x] += s1[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s1[0];
}

// --------------------------------------------------------------- launch

namespace {

dim3 grid_for(uint64_t blocks) {
    if (blocks <= 0x7fffffffULL) return dim3((unsigned)blocks, 1, 1);
    unsigned x = 1u << 20;
    return dim3(x, (unsigned)((blocks + x - 1) / x), 1);
}

uint64_t tile_blocks(const GemmArgs& g) {
    return 1ull << ((g.m_log - g.tm) + (g.n_log - g.tn) + g.b_log + g.split_log);
}

// A tile must fit the step: tile_index shifts by m_log - tm and n_log - tn.
bool tile_fits(const GemmArgs& g) {
    return g.tm >= 0 && g.tn >= 0 && g.tm <= g.m_log && g.tn <= g.n_log && g.split_log >= 0 &&
           g.split_log <= g.k_log && (g.m_log - g.tm) + (g.n_log - g.tn) + g.b_log + g.split_log < 62;
}

}  // namespace

hipError_t launch_valu(int storage, const GemmArgs& g, int R, hipStream_t s) {
    if (!tile_fits(g)) return hipErrorInvalidValue;
    const size_t esz = storage == ST_C128 ? 16 : 8;
    const size_t ab = (size_t)((1 << g.tk) * ((1 << g.tm) + (1 << g.tn)));
    const size_t st = (size_t)1 << (g.tm + g.tn);
    const size_t smem = std::max(ab, st) * esz;
    const dim3 grid = grid_for(tile_blocks(g));
    if (grid.y > 1 && (uint64_t)grid.x * grid.y != tile_blocks(g)) return hipErrorInvalidValue;
#define TN_VALU(T, RR) hipLaunchKernelGGL((k_valu<T, RR>), grid, dim3(256), smem, s, g)
    if (storage == ST_C128) {
        switch (R) {
            case 1: TN_VALU(double2, 1); break;
            case 2: TN_VALU(double2, 2); break;
            case 4: TN_VALU(double2, 4); break;
            default: TN_VALU(double2, 8); break;
        }
    } else {
        switch (R) {
            case 1: TN_VALU(float2, 1); break;
            case 2: TN_VALU(float2, 2); break;
            case 4: TN_VALU(float2, 4); break;
            default: TN_VALU(float2, 8); break;
        }
    }
#undef TN_VALU
    return hipGetLastError();
}

hipError_t launch_stream(int storage, const GemmArgs& g, hipStream_t s) {
    if (g.k_log > 4 || g.n_log > 4) return hipErrorInvalidValue;
    if (storage == ST_C128) {
        const uint64_t blocks = std::max<uint64_t>(1, (1ull << g.m_log) / 256);
        if (g.m_log < 8) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_stream<double2, 1>), dim3((unsigned)blocks, 1u << g.b_log), dim3(256), 0, s, g);
    } else {
        if (g.m_log < 9) return hipErrorInvalidValue;
        const uint64_t blocks = (1ull << g.m_log) / 512;
        hipLaunchKernelGGL((k_stream<float2, 2>), dim3((unsigned)blocks, 1u << g.b_log), dim3(256), 0, s, g);
    }
    return hipGetLastError();
}

hipError_t launch_skinny(const GemmArgs& g, hipStream_t s) {
    if (g.n_log < 4 || g.n_log > 6 || g.k_log < 1 || g.k_log > 6 || g.k_log + g.n_log > 12 || g.m_log < 7 ||
        g.b_log > 16 || g.tm != 5 || g.tn != 4 || g.ep_n != 9)
        return hipErrorInvalidValue;
    const uint64_t tiles = 1ull << (g.m_log - 7);
    // enough blocks to fill the chip several times, each walking several tiles
    const int want_log = std::max(0, 12 - g.b_log);
    const unsigned bx = (unsigned)std::min<uint64_t>(tiles, 1ull << want_log);
    const dim3 grid(bx, 1u << g.b_log);
#define TN_SK(KT, NB) hipLaunchKernelGGL((k_skinny<KT, NB>), grid, dim3(256), 0, s, g)
#define TN_SK_N(KT)                    \
    switch (g.n_log) {                 \
        case 4: TN_SK(KT, 1); break;   \
        case 5: TN_SK(KT, 2); break;   \
        default: TN_SK(KT, 4); break;  \
    }
    switch (g.k_log) {
        case 1: TN_SK_N(2); break;
        case 2: TN_SK_N(4); break;
        case 3: TN_SK_N(8); break;
        case 4: TN_SK_N(16); break;
        case 5: TN_SK_N(32); break;
        default:
            if (g.n_log == 6) TN_SK(64, 4);
            else if (g.n_log == 5) TN_SK(64, 2);
            else TN_SK(64, 1);
            break;
    }
#undef TN_SK_N
#undef TN_SK
    return hipGetLastError();
}

template <bool NT>
static void launch_panel3_t(int tile, const GemmArgs& g, dim3 grid, hipStream_t s) {
    switch (tile & 3) {
        case 0: hipLaunchKernelGGL((k_panel3<32, 4, NT>), grid, dim3(256), 0, s, g); break;
        case 1: hipLaunchKernelGGL((k_panel3<16, 4, NT>), grid, dim3(256), 0, s, g); break;
        case 2: hipLaunchKernelGGL((k_panel3<32, 2, NT>), grid, dim3(256), 0, s, g); break;
        default: hipLaunchKernelGGL((k_panel3<16, 2, NT>), grid, dim3(256), 0, s, g); break;
    }
}

template <bool NT>
static void launch_panel_t(int tile, const GemmArgs& g, dim3 grid, hipStream_t s) {
    switch (tile & 3) {
        case 0: hipLaunchKernelGGL((k_panel<32, 4, NT>), grid, dim3(256), 0, s, g); break;
        case 1: hipLaunchKernelGGL((k_panel<16, 4, NT>), grid, dim3(256), 0, s, g); break;
        case 2: hipLaunchKernelGGL((k_panel<32, 2, NT>), grid, dim3(256), 0, s, g); break;
        default: hipLaunchKernelGGL((k_panel<16, 2, NT>), grid, dim3(256), 0, s, g); break;
    }
}

hipError_t launch_panel(int tile, const GemmArgs& g, hipStream_t s) {
    // tile: bit 0 -> KC = 16 (else 32), bit 1 -> NB = 2 (else 4), bit 4 ->
    // non-temporal A loads, bit 5 -> three real products per complex
    // multiply-add (k_panel3), bit 7 -> k_panel3 with A staged in LDS by
    // direct loads (KC = 16, no bit 4)
    const int kc_log = (tile & 1) ? 4 : 5, nb_log = (tile & 2) ? 1 : 2;
    if (tile < 0 || (tile & ~179) || g.tm != 7 || g.tn != 4 + nb_log || !tile_fits(g) || g.k_log < kc_log ||
        g.ep_n != 11 || g.split_log != 0 || ((tile & 128) && (tile & 49) != 33))
        return hipErrorInvalidValue;
    const dim3 grid = grid_for(tile_blocks(g));
    if (tile & 128) {
        if (tile & 2) hipLaunchKernelGGL((k_panel3d<2>), grid, dim3(256), 0, s, g);
        else hipLaunchKernelGGL((k_panel3d<4>), grid, dim3(256), 0, s, g);
    } else if (tile & 32) {
        if (tile & 16) launch_panel3_t<true>(tile, g, grid, s);
        else launch_panel3_t<false>(tile, g, grid, s);
    } else {
        if (tile & 16) launch_panel_t<true>(tile, g, grid, s);
        else launch_panel_t<false>(tile, g, grid, s);
    }
    return hipGetLastError();
}

hipError_t launch_splitk_reduce(int storage, const GemmArgs& g, hipStream_t s) {
    const uint64_t total = 1ull << (g.m_log + g.n_log + g.b_log);
    const dim3 grid = grid_for((total + 255) / 256);
    if (storage == ST_C128) hipLaunchKernelGGL(k_splitk_red<double2>, grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL(k_splitk_red<float2>, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_lp(int tile, const GemmArgs& g, dim3 grid, hipStream_t s) {
    switch (tile) {
        case 0: hipLaunchKernelGGL((k_mfma_lp<4, 4, 2, 2, MODE>), grid, dim3(256), 0, s, g); break;
        case 1: hipLaunchKernelGGL((k_mfma_lp<2, 2, 2, 2, MODE>), grid, dim3(256), 0, s, g); break;
        case 2: hipLaunchKernelGGL((k_mfma_lp<2, 2, 4, 1, MODE>), grid, dim3(256), 0, s, g); break;
        case 3: hipLaunchKernelGGL((k_mfma_lp<1, 1, 4, 1, MODE>), grid, dim3(256), 0, s, g); break;
        case 4: hipLaunchKernelGGL((k_mfma_lp<4, 1, 4, 1, MODE>), grid, dim3(256), 0, s, g); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MODE, bool PRE, bool NT>
static hipError_t launch_panel_lp_t(int tile, const GemmArgs& g, dim3 grid, hipStream_t s) {
    if (tile & 64) {   // KC = 16 only (KC = 32 spills at two waves per SIMD)
        hipLaunchKernelGGL((k_panel_lp<16, 8, MODE, PRE, NT>), grid, dim3(256), 0, s, g);
        return hipGetLastError();
    }
    switch (tile & 3) {
        case 0: hipLaunchKernelGGL((k_panel_lp<32, 4, MODE, PRE, NT>), grid, dim3(256), 0, s, g); break;
        case 1: hipLaunchKernelGGL((k_panel_lp<16, 4, MODE, PRE, NT>), grid, dim3(256), 0, s, g); break;
        case 2: hipLaunchKernelGGL((k_panel_lp<32, 2, MODE, PRE, NT>), grid, dim3(256), 0, s, g); break;
        default: hipLaunchKernelGGL((k_panel_lp<16, 2, MODE, PRE, NT>), grid, dim3(256), 0, s, g); break;
    }
    return hipGetLastError();
}

hipError_t launch_panel_lp(int mode, int tile, const GemmArgs& g, uint32_t* conv, hipStream_t s) {
    // tile bits as in launch_panel; bit 4 (non-temporal A loads) applies to
    // A split in registers (conv = null) only; bit 6: NB = 8 (KC = 16)
    const int kc_log = (tile & 1) ? 4 : 5, nb_log = (tile & 64) ? 3 : ((tile & 2) ? 1 : 2);
    if (tile < 0 || (tile & ~83) || ((tile & 64) && (tile & 3) != 1) || (conv && (tile & 16)) || g.tm != 7 || g.tn != 4 + nb_log || !tile_fits(g) ||
        g.k_log < kc_log || g.ep_n != 11 || g.split_log != 0 || (mode != LP_SPLIT_FP16 && mode != LP_BF16))
        return hipErrorInvalidValue;
    const dim3 grid = grid_for(tile_blocks(g));
    if (!conv) {
        const bool nt = tile & 16;
        if (mode == LP_SPLIT_FP16)
            return nt ? launch_panel_lp_t<LP_SPLIT_FP16, false, true>(tile, g, grid, s)
                      : launch_panel_lp_t<LP_SPLIT_FP16, false, false>(tile, g, grid, s);
        return nt ? launch_panel_lp_t<LP_BF16, false, true>(tile, g, grid, s)
                  : launch_panel_lp_t<LP_BF16, false, false>(tile, g, grid, s);
    }
    // one pass over A into word planes, then the GEMM on the planes
    const uint64_t na = 1ull << (g.m_log + g.b_log + g.k_log);
    uint32_t* hi = conv;
    uint32_t* lo = conv + na;
    const dim3 cgrid((unsigned)std::min<uint64_t>(((na >> 2) + 255) / 256, 16384));
    if (mode == LP_SPLIT_FP16) hipLaunchKernelGGL(k_lp_convert_a<LP_SPLIT_FP16>, cgrid, dim3(256), 0, s, g, hi, lo);
    else hipLaunchKernelGGL(k_lp_convert_a<LP_BF16>, cgrid, dim3(256), 0, s, g, hi, lo);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    GemmArgs h = g;
    h.A = hi;
    h.a_lo = lo;
    h.sa_n = 0;   // the planes are already slice-selected
    if (mode == LP_SPLIT_FP16) return launch_panel_lp_t<LP_SPLIT_FP16, true, false>(tile, h, grid, s);
    return launch_panel_lp_t<LP_BF16, true, false>(tile, h, grid, s);
}

hipError_t launch_fill(float* p, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;   // nothing to clear (e.g. every tensor slice-invariant)
    hipLaunchKernelGGL(k_fill, grid_for((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_mfma(int mode, int tile, const GemmArgs& g, hipStream_t s) {
    if (!tile_fits(g)) return hipErrorInvalidValue;
    const dim3 grid = grid_for(tile_blocks(g));
    if (mode == LP_SPLIT_FP16) return launch_lp<LP_SPLIT_FP16>(tile, g, grid, s);
    if (mode == LP_FP16) return launch_lp<LP_FP16>(tile, g, grid, s);
    if (mode == LP_BF16) return launch_lp<LP_BF16>(tile, g, grid, s);
    switch (tile) {
        case 0: hipLaunchKernelGGL((k_mfma_c64<4, 4, 2, 2>), grid, dim3(256), 0, s, g); break;
        case 1: hipLaunchKernelGGL((k_mfma_c64<2, 2, 2, 2>), grid, dim3(256), 0, s, g); break;
        case 2: hipLaunchKernelGGL((k_mfma_c64<2, 2, 4, 1>), grid, dim3(256), 0, s, g); break;
        case 3: hipLaunchKernelGGL((k_mfma_c64<1, 1, 4, 1>), grid, dim3(256), 0, s, g); break;
        case 4: hipLaunchKernelGGL((k_mfma_c64<4, 1, 4, 1>), grid, dim3(256), 0, s, g); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_slice_sum(int storage, const void* root, double* acc, int res_log, int b_log,
                            const uint32_t* d_mask, uint64_t beta0, uint64_t beta1, hipStream_t s,
                            const uint64_t* d_slice, const uint8_t* r_bit, const uint8_t* r_pos, int r_n) {
    (void)b_log;
    RootSel rs{};
    rs.d_slice = d_slice;
    rs.n = r_n;
    for (int i = 0; i < r_n && i < 8; ++i) {
        rs.bit[i] = r_bit[i];
        rs.pos[i] = r_pos[i];
    }
    const uint64_t n = 1ull << res_log;
    const dim3 grid = grid_for((n + 255) / 256);
    if (storage == ST_C128)
        hipLaunchKernelGGL(k_slice_sum<double2>, grid, dim3(256), 0, s, reinterpret_cast<const double2*>(root),
                           reinterpret_cast<double2*>(acc), res_log, d_mask, beta0, beta1, rs);
    else
        hipLaunchKernelGGL(k_slice_sum<float2>, grid, dim3(256), 0, s, reinterpret_cast<const float2*>(root),
                           reinterpret_cast<double2*>(acc), res_log, d_mask, beta0, beta1, rs);
    return hipGetLastError();
}

hipError_t launch_group_set(GroupState* st, uint64_t first_group, hipStream_t s) {
    hipLaunchKernelGGL(k_group_set, dim3(1), dim3(64), 0, s, st, first_group);
    return hipGetLastError();
}

hipError_t launch_group_begin(GroupState* st, int batch_log2, hipStream_t s) {
    hipLaunchKernelGGL(k_group_begin, dim3(1), dim3(64), 0, s, st, batch_log2);
    return hipGetLastError();
}

hipError_t launch_copy_acc(const double* src, double* dst, uint64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_copy, grid_for((n + 255) / 256), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_xeb_partials(const double* amps, uint64_t n, double w, double* part, int blocks,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_xeb_partials, dim3(blocks), dim3(256), 0, s, reinterpret_cast<const double2*>(amps), n,
                       w, part);
    return hipGetLastError();
}

hipError_t launch_xeb_cond(const double* amps, uint64_t n, double w, double inv_sum, double* part, int blocks,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_xeb_cond, dim3(blocks), dim3(256), 0, s, reinterpret_cast<const double2*>(amps), n, w,
                       inv_sum, part);
    return hipGetLastError();
}

}  // namespace tn

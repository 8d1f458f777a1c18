// Device kernels of the contraction steps (declarations shared with the
// launcher).  Every step computes C[b, m, n] = sum_k A[k, b, m] * B[k, b, n]
// over complex numbers, with A and B plain strided arrays and C written to
// arbitrary address bits (the permutation into the consumer's layout happens
// while the tile is staged through LDS).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tn {

constexpr int kMaxBits = 40;

struct GemmArgs {
    const void* A;
    const void* B;
    void* C;
    void* scratch;          // split-K partial tiles
    int m_log, n_log, k_log, b_log;
    int tm, tn, tk;         // tile sizes (log2): m, n, k per chunk
    int split_log;          // K split into 2^split_log parts (partials to scratch)
    int ep_n;               // number of tile bits in the epilogue decode
    uint8_t ep_pos[16];     // address bit of the i-th lowest tile bit of C
    uint8_t ep_src[16];     // logical source: < 32 -> m bit, >= 32 -> n bit (src - 32)
    uint8_t cpm[kMaxBits], cpn[kMaxBits], cpb[kMaxBits];
    const uint32_t* a_lo;   // k_panel_lp on pre-split A: lo word plane (A then points at the hi plane)
    const float* amax;      // max |re|,|im| of A and B (low-precision MFMA scaling), or null
    const float* bmax;
    float* cmax;            // producer epilogue: atomic max of |re|,|im| of C, or null
    // Slice selection read from device memory (graph replays): operand X gets
    // offset sum_i bit(slice, x_bit[i]) << x_pos[i] elements, slice = *d_slice.
    const uint64_t* d_slice;
    uint8_t sa_n, sb_n;
    uint8_t sa_bit[8], sa_pos[8], sb_bit[8], sb_pos[8];
};

// Device-resident state of graph replays.
struct GroupState {
    uint64_t next_group;    // launch group o of the next replay
    uint64_t slice_base;    // o << batch_log2 of the current replay
};

// low-precision MFMA modes
enum LpMode : int { LP_SPLIT_FP16 = 0, LP_FP16 = 1, LP_BF16 = 2 };

// storage kinds
enum Storage : int { ST_C64 = 0, ST_C128 = 1, ST_BF16 = 2 };

hipError_t launch_valu(int storage, const GemmArgs& g, int R, hipStream_t s);
hipError_t launch_stream(int storage, const GemmArgs& g, hipStream_t s);
hipError_t launch_skinny(const GemmArgs& g, hipStream_t s);   // complex64 storage, FP32 MFMA
hipError_t launch_panel(int tile, const GemmArgs& g, hipStream_t s);   // complex64, FP32 MFMA
// Mixed-precision panel (mode LP_SPLIT_FP16 or LP_BF16).  conv: scratch of
// 2 * 2^(m+b+k) words for the split A planes, or null to split A in the GEMM.
hipError_t launch_panel_lp(int mode, int tile, const GemmArgs& g, uint32_t* conv, hipStream_t s);
hipError_t launch_splitk_reduce(int storage, const GemmArgs& g, hipStream_t s);
hipError_t launch_mfma(int mode, int tile, const GemmArgs& g, hipStream_t s);   // mode -1: FP32, else LpMode
hipError_t launch_fill(float* p, uint64_t n, hipStream_t s);
hipError_t launch_group_set(GroupState* st, uint64_t first_group, hipStream_t s);
hipError_t launch_group_begin(GroupState* st, int batch_log2, hipStream_t s);
hipError_t launch_slice_sum(int storage, const void* root, double* acc, int res_log, int b_log,
                            const uint32_t* d_mask, uint64_t beta0, uint64_t beta1, hipStream_t s,
                            const uint64_t* d_slice = nullptr, const uint8_t* r_bit = nullptr,
                            const uint8_t* r_pos = nullptr, int r_n = 0);
hipError_t launch_copy_acc(const double* src, double* dst, uint64_t n, hipStream_t s);
// acc[i] += part[i] and acc[i] = 0 over n complex128 entries (lanes.hip)
hipError_t launch_acc_add(double* acc, const double* part, uint64_t n, hipStream_t s);
hipError_t launch_acc_zero(double* acc, uint64_t n, hipStream_t s);
hipError_t launch_xeb_partials(const double* amps, uint64_t n, double w, double* part, int blocks,
                               hipStream_t s);
hipError_t launch_xeb_cond(const double* amps, uint64_t n, double w, double inv_sum, double* part,
                           int blocks, hipStream_t s);

}  // namespace tn

// Kernel classes and tile shapes shared by the planner and the launcher.
#pragma once

#include <algorithm>
#include <cstdint>

#include "../../include/tn.h"

namespace tn {

// MFMA tile shapes: complex M x N per workgroup of 4 waves.
struct MfmaTile {
    int tm_log, tn_log;   // log2 of the complex tile
    int waves_m, waves_n; // wave grid (waves_m * waves_n = 4)
    int tk_max_log;       // largest K chunk (complex, log2) the LDS tile holds
};
constexpr MfmaTile kMfmaTiles[] = {
    {7, 6, 2, 2, 4},   // 128 x 64: each wave 64 rows x 64 real columns
    {6, 5, 2, 2, 4},   // 64 x 32
    {7, 4, 4, 1, 4},   // 128 x 16
    {6, 3, 4, 1, 4},   // 64 x 8
    {8, 3, 4, 1, 3},   // 256 x 8
};
constexpr int kNumMfmaTiles = sizeof(kMfmaTiles) / sizeof(kMfmaTiles[0]);

inline bool mfma_capable(tn_precision p) { return p != TN_C128; }
inline bool lp_prec(tn_precision p) { return p == TN_SPLIT_FP16 || p == TN_BF16; }

// Skinny MFMA kernel: N = 16..64 complex columns, K = 2..64, B of at most 4096
// complex elements (held in LDS), 128-row tiles, complex64 storage.
inline bool skinny_ok(int m, int n, int k, int b, tn_precision prec) {
    return mfma_capable(prec) && n >= 4 && n <= 6 && k >= 1 && k <= 6 && k + n <= 12 && m >= 7 && b <= 16;
}

// Panel MFMA kernel: 128 rows x 16 NB columns per block, K in chunks of KC;
// FP32 for complex64, FP16/BF16 MFMA for the mixed forms (complex64
// storage).  Tile id: bit 0 -> KC = 16 (else 32), bit 1 -> NB = 2 (else 4),
// bit 2 -> FP32 MFMA even in a mixed form (the autotuner may pick it where
// the low-precision GEMM is not faster), bit 3 -> a mixed-form GEMM splits A
// in registers instead of reading planes split by a separate pass, bit 4 ->
// A loaded with non-temporal loads (FP32 panels and A split in registers),
// bit 5 -> complex64 panel with three real products per complex
// multiply-add (Gauss's form) instead of four, bit 6 -> NB = 8 (mixed-form
// GEMM only, with KC = 16: 128 complex columns per block, so each A element
// is loaded and split once per 128 columns instead of once per 32 or 64),
// bit 7 -> the three-product complex64 panel with its A chunks moved into
// LDS by direct global-to-LDS loads (with bits 0 and 5; k_panel3d).
constexpr int kNumPanelTiles = 4;
inline int panel_kc_log(int tile) { return (tile & 1) ? 4 : 5; }
inline int panel_tn_log(int tile) { return (tile & 64) ? 7 : ((tile & 2) ? 5 : 6); }
inline bool panel_fp32(int tile, tn_precision prec) { return prec == TN_C64 || (tile & 4); }
inline bool panel_ok(int m, int n, int k, int b, tn_precision prec, int tile) {
    return mfma_capable(prec) && m >= 7 && n >= panel_tn_log(tile) && k >= panel_kc_log(tile) &&
           (m - 7) + (n - panel_tn_log(tile)) + b < 40;
}

// Choose the kernel class and tile for C[b,m,n] = sum_k A[k,b,m] B[k,b,n]
// (all sizes log2).  Dense steps go to MFMA tiles; steps whose output is tiny
// but whose contracted dimension is long are split along K; everything else
// (the big-times-small steps that dominate bond-dimension-2 networks) runs on
// the streaming kernel, or the generic VALU tile kernel.
inline void choose_kernel(int m, int n, int k, int b, tn_precision prec, int& kernel, int& tile,
                          int& splitk_log) {
    kernel = 0;
    tile = 0;
    splitk_log = 0;
    // many rows against a small B: stream A once through the skinny kernel
    if (skinny_ok(m, n, k, b, prec) && m + b >= 14) {
        kernel = 4;
        return;
    }
    // dense complex64 steps: panel kernel, widest N tile that fits
    for (int t : {0, 2})
        if (panel_ok(m, n, k, b, prec, t) && k >= 6) {
            kernel = 5;
            tile = t;
            return;
        }
    if (mfma_capable(prec) && m >= 6 && n >= 3 && k >= 2) {
        int best = -1;
        for (int t = 0; t < kNumMfmaTiles; ++t) {
            const MfmaTile& T = kMfmaTiles[t];
            if (T.tm_log > m || T.tn_log > n) continue;
            const int grid_log = (m - T.tm_log) + (n - T.tn_log) + b;
            if (grid_log >= 9) { best = t; break; }
            if (best < 0 || grid_log > (m - kMfmaTiles[best].tm_log) + (n - kMfmaTiles[best].tn_log) + b)
                best = t;
        }
        if (best >= 0) {
            kernel = 1;
            tile = best;
            return;
        }
    }
    // big-times-small: streaming kernel (one pass over A, all K loads in flight)
    if (k <= 4 && n <= 4 && k + n <= 6 && m >= (prec == TN_C128 ? 8 : 9) && b <= 16) {
        kernel = 3;
        return;
    }
    if (m + n + b <= 14 && k >= 12) {
        kernel = 2;
        // aim for ~2^10 workgroups, each with at least 2^8 of K
        const int out_tiles_log = std::max(0, m + n + b - 8);
        splitk_log = std::max(0, std::min(k - 8, 10 - out_tiles_log));
        return;
    }
}

}  // namespace tn

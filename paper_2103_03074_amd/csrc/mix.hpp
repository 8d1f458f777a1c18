// Top-k selection of the computed probabilities and mixing with random
// bitstrings.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

namespace tn {

// Whole n-bit strings of open-qubit indices: bit pos[j] holds the j-th open
// qubit (the (n_open - 1 - j)-th bit of the index); base holds s1.
struct MixBits {
    uint64_t base;
    int n_open;
    uint8_t pos[64];
};

uint64_t mix_workspace_bytes(uint64_t n);

// d_out[0, k): the k most probable indices (ties to the lower index) as whole
// bitstrings in increasing index order; d_out[k, k + n_random): the random
// words masked to n_qubits bits.  p_top receives the sum of the selected
// probabilities.  Synchronises the stream.
std::string mix_topk(const double* d_amps, uint64_t n, uint64_t k, const MixBits& mb, const uint64_t* d_words,
                     uint64_t n_random, int n_qubits, uint64_t* d_out, void* ws, hipStream_t s, double& p_top);

}  // namespace tn

// Sampling from the conditional distribution of the open qubits.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace tn {

// Float64 elements of workspace that launch_sample needs for n probabilities
// (the cdf plus the block sums of every scan level).
uint64_t sample_workspace_elems(uint64_t n);

// amps: n complex128 amplitudes; u: n_samples uniforms in [0, 1); out:
// n_samples indices; ws: sample_workspace_elems(n) doubles.  Asynchronous.
hipError_t launch_sample(const double* amps, uint64_t n, const double* u, uint64_t n_samples, uint64_t* out,
                         double* ws, hipStream_t s);

// Same with the workspace in a file-scope device array (no allocation):
// n <= 2^kStaticSampleMaxOpen.  Calls that overlap on one GPU share the
// array and race.
constexpr int kStaticSampleMaxOpen = 20;
hipError_t launch_sample_static(const double* amps, uint64_t n, const double* u, uint64_t n_samples, uint64_t* out,
                                hipStream_t s);

}  // namespace tn

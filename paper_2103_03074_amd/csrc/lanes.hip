// Accumulator merge for concurrent lanes of launch groups: each extra lane
// sums its subtasks' results into a private float64 accumulator, and the
// caller's accumulator takes the lanes' sums in lane order once every lane
// has finished (section "The algorithm": the subtasks of a sliced network
// are independent and their results add up).
#include "kernels.hpp"

namespace tn {

namespace {

__global__ void __launch_bounds__(256) k_acc_add(double2* acc, const double2* part, uint64_t n) {
    const uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    double2 a = acc[r];
    const double2 b = part[r];
    a.x += b.x;
    a.y += b.y;
    acc[r] = a;
}

__global__ void __launch_bounds__(256) k_acc_zero(double2* acc, uint64_t n) {
    const uint64_t r = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (r < n) acc[r] = make_double2(0.0, 0.0);
}

}  // namespace

hipError_t launch_acc_add(double* acc, const double* part, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (n > (uint64_t)256 * 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_acc_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<double2*>(acc), reinterpret_cast<const double2*>(part), n);
    return hipGetLastError();
}

hipError_t launch_acc_zero(double* acc, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (n > (uint64_t)256 * 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_acc_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<double2*>(acc), n);
    return hipGetLastError();
}

}  // namespace tn

// Layout transposes between the ABI layout (element-major) and the coefficient-major device layout.
#include "kernels_common.hpp"

namespace ridg {

// ---------------------------------------------------------------- layout transposes
__global__ void aos_to_soa_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t nel, int nm) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nel * nm) return;
  int64_t e = t / nm;
  int k = (int)(t % nm);
  dst[(int64_t)k * nel + e] = src[t];
}

__global__ void soa_to_aos_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t nel, int nm) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nel * nm) return;
  int64_t e = t / nm;
  int k = (int)(t % nm);
  dst[t] = src[(int64_t)k * nel + e];
}

__global__ void check_finite_kernel(const double* __restrict__ x, int64_t n, int32_t* flag) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n && !isfinite(x[t])) flag[0] = 1;
}

int launch_aos_to_soa(const double* src, double* dst, int64_t nel, int nmodes, void* stream) {
  int64_t n = nel * nmodes;
  if (n == 0) return 0;
  hipLaunchKernelGGL(aos_to_soa_kernel, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, src, dst, nel, nmodes);
  return (int)hipGetLastError();
}

int launch_soa_to_aos(const double* src, double* dst, int64_t nel, int nmodes, void* stream) {
  int64_t n = nel * nmodes;
  if (n == 0) return 0;
  hipLaunchKernelGGL(soa_to_aos_kernel, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, src, dst, nel, nmodes);
  return (int)hipGetLastError();
}

int launch_check_finite(const double* x, int64_t n, int32_t* flag, void* stream) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(check_finite_kernel, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, x, n, flag);
  return (int)hipGetLastError();
}


}  // namespace ridg

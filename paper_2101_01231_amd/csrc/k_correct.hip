// Explicit flux-form correction (Sec. 2.3), FP64.
#include "kernels_common.hpp"

namespace ridg {

// ---------------------------------------------------------------- correction
template <int D, int M, bool AFFINE>
__global__ __launch_bounds__(256) void correct_kernel(DevGeom g, double dt, const double* __restrict__ Q,
                                                      const double* __restrict__ W, double* __restrict__ Qout,
                                                      DevTensors t) {
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  const int64_t e = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (e >= nel) return;
  correct_elem<D, M, AFFINE>(g, dt, Q, W, Qout, t, e, nel);
}

template <int D, int M>
struct CorrectL {
  static int run(int flux, const DevGeom& g, double dt, const double* Q, const double* W, double* Qout,
                 const DevTensors& t, void* stream) {
    const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
    if (flux == RIDG_FLUX_CONST)
      hipLaunchKernelGGL((correct_kernel<D, M, false>), dim3(grid_for(nel, 256)), dim3(256), 0,
                         (hipStream_t)stream, g, dt, Q, W, Qout, t);
    else
      hipLaunchKernelGGL((correct_kernel<D, M, true>), dim3(grid_for(nel, 256)), dim3(256), 0,
                         (hipStream_t)stream, g, dt, Q, W, Qout, t);
    return (int)hipGetLastError();
  }
};

int launch_correct(int d, int M, int flux, const DevGeom& g, double dt, const double* Q, const double* W,
                   double* Qout, const DevTensors& t, void* stream) {
  return dispatch_dm<CorrectL>(d, M, flux, g, dt, Q, W, Qout, t, stream);
}


}  // namespace ridg

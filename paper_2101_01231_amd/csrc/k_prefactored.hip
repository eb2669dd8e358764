// Constant-velocity prediction with the host-prefactored operator G (Sec. 2.2, one linear solve).
#include "kernels_common.hpp"

namespace ridg {

// ---------------------------------------------------------------- prefactored prediction
// Constant velocity: W_e = sum_tap G_tap Q_{e + off_tap} (Sec. 2.2 system solved once on the host).
struct Taps {
  int8_t off[kMaxBlocks][3];
};

template <int D, int M>
__global__ __launch_bounds__(256) void predict_prefactored_kernel(DevGeom g, const double* __restrict__ Q,
                                                                  double* __restrict__ W,
                                                                  const double* __restrict__ G, Taps taps,
                                                                  int ntaps) {
  constexpr int NS = n_space(D, M), NT = n_spacetime(D, M);
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nel) return;
  int idx[3];
  elem_idx(g, e, idx);
  double w[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) w[k] = 0.0;
  for (int t = 0; t < ntaps; ++t) {
    const int64_t src = elem_lin(g, idx[0] + taps.off[t][0], idx[1] + taps.off[t][1], idx[2] + taps.off[t][2]);
    double q[NS];
#pragma unroll
    for (int l = 0; l < NS; ++l) q[l] = Q[(int64_t)l * nel + src];
    const double* Gt = G + (size_t)t * NT * NS;
#pragma unroll
    for (int k = 0; k < NT; ++k)
#pragma unroll
      for (int l = 0; l < NS; ++l) w[k] = fma(Gt[k * NS + l], q[l], w[k]);
  }
#pragma unroll
  for (int k = 0; k < NT; ++k) W[(int64_t)k * nel + e] = w[k];
}

template <int D, int M>
struct PrefactoredL {
  static int run(const DevGeom& g, const double* Q, double* W, const double* G, const int32_t* taps, int ntaps,
                 void* stream) {
    Taps tp;
    for (int t = 0; t < kMaxBlocks; ++t)
      for (int i = 0; i < 3; ++i) tp.off[t][i] = (t < ntaps) ? (int8_t)taps[3 * t + i] : 0;
    const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
    hipLaunchKernelGGL((predict_prefactored_kernel<D, M>), dim3(grid_for(nel, 256)), dim3(256), 0,
                       (hipStream_t)stream, g, Q, W, G, tp, ntaps);
    return (int)hipGetLastError();
  }
};

int launch_predict_prefactored(int d, int M, const DevGeom& g, const double* Q, double* W, const double* G,
                               const int32_t* taps, int ntaps, void* stream) {
  return dispatch_dm<PrefactoredL>(d, M, g, Q, W, G, taps, ntaps, stream);
}


}  // namespace ridg

// Constant-velocity prediction with the host-prefactored operator G (Sec. 2.2, one linear solve),
// and the fused small-mesh kernel that runs whole RIDG steps (prediction, then correction, Sec.
// 2.3) on one workgroup with the mesh state resident in LDS.
#include "kernels_common.hpp"

namespace ridg {

template <int D, int M>
__global__ __launch_bounds__(256) void predict_prefactored_kernel(DevGeom g, const double* __restrict__ Q,
                                                                  double* __restrict__ W,
                                                                  const double* __restrict__ G, Taps taps,
                                                                  int ntaps) {
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  const int64_t e = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (e >= nel) return;
  predict_prefactored_elem<D, M>(g, Q, W, G, taps, ntaps, e, nel);
}

// n_steps full steps with a workgroup-wide barrier between the prediction of every element and
// the correction (which reads the face neighbours' predictions). Q and W live in LDS; the
// correction updates Q in place (each element writes only its own coefficients).
constexpr int kFusedThreads = 1024;
constexpr int64_t kFusedLdsBytes = 160 * 1024;

template <int D, int M>
__global__ __launch_bounds__(kFusedThreads) void fused_prefactored_kernel(DevGeom g, double dt,
                                                                         const double* __restrict__ Qin,
                                                                         double* __restrict__ Qout,
                                                                         const double* __restrict__ G, Taps taps,
                                                                         int ntaps, DevTensors t, int n_steps) {
  constexpr int NS = n_space(D, M);
  extern __shared__ double sm[];
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  double* sQ = sm;
  double* sW = sm + (size_t)NS * nel;
  for (int64_t q = threadIdx.x; q < (int64_t)NS * nel; q += blockDim.x) sQ[q] = Qin[q];
  __syncthreads();
  for (int s = 0; s < n_steps; ++s) {
    for (int64_t e = threadIdx.x; e < nel; e += blockDim.x) predict_prefactored_elem<D, M>(g, sQ, sW, G, taps, ntaps, e, nel);
    __syncthreads();
    for (int64_t e = threadIdx.x; e < nel; e += blockDim.x) correct_elem<D, M, false>(g, dt, sQ, sW, sQ, t, e, nel);
    __syncthreads();
  }
  for (int64_t q = threadIdx.x; q < (int64_t)NS * nel; q += blockDim.x) Qout[q] = sQ[q];
}

static Taps make_taps(const int32_t* taps, int ntaps) {
  Taps tp;
  for (int t = 0; t < kMaxBlocks; ++t)
    for (int i = 0; i < 3; ++i) tp.off[t][i] = (t < ntaps) ? (int8_t)taps[3 * t + i] : 0;
  return tp;
}

template <int D, int M>
struct PrefactoredL {
  static int run(const DevGeom& g, const double* Q, double* W, const double* G, const int32_t* taps, int ntaps,
                 void* stream) {
    const Taps tp = make_taps(taps, ntaps);
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

template <int D, int M>
struct FusedFitsL {
  static int run(int64_t nel) {
    return (int64_t)(n_space(D, M) + n_spacetime(D, M)) * 8 * nel <= kFusedLdsBytes ? 1 : 0;
  }
};

int fused_fits(int d, int M, int64_t nel) { return dispatch_dm<FusedFitsL>(d, M, nel); }

template <int D, int M>
struct FusedL {
  static int run(const DevGeom& g, double dt, const double* Qin, double* Qout, const double* G, const int32_t* taps,
                 int ntaps, const DevTensors& t, int n_steps, void* stream) {
    const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
    const int64_t bytes = (int64_t)(n_space(D, M) + n_spacetime(D, M)) * 8 * nel;
    if (bytes > kFusedLdsBytes) return (int)hipErrorInvalidValue;
    static bool attr = [] {
      return hipFuncSetAttribute((const void*)fused_prefactored_kernel<D, M>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFusedLdsBytes) == hipSuccess;
    }();
    if (!attr && bytes > 64 * 1024) return (int)hipErrorInvalidValue;
    const Taps tp = make_taps(taps, ntaps);
    hipLaunchKernelGGL((fused_prefactored_kernel<D, M>), dim3(1), dim3(kFusedThreads), (size_t)bytes,
                       (hipStream_t)stream, g, dt, Qin, Qout, G, tp, ntaps, t, n_steps);
    return (int)hipGetLastError();
  }
};

int launch_fused_prefactored(int d, int M, const DevGeom& g, double dt, const double* Qin, double* Qout,
                             const double* G, const int32_t* taps, int ntaps, const DevTensors& t, int n_steps,
                             void* stream) {
  return dispatch_dm<FusedL>(d, M, g, dt, Qin, Qout, G, taps, ntaps, t, n_steps, stream);
}

// ---------------------------------------------------------------- tap-form updates (constant velocity)
// out_e = base_e + sum_t A_t in_{e + off_t}: the correction from the predictions (R = theta rows,
// C = theta_T columns) or the composed prediction + correction acting on the state directly
// (R = C = theta). Operators are uniform across threads (scalar loads).
template <int D, int R, int C>
__global__ __launch_bounds__(256) void tap_update_kernel(DevGeom g, const double* __restrict__ in,
                                                         const double* __restrict__ base, double* __restrict__ out,
                                                         const double* __restrict__ A, TapsN taps, int ntaps) {
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  const int64_t e = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (e >= nel) return;
  tap_update_elem<R, C>(g, in, base, out, A, taps, ntaps, e, nel);
}

template <int D, int M>
struct TapL {
  static int run(int kind, const DevGeom& g, const double* in, const double* base, double* out, const double* A,
                 const int32_t* taps, int ntaps, void* stream) {
    constexpr int NS = n_space(D, M), NT = n_spacetime(D, M);
    if (ntaps > kMaxTapUpdate) return (int)hipErrorInvalidValue;
    TapsN tp;
    for (int t = 0; t < kMaxTapUpdate; ++t)
      for (int i = 0; i < 3; ++i) tp.off[t][i] = (t < ntaps) ? (int8_t)taps[3 * t + i] : 0;
    const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
    if (kind == 0)
      hipLaunchKernelGGL((tap_update_kernel<D, NS, NT>), dim3(grid_for(nel, 256)), dim3(256), 0, (hipStream_t)stream,
                         g, in, base, out, A, tp, ntaps);
    else
      hipLaunchKernelGGL((tap_update_kernel<D, NS, NS>), dim3(grid_for(nel, 256)), dim3(256), 0, (hipStream_t)stream,
                         g, in, base, out, A, tp, ntaps);
    return (int)hipGetLastError();
  }
};

int launch_tap_update(int d, int M, int kind, const DevGeom& g, const double* in, const double* base, double* out,
                      const double* A, const int32_t* taps, int ntaps, void* stream) {
  return dispatch_dm<TapL>(d, M, kind, g, in, base, out, A, taps, ntaps, stream);
}

template <int D, int NS>
static int composite_ns(const DevGeom& g, const double* in, double* out, const double* A, const int32_t* taps,
                        int ntaps, void* stream) {
  if (ntaps > kMaxTapUpdate) return (int)hipErrorInvalidValue;
  TapsN tp;
  for (int t = 0; t < kMaxTapUpdate; ++t)
    for (int i = 0; i < 3; ++i) tp.off[t][i] = (t < ntaps) ? (int8_t)taps[3 * t + i] : 0;
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  hipLaunchKernelGGL((tap_update_kernel<D, NS, NS>), dim3(grid_for(nel, 256)), dim3(256), 0, (hipStream_t)stream, g,
                     in, in, out, A, tp, ntaps);
  return (int)hipGetLastError();
}

int launch_tap_composite_ns(int d, int ns, const DevGeom& g, const double* in, double* out, const double* A,
                            const int32_t* taps, int ntaps, void* stream) {
#define RIDG_TC(DD, NN) \
  if (d == DD && ns == NN) return composite_ns<DD, NN>(g, in, out, A, taps, ntaps, stream);
  RIDG_TC(1, 1) RIDG_TC(1, 2) RIDG_TC(1, 3) RIDG_TC(1, 4) RIDG_TC(1, 5) RIDG_TC(1, 6) RIDG_TC(1, 7) RIDG_TC(1, 8)
  RIDG_TC(1, 9) RIDG_TC(1, 10) RIDG_TC(1, 11) RIDG_TC(1, 12)
  RIDG_TC(2, 1) RIDG_TC(2, 4) RIDG_TC(2, 9) RIDG_TC(2, 16) RIDG_TC(2, 25)
#undef RIDG_TC
  return (int)hipErrorInvalidValue;
}

}  // namespace ridg

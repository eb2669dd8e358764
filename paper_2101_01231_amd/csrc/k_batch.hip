// Shared launches for serving: one prediction kernel and one correction kernel advance a step of
// several independent constant-velocity problems of the same dimension and order (the correction
// in the same tap form as a single problem's default step). Each problem is
// described by value in the kernel arguments (no device-side table to manage); a workgroup finds
// its problem from the block ranges. The per-element arithmetic is exactly that of the
// single-problem kernels, so a problem's result does not depend on what it is batched with.
#include "kernels_common.hpp"

namespace ridg {

template <int D, int M>
__global__ __launch_bounds__(256) void batch_predict_kernel(BatchArgs args) {
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  int r = 0;
  for (int q = 1; q < args.count; ++q)
    if (blk >= args.d[q].block_begin) r = q;
  const BatchDesc& bd = args.d[r];
  const int64_t e = (blk - bd.block_begin) * 256 + threadIdx.x;
  if (e >= bd.nel) return;
  DevGeom g{};
  g.d = D;
  g.n0 = bd.n[0];
  g.n1 = bd.n[1];
  g.n2 = bd.n[2];
  g.h0 = bd.h[0];
  g.h1 = bd.h[1];
  g.h2 = bd.h[2];
  Taps tp;
#pragma unroll
  for (int t = 0; t < kBatchTaps; ++t)
#pragma unroll
    for (int i = 0; i < 3; ++i) tp.off[t][i] = bd.taps[t][i];
  predict_prefactored_elem<D, M>(g, bd.Qin, bd.W, bd.G, tp, bd.ntaps, e, bd.nel);
}

struct BatchTaps {
  int8_t off[7][3];
};

template <int D, int M>
__global__ __launch_bounds__(256) void batch_correct_kernel(BatchArgs args) {
  constexpr int NS = n_space(D, M), NT = n_spacetime(D, M);
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  int r = 0;
  for (int q = 1; q < args.count; ++q)
    if (blk >= args.d[q].block_begin) r = q;
  const BatchDesc& bd = args.d[r];
  const int64_t e = (blk - bd.block_begin) * 256 + threadIdx.x;
  if (e >= bd.nel) return;
  DevGeom g{};
  g.d = D;
  g.n0 = bd.n[0];
  g.n1 = bd.n[1];
  g.n2 = bd.n[2];
  BatchTaps tp;
#pragma unroll
  for (int t = 0; t < 7; ++t)
#pragma unroll
    for (int i = 0; i < 3; ++i) tp.off[t][i] = bd.dtaps[t][i];
  tap_update_elem<NS, NT>(g, bd.W, bd.Qin, bd.Qout, bd.Dc, tp, bd.ndtaps, e, bd.nel);
}

template <int D, int M>
struct BatchL {
  static int run(const BatchArgs& a, const DevTensors& t, void* stream) {
    if (a.count <= 0) return 0;
    const int64_t blocks = a.d[a.count - 1].block_begin + (a.d[a.count - 1].nel + 255) / 256;
    hipLaunchKernelGGL((batch_predict_kernel<D, M>), dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a);
    int err = (int)hipGetLastError();
    if (err) return err;
    (void)t;
    hipLaunchKernelGGL((batch_correct_kernel<D, M>), dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a);
    return (int)hipGetLastError();
  }
};

int launch_batch_step(int d, int M, const BatchArgs& args, const DevTensors& t, void* stream) {
  return dispatch_dm<BatchL>(d, M, args, t, stream);
}

}  // namespace ridg

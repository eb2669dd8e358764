// Temporal blocking of the 2D composite constant-velocity step (prediction and correction composed
// into taps K_o acting on the state, Sec. 2.2-2.3): Q'_e = Q_e + sum_o K_o Q_{e+o}, kTBlockSteps steps
// per launch.
//
// One workgroup owns a 16 x 16 tile. The state after s more steps at the tile depends on the state
// over the tile grown by s times the taps' reach on each side, so the workgroup loads that region
// (all theta coefficients) into LDS once and advances it step by step between two LDS buffers, each
// step on a region one reach smaller, until only the tile is left, which it writes back. No grid-wide
// synchronisation is needed; the price is the recomputed margin (at 16 x 16 and four steps of reach
// 2, 1.4x the tile's arithmetic). The taps, the operator entries and the order of every fused
// multiply-add are those of the one-step composite kernel, so the results are identical to four of
// its launches.
#include "kernels_common.hpp"
#include "k_tblock.hpp"

namespace ridg {

namespace {
constexpr int kTT = 16;                       // tile edge
constexpr int kTMaxTaps = 9;                  // a 3 x 3 window of offsets
constexpr int kTRegion = kTT + 2 * kTBlockSteps;  // region edge bound (reach <= 2 per step)
// Two wavefronts per SIMD with one tile per CU. Measured per step on the 256^2 order-3 workload:
// 4.99 us at 256 threads, 3.75 at 512, 3.63 at 1024; eight steps per launch (a 32 x 32 region)
// 5.28 us at 512 threads; one launch per step 6.6 us.
constexpr int kTThreads = 512;

struct TBlockTaps {
  int8_t off[kTMaxTaps][2];
  int8_t lo[2], hi[2];
};
}  // namespace

template <int NS>
__global__ __launch_bounds__(kTThreads) void tap_tblock_kernel(DevGeom g, const double* __restrict__ in,
                                                         double* __restrict__ out, const double* __restrict__ A,
                                                         TBlockTaps tb, int ntaps) {
  constexpr int PL = kTRegion * kTRegion;  // LDS plane of one coefficient
  __shared__ double buf[2][NS * PL];
  const int sx = kTT + kTBlockSteps * (tb.hi[0] - tb.lo[0]), sy = kTT + kTBlockSteps * (tb.hi[1] - tb.lo[1]);
  const int ntx = g.n0 / kTT;
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);
  const int x0 = (int)(b % ntx) * kTT, y0 = (int)(b / ntx) * kTT;
  const int rx0 = x0 + kTBlockSteps * tb.lo[0], ry0 = y0 + kTBlockSteps * tb.lo[1];  // region origin
  const int64_t nel = (int64_t)g.n0 * g.n1;
  for (int i = threadIdx.x; i < NS * sx * sy; i += kTThreads) {
    const int l = i / (sx * sy), rr = i - l * (sx * sy), yy = rr / sx, xx = rr - yy * sx;
    buf[0][l * PL + yy * sx + xx] = in[(int64_t)l * nel + elem_lin(g, rx0 + xx, ry0 + yy, 0)];
  }
  __syncthreads();
  for (int s = 1; s <= kTBlockSteps; ++s) {
    const double* src = buf[(s - 1) & 1];
    double* dst = buf[s & 1];
    // step s produces region coordinates [ax, bx) x [ay, by): its taps read step s - 1's region
    const int ax = -s * tb.lo[0], bx = sx - s * tb.hi[0], ay = -s * tb.lo[1], by = sy - s * tb.hi[1];
    const int wx = bx - ax, cnt = wx * (by - ay);
    for (int i = threadIdx.x; i < cnt; i += kTThreads) {
      const int yr = ay + i / wx, xr = ax + i % wx;
      double acc[NS];
#pragma unroll
      for (int k = 0; k < NS; ++k) acc[k] = 0.0;
      for (int t = 0; t < ntaps; ++t) {
        const int idx = (yr + tb.off[t][1]) * sx + (xr + tb.off[t][0]);
        double x[NS];
#pragma unroll
        for (int l = 0; l < NS; ++l) x[l] = src[l * PL + idx];
        const double* At = A + (size_t)t * NS * NS;
#pragma unroll
        for (int k = 0; k < NS; ++k)
#pragma unroll
          for (int l = 0; l < NS; ++l) acc[k] = fma(At[k * NS + l], x[l], acc[k]);
      }
      const int me = yr * sx + xr;
#pragma unroll
      for (int k = 0; k < NS; ++k) dst[k * PL + me] = src[k * PL + me] + acc[k];
    }
    __syncthreads();
  }
  const double* fin = buf[kTBlockSteps & 1];
  const int fx = -kTBlockSteps * tb.lo[0], fy = -kTBlockSteps * tb.lo[1];
  for (int i = threadIdx.x; i < NS * kTT * kTT; i += kTThreads) {
    const int l = i / (kTT * kTT), rr = i - l * (kTT * kTT), yy = rr / kTT, xx = rr - yy * kTT;
    out[(int64_t)l * nel + (int64_t)(x0 + xx) + (int64_t)g.n0 * (y0 + yy)] = fin[l * PL + (fy + yy) * sx + fx + xx];
  }
}

bool tblock_shape_supported(int d, int ns, int n0, int n1) {
  return d == 2 && (ns == 1 || ns == 3 || ns == 6 || ns == 10 || ns == 15) && n0 % kTT == 0 && n1 % kTT == 0;
}

bool tblock_taps_supported(const int32_t* taps, int ntaps) {
  if (ntaps < 1 || ntaps > kTMaxTaps) return false;
  for (int i = 0; i < 2; ++i) {
    int lo = 0, hi = 0;
    for (int t = 0; t < ntaps; ++t) {
      lo = taps[3 * t + i] < lo ? taps[3 * t + i] : lo;
      hi = taps[3 * t + i] > hi ? taps[3 * t + i] : hi;
    }
    if (hi - lo > 2) return false;
  }
  for (int t = 0; t < ntaps; ++t)
    if (taps[3 * t + 2] != 0) return false;
  return true;
}

template <int NS>
static int tblock_ns(const DevGeom& g, const double* in, double* out, const double* A, const int32_t* taps, int ntaps,
                     void* stream) {
  TBlockTaps tb{};
  for (int t = 0; t < ntaps; ++t)
    for (int i = 0; i < 2; ++i) tb.off[t][i] = (int8_t)taps[3 * t + i];
  for (int i = 0; i < 2; ++i) {
    int lo = 0, hi = 0;
    for (int t = 0; t < ntaps; ++t) {
      lo = taps[3 * t + i] < lo ? taps[3 * t + i] : lo;
      hi = taps[3 * t + i] > hi ? taps[3 * t + i] : hi;
    }
    tb.lo[i] = (int8_t)lo;
    tb.hi[i] = (int8_t)hi;
  }
  const int64_t blocks = (int64_t)(g.n0 / kTT) * (g.n1 / kTT);
  hipLaunchKernelGGL((tap_tblock_kernel<NS>), dim3((unsigned)blocks), dim3(kTThreads), 0, (hipStream_t)stream, g, in, out, A,
                     tb, ntaps);
  return (int)hipGetLastError();
}

int launch_tap_tblock(int ns, const DevGeom& g, const double* in, double* out, const double* A, const int32_t* taps,
                      int ntaps, void* stream) {
  if (!tblock_shape_supported(g.d, ns, g.n0, g.n1) || !tblock_taps_supported(taps, ntaps) || in == out)
    return (int)hipErrorInvalidValue;
  switch (ns) {
    case 1: return tblock_ns<1>(g, in, out, A, taps, ntaps, stream);
    case 3: return tblock_ns<3>(g, in, out, A, taps, ntaps, stream);
    case 6: return tblock_ns<6>(g, in, out, A, taps, ntaps, stream);
    case 10: return tblock_ns<10>(g, in, out, A, taps, ntaps, stream);
    case 15: return tblock_ns<15>(g, in, out, A, taps, ntaps, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

}  // namespace ridg

// Composite constant-velocity step in 3D (prediction and correction composed into taps K_o acting on
// the state, Sec. 2.2-2.3): Q'_e = Q_e + sum_o K_o Q_{e+o}, marched along z.
//
// One workgroup of 16 x 16 threads owns a 16 x 16 column of the mesh over tz planes. The taps span at
// most three z-planes; a ring of three state planes (the 16 x 16 tile plus the x/y halo of the taps,
// all theta coefficients) lives in LDS, and each step of the march loads one new plane from HBM, so
// every state value is fetched about (16 + halo)^2 / 16^2 x (tz + 2) / tz times instead of once per
// tap. Each thread then applies all taps to its element from LDS; the operator K (wave-uniform) comes
// through scalar loads.
#include "kernels_common.hpp"
#include "k_stencil3d.hpp"

namespace ridg {

namespace {
constexpr int kZT = 16;       // tile edge in x and y
constexpr int kZRing = 3;     // planes held (the taps' z-span is at most 3)
constexpr int kZBatch = 8;    // plane loads in flight per thread
}  // namespace

template <int NS>
__global__ __launch_bounds__(kZT* kZT) void tap_zmarch_kernel(DevGeom g, const double* __restrict__ in,
                                                             double* __restrict__ out, const double* __restrict__ A,
                                                             TapsN taps, int ntaps, ZMarch zm) {
  __shared__ double ring[kZRing * NS * (kZT + 2) * (kZT + 2)];  // [kZRing][NS][sy][sx], sx, sy <= kZT + 2
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  const int sx = kZT + zm.hi[0] - zm.lo[0], sy = kZT + zm.hi[1] - zm.lo[1], pl = sx * sy;
  const int ntx = g.n0 / kZT, nty = g.n1 / kZT;
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);
  const int x0 = (int)(b % ntx) * kZT, y0 = (int)((b / ntx) % nty) * kZT, z0 = (int)(b / ((int64_t)ntx * nty)) * zm.tz;
  const int tx = threadIdx.x % kZT, ty = threadIdx.x / kZT;
  // plane of relative index r (absolute z0 + lo_z + r) into ring slot r % kZRing
  auto load_plane = [&](int r) {
    double* dst = ring + (size_t)(r % kZRing) * NS * pl;
    const int z = z0 + zm.lo[2] + r;
    const int total = NS * pl;
    for (int i0 = threadIdx.x; i0 < total; i0 += kZT * kZT * kZBatch) {
      double v[kZBatch];
#pragma unroll
      for (int u = 0; u < kZBatch; ++u) {
        const int i = i0 + u * kZT * kZT;
        const int ic = i < total ? i : 0;
        const int l = ic / pl, rr = ic - l * pl, yy = rr / sx, xx = rr - yy * sx;
        v[u] = in[(int64_t)l * nel + elem_lin(g, x0 + zm.lo[0] + xx, y0 + zm.lo[1] + yy, z)];
      }
#pragma unroll
      for (int u = 0; u < kZBatch; ++u) {
        const int i = i0 + u * kZT * kZT;
        if (i < total) dst[i] = v[u];
      }
    }
  };
  const int zspan = zm.hi[2] - zm.lo[2];
  for (int r = 0; r < zspan; ++r) load_plane(r);
  for (int z = 0; z < zm.tz; ++z) {
    load_plane(z + zspan);
    __syncthreads();
    double acc[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] = 0.0;
    for (int t = 0; t < ntaps; ++t) {
      const int slot = (z + taps.off[t][2] - zm.lo[2]) % kZRing;
      const int idx = (ty + taps.off[t][1] - zm.lo[1]) * sx + (tx + taps.off[t][0] - zm.lo[0]);
      const double* src = ring + (size_t)slot * NS * pl + idx;
      double q[NS];
#pragma unroll
      for (int l = 0; l < NS; ++l) q[l] = src[l * pl];
      const double* At = A + (size_t)t * NS * NS;
#pragma unroll
      for (int k = 0; k < NS; ++k)
#pragma unroll
        for (int l = 0; l < NS; ++l) acc[k] = fma(At[k * NS + l], q[l], acc[k]);
    }
    const int slot0 = (z - zm.lo[2]) % kZRing;
    const double* own = ring + (size_t)slot0 * NS * pl + (ty - zm.lo[1]) * sx + (tx - zm.lo[0]);
    const int64_t e = (int64_t)(x0 + tx) + (int64_t)g.n0 * ((int64_t)(y0 + ty) + (int64_t)g.n1 * (z0 + z));
#pragma unroll
    for (int k = 0; k < NS; ++k) out[(int64_t)k * nel + e] = own[k * pl] + acc[k];
    __syncthreads();  // every thread is done with the oldest plane before it is overwritten
  }
}

template <int NS>
static int zmarch_ns(const DevGeom& g, const double* in, double* out, const double* A, const int32_t* taps,
                     int ntaps, void* stream) {
  if (ntaps < 1 || ntaps > kMaxTapUpdate) return (int)hipErrorInvalidValue;
  TapsN tp;
  ZMarch zm{};
  for (int t = 0; t < kMaxTapUpdate; ++t)
    for (int i = 0; i < 3; ++i) tp.off[t][i] = (t < ntaps) ? (int8_t)taps[3 * t + i] : 0;
  for (int i = 0; i < 3; ++i) {
    int lo = 0, hi = 0;
    for (int t = 0; t < ntaps; ++t) {
      lo = taps[3 * t + i] < lo ? taps[3 * t + i] : lo;
      hi = taps[3 * t + i] > hi ? taps[3 * t + i] : hi;
    }
    if (hi - lo > kZRing - 1) return (int)hipErrorInvalidValue;  // the ring and the halos assume a span <= 2
    zm.lo[i] = (int8_t)lo;
    zm.hi[i] = (int8_t)hi;
  }
  if (!zmarch_supported(g.d, NS, g.n0, g.n1, g.n2)) return (int)hipErrorInvalidValue;
  zm.tz = (g.n2 % 8 == 0) ? 8 : g.n2;
  const int64_t blocks = (int64_t)(g.n0 / kZT) * (g.n1 / kZT) * (g.n2 / zm.tz);
  hipLaunchKernelGGL((tap_zmarch_kernel<NS>), dim3((unsigned)blocks), dim3(kZT * kZT), 0, (hipStream_t)stream, g,
                     in, out, A, tp, ntaps, zm);
  return (int)hipGetLastError();
}

// The one-element-per-thread composite step for two z-neighbours (x, y, 2 z2) and (x, y, 2 z2 + 1)
// per thread. The taps come in column order (same (x, y) offset, increasing z), so the value that the
// upper element reads for tap (ox, oy, oz) is the one the lower element needs for the column's next
// tap (ox, oy, oz + 1): it is kept instead of loaded again, and a column of three taps costs four
// loads of the theta coefficients instead of six. (At 128^3, order 3, the one-element kernel keeps
// the texture-address unit busy 91% of the time and the VALU 55%.) Each element sums its taps in list
// order with tap_update_elem's fused multiply-adds, so the result is bitwise the same.
//
// Where n1 is a multiple of 8 and a band of n1 / 8 rows holds whole workgroups (`banded`), the
// workgroups of each XCD (workgroup b runs on XCD b % 8) take one such band in y, band-plane after
// band-plane along z, so the neighbours they read one and two planes back are more often still in
// that XCD's L2: at 128^3, order 3, 1.52 against 1.78 GB fetched per launch and 0.273 against 0.285
// ms; otherwise consecutive pairs of planes are spread over the XCDs in contiguous ranges.
template <int NS>
__global__ __launch_bounds__(256) void tap_z2_kernel(DevGeom g, const double* __restrict__ in,
                                                     double* __restrict__ out, const double* __restrict__ A,
                                                     TapsN taps, int ntaps, int banded) {
  const int64_t plane = (int64_t)g.n0 * g.n1, nel = plane * g.n2;
  int64_t e0;
  if (banded) {
    const int band = g.n1 / 8;
    const int64_t per_plane = (int64_t)g.n0 * band / 256;  // workgroups per band-plane
    const int xcd = (int)(blockIdx.x % 8);
    const int64_t j = blockIdx.x / 8;
    const int64_t zp = j / per_plane, r = j - zp * per_plane;
    const int64_t local = r * 256 + threadIdx.x;
    const int x = (int)(local % g.n0), y = xcd * band + (int)(local / g.n0);
    e0 = (int64_t)x + (int64_t)g.n0 * ((int64_t)y + (int64_t)g.n1 * (2 * zp));
  } else {
    const int64_t p = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (p >= nel / 2) return;
    e0 = p % plane + 2 * plane * (p / plane);
  }
  const int64_t e1 = e0 + plane;
  int idx[3];
  elem_idx(g, e0, idx);
  double acc0[NS], acc1[NS], up[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) acc0[k] = acc1[k] = up[k] = 0.0;
  int px = 0, py = 0, pz = 0;
  bool have = false;  // `up` holds the value at (px, py, pz + 1)
  for (int t = 0; t < ntaps; ++t) {
    const int ox = taps.off[t][0], oy = taps.off[t][1], oz = taps.off[t][2];
    double x0[NS];
    if (have && ox == px && oy == py && oz == pz + 1) {
#pragma unroll
      for (int l = 0; l < NS; ++l) x0[l] = up[l];
    } else {
      const int64_t s0 = elem_lin(g, idx[0] + ox, idx[1] + oy, idx[2] + oz);
#pragma unroll
      for (int l = 0; l < NS; ++l) x0[l] = in[(int64_t)l * nel + s0];
    }
    const int64_t s1 = elem_lin(g, idx[0] + ox, idx[1] + oy, idx[2] + oz + 1);
#pragma unroll
    for (int l = 0; l < NS; ++l) up[l] = in[(int64_t)l * nel + s1];
    px = ox;
    py = oy;
    pz = oz;
    have = true;
    const double* At = A + (size_t)t * NS * NS;
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
      for (int l = 0; l < NS; ++l) {
        const double a = At[k * NS + l];
        acc0[k] = fma(a, x0[l], acc0[k]);
        acc1[k] = fma(a, up[l], acc1[k]);
      }
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    out[(int64_t)k * nel + e0] = in[(int64_t)k * nel + e0] + acc0[k];
    out[(int64_t)k * nel + e1] = in[(int64_t)k * nel + e1] + acc1[k];
  }
}

bool z2_supported(int d, int ns, int n2) {
  return d == 3 && n2 % 2 == 0 && (ns == 1 || ns == 4 || ns == 10);  // order 4 and up: 168+ VGPRs
}

template <int NS>
static int z2_ns(const DevGeom& g, const double* in, double* out, const double* A, const int32_t* taps, int ntaps,
                 void* stream) {
  if (ntaps < 1 || ntaps > kMaxTapUpdate || in == out) return (int)hipErrorInvalidValue;
  TapsN tp;
  for (int t = 0; t < kMaxTapUpdate; ++t)
    for (int i = 0; i < 3; ++i) tp.off[t][i] = (t < ntaps) ? (int8_t)taps[3 * t + i] : 0;
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  // bands: whole workgroups per band-plane, and the grid (nel / 512 workgroups) a multiple of 8
  const int banded = g.n1 % 8 == 0 && ((int64_t)g.n0 * (g.n1 / 8)) % 256 == 0 ? 1 : 0;
  hipLaunchKernelGGL((tap_z2_kernel<NS>), dim3(grid_for(nel / 2, 256)), dim3(256), 0, (hipStream_t)stream, g, in, out,
                     A, tp, ntaps, banded);
  return (int)hipGetLastError();
}

int launch_tap_z2(int ns, const DevGeom& g, const double* in, double* out, const double* A, const int32_t* taps,
                  int ntaps, void* stream) {
  if (!z2_supported(g.d, ns, g.n2)) return (int)hipErrorInvalidValue;
  switch (ns) {
    case 1: return z2_ns<1>(g, in, out, A, taps, ntaps, stream);
    case 4: return z2_ns<4>(g, in, out, A, taps, ntaps, stream);
    case 10: return z2_ns<10>(g, in, out, A, taps, ntaps, stream);
    default: return (int)hipErrorInvalidValue;
  }
}

bool zmarch_supported(int d, int ns, int n0, int n1, int n2) {
  return d == 3 && (ns == 4 || ns == 10) && n0 % kZT == 0 && n1 % kZT == 0 && (n2 % 8 == 0 || n2 <= 64);
}

int launch_tap_zmarch(int ns, const DevGeom& g, const double* in, double* out, const double* A, const int32_t* taps,
                      int ntaps, void* stream) {
  if (ns == 4) return zmarch_ns<4>(g, in, out, A, taps, ntaps, stream);
  if (ns == 10) return zmarch_ns<10>(g, in, out, A, taps, ntaps, stream);
  return (int)hipErrorInvalidValue;
}

}  // namespace ridg

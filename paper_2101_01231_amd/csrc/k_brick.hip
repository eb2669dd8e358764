// Fused constant-velocity step on bricks of a 3D mesh (Sec. 2.2 prediction, Sec. 2.3 correction):
//
//   W_f = sum_s G_s Q_{f+s}          (prediction, G = E_c A^-1 C from the host FP64 factorisation)
//   Q'_e = Q_e + sum_t D_t W_{e+t}    (correction taps: own element and inflow faces)
//
// One workgroup owns a brick of 16 x BY x BZ elements. It stages the state of the brick and of its
// upwind neighbourhood in LDS (each state read from HBM about once), computes the predictions of the
// brick and of the one-element upwind halo its correction reads as stacked-right-hand-side products
// on the matrix cores, keeps them in LDS, then applies the correction in FP64. The products run in
// FP64 (v_mfma_f64_16x16x4f64) or, for the reduced-precision path, with FP32 operands and FP32
// accumulation (v_mfma_f32_16x16x4f32); the correction, and with it the flux-form update that
// conserves the element averages, is FP64 in both.
//
// Matrix-core lane layouts (16x16x4, A 16x4, B 4x16, D 16x16): lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; the FP64 result register r of lane l is D[4 r + l / 16][l % 16], the FP32 one
// D[4 (l / 16) + r][l % 16].
#include "kernels_common.hpp"

namespace ridg {

typedef float brick_v4f __attribute__((ext_vector_type(4)));
typedef double brick_v4d __attribute__((ext_vector_type(4)));

template <class T>
struct BrickMfma;
template <>
struct BrickMfma<double> {
  using V = brick_v4d;
  static __device__ __forceinline__ V step(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int kq) { return 4 * r + kq; }
};
template <>
struct BrickMfma<float> {
  using V = brick_v4f;
  static __device__ __forceinline__ V step(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int r, int kq) { return 4 * kq + r; }
};

// FP64 stages bricks of 16 x 4 x 2 (LDS 65 KB at order 3), FP32 bricks of 16 x 4 x 4 (51 KB).
template <class T>
constexpr int kBrickZ = std::is_same<T, double>::value ? 2 : 4;
template <class T>
constexpr int kBrickThreads = 16 * 4 * kBrickZ<T>;  // one output element per thread in the correction

constexpr int kBrickBatch = 8;  // state reads in flight per thread while staging

template <int M, class T>
struct BrickCfg {
  static constexpr int NS = n_space(3, M), NT = n_spacetime(3, M);
  static constexpr int BX = 16, BY = 4, BZ = kBrickZ<T>;
  static constexpr int THREADS = kBrickThreads<T>;
  static constexpr int WAVES = THREADS / 64;
  static constexpr int CQ = (NS + 3) / 4;        // K chunks of 4 state coefficients per tap
  static constexpr int QXM = BX + 2, QYM = BY + 2, QZM = BZ + 2;  // largest Q region (halo 2 per axis)
  static constexpr int WXM = BX + 1, WYM = BY + 1, WZM = BZ + 1;  // largest W region (halo 1 per axis)
  static constexpr int NQ = QXM * QYM * QZM, NW = WXM * WYM * WZM;
  static constexpr size_t LDS = sizeof(T) * ((size_t)NS * NQ + (size_t)NT * NW);
  static_assert(NT <= 16, "one 16-row tile of the prediction operator");
};

template <int M, class T>
__global__ __launch_bounds__(kBrickThreads<T>) void brick_step_kernel(DevGeom g, const double* __restrict__ Q,
                                                                            double* __restrict__ Qout,
                                                                            const T* __restrict__ gfrag,
                                                                            const double* __restrict__ Dc,
                                                                            BrickTaps tp) {
  using C = BrickCfg<M, T>;
  using MF = BrickMfma<T>;
  constexpr int NS = C::NS, NT = C::NT, CQ = C::CQ, BX = C::BX, BY = C::BY, BZ = C::BZ;
  __shared__ T sQ[NS][C::NQ];
  __shared__ T sW[NT][C::NW];
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  const int nbx = g.n0 / BX, nby = g.n1 / BY;
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);
  const int x0 = (int)(b % nbx) * BX, y0 = (int)((b / nbx) % nby) * BY, z0 = (int)(b / ((int64_t)nbx * nby)) * BZ;
  // regions: W = brick + [wlo, whi] per axis (the correction taps), Q = W region + the prediction taps
  const int QX = BX + tp.qhi[0] - tp.qlo[0], QY = BY + tp.qhi[1] - tp.qlo[1], QZ = BZ + tp.qhi[2] - tp.qlo[2];
  const int WX = BX + tp.whi[0] - tp.wlo[0], WY = BY + tp.whi[1] - tp.wlo[1], WZ = BZ + tp.whi[2] - tp.wlo[2];
  const int nq = QX * QY * QZ, nw = WX * WY * WZ;
  // this thread's output element and its state (the base of the correction), requested first
  const int ox = threadIdx.x % BX, oy = (threadIdx.x / BX) % BY, oz = threadIdx.x / (BX * BY);
  const int64_t e = (int64_t)(x0 + ox) + (int64_t)g.n0 * ((int64_t)(y0 + oy) + (int64_t)g.n1 * (z0 + oz));
  double qe[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) qe[k] = Q[(int64_t)k * nel + e];
  // 1. the state of the Q region into LDS (x fastest: consecutive threads read consecutive elements),
  // kBrickBatch independent reads in flight per thread
  for (int i0 = threadIdx.x; i0 < NS * nq; i0 += C::THREADS * kBrickBatch) {
    T v[kBrickBatch];
#pragma unroll
    for (int u = 0; u < kBrickBatch; ++u) {
      const int i = i0 + u * C::THREADS;
      const int ic = i < NS * nq ? i : 0;
      const int c = ic / nq, r = ic - c * nq;
      const int qx = r % QX, qy = (r / QX) % QY, qz = r / (QX * QY);
      v[u] = (T)Q[(int64_t)c * nel + elem_lin(g, x0 + tp.qlo[0] + qx, y0 + tp.qlo[1] + qy, z0 + tp.qlo[2] + qz)];
    }
#pragma unroll
    for (int u = 0; u < kBrickBatch; ++u) {
      const int i = i0 + u * C::THREADS;
      if (i < NS * nq) sQ[i / nq][i % nq] = v[u];
    }
  }
  // the operator's A fragments stay in registers
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kq = lane >> 4;
  T af[8][CQ];
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int q = 0; q < CQ; ++q) af[t][q] = t < tp.ng ? gfrag[((size_t)t * CQ + q) * 64 + lane] : (T)0;
  __syncthreads();
  // 2. predictions of the W region, 16 elements per matrix-core tile
  const int ntiles = (nw + 15) / 16;
  for (int tile = wave; tile < ntiles; tile += C::WAVES) {
    const int ew = tile * 16 + col;
    const bool valid = ew < nw;
    const int ec = valid ? ew : 0;  // columns past the region compute element 0 again and are dropped
    const int wx = ec % WX, wy = (ec / WX) % WY, wz = ec / (WX * WY);
    const int bx = wx + tp.wlo[0] - tp.qlo[0], by = wy + tp.wlo[1] - tp.qlo[1], bz = wz + tp.wlo[2] - tp.qlo[2];
    typename MF::V acc = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if (t >= tp.ng) break;
      const int r = (bx + tp.g[t][0]) + QX * ((by + tp.g[t][1]) + QY * (bz + tp.g[t][2]));
#pragma unroll
      for (int q = 0; q < CQ; ++q) {
        const int c = 4 * q + kq;
        const T bv = c < NS ? sQ[c < NS ? c : 0][r] : (T)0;
        acc = MF::step(af[t][q], bv, acc);
      }
    }
    if (valid) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = MF::row(i, kq);
        if (row < NT) sW[row][ew] = acc[i];
      }
    }
  }
  __syncthreads();
  // 3. FP64 correction, one output element per thread (taps uniform: scalar loads of D)
  double acc[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) acc[k] = 0.0;
  for (int t = 0; t < tp.nd; ++t) {
    const int r = (ox - tp.wlo[0] + tp.d[t][0]) + WX * ((oy - tp.wlo[1] + tp.d[t][1]) + WY * (oz - tp.wlo[2] + tp.d[t][2]));
    double w[NT];
#pragma unroll
    for (int l = 0; l < NT; ++l) w[l] = (double)sW[l][r];
    const double* Dt = Dc + (size_t)t * NS * NT;
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
      for (int l = 0; l < NT; ++l) acc[k] = fma(Dt[k * NT + l], w[l], acc[k]);
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) Qout[(int64_t)k * nel + e] = qe[k] + acc[k];
}

template <int M>
struct BrickL {
  template <class T>
  static int go(const DevGeom& g, const double* Q, double* Qout, const void* frag, const double* Dc,
                const BrickTaps& tp, void* stream) {
    using C = BrickCfg<M, T>;
    if (g.n0 % C::BX || g.n1 % C::BY || g.n2 % C::BZ) return (int)hipErrorInvalidValue;
    const int64_t blocks = (int64_t)(g.n0 / C::BX) * (g.n1 / C::BY) * (g.n2 / C::BZ);
    hipLaunchKernelGGL((brick_step_kernel<M, T>), dim3((unsigned)blocks), dim3(C::THREADS), 0, (hipStream_t)stream, g,
                       Q, Qout, (const T*)frag, Dc, tp);
    return (int)hipGetLastError();
  }
};

bool brick_supported(int d, int M, const int n[3], bool f32) {
  if (d != 3 || (M != 2 && M != 3)) return false;
  const int bz = f32 ? BrickCfg<3, float>::BZ : BrickCfg<3, double>::BZ;
  return n[0] % 16 == 0 && n[1] % 4 == 0 && n[2] % bz == 0;
}

int launch_brick_step(int M, bool f32, const DevGeom& g, const double* Q, double* Qout, const void* frag,
                      const double* Dc, const BrickTaps& tp, void* stream) {
  if (tp.ng < 1 || tp.ng > 8 || tp.nd < 1 || tp.nd > 4) return (int)hipErrorInvalidValue;
  for (int i = 0; i < 3; ++i)  // the halos the shared-memory regions are sized for
    if (tp.wlo[i] < -1 || tp.whi[i] > 1 || tp.qlo[i] < -2 || tp.qhi[i] > 2 || tp.qhi[i] - tp.qlo[i] > 2 ||
        tp.whi[i] - tp.wlo[i] > 1)
      return (int)hipErrorInvalidValue;
  if (M == 2) return f32 ? BrickL<2>::go<float>(g, Q, Qout, frag, Dc, tp, stream)
                         : BrickL<2>::go<double>(g, Q, Qout, frag, Dc, tp, stream);
  if (M == 3) return f32 ? BrickL<3>::go<float>(g, Q, Qout, frag, Dc, tp, stream)
                         : BrickL<3>::go<double>(g, Q, Qout, frag, Dc, tp, stream);
  return (int)hipErrorInvalidValue;
}

}  // namespace ridg

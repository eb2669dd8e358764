// Constant-velocity tap operators on the matrix cores (FP64 MFMA): the prefactored prediction
// W = sum_s G_s Q_{e+s} (Sec. 2.2), the correction Q' = Q + sum_t D_t W_{e+t} (Sec. 2.3) and their
// composition are one stacked-right-hand-side product each,
//
//   out[R x N] = base + [A_0 | A_1 | ... ] (R x ntaps*C) . [in_{e+off_0} ; in_{e+off_1} ; ...] (ntaps*C x N),
//
// with N the elements. A wavefront computes a 16-element column tile with v_mfma_f64_16x16x4f64:
// rows of A in 16-row tiles, K in chunks of 4 columns of one tap (C padded to a multiple of 4 per
// tap, so a chunk never straddles two taps and each lane needs one neighbour index per tap).
//
// Lane layout of v_mfma_f64_16x16x4f64 (A 16x4, B 4x16, D 16x16): lane l holds A[l % 16][l / 16],
// B[l / 16][l % 16] and D[4 r + l / 16][l % 16] in its r-th result register, r = 0..3.
//
// The A fragments are precomputed on the host in exactly that order ([row tile][tap][chunk][lane])
// and staged once per workgroup in LDS (read through the caches when they exceed it); each
// workgroup then sweeps a contiguous range of tiles,
// so consecutive workgroups (spread over the XCDs) work on distant parts of the mesh while the
// taps of one workgroup's tiles stay close in its XCD's L2.
#include "kernels_common.hpp"

namespace ridg {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kMfmaWaves = 8;

// One wavefront: column tiles tile = t_begin + first, t_begin + first + stride, ... < t_end of the
// product out = base + sum_t A_t in_{e+off_t}; A fragments at fsrc (LDS or global).
template <int R, int C, class TAPS>
__device__ inline void mfma_tiles(const DevGeom& g, const double* __restrict__ in, const double* __restrict__ base,
                                  double* __restrict__ out, const double* fsrc, const TAPS& taps, int ntaps,
                                  int64_t t_begin, int64_t t_end, int first, int stride) {
  constexpr int MT = (R + 15) / 16;  // 16-row tiles of the operator
  constexpr int CQ = (C + 3) / 4;    // K chunks per tap
  const int lane = threadIdx.x & 63;
  const int kq = lane >> 4;  // K index within a chunk (B) / row group (D)
  const int col = lane & 15;
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  // rows of whole tiles (n0 a multiple of 16): a tile lies in one x-row, so the y and z parts of
  // every neighbour index are wave-uniform and only the x wrap is per lane
  const bool rows = g.n0 % 16 == 0;
  for (int64_t tile = t_begin + first; tile < t_end; tile += stride) {
    const int64_t e = tile * 16 + col;
    const bool valid = e < nel;
    int idx[3];
    elem_idx(g, valid ? e : nel - 1, idx);
    int yz[2] = {0, 0};  // uniform y, z of the tile (rows only)
    if (rows) {
      yz[0] = __builtin_amdgcn_readfirstlane(idx[1]);
      yz[1] = __builtin_amdgcn_readfirstlane(idx[2]);
    }
    v4d acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = v4d{0.0, 0.0, 0.0, 0.0};
    auto nbr = [&](int t) -> int64_t {
      if (rows) {
        const int64_t row = (int64_t)wrap(yz[0] + taps.off[t][1], g.n1) + (int64_t)g.n1 * wrap(yz[1] + taps.off[t][2], g.n2);
        return (int64_t)wrap(idx[0] + taps.off[t][0], g.n0) + (int64_t)g.n0 * row;
      }
      return (int64_t)wrap(idx[0] + taps.off[t][0], g.n0) +
             (int64_t)g.n0 * ((int64_t)wrap(idx[1] + taps.off[t][1], g.n1) + (int64_t)g.n1 * wrap(idx[2] + taps.off[t][2], g.n2));
    };
    // B operands of one tap: column 4 q + kq of the neighbour (columns past C meet zero rows of
    // A; the load index is clamped to stay inside `in`)
    auto load_b = [&](int t, double (&b)[CQ]) {
      const int64_t ne = nbr(t);
#pragma unroll
      for (int q = 0; q < CQ; ++q) {
        const int c = 4 * q + kq;
        b[q] = in[(int64_t)(c < C ? c : C - 1) * nel + ne];
      }
    };
    double b[CQ];
    load_b(0, b);
    for (int t = 0; t < ntaps; ++t) {
      double bn[CQ];  // the next tap's operands are requested before this tap's products
      const bool more = t + 1 < ntaps;
      if (more) load_b(t + 1, bn);
      const double* ft = fsrc + (size_t)t * CQ * 64 + lane;
#pragma unroll
      for (int q = 0; q < CQ; ++q) {
        const double bq = 4 * q + kq < C ? b[q] : 0.0;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          acc[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ft[((size_t)mt * ntaps * CQ + q) * 64], bq, acc[mt], 0, 0, 0);
      }
      if (more) {
#pragma unroll
        for (int q = 0; q < CQ; ++q) b[q] = bn[q];
      }
    }
    if (valid) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * mt + 4 * r + kq;
          if (row < R) {
            const int64_t o = (int64_t)row * nel + e;
            out[o] = base ? base[o] + acc[mt][r] : acc[mt][r];
          }
        }
    }
  }
}

template <int R, int C, bool LDS_FRAG>
__global__ __launch_bounds__(64 * kMfmaWaves) void tap_mfma_kernel(DevGeom g, const double* __restrict__ in,
                                                                   const double* __restrict__ base,
                                                                   double* __restrict__ out,
                                                                   const double* __restrict__ frag, TapsN taps,
                                                                   int ntaps, int64_t tiles_per_group) {
  constexpr int MT = (R + 15) / 16, CQ = (C + 3) / 4;
  extern __shared__ double s_frag[];  // [MT][ntaps][CQ][64]
  const double* fsrc = frag;           // operators too large for LDS are read through the caches
  if constexpr (LDS_FRAG) {
    const int nfrag = MT * ntaps * CQ * 64;
    for (int i = threadIdx.x; i < nfrag; i += blockDim.x) s_frag[i] = frag[i];
    __syncthreads();
    fsrc = s_frag;
  }
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  const int64_t ntiles = (nel + 15) / 16;
  const int64_t t_begin = xcd_block(blockIdx.x, gridDim.x) * tiles_per_group;
  const int64_t t_end = t_begin + tiles_per_group < ntiles ? t_begin + tiles_per_group : ntiles;
  mfma_tiles<R, C>(g, in, base, out, fsrc, taps, ntaps, t_begin, t_end, threadIdx.x >> 6, kMfmaWaves);
}

// Shared launch for several problems of one (dimension, order) family (serving): a workgroup finds
// its problem from the group ranges; per element the arithmetic is that of tap_mfma_kernel, so a
// problem's result does not depend on what it is batched with. Fragments are read through the caches.
template <int R, int C>
__global__ __launch_bounds__(64 * kMfmaWaves) void batch_mfma_kernel(BatchMfmaArgs args) {
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  int r = 0;
  for (int q = 1; q < args.count; ++q)
    if (blk >= args.d[q].group_begin) r = q;
  const BatchMfmaDesc& bd = args.d[r];
  DevGeom g{};
  g.n0 = bd.n[0];
  g.n1 = bd.n[1];
  g.n2 = bd.n[2];
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  const int64_t ntiles = (nel + 15) / 16;
  const int64_t t_begin = (blk - bd.group_begin) * bd.tiles_per_group;
  const int64_t t_end = t_begin + bd.tiles_per_group < ntiles ? t_begin + bd.tiles_per_group : ntiles;
  BatchMfmaTaps tp;
#pragma unroll
  for (int t = 0; t < kBatchTaps; ++t)
#pragma unroll
    for (int i = 0; i < 3; ++i) tp.off[t][i] = bd.taps[t][i];
  mfma_tiles<R, C>(g, bd.in, bd.base, bd.out, bd.frag, tp, bd.ntaps, t_begin, t_end, threadIdx.x >> 6, kMfmaWaves);
}

template <int R, int C>
static int launch_rc(const DevGeom& g, const double* in, const double* base, double* out, const double* frag,
                     const int32_t* taps, int ntaps, void* stream) {
  constexpr int MT = (R + 15) / 16, CQ = (C + 3) / 4;
  if (ntaps <= 0 || ntaps > kMaxTapUpdate) return (int)hipErrorInvalidValue;
  const size_t lds = (size_t)MT * ntaps * CQ * 64 * 8;
  static const bool attr = hipFuncSetAttribute((const void*)tap_mfma_kernel<R, C, true>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)kMfmaMaxLds) == hipSuccess;
  const bool in_lds = lds <= (attr ? kMfmaMaxLds : (size_t)64 * 1024);
  TapsN tp;
  for (int t = 0; t < kMaxTapUpdate; ++t)
    for (int i = 0; i < 3; ++i) tp.off[t][i] = (t < ntaps) ? (int8_t)taps[3 * t + i] : 0;
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  const int64_t ntiles = (nel + 15) / 16;
  // enough workgroups to fill the chip several times over; each sweeps a contiguous tile range
  const int64_t per = mfma_tiles_per_group(nel, in_lds ? lds : 0);
  const int64_t groups = (ntiles + per - 1) / per;
  if (in_lds)
    hipLaunchKernelGGL((tap_mfma_kernel<R, C, true>), dim3((unsigned)groups), dim3(64 * kMfmaWaves), lds,
                       (hipStream_t)stream, g, in, base, out, frag, tp, ntaps, per);
  else
    hipLaunchKernelGGL((tap_mfma_kernel<R, C, false>), dim3((unsigned)groups), dim3(64 * kMfmaWaves), 0,
                       (hipStream_t)stream, g, in, base, out, frag, tp, ntaps, per);
  return (int)hipGetLastError();
}

template <int D, int M>
struct MfmaL {
  static int run(int kind, const DevGeom& g, const double* in, const double* base, double* out, const double* frag,
                 const int32_t* taps, int ntaps, void* stream) {
    constexpr int NS = n_space(D, M), NT = n_spacetime(D, M);
    if (kind == kMfmaPredict) return launch_rc<NT, NS>(g, in, base, out, frag, taps, ntaps, stream);
    if (kind == kMfmaCorrect) return launch_rc<NS, NT>(g, in, base, out, frag, taps, ntaps, stream);
    return launch_rc<NS, NS>(g, in, base, out, frag, taps, ntaps, stream);
  }
};

int launch_tap_mfma(int d, int M, int kind, const DevGeom& g, const double* in, const double* base, double* out,
                    const double* frag, const int32_t* taps, int ntaps, void* stream) {
  return dispatch_dm<MfmaL>(d, M, kind, g, in, base, out, frag, taps, ntaps, stream);
}

int mfma_tiles_per_group(int64_t nel, size_t lds_bytes) {
  // one round of resident workgroups: up to 8 per CU, fewer when the staged fragments fill the LDS
  int64_t resident = 8;
  if (lds_bytes > 0 && (int64_t)(kMfmaMaxLds / lds_bytes) < resident) resident = (int64_t)(kMfmaMaxLds / lds_bytes);
  if (resident < 1) resident = 1;
  const int64_t ntiles = (nel + 15) / 16;
  int64_t groups = (ntiles + kMfmaWaves - 1) / kMfmaWaves;
  if (groups > 256 * resident) groups = 256 * resident;
  return (int)((ntiles + groups - 1) / groups);
}

template <int D, int M>
struct BatchMfmaL {
  static int run(int kind, const BatchMfmaArgs& a, int64_t groups, void* stream) {
    constexpr int NS = n_space(D, M), NT = n_spacetime(D, M);
    if (a.count <= 0 || groups <= 0) return 0;
    if (kind == kMfmaPredict)
      hipLaunchKernelGGL((batch_mfma_kernel<NT, NS>), dim3((unsigned)groups), dim3(64 * kMfmaWaves), 0,
                         (hipStream_t)stream, a);
    else
      hipLaunchKernelGGL((batch_mfma_kernel<NS, NT>), dim3((unsigned)groups), dim3(64 * kMfmaWaves), 0,
                         (hipStream_t)stream, a);
    return (int)hipGetLastError();
  }
};

int launch_batch_mfma(int d, int M, int kind, const BatchMfmaArgs& args, int64_t groups, void* stream) {
  if (kind != kMfmaPredict && kind != kMfmaCorrect) return (int)hipErrorInvalidValue;
  return dispatch_dm<BatchMfmaL>(d, M, kind, args, groups, stream);
}

}  // namespace ridg

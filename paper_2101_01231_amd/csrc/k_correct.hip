// Explicit flux-form correction (Sec. 2.3), FP64.
#include "kernels_common.hpp"

namespace ridg {

// ---------------------------------------------------------------- correction
// Q'_e = Q_e + 2^-d [ sum_i sum_p V_ip Cv_ip W_e - sum_faces sum_p V_ip (CFo W_e | CFn W_nbr) ]
template <int D, int M, bool AFFINE>
__global__ __launch_bounds__(256) void correct_kernel(DevGeom g, double dt, const double* __restrict__ Q,
                                                      const double* __restrict__ W, double* __restrict__ Qout,
                                                      DevTensors t) {
  constexpr int NS = n_space(D, M), NT = n_spacetime(D, M), NP = D + 1;
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nel) return;
  int idx[3];
  elem_idx(g, e, idx);
  double V[D][D + 1];
  vel_modes<D>(g, idx, dt, V);
  double we[NT], acc[NS];
#pragma unroll
  for (int l = 0; l < NT; ++l) we[l] = W[(int64_t)l * nel + e];
#pragma unroll
  for (int k = 0; k < NS; ++k) acc[k] = 0.0;
#pragma unroll 1
  for (int i = 0; i < D; ++i) {
#pragma unroll 1
    for (int p = 0; p < NP; ++p) {
      if (p == 1 + i || (!AFFINE && p > 0)) continue;
      const double vp = V[i][p];
      const double* cv = t.Cv + ((size_t)i * NP + p) * NS * NT;
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < NT; ++l) s = fma(cv[k * NT + l], we[l], s);
        acc[k] = fma(vp, s, acc[k]);
      }
    }
#pragma unroll 1
    for (int sd = 0; sd < 2; ++sd) {
      const int s = sd ? 1 : -1;
      const int side = face_side<D>(g, idx, i, s);
      double wn[NT];
      const double* tens;
      if (side == 0) {
#pragma unroll
        for (int l = 0; l < NT; ++l) wn[l] = we[l];
        tens = t.CFo;
      } else {
        int j[3] = {idx[0], idx[1], idx[2]};
        j[i] += s;
        const int64_t en = elem_lin(g, j[0], j[1], j[2]);
#pragma unroll
        for (int l = 0; l < NT; ++l) wn[l] = W[(int64_t)l * nel + en];
        tens = t.CFn;
      }
#pragma unroll 1
      for (int p = 0; p < NP; ++p) {
        if (p == 1 + i || (!AFFINE && p > 0)) continue;
        const double vp = V[i][p];
        const double* cf = tens + (((size_t)i * 2 + sd) * NP + p) * NS * NT;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          double s2 = 0.0;
#pragma unroll
          for (int l = 0; l < NT; ++l) s2 = fma(cf[k * NT + l], wn[l], s2);
          acc[k] = fma(-vp, s2, acc[k]);
        }
      }
    }
  }
  constexpr double scale = 1.0 / (double)(1 << D);
#pragma unroll
  for (int k = 0; k < NS; ++k) Qout[(int64_t)k * nel + e] = fma(acc[k], scale, Q[(int64_t)k * nel + e]);
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

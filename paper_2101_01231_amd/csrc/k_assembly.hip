// The three ways Sec. 3 compares of assembling the Newton Jacobian of the prediction's volume flux
// term for a nonlinear flux (Burgers, F(w) = w^2 / 2 on every axis, F'(w) = w), one space-time element
// per workgroup:
//   quadrature      J_kl = -c sum_pt w_pt sum_i d_xi_i Psi_k(pt) F'(w(pt)) Psi_l(pt)         (eq. Jacobian)
//   quasi-quadrature-free: F'_p = projection of F'(w) on Psi (eq. Jacproj, quadrature once per mode),
//                   J_kl = -c sum_p beta_{k l p} F'_p with the exact triple products   (eq. Jacobian2)
//   perturbation    J_kl = (R_k(W + eps e_l) - R_k(W - eps e_l)) / (2 eps), R_k the residual volume term
//                   -c sum_pt w_pt sum_i d_xi_i Psi_k F(w): one residual evaluation per unknown.
// Quadrature and perturbation accumulate 4 x 4 register tiles of J over the points; the point values
// of w are staged in LDS.
#include "kernels_common.hpp"

namespace ridg {

namespace {
constexpr int kAsmThreads = 256;
constexpr double kAsmEps = 1e-3;
}  // namespace

__global__ __launch_bounds__(kAsmThreads) void assembly_kernel(int method, AsmDev t, const double* __restrict__ W,
                                                               double c, double* __restrict__ J) {
  extern __shared__ double sh[];  // [nq] point values of w, then [nt] projection of F'(w)
  const int nt = t.nt, nq = t.nq, tid = threadIdx.x;
  const int64_t e = blockIdx.x;
  double* s_w = sh;
  double* s_fp = sh + nq;
  const double* We = W + e * nt;
  double* Je = J + e * (int64_t)nt * nt;
  for (int pt = tid; pt < nq; pt += kAsmThreads) {
    double v = 0.0;
    for (int l = 0; l < nt; ++l) v = fma(t.psiv[(size_t)l * nq + pt], We[l], v);
    s_w[pt] = v;
  }
  __syncthreads();
  if (method == kAsmQqf) {
    for (int p = tid; p < nt; p += kAsmThreads) {
      double v = 0.0;
      for (int pt = 0; pt < nq; ++pt) v = fma(t.projw[(size_t)p * nq + pt], s_w[pt], v);  // F'(w) = w
      s_fp[p] = v;
    }
    __syncthreads();
    for (int kl = tid; kl < nt * nt; kl += kAsmThreads) {
      double s = 0.0;
      for (int q = t.rptr[kl]; q < t.rptr[kl + 1]; ++q) s = fma(t.bval[q], s_fp[t.bp[q]], s);
      Je[kl] = -c * s;
    }
    return;
  }
  const int nb = (nt + 3) / 4;
  for (int tile = tid; tile < nb * nb; tile += kAsmThreads) {
    const int k0 = (tile / nb) * 4, l0 = (tile % nb) * 4;
    int kr[4], lr[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      kr[a] = min(k0 + a, nt - 1);  // rows past nt repeat the last one and are not stored
      lr[a] = min(l0 + a, nt - 1);
    }
    double acc[4][4] = {};
    for (int pt = 0; pt < nq; ++pt) {
      const double w = s_w[pt];
      double dk[4], pl[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        dk[a] = t.dsum[(size_t)kr[a] * nq + pt];
        pl[a] = t.psiv[(size_t)lr[a] * nq + pt];
      }
      double g[4];
      if (method == kAsmQuadrature) {
#pragma unroll
        for (int b = 0; b < 4; ++b) g[b] = w * pl[b];
      } else {  // F(w + eps psi_l) - F(w - eps psi_l), F(x) = x^2 / 2
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const double up = w + kAsmEps * pl[b], dn = w - kAsmEps * pl[b];
          g[b] = (0.5 * up * up - 0.5 * dn * dn) * (0.5 / kAsmEps);
        }
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(dk[a], g[b], acc[a][b]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (k0 + a < nt && l0 + b < nt) Je[(size_t)(k0 + a) * nt + l0 + b] = -c * acc[a][b];
  }
}

int launch_assembly(int method, const AsmDev& t, int64_t n_elements, const double* W, double c, double* J,
                    void* stream) {
  if (method < kAsmQuadrature || method > kAsmPerturbation || n_elements < 0 || n_elements > (int64_t)1 << 31)
    return (int)hipErrorInvalidValue;
  if (n_elements == 0) return 0;
  const size_t lds = ((size_t)t.nq + t.nt) * sizeof(double);
  if (lds > 64 * 1024) return (int)hipErrorInvalidValue;
  hipLaunchKernelGGL(assembly_kernel, dim3((unsigned)n_elements), dim3(kAsmThreads), lds, (hipStream_t)stream,
                     method, t, W, c, J);
  return (int)hipGetLastError();
}

}  // namespace ridg

// Region solves by upwind elimination plans (Sec. 2.2 and Sec. 3): the layout with two regions per packed segment.
#include "kernels_common.hpp"

namespace ridg {

// Two regions per packed segment (same plan): every tensor row is loaded once for both, and the
// two block eliminations are interleaved (seg_solve2). FP64.
template <int D, int M>
__global__ __launch_bounds__(256) void predict_plans2_kernel(DevGeom g, double dt, const double* __restrict__ Q,
                                                             double* __restrict__ W, PlanTables t,
                                                             const PlanRec* __restrict__ plans,
                                                             const int32_t* __restrict__ items,
                                                             const int32_t* __restrict__ item_plan,
                                                             int64_t n_items) {
  using C = PlanCfg<D, M, false>;
  constexpr int NT = C::NT, S = C::S, NB = C::NB, LB = C::LB, SEGW = C::SEGW;
  __shared__ double s_w[C::WAVES][S][2][NB][NT];
  __shared__ double s_piv[C::WAVES][S][4 * (NT + 2)];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const bool tail = lane >= S * SEGW;
  const int seg = tail ? 0 : lane / SEGW;
  const int k = tail ? lane - S * SEGW : lane % SEGW;
  const bool idle = tail || k >= NT;
  const int64_t wave_first = (xcd_block(blockIdx.x, gridDim.x) * C::WAVES + wave) * S * 2;
  if (wave_first >= n_items) return;  // the list is padded to 2 S
  int addr[LB > 0 ? LB : 1];
#pragma unroll
  for (int r = 0; r < LB; ++r) addr[r] = 4 * (tail ? lane : seg * SEGW + (k + (1 << r)) % SEGW);
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  int32_t e[2];
  bool write[2];
  int base[2][3];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    e[u] = items[wave_first + seg * 2 + u];
    write[u] = e[u] >= 0 && !idle;
    if (e[u] < 0) e[u] = -e[u] - 1;
    elem_idx(g, e[u], base[u]);
  }
  const int pid = __builtin_amdgcn_readfirstlane(item_plan[wave_first]);
  const PlanRec* pr = plans + pid;
  const int nb = pr->nb;
  double* sw0 = &s_w[wave][seg][0][0][0];
  double* sw1 = &s_w[wave][seg][1][0][0];
  double* spiv = &s_piv[wave][seg][0];
  const int kr = idle ? 0 : k;
  const int ccl = t.cc_idx[kr];
  const double ccv = t.cc_val[kr];
  for (int b = 0; b < nb; ++b) {
    const PlanBlock blk = pr->blk[b];
    int mask = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
      mask |= ((blk.src[2 * i] == kOwn ? 1 : 0) | (blk.src[2 * i + 1] == kOwn ? 2 : 0)) << (2 * i);
    int64_t ge[2];
    double V0[2][D];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int gi[3] = {wrap(base[u][0] + blk.off[0], g.n0), wrap(base[u][1] + blk.off[1], g.n1),
                         wrap(base[u][2] + blk.off[2], g.n2)};
      ge[u] = (int64_t)gi[0] + (int64_t)g.n0 * ((int64_t)gi[1] + (int64_t)g.n1 * gi[2]);
#pragma unroll
      for (int i = 0; i < D; ++i) {
        double v = g.a[i];
#pragma unroll
        for (int j = 0; j < D; ++j) v += g.g[i][j] * ((gi[j] + 0.5) * geom_h(g, j));
        V0[u][i] = v * dt / geom_h(g, i);
      }
    }
    double a[2][NT];
    {
      const double* a0 = t.A0 + ((size_t)mask * NT + kr) * NT;
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        const double v = a0[l];
        a[0][l] = v;
        a[1][l] = v;
      }
    }
#pragma unroll 1
    for (int i = 0; i < D; ++i) {
      const double v0 = sel<D>(V0[0], i), v1 = sel<D>(V0[1], i);
      const double* kk = t.K + (((size_t)i * 4 + ((mask >> (2 * i)) & 3)) * NT + kr) * NT;
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        const double kv = kk[l];
        a[0][l] = fma(v0, kv, a[0][l]);
        a[1][l] = fma(v1, kv, a[1][l]);
      }
    }
    double rhs[2] = {ccv * Q[(int64_t)ccl * nel + ge[0]], ccv * Q[(int64_t)ccl * nel + ge[1]]};
#pragma unroll 1
    for (int i = 0; i < D; ++i) {
      const double v0 = sel<D>(V0[0], i), v1 = sel<D>(V0[1], i);
#pragma unroll 1
      for (int sd = 0; sd < 2; ++sd) {
        const int src = blk.src[2 * i + sd];
        if (src == kOwn) continue;
        const double* f0 = t.Fn0 + (((size_t)i * 2 + sd) * NT + kr) * NT;
        const double* fc = t.FnC + (((size_t)i * 2 + sd) * NT + kr) * NT;
        const double* w0 = sw0 + src * NT;
        const double* w1 = sw1 + src * NT;
        double acc0 = 0.0, acc1 = 0.0;
#pragma unroll
        for (int l = 0; l < NT; ++l) {
          const double fv = f0[l], cv = fc[l];
          acc0 = fma(fma(v0, fv, cv), w0[l], acc0);
          acc1 = fma(fma(v1, fv, cv), w1[l], acc1);
        }
        rhs[0] -= acc0;
        rhs[1] -= acc1;
      }
    }
    seg_solve2<NT, LB, C::POW2, SEGW>(a, rhs, k, idle, addr, spiv, sw0 + b * NT, sw1 + b * NT);
  }
  if (write[0]) W[(int64_t)k * nel + e[0]] = sw0[(nb - 1) * NT + k];
  if (write[1]) W[(int64_t)k * nel + e[1]] = sw1[(nb - 1) * NT + k];
}

template <int D, int M>
struct Plans2L {
  static int run(const DevGeom& g, double dt, const double* Q, double* W, const PlanTables& t, const PlanRec* plans,
                 const int32_t* items, const int32_t* item_plan, int64_t n_items, void* stream) {
    if (n_spacetime(D, M) > 64) return (int)hipErrorInvalidValue;
    using C = PlanCfg<D, M, false>;
    const int64_t per_block = (int64_t)C::WAVES * C::S * 2;
    const int64_t blocks = (n_items + per_block - 1) / per_block;
    if (blocks == 0) return 0;
    hipLaunchKernelGGL((predict_plans2_kernel<D, M>), dim3((unsigned)blocks), dim3(64 * C::WAVES), 0,
                       (hipStream_t)stream, g, dt, Q, W, t, plans, items, item_plan, n_items);
    return (int)hipGetLastError();
  }
};

int launch_plans2(int d, int M, const DevGeom& g, double dt, const double* Q, double* W, const PlanTables& t,
                  const PlanRec* plans, const int32_t* items, const int32_t* item_plan, int64_t n_items, void* stream) {
  return dispatch_dm<Plans2L>(d, M, g, dt, Q, W, t, plans, items, item_plan, n_items, stream);
}

}  // namespace ridg

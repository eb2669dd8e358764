// Region solves by upwind elimination plans (Sec. 2.2 and Sec. 3), FP64 and FP32 with FP64 refinement.
#include "kernels_common.hpp"
#include "plans_nr.hpp"

namespace ridg {


template <int D, int M, bool PADDED, bool F32 = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PlanCfg<D, M, PADDED>::MIN_WAVES))) void predict_plans_kernel(DevGeom g, double dt, const double* __restrict__ Q,
                                                            double* __restrict__ W, PlanTables t,
                                                            const PlanRec* __restrict__ plans,
                                                            const int32_t* __restrict__ items,
                                                            const int32_t* __restrict__ item_plan,
                                                            int64_t n_items, int refine) {
  using C = PlanCfg<D, M, PADDED>;
  constexpr int NT = C::NT, S = C::S, NB = C::NB, LB = C::LB, SEGW = C::SEGW;
  __shared__ double s_w[C::WAVES][S][NB][NT];
  __shared__ double s_piv[C::WAVES][S][2 * (NT + 2)];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const bool tail = lane >= S * SEGW;  // lanes past the last whole segment
  const int seg = tail ? 0 : lane / SEGW;
  const int k = tail ? lane - S * SEGW : lane % SEGW;
  const bool idle = tail || k >= NT;   // no row (tail lanes, padding rows of a padded segment)
  const int64_t wave_first = (xcd_block(blockIdx.x, gridDim.x) * C::WAVES + wave) * S;
  if (wave_first >= n_items) return;  // whole wavefront idle (the list is padded to S)
  int addr[LB > 0 ? LB : 1];
#pragma unroll
  for (int r = 0; r < LB; ++r) addr[r] = 4 * (tail ? lane : seg * SEGW + (k + (1 << r)) % SEGW);
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  int32_t e = items[wave_first + seg];
  const bool write = e >= 0 && !idle;  // idle already covers k >= NT
  if (e < 0) e = -e - 1;
  int base[3];
  elem_idx(g, e, base);
  const int pid = __builtin_amdgcn_readfirstlane(item_plan[wave_first]);  // one plan per wavefront
  const PlanRec* pr = plans + pid;
  const int nb = pr->nb;
  double* sw = &s_w[wave][seg][0][0];
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
    const int gi[3] = {wrap(base[0] + blk.off[0], g.n0), wrap(base[1] + blk.off[1], g.n1),
                       wrap(base[2] + blk.off[2], g.n2)};
    const int64_t ge = (int64_t)gi[0] + (int64_t)g.n0 * ((int64_t)gi[1] + (int64_t)g.n1 * gi[2]);
    double V0[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double v = g.a[i];
#pragma unroll
      for (int j = 0; j < D; ++j) v += g.g[i][j] * ((gi[j] + 0.5) * geom_h(g, j));
      V0[i] = v * dt / geom_h(g, i);
    }
    // row kr of the diagonal block: A0[mask] + sum_i V_i0 K_i[mask_i]
    double a[NT];
    {
      const double* a0 = t.A0 + ((size_t)mask * NT + kr) * NT;
#pragma unroll
      for (int l = 0; l < NT; ++l) a[l] = a0[l];
    }
#pragma unroll 1
    for (int i = 0; i < D; ++i) {
      const double vi = sel<D>(V0, i);
      const double* kk = t.K + (((size_t)i * 4 + ((mask >> (2 * i)) & 3)) * NT + kr) * NT;
#pragma unroll
      for (int l = 0; l < NT; ++l) a[l] = fma(vi, kk[l], a[l]);
    }
    // right-hand side: causal source minus the upwind couplings to solved blocks
    double rhs = ccv * Q[(int64_t)ccl * nel + ge];
#pragma unroll 1
    for (int i = 0; i < D; ++i) {
      const double vi = sel<D>(V0, i);
#pragma unroll 1
      for (int sd = 0; sd < 2; ++sd) {
        const int src = blk.src[2 * i + sd];
        if (src == kOwn) continue;
        const double* f0 = t.Fn0 + (((size_t)i * 2 + sd) * NT + kr) * NT;
        const double* fc = t.FnC + (((size_t)i * 2 + sd) * NT + kr) * NT;
        const double* wsrc = sw + src * NT;
        double acc = 0.0;
#pragma unroll
        for (int l = 0; l < NT; ++l) acc = fma(fma(vi, f0[l], fc[l]), wsrc[l], acc);
        rhs -= acc;
      }
    }
    if constexpr (F32)
      seg_solve_f32r<NT, LB, C::POW2, SEGW>(a, rhs, refine, k, idle, addr, spiv, sw + b * NT);
    else
      seg_solve<NT, LB, C::POW2, SEGW>(a, rhs, k, idle, addr, spiv, sw + b * NT);
  }
  if (write) W[(int64_t)k * nel + e] = sw[(nb - 1) * NT + k];
}

template <int D, int M>
struct IpwL {
  static int run(int layout) {
    if (layout == 2) return 2 * PlanCfg<D, M, false>::S;
    if (layout == 3) return PlanCfg2R<D, M>::S;
    if (layout == 4) return PlanCfgDpp<D, M>::S;
    if (layout == kStaticPivotLayout) return PlanCfgSp<D, M>::S;
    return layout ? PlanCfg<D, M, true>::S : PlanCfg<D, M, false>::S;
  }
};
int items_per_wave(int d, int M, int layout) { return dispatch_dm<IpwL>(d, M, layout); }

template <int D, int M, bool PADDED>
static int launch_plans(int precision, int refine, const DevGeom& g, double dt, const double* Q, double* W,
                        const PlanTables& t, const PlanRec* plans, const int32_t* items, const int32_t* item_plan,
                        int64_t n_items, void* stream) {
  using C = PlanCfg<D, M, PADDED>;
  const int64_t per_block = (int64_t)C::WAVES * C::S;
  const int64_t blocks = (n_items + per_block - 1) / per_block;
  if (blocks == 0) return 0;
  if (precision == RIDG_FP32_REFINE)
    hipLaunchKernelGGL((predict_plans_kernel<D, M, PADDED, true>), dim3((unsigned)blocks), dim3(64 * C::WAVES), 0,
                       (hipStream_t)stream, g, dt, Q, W, t, plans, items, item_plan, n_items, refine);
  else
    hipLaunchKernelGGL((predict_plans_kernel<D, M, PADDED, false>), dim3((unsigned)blocks), dim3(64 * C::WAVES), 0,
                       (hipStream_t)stream, g, dt, Q, W, t, plans, items, item_plan, n_items, 0);
  return (int)hipGetLastError();
}

template <int D, int M>
struct PlansL {
  static int run(int layout, int precision, int refine, const DevGeom& g, double dt, const double* Q, double* W,
                 const PlanTables& t, const PlanRec* plans, const int32_t* items, const int32_t* item_plan,
                 int64_t n_items, void* stream) {
    if (n_spacetime(D, M) > 64) return (int)hipErrorInvalidValue;
    if (layout == kStaticPivotLayout)
      return launch_plans_sp(D, M, precision, refine, g, dt, Q, W, t, plans, items, item_plan, n_items, stream);
    if (layout >= 2) {  // FP64-only layouts, each compiled in its own unit
      if (precision != RIDG_FP64) return (int)hipErrorInvalidValue;
      if (layout == 2) return launch_plans2(D, M, g, dt, Q, W, t, plans, items, item_plan, n_items, stream);
      if (layout == 3) return launch_plans_2rows(D, M, g, dt, Q, W, t, plans, items, item_plan, n_items, stream);
      return launch_plans_dpp(D, M, g, dt, Q, W, t, plans, items, item_plan, n_items, stream);
    }
    if (layout)
      return launch_plans<D, M, true>(precision, refine, g, dt, Q, W, t, plans, items, item_plan, n_items, stream);
    return launch_plans<D, M, false>(precision, refine, g, dt, Q, W, t, plans, items, item_plan, n_items, stream);
  }
};

int launch_predict_plans(int d, int M, int layout, int precision, int refine, const DevGeom& g, double dt,
                         const double* Q, double* W, const PlanTables& t, const PlanRec* plans, const int32_t* items,
                         const int32_t* item_plan, int64_t n_items, void* stream) {
  return dispatch_dm<PlansL>(d, M, layout, precision, refine, g, dt, Q, W, t, plans, items, item_plan, n_items,
                             stream);
}


}  // namespace ridg

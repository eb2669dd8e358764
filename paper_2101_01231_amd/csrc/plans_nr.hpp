// Region solves by upwind elimination plans (Sec. 2.2 and Sec. 3): the kernel of the layouts with
// several rows per lane, instantiated per layout in k_plans_nr.hip and k_plans_dpp.hip.
#pragma once
#include "kernels_common.hpp"

namespace ridg {

constexpr int kLoadChunk = 4;  // table loads between scheduling barriers

// Several rows per lane (PlanCfgNR): RPL rows of a region's block system in each lane of a
// SEGW-lane segment, each pivot row read once for RPL rows. FP64; bitwise the results of the
// packed layout. Table rows are addressed by 32-bit byte offsets and loaded kLoadChunk at a time
// (scheduling barriers), which keeps the loads in flight, and with them the registers, bounded.
template <int D, int M, int RPL, int SEGW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PlanCfgNR<D, M, RPL, SEGW>::MIN_WAVES))) void
predict_plans_nr_kernel(DevGeom g, double dt, const double* __restrict__ Q, double* __restrict__ W, PlanTables t,
                        const PlanRec* __restrict__ plans, const int32_t* __restrict__ items,
                        const int32_t* __restrict__ item_plan, int64_t n_items) {
  using C = PlanCfgNR<D, M, RPL, SEGW>;
  constexpr int NT = C::NT, S = C::S, NB = C::NB, LB = C::LB;
  __shared__ double s_w[C::WAVES][S][NB][NT];
  __shared__ double s_piv[C::WAVES][S][2 * (NT + 2)];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const bool tail = lane >= S * SEGW;
  const int seg = tail ? 0 : lane / SEGW;
  const int k = tail ? lane - S * SEGW : lane % SEGW;
  bool idle[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) idle[u] = tail || k + u * SEGW >= NT;
  const int64_t wave_first = (xcd_block(blockIdx.x, gridDim.x) * C::WAVES + wave) * S;
  if (wave_first >= n_items) return;  // the list is padded to S
  int addr[LB > 0 ? LB : 1];
#pragma unroll
  for (int r = 0; r < LB; ++r) addr[r] = 4 * (tail ? lane : seg * SEGW + (k + (1 << r)) % SEGW);
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  int32_t e = items[wave_first + seg];
  const bool write = e >= 0 && !tail;
  if (e < 0) e = -e - 1;
  int base[3];
  elem_idx(g, e, base);
  const int pid = __builtin_amdgcn_readfirstlane(item_plan[wave_first]);
  const PlanRec* pr = plans + pid;
  const int nb = pr->nb;
  double* sw = &s_w[wave][seg][0][0];
  double* spiv = &s_piv[wave][seg][0];
  unsigned rb[RPL];  // byte offset of the lane's rows within a theta_T x theta_T table
  int ccl[RPL];
  double ccv[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int kr = idle[u] ? 0 : k + u * SEGW;
    rb[u] = (unsigned)kr * (unsigned)(NT * 8);
    ccl[u] = t.cc_idx[kr];
    ccv[u] = t.cc_val[kr];
  }
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
    double a[RPL][NT];
    {
      const char* a0 = (const char*)t.A0 + (unsigned)mask * (unsigned)(NT * NT * 8);
#pragma unroll
      for (int u = 0; u < RPL; ++u)
#pragma unroll
        for (int l = 0; l < NT; ++l) a[u][l] = *(const double*)(a0 + (rb[u] + (unsigned)(l * 8)));
    }
#pragma unroll 1
    for (int i = 0; i < D; ++i) {
      const double vi = sel<D>(V0, i);
      const char* kk = (const char*)t.K + (unsigned)(i * 4 + ((mask >> (2 * i)) & 3)) * (unsigned)(NT * NT * 8);
#pragma unroll
      for (int u = 0; u < RPL; ++u)
#pragma unroll
        for (int l = 0; l < NT; ++l) {
          a[u][l] = fma(vi, *(const double*)(kk + (rb[u] + (unsigned)(l * 8))), a[u][l]);
          if (l % kLoadChunk == kLoadChunk - 1) __builtin_amdgcn_sched_barrier(0);
        }
    }
    double rhs[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) rhs[u] = ccv[u] * Q[(int64_t)ccl[u] * nel + ge];
#pragma unroll 1
    for (int i = 0; i < D; ++i) {
      const double vi = sel<D>(V0, i);
#pragma unroll 1
      for (int sd = 0; sd < 2; ++sd) {
        const int src = blk.src[2 * i + sd];
        if (src == kOwn) continue;
        const unsigned toff = (unsigned)(i * 2 + sd) * (unsigned)(NT * NT * 8);
        const char* f0 = (const char*)t.Fn0 + toff;
        const char* fc = (const char*)t.FnC + toff;
        const double* wsrc = sw + src * NT;
        double acc[RPL];
#pragma unroll
        for (int u = 0; u < RPL; ++u) acc[u] = 0.0;
#pragma unroll
        for (int l = 0; l < NT; ++l) {
          const double w = wsrc[l];
#pragma unroll
          for (int u = 0; u < RPL; ++u) {
            const unsigned o = rb[u] + (unsigned)(l * 8);
            acc[u] = fma(fma(vi, *(const double*)(f0 + o), *(const double*)(fc + o)), w, acc[u]);
          }
          if (l % kLoadChunk == kLoadChunk - 1) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int u = 0; u < RPL; ++u) rhs[u] -= acc[u];
      }
    }
    seg_solve_nr<C>(a, rhs, k, idle, addr, spiv, sw + b * NT);
  }
  if (write) {
#pragma unroll
    for (int u = 0; u < RPL; ++u)
      if (!idle[u]) W[(int64_t)(k + u * SEGW) * nel + e] = sw[(nb - 1) * NT + k + u * SEGW];
  }
}

template <class C, int D, int M>
static int launch_nr(const DevGeom& g, double dt, const double* Q, double* W, const PlanTables& t,
                     const PlanRec* plans, const int32_t* items, const int32_t* item_plan, int64_t n_items,
                     void* stream) {
  const int64_t per_block = (int64_t)C::WAVES * C::S;
  const int64_t blocks = (n_items + per_block - 1) / per_block;
  if (blocks == 0) return 0;
  hipLaunchKernelGGL((predict_plans_nr_kernel<D, M, C::RPL, C::SEGW>), dim3((unsigned)blocks), dim3(64 * C::WAVES),
                     0, (hipStream_t)stream, g, dt, Q, W, t, plans, items, item_plan, n_items);
  return (int)hipGetLastError();
}

}  // namespace ridg

// Region solves by upwind elimination plans (Sec. 2.2 and Sec. 3) with several rows per lane: the
// partial-pivoting kernel (layouts 3 and 4, instantiated in k_plans_nr.hip and k_plans_dpp.hip) and
// the static-pivot kernel (layout 5, FP64 or FP32 with FP64-residual refinement, k_plans_sp.hip).
#pragma once
#include "kernels_common.hpp"

namespace ridg {

constexpr int kLoadChunk = 4;  // table loads between scheduling barriers
#ifndef RIDG_PIV_CHUNK
#define RIDG_PIV_CHUNK 8
#endif
constexpr int kPivChunk = RIDG_PIV_CHUNK;  // pivot-row LDS reads between scheduling barriers (static pivots)
#ifndef RIDG_SP_LOOKAHEAD
#define RIDG_SP_LOOKAHEAD false
#endif

// Geometry of the static-pivot layout (5): the layout-4 segments, except at 2D order 4 (theta_T =
// 20), where two rows per lane in 10-lane segments at three wavefronts per SIMD (FP64, 168 VGPRs)
// measured 1.059 ms per prediction against 1.117 ms for three rows per lane in 8-lane segments at two
// (FP32: 1.80 against 1.88 ms, at two wavefronts). Its segments per wavefront also set how the host
// groups and pads the layout's work list.
template <int D, int M>
using PlanCfgSp = typename std::conditional<D == 2 && M == 4, PlanCfg2R<D, M>, PlanCfgDpp<D, M>>::type;

// Per-lane state of the several-rows layouts: RPL rows of a region's block system in each lane of
// a SEGW-lane segment; rows k + SEGW u (u < RPL) of every block, rows >= theta_T idle.
template <class C>
struct RowsCtx {
  int k;                 // lane within the segment
  bool idle[C::RPL];     // no row in this slot
  unsigned rb[C::RPL];   // byte offset of the slot's row within a theta_T x theta_T table
  int ccl[C::RPL];       // causal source: the spatial mode coupled to the row
  double ccv[C::RPL];    // and its coefficient
  int base[3];           // region centre
};

// Row index (block offset, mask, global element, V_i0) of plan block b.
template <int D>
struct BlockGeo {
  int mask;
  int64_t ge;
  double V0[D];
};

template <int D>
__device__ __forceinline__ BlockGeo<D> block_geo(const DevGeom& g, double dt, const PlanBlock& blk, const int (&base)[3]) {
  BlockGeo<D> r;
  r.mask = 0;
#pragma unroll
  for (int i = 0; i < D; ++i)
    r.mask |= ((blk.src[2 * i] == kOwn ? 1 : 0) | (blk.src[2 * i + 1] == kOwn ? 2 : 0)) << (2 * i);
  const int gi[3] = {wrap(base[0] + blk.off[0], g.n0), wrap(base[1] + blk.off[1], g.n1),
                     wrap(base[2] + blk.off[2], g.n2)};
  r.ge = (int64_t)gi[0] + (int64_t)g.n0 * ((int64_t)gi[1] + (int64_t)g.n1 * gi[2]);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double v = g.a[i];
#pragma unroll
    for (int j = 0; j < D; ++j) v += g.g[i][j] * ((gi[j] + 0.5) * geom_h(g, j));
    r.V0[i] = v * dt / geom_h(g, i);
  }
  return r;
}

// Diagonal block rows A0[mask] + sum_i V_i0 K_i[mask_i] (FP64), the arithmetic of every layout.
// Table rows are read kLoadChunk entries at a time between scheduling barriers. (Keeping two such
// chunks in flight, or larger chunks, measured slower on the 512^2 order-4 rotation: 1.09-1.40 ms
// against 1.04 ms per prediction; the table reads are bound by the rate at which the 64 lane
// addresses of each load are processed, not by their latency.)
template <class C, int D>
__device__ __forceinline__ void assemble_rows(const PlanTables& t, const RowsCtx<C>& x, const BlockGeo<D>& bg,
                                              double (&a)[C::RPL][C::NT]) {
  constexpr int NT = C::NT, RPL = C::RPL;
  const char* a0 = (const char*)t.A0 + (unsigned)bg.mask * (unsigned)(NT * NT * 8);
  double V0[D];  // a local copy: selecting from the struct member is lowered to a stack load
#pragma unroll
  for (int i = 0; i < D; ++i) V0[i] = bg.V0[i];
#pragma unroll
  for (int u = 0; u < RPL; ++u)
#pragma unroll
    for (int l = 0; l < NT; ++l) a[u][l] = *(const double*)(a0 + (x.rb[u] + (unsigned)(l * 8)));
#pragma unroll 1
  for (int i = 0; i < D; ++i) {
    const double vi = sel<D>(V0, i);
    const char* kk = (const char*)t.K + (unsigned)(i * 4 + ((bg.mask >> (2 * i)) & 3)) * (unsigned)(NT * NT * 8);
#pragma unroll
    for (int u = 0; u < RPL; ++u)
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        a[u][l] = fma(vi, *(const double*)(kk + (x.rb[u] + (unsigned)(l * 8))), a[u][l]);
        if (l % kLoadChunk == kLoadChunk - 1) __builtin_amdgcn_sched_barrier(0);
      }
  }
}

// Right-hand side of the block rows: causal source minus the upwind couplings to solved blocks.
template <class C, int D>
__device__ __forceinline__ void assemble_rhs(const DevGeom& g, const double* __restrict__ Q, const PlanTables& t,
                                             const RowsCtx<C>& x, const BlockGeo<D>& bg, const PlanBlock& blk,
                                             const double* sw, int64_t nel, double (&rhs)[C::RPL]) {
  constexpr int NT = C::NT, RPL = C::RPL;
  double V0[D];
#pragma unroll
  for (int i = 0; i < D; ++i) V0[i] = bg.V0[i];
#pragma unroll
  for (int u = 0; u < RPL; ++u) rhs[u] = x.ccv[u] * Q[(int64_t)x.ccl[u] * nel + bg.ge];
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
          const unsigned o = x.rb[u] + (unsigned)(l * 8);
          acc[u] = fma(fma(vi, *(const double*)(f0 + o), *(const double*)(fc + o)), w, acc[u]);
        }
        if (l % kLoadChunk == kLoadChunk - 1) __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int u = 0; u < RPL; ++u) rhs[u] -= acc[u];
    }
  }
}

// Gauss-Jordan without row exchanges (static pivots: row c is the pivot of column c), RPL rows per
// lane. Row c + 1 is eliminated first and published (with its reciprocal pivot) to the other LDS
// buffer before the remaining rows, so its store and the reciprocal overlap the column's bulk of
// FMAs; one wave-level sync per column. x[r] = rhs_r / a_rr at the end (Gauss-Jordan leaves the
// diagonal). The host enables this only where elimination in natural order is measured stable on
// the problem's velocity range.
template <class C, bool LOOKAHEAD>
__device__ __forceinline__ void seg_solve_sp(double (&a)[C::RPL][C::NT], double (&rhs)[C::RPL], int k,
                                    const bool (&idle)[C::RPL], double* piv, double* x) {
  constexpr int NT = C::NT, RPL = C::RPL, SEGW = C::SEGW;
  constexpr int PS = NT + 2;
  static_assert(2 * PS <= 256, "ds_write2_b64 offsets are 8-bit");
  double inv[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) inv[u] = 0.0;
  const unsigned pbase = lds_addr(piv);
  if (k == 0 && !idle[0]) {  // row 0: slot 0 of lane 0
    inv[0] = recip(a[0][0]);
    publish_row<0, 1, NT>(pbase, a[0], rhs[0], inv[0]);
  }
  wave_sync();
  static_for<0, NT>([&](auto CC) {
    constexpr int c = decltype(CC)::value;
    constexpr int uc = c / SEGW, kc = c % SEGW;
    constexpr int c1 = c + 1, u1 = c1 / SEGW, k1 = c1 % SEGW;
    const double* pv = piv + (c & 1) * PS;
    const double ip = pv[NT + 1];
    double l[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) l[u] = (idle[u] || (u == uc && k == kc)) ? 0.0 : a[u][c] * ip;
    if constexpr (LOOKAHEAD && c1 < NT) {  // the next pivot row first
#pragma unroll
      for (int j = c + 1; j < NT; ++j) a[u1][j] = fma(-l[u1], pv[j], a[u1][j]);
      rhs[u1] = fma(-l[u1], pv[NT], rhs[u1]);
      if (k == k1 && !idle[u1]) {
        inv[u1] = recip(a[u1][c1]);
        publish_row<(c1 & 1) * PS, c1 + 1, NT>(pbase, a[u1], rhs[u1], inv[u1]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    constexpr int skip = (LOOKAHEAD && c1 < NT) ? u1 : -1;
#pragma unroll
    for (int j = c + 1; j < NT; ++j) {
      const double vj = pv[j];
#pragma unroll
      for (int u = 0; u < RPL; ++u)
        if (u != skip) a[u][j] = fma(-l[u], vj, a[u][j]);
      if ((j - c) % kPivChunk == 0) __builtin_amdgcn_sched_barrier(0);
    }
    {
      const double pr = pv[NT];
#pragma unroll
      for (int u = 0; u < RPL; ++u)
        if (u != skip) rhs[u] = fma(-l[u], pr, rhs[u]);
    }
    if constexpr (!LOOKAHEAD && c1 < NT) {
      // every lane forms the reciprocal for its slot-u1 row (no divergent arithmetic); only the
      // lane holding row c + 1 keeps it and stores the row
      const double r1 = recip(a[u1][c1]);
      const bool mine = (k == k1) && !idle[u1];
      inv[u1] = mine ? r1 : inv[u1];
      __builtin_amdgcn_sched_barrier(0);
      if (mine) publish_row<(c1 & 1) * PS, c1 + 1, NT>(pbase, a[u1], rhs[u1], r1);
    }
    // every row's update of this column completes here: with static pivots only row c + 1 is
    // needed by the next column, and deferring the others (which the compiler otherwise does)
    // keeps pivot rows live across columns; the empty asm statements emit no instructions
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
#pragma unroll
      for (int j = c + 1; j < NT; ++j) asm volatile("" : "+v"(a[u][j]));
      asm volatile("" : "+v"(rhs[u]));
    }
    wave_sync();
  });
#pragma unroll
  for (int u = 0; u < RPL; ++u)
    if (!idle[u]) x[k + u * SEGW] = rhs[u] * inv[u];
  wave_sync();
}

// Reduced-precision static-pivot solve: the FP64-assembled block rows are rounded to FP32 and
// eliminated as seg_solve_sp does (FP32 rows, multipliers kept in place of the eliminated
// entries); then `refine` sweeps of iterative refinement: the residual r = b - A x is formed in
// FP64 from the FP64 block rows (re-assembled from the tables, not kept in registers) and the FP64
// solution x in LDS, and the correction is the FP32 elimination replayed on r.
template <class C, int D>
__device__ __forceinline__ void seg_solve_sp_f32r(const PlanTables& t, const RowsCtx<C>& cx, const BlockGeo<D>& bg,
                                         const double (&rhs64)[C::RPL], int refine, double* pivd, double* x) {
  constexpr int NT = C::NT, RPL = C::RPL, SEGW = C::SEGW;
  constexpr int PS = NT + 2;
  const int k = cx.k;
  float a[RPL][NT];
  {  // entry by entry: A0 + V_0 K_0 + ... in FP64 (the arithmetic of assemble_rows), then rounded
    const char* a0 = (const char*)t.A0 + (unsigned)bg.mask * (unsigned)(NT * NT * 8);
    const char* kt[D];
#pragma unroll
    for (int i = 0; i < D; ++i)
      kt[i] = (const char*)t.K + (unsigned)(i * 4 + ((bg.mask >> (2 * i)) & 3)) * (unsigned)(NT * NT * 8);
#pragma unroll
    for (int u = 0; u < RPL; ++u)
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        const unsigned o = cx.rb[u] + (unsigned)(l * 8);
        double e = *(const double*)(a0 + o);
#pragma unroll
        for (int i = 0; i < D; ++i) e = fma(bg.V0[i], *(const double*)(kt[i] + o), e);
        a[u][l] = (float)e;
        if (l % kLoadChunk == kLoadChunk - 1) __builtin_amdgcn_sched_barrier(0);
      }
  }
  float rhs[RPL], inv[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    rhs[u] = (float)rhs64[u];
    inv[u] = 0.0f;
  }
  float* piv = (float*)pivd;
  volatile __attribute__((address_space(3))) float* vpiv = (volatile __attribute__((address_space(3))) float*)piv;
  auto publish = [&](int off, int c, const float (&row)[NT], float r, float iv) {
#pragma unroll
    for (int j = 0; j < NT; ++j)
      if (j > c) vpiv[off + j] = row[j];
    vpiv[off + NT] = r;
    vpiv[off + NT + 1] = iv;
  };
  if (k == 0 && !cx.idle[0]) {
    inv[0] = recipf(a[0][0]);
    publish(0, 0, a[0], rhs[0], inv[0]);
  }
  wave_sync();
  static_for<0, NT>([&](auto CC) {
    constexpr int c = decltype(CC)::value;
    constexpr int uc = c / SEGW, kc = c % SEGW;
    constexpr int c1 = c + 1, u1 = c1 / SEGW, k1 = c1 % SEGW;
    const float* pv = piv + (c & 1) * PS;
    const float ip = pv[NT + 1];
    float l[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      l[u] = (cx.idle[u] || (u == uc && k == kc)) ? 0.0f : a[u][c] * ip;
      a[u][c] = (u == uc && k == kc) ? a[u][c] : l[u];  // the multiplier replaces the eliminated entry
    }
#pragma unroll
    for (int j = c + 1; j < NT; ++j) {
      const float vj = pv[j];
#pragma unroll
      for (int u = 0; u < RPL; ++u) a[u][j] = fmaf(-l[u], vj, a[u][j]);
    }
    {
      const float pr = pv[NT];
#pragma unroll
      for (int u = 0; u < RPL; ++u) rhs[u] = fmaf(-l[u], pr, rhs[u]);
    }
    if constexpr (c1 < NT) {
      const float r1 = recipf(a[u1][c1]);
      const bool mine = (k == k1) && !cx.idle[u1];
      inv[u1] = mine ? r1 : inv[u1];
      if (mine) publish((c1 & 1) * PS, c1, a[u1], rhs[u1], r1);
    }
    // the column completes here (see seg_solve_sp); the empty asm statements emit no instructions
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
#pragma unroll
      for (int j = c; j < NT; ++j) asm volatile("" : "+v"(a[u][j]));
      asm volatile("" : "+v"(rhs[u]));
    }
    wave_sync();
  });
#pragma unroll
  for (int u = 0; u < RPL; ++u)
    if (!cx.idle[u]) x[k + u * SEGW] = (double)(rhs[u] * inv[u]);
  wave_sync();
  for (int it = 0; it < refine; ++it) {
    // r = b - A x in FP64: the block rows are re-assembled entry by entry from the tables
    double res[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) res[u] = rhs64[u];
    {
      const char* a0 = (const char*)t.A0 + (unsigned)bg.mask * (unsigned)(NT * NT * 8);
      const char* kt[D];
#pragma unroll
      for (int i = 0; i < D; ++i)
        kt[i] = (const char*)t.K + (unsigned)(i * 4 + ((bg.mask >> (2 * i)) & 3)) * (unsigned)(NT * NT * 8);
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        const double xl = x[l];
#pragma unroll
        for (int u = 0; u < RPL; ++u) {
          const unsigned o = cx.rb[u] + (unsigned)(l * 8);
          double e = *(const double*)(a0 + o);
#pragma unroll
          for (int i = 0; i < D; ++i) e = fma(bg.V0[i], *(const double*)(kt[i] + o), e);
          res[u] = fma(-e, xl, res[u]);
        }
        if (l % kLoadChunk == kLoadChunk - 1) __builtin_amdgcn_sched_barrier(0);
      }
    }
    float r[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) r[u] = cx.idle[u] ? 0.0f : (float)res[u];
    // replay of the elimination on r (multipliers in a[u][c], pivot rows publish their value)
    static_for<0, NT>([&](auto CC) {
      constexpr int c = decltype(CC)::value;
      constexpr int uc = c / SEGW, kc = c % SEGW;
      if (k == kc && !cx.idle[uc]) vpiv[(c & 1) * PS] = r[uc];
      wave_sync();
      const float pvv = piv[(c & 1) * PS];
#pragma unroll
      for (int u = 0; u < RPL; ++u)
        if (!(u == uc && k == kc)) r[u] = fmaf(-a[u][c], pvv, r[u]);
#pragma unroll
      for (int u = 0; u < RPL; ++u) asm volatile("" : "+v"(r[u]));
    });
#pragma unroll
    for (int u = 0; u < RPL; ++u)
      if (!cx.idle[u]) x[k + u * SEGW] += (double)(r[u] * inv[u]);
    wave_sync();
  }
}

// The kernel body of the several-rows layouts. SOLVE: 0 = Gauss-Jordan with partial pivoting
// (seg_solve_nr), 1 = static pivots (seg_solve_sp), 2 = static pivots in FP32 with FP64 refinement.
// Table rows are addressed by 32-bit byte offsets and loaded kLoadChunk at a time (scheduling
// barriers), which keeps the loads in flight, and with them the registers, bounded.
template <int D, int M, int RPL, int SEGW, int SOLVE>
__device__ __forceinline__ void plans_rows_body(const DevGeom& g, double dt, const double* __restrict__ Q,
                                                double* __restrict__ W, const PlanTables& t,
                                                const PlanRec* __restrict__ plans, const int32_t* __restrict__ items,
                                                const int32_t* __restrict__ item_plan, int64_t n_items, int refine,
                                                double* s_w_wave, double* s_piv_wave) {
  using C = PlanCfgNR<D, M, RPL, SEGW>;
  constexpr int NT = C::NT, S = C::S, NB = C::NB, LB = C::LB;
  const int lane = threadIdx.x & 63;
  const bool tail = lane >= S * SEGW;
  const int seg = tail ? 0 : lane / SEGW;
  RowsCtx<C> cx;
  cx.k = tail ? lane - S * SEGW : lane % SEGW;
  const int k = cx.k;
#pragma unroll
  for (int u = 0; u < RPL; ++u) cx.idle[u] = tail || k + u * SEGW >= NT;
  const int wave = threadIdx.x >> 6;
  const int64_t wave_first = (xcd_block(blockIdx.x, gridDim.x) * C::WAVES + wave) * S;
  if (wave_first >= n_items) return;  // the list is padded to S
  int addr[LB > 0 ? LB : 1];
#pragma unroll
  for (int r = 0; r < LB; ++r) addr[r] = 4 * (tail ? lane : seg * SEGW + (k + (1 << r)) % SEGW);
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  int32_t e = items[wave_first + seg];
  const bool write = e >= 0 && !tail;
  if (e < 0) e = -e - 1;
  elem_idx(g, e, cx.base);
  const int pid = __builtin_amdgcn_readfirstlane(item_plan[wave_first]);
  const PlanRec* pr = plans + pid;
  const int nb = pr->nb;
  double* sw = s_w_wave + (size_t)seg * NB * NT;
  double* spiv = s_piv_wave + (size_t)seg * 2 * (NT + 2);
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int kr = cx.idle[u] ? 0 : k + u * SEGW;
    cx.rb[u] = (unsigned)kr * (unsigned)(NT * 8);
    cx.ccl[u] = t.cc_idx[kr];
    cx.ccv[u] = t.cc_val[kr];
  }
  for (int b = 0; b < nb; ++b) {
    const PlanBlock blk = pr->blk[b];
    const BlockGeo<D> bg = block_geo<D>(g, dt, blk, cx.base);
    double rhs[RPL];
    if constexpr (SOLVE == 2) {
      assemble_rhs<C, D>(g, Q, t, cx, bg, blk, sw, nel, rhs);
      seg_solve_sp_f32r<C, D>(t, cx, bg, rhs, refine, spiv, sw + b * NT);
    } else {
      double a[RPL][NT];
      assemble_rows<C, D>(t, cx, bg, a);
      assemble_rhs<C, D>(g, Q, t, cx, bg, blk, sw, nel, rhs);
      if constexpr (SOLVE == 1)
        seg_solve_sp<C, RIDG_SP_LOOKAHEAD>(a, rhs, k, cx.idle, spiv, sw + b * NT);
      else
        seg_solve_nr<C>(a, rhs, k, cx.idle, addr, spiv, sw + b * NT);
    }
  }
  if (write) {
#pragma unroll
    for (int u = 0; u < RPL; ++u)
      if (!cx.idle[u]) W[(int64_t)(k + u * SEGW) * nel + e] = sw[(nb - 1) * NT + k + u * SEGW];
  }
}

// Several rows per lane (PlanCfgNR), partial pivoting: RPL rows of a region's block system in each
// lane of a SEGW-lane segment, each pivot row read once for RPL rows. FP64; bitwise the results of
// the packed layout.
template <int D, int M, int RPL, int SEGW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PlanCfgNR<D, M, RPL, SEGW>::MIN_WAVES))) void
predict_plans_nr_kernel(DevGeom g, double dt, const double* __restrict__ Q, double* __restrict__ W, PlanTables t,
                        const PlanRec* __restrict__ plans, const int32_t* __restrict__ items,
                        const int32_t* __restrict__ item_plan, int64_t n_items) {
  using C = PlanCfgNR<D, M, RPL, SEGW>;
  __shared__ double s_w[C::WAVES][C::S][C::NB][C::NT];
  __shared__ double s_piv[C::WAVES][C::S][2 * (C::NT + 2)];
  const int wave = threadIdx.x >> 6;
  plans_rows_body<D, M, RPL, SEGW, 0>(g, dt, Q, W, t, plans, items, item_plan, n_items, 0, &s_w[wave][0][0][0],
                                      &s_piv[wave][0][0]);
}

// Static pivots (layout 5): FP64 (F32 = false) or FP32 with `refine` FP64-residual sweeps. The FP64
// kernel takes the geometry's register budget hint; the FP32 one, which also holds the refinement's
// FP64 rows, keeps the compiler's choice (capped at three wavefronts it spills heavily).
template <int D, int M, int RPL, int SEGW, bool F32>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(F32 ? 1 : PlanCfgNR<D, M, RPL, SEGW>::MIN_WAVES))) void predict_plans_sp_kernel(DevGeom g, double dt, const double* __restrict__ Q,
                                                               double* __restrict__ W, PlanTables t,
                                                               const PlanRec* __restrict__ plans,
                                                               const int32_t* __restrict__ items,
                                                               const int32_t* __restrict__ item_plan, int64_t n_items,
                                                               int refine) {
  using C = PlanCfgNR<D, M, RPL, SEGW>;
  __shared__ double s_w[C::WAVES][C::S][C::NB][C::NT];
  __shared__ double s_piv[C::WAVES][C::S][2 * (C::NT + 2)];
  const int wave = threadIdx.x >> 6;
  plans_rows_body<D, M, RPL, SEGW, F32 ? 2 : 1>(g, dt, Q, W, t, plans, items, item_plan, n_items, refine,
                                                &s_w[wave][0][0][0], &s_piv[wave][0][0]);
}

template <class C, int D, int M>
static int launch_nr(const DevGeom& g, double dt, const double* Q, double* W, const PlanTables& t,
                     const PlanRec* plans, const int32_t* items, const int32_t* item_plan, int64_t n_items,
                     void* stream) {
  if (n_items % C::S) return (int)hipErrorInvalidValue;  // the list is padded to whole wavefronts
  const int64_t per_block = (int64_t)C::WAVES * C::S;
  const int64_t blocks = (n_items + per_block - 1) / per_block;
  if (blocks == 0) return 0;
  hipLaunchKernelGGL((predict_plans_nr_kernel<D, M, C::RPL, C::SEGW>), dim3((unsigned)blocks), dim3(64 * C::WAVES),
                     0, (hipStream_t)stream, g, dt, Q, W, t, plans, items, item_plan, n_items);
  return (int)hipGetLastError();
}

}  // namespace ridg

// HIP kernels of libridg for gfx950 (MI355X): the RIDG prediction (Sec. 2.2 of
// arXiv 2101.01231) and correction (Sec. 2.3) on a periodic Cartesian mesh.
//
// State and prediction arrays are coefficient-major in HBM (Q[k * nel + e],
// W[k * nel + e]) so that neighbouring threads/elements read neighbouring
// addresses. Element e = i0 + n0 (i1 + n1 i2).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>

#include "ridg_internal.hpp"

namespace ridg {

// ---------------------------------------------------------------- sizes
__host__ __device__ constexpr int binom(int n, int k) {
  int r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}
__host__ __device__ constexpr int n_space(int D, int M) { return binom(M - 1 + D, D); }
__host__ __device__ constexpr int n_spacetime(int D, int M) { return binom(M + D, D + 1); }
__host__ __device__ constexpr int pow3(int D) { return D == 1 ? 3 : (D == 2 ? 9 : 27); }
__host__ __device__ constexpr int seg_width(int nt) {
  return nt <= 1 ? 1 : nt <= 2 ? 2 : nt <= 4 ? 4 : nt <= 8 ? 8 : nt <= 16 ? 16 : nt <= 32 ? 32 : 64;
}

// ---------------------------------------------------------------- geometry helpers
__device__ inline void elem_idx(const DevGeom& g, int64_t e, int idx[3]) {
  idx[0] = (int)(e % g.n0);
  int64_t r = e / g.n0;
  idx[1] = (int)(r % g.n1);
  idx[2] = (int)(r / g.n1);
}

__device__ inline int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ inline int64_t elem_lin(const DevGeom& g, int i0, int i1, int i2) {
  return (int64_t)wrap(i0, g.n0) + (int64_t)g.n0 * ((int64_t)wrap(i1, g.n1) + (int64_t)g.n1 * wrap(i2, g.n2));
}

__device__ inline double geom_h(const DevGeom& g, int i) { return i == 0 ? g.h0 : (i == 1 ? g.h1 : g.h2); }

// nu_i(xi) = c0[i] + sum_j c[i][j] xi_j; projected on p-modes {1, psi_1(xi_j)}: V[i][0] = c0, V[i][1+j] = c_ij / sqrt3
template <int D>
__device__ inline void vel_modes(const DevGeom& g, const int idx[3], double dt, double V[D][D + 1]) {
  const double inv_sqrt3 = 0.57735026918962576451;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double v = g.a[i];
#pragma unroll
    for (int j = 0; j < D; ++j) v += g.g[i][j] * ((idx[j] + 0.5) * geom_h(g, j));
    const double hi = geom_h(g, i);
    V[i][0] = v * dt / hi;
#pragma unroll
    for (int j = 0; j < D; ++j) V[i][1 + j] = g.g[i][j] * (0.5 * geom_h(g, j)) * dt / hi * inv_sqrt3;
  }
}

// upwind side of face (i, s): 0 own trace, 1 neighbour trace (same rule as the host plans)
template <int D>
__device__ inline int face_side(const DevGeom& g, const int idx[3], int i, int s) {
  double v = g.a[i], spread = 0.0;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    v += g.g[i][j] * ((idx[j] + 0.5) * geom_h(g, j));
    spread += fabs(g.g[i][j] * (0.5 * geom_h(g, j)));
  }
  const double hi = geom_h(g, i);
  const double c0 = v / hi;
  spread /= hi;
  const double tol = 1e-12 * (fabs(c0) + spread);
  return (s * c0 - spread >= -tol) ? 0 : 1;
}

// element i of a small register array without dynamic indexing (a select chain)
template <int D>
__device__ inline double sel(const double (&v)[D], int i) {
  double r = v[0];
#pragma unroll
  for (int j = 1; j < D; ++j) r = (i == j) ? v[j] : r;
  return r;
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------- layout transposes
__global__ void aos_to_soa_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t nel, int nm) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nel * nm) return;
  int64_t e = t / nm;
  int k = (int)(t % nm);
  dst[(int64_t)k * nel + e] = src[t];
}

__global__ void soa_to_aos_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t nel, int nm) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nel * nm) return;
  int64_t e = t / nm;
  int k = (int)(t % nm);
  dst[t] = src[(int64_t)k * nel + e];
}

__global__ void check_finite_kernel(const double* __restrict__ x, int64_t n, int32_t* flag) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n && !isfinite(x[t])) flag[0] = 1;
}

// ---------------------------------------------------------------- prefactored prediction
// Constant velocity: W_e = sum_tap G_tap Q_{e + off_tap} (Sec. 2.2 system solved once on the host).
struct Taps {
  int8_t off[kMaxBlocks][3];
};

template <int D, int M>
__global__ __launch_bounds__(256) void predict_prefactored_kernel(DevGeom g, const double* __restrict__ Q,
                                                                  double* __restrict__ W,
                                                                  const double* __restrict__ G, Taps taps,
                                                                  int ntaps) {
  constexpr int NS = n_space(D, M), NT = n_spacetime(D, M);
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nel) return;
  int idx[3];
  elem_idx(g, e, idx);
  double w[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) w[k] = 0.0;
  for (int t = 0; t < ntaps; ++t) {
    const int64_t src = elem_lin(g, idx[0] + taps.off[t][0], idx[1] + taps.off[t][1], idx[2] + taps.off[t][2]);
    double q[NS];
#pragma unroll
    for (int l = 0; l < NS; ++l) q[l] = Q[(int64_t)l * nel + src];
    const double* Gt = G + (size_t)t * NT * NS;
#pragma unroll
    for (int k = 0; k < NT; ++k)
#pragma unroll
      for (int l = 0; l < NS; ++l) w[k] = fma(Gt[k * NS + l], q[l], w[k]);
  }
#pragma unroll
  for (int k = 0; k < NT; ++k) W[(int64_t)k * nel + e] = w[k];
}

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

// ---------------------------------------------------------------- region solve by upwind plans
// A wavefront holds S = floor(64 / theta_T) segments of theta_T consecutive lanes, one region per
// segment; lane k of a segment owns row k of each block system. Blocks are solved in the plan's
// topological order: the diagonal block (time term - internal flux + own-trace faces, assembled
// from precombined exact tensors and the projected velocity, Sec. 3) is eliminated with partial
// pivoting, the pivot row being found by a segment-wide argmax over lanes; inflow faces inside
// the region move the upwind neighbour's already-solved W to the right-hand side.
template <int D, int M, bool PADDED = false>
struct PlanCfg {
  static constexpr int NS = n_space(D, M);
  static constexpr int NT = n_spacetime(D, M);
  // segment width: theta_T lanes (packed) or the next power of two (padded, DPP reductions)
  static constexpr int SEGW = PADDED ? seg_width(NT) : NT;
  static constexpr int S = SEGW <= 64 ? 64 / SEGW : 1;      // segments (regions) per wavefront
  static constexpr bool POW2 = (SEGW & (SEGW - 1)) == 0;     // segments align with DPP rows
  static constexpr int LB = SEGW <= 1 ? 0 : SEGW <= 2 ? 1 : SEGW <= 4 ? 2 : SEGW <= 8 ? 3 : SEGW <= 16 ? 4 : SEGW <= 32 ? 5 : 6;
  static constexpr int NB = D == 3 ? 8 : pow3(D);            // plan blocks (larger plans use the dense path)
  static constexpr int WAVES = 4;
};

// Segment-wide maximum of a 32-bit key (every lane of the segment ends with it).
// Power-of-two segments: butterfly of DPP lane permutations inside 16-lane rows, a swizzle (xor 16)
// inside 32 lanes and readlane across the two halves of a 64-lane segment.
template <int CTRL>
__device__ inline unsigned dpp_mov(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}

template <int SEG>
__device__ inline unsigned seg_max_pow2(unsigned key) {
  if (SEG > 1) key = max(key, dpp_mov<0xB1>(key));   // quad_perm [1,0,3,2]
  if (SEG > 2) key = max(key, dpp_mov<0x4E>(key));   // quad_perm [2,3,0,1]
  if (SEG > 4) key = max(key, dpp_mov<0x141>(key));  // row_half_mirror
  if (SEG > 8) key = max(key, dpp_mov<0x140>(key));  // row_mirror
  if (SEG > 16) key = max(key, (unsigned)__builtin_amdgcn_ds_swizzle((int)key, 0x401F));  // xor 16
  if (SEG > 32) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)key, 0);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)key, 32);
    key = max(lo, hi);
  }
  return key;
}

// Other segment widths: log2 rounds of a cyclic rotation inside the segment (ds_bpermute); after
// round r every lane holds the maximum over 2^r consecutive lanes of its segment.
template <int NT, int LB>
__device__ inline unsigned seg_max_rot(unsigned key, const int (&addr)[LB > 0 ? LB : 1]) {
#pragma unroll
  for (int r = 0; r < LB; ++r) key = max(key, (unsigned)__builtin_amdgcn_ds_bpermute(addr[r], (int)key));
  return key;
}

// 1/x to full FP64 precision: hardware reciprocal estimate and two Newton steps.
__device__ inline double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Gauss-Jordan elimination with partial pivoting of [A | b], row k of A in lane k of the segment.
// The pivot of column c is the unused row of largest |a_c|, compared on a 32-bit key (the FP32
// image of |a_c| with its low bits replaced by the row, ties to the lowest row). The pivot row,
// its right-hand side and 1/pivot are published to LDS (two alternating buffers, so one wave-level
// sync per column suffices) and every other row, earlier pivot rows included, is reduced by it.
// After the last column, pivot row p_c holds x_c = rhs / a_c, written to x[c] (LDS).
template <int NT, int LB, bool POW2, int SEGW = NT>
__device__ inline void seg_solve(double (&a)[NT], double& rhs, int k, bool idle, const int (&addr)[LB > 0 ? LB : 1],
                                 double* piv, double* x) {
  constexpr unsigned LMASK = (1u << LB) - 1u;
  constexpr int PS = NT + 2;  // published row: a[c+1..NT-1], rhs, 1/pivot
  bool used = idle;
  int mystep = -1;
  double myinv = 0.0;
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    double* pv = piv + (c & 1) * PS;
    unsigned key = 0u;
    if (!used) key = (__float_as_uint((float)fabs(a[c])) & ~LMASK) | (LMASK - (unsigned)k);
    if constexpr (POW2)
      key = seg_max_pow2<SEGW>(key);
    else
      key = seg_max_rot<SEGW, LB>(key, addr);
    const int p = (int)(LMASK - (key & LMASK));
    const bool is_piv = (k == p) && !idle;
    if (is_piv) {
      myinv = recip(a[c]);
      // one 64-bit store per value: lets the register allocator keep a[] in place
      volatile __attribute__((address_space(3))) double* vp = (volatile __attribute__((address_space(3))) double*)pv;
#pragma unroll
      for (int j = c + 1; j < NT; ++j) vp[j] = a[j];
      vp[NT] = rhs;
      vp[NT + 1] = myinv;
      used = true;
      mystep = c;
    }
    wave_sync();
    if (!is_piv && !idle) {
      const double l = a[c] * pv[NT + 1];
#pragma unroll
      for (int j = c + 1; j < NT; ++j) a[j] = fma(-l, pv[j], a[j]);
      rhs = fma(-l, pv[NT], rhs);
    }
  }
  if (mystep >= 0) x[mystep] = rhs * myinv;
  wave_sync();
}

// Reduced-precision variant: Gauss-Jordan with partial pivoting in FP32 on the FP32 image of the
// FP64-assembled block, then `refine` sweeps of iterative refinement: the residual r = b - A x is
// formed in FP64 from the FP64 row, and the correction is obtained by replaying the FP32
// elimination (stored multipliers, same pivot order) on r. x is kept in FP64.
template <int NT, int LB, bool POW2, int SEGW>
__device__ inline void seg_solve_f32r(const double (&a64)[NT], double rhs64, int refine, int k, bool idle,
                                      const int (&addr)[LB > 0 ? LB : 1], double* pivbuf, double* x) {
  constexpr unsigned LMASK = (1u << LB) - 1u;
  constexpr int PS = NT + 2;
  float a[NT], lm[NT];
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    a[l] = (float)a64[l];
    lm[l] = 0.0f;
  }
  float r = (float)rhs64;
  bool used = idle;
  int mystep = -1;
  float myinv = 0.0f;
  float* pbase = (float*)pivbuf;
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    float* pv = pbase + (c & 1) * PS;
    unsigned key = 0u;
    if (!used) key = (__float_as_uint(fabsf(a[c])) & ~LMASK) | (LMASK - (unsigned)k);
    if constexpr (POW2)
      key = seg_max_pow2<SEGW>(key);
    else
      key = seg_max_rot<SEGW, LB>(key, addr);
    const int p = (int)(LMASK - (key & LMASK));
    const bool is_piv = (k == p) && !idle;
    if (is_piv) {
      myinv = 1.0f / a[c];
      volatile __attribute__((address_space(3))) float* vp = (volatile __attribute__((address_space(3))) float*)pv;
#pragma unroll
      for (int j = c + 1; j < NT; ++j) vp[j] = a[j];
      vp[NT] = r;
      vp[NT + 1] = myinv;
      used = true;
      mystep = c;
    }
    wave_sync();
    if (!is_piv && !idle) {
      const float l = a[c] * pv[NT + 1];
      lm[c] = l;
#pragma unroll
      for (int j = c + 1; j < NT; ++j) a[j] = fmaf(-l, pv[j], a[j]);
      r = fmaf(-l, pv[NT], r);
    }
  }
  if (mystep >= 0) x[mystep] = (double)(r * myinv);
  wave_sync();
  for (int it = 0; it < refine; ++it) {
    double res = rhs64;
#pragma unroll
    for (int l = 0; l < NT; ++l) res = fma(-a64[l], x[l], res);
    float rr = idle ? 0.0f : (float)res;
#pragma unroll
    for (int c = 0; c < NT; ++c) {
      float* pv = pbase + (c & 1) * PS;
      if (mystep == c) pv[0] = rr;
      wave_sync();
      rr = fmaf(-lm[c], pv[0], rr);  // lm[c] = 0 on the pivot row of column c and on idle lanes
    }
    wave_sync();
    if (mystep >= 0) x[mystep] += (double)(rr * myinv);
    wave_sync();
  }
}

template <int D, int M, bool PADDED, bool F32 = false>
__global__ __launch_bounds__(256) void predict_plans_kernel(DevGeom g, double dt, const double* __restrict__ Q,
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
  const int64_t wave_first = ((int64_t)blockIdx.x * C::WAVES + wave) * S;
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

// ---------------------------------------------------------------- cyclic regions by tearing
// Regions whose centre lies on a dependency cycle (around a point where the flow circulates) are
// solved on the same block structure: block 0 of the plan is a tear block whose unknowns x break
// every cycle. The other ancestor blocks are eliminated in upwind order with 1 + theta_T
// right-hand sides, giving W_r = alpha_r + B_r x; the tear block's own equations then form one
// theta_T x theta_T system for x, and W_centre = alpha_c + B_c x. This solves exactly the region
// system of eq. (pred_full_system) restricted to the centre's ancestors.
template <int NT, int LB, bool POW2, int R>
__device__ inline void seg_solve_multi(double (&a)[NT], double (&rhs)[R], int k, bool idle,
                                       const int (&addr)[LB > 0 ? LB : 1], double* piv, double* x) {
  constexpr unsigned LMASK = (1u << LB) - 1u;
  bool used = idle;
  int mystep = -1;
  double myinv = 0.0;
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    unsigned key = 0u;
    if (!used) key = (__float_as_uint((float)fabs(a[c])) & ~LMASK) | (LMASK - (unsigned)k);
    if constexpr (POW2)
      key = seg_max_pow2<(NT > 1 ? NT : 1)>(key);
    else
      key = seg_max_rot<NT, LB>(key, addr);
    const int p = (int)(LMASK - (key & LMASK));
    if (k == p && !idle) {
      myinv = recip(a[c]);
#pragma unroll
      for (int j = c + 1; j < NT; ++j) piv[j] = a[j];
#pragma unroll
      for (int j = 0; j < R; ++j) piv[NT + j] = rhs[j];
      piv[NT + R] = myinv;
      used = true;
      mystep = c;
    }
    wave_sync();
    if (!used) {
      const double l = a[c] * piv[NT + R];
#pragma unroll
      for (int j = c + 1; j < NT; ++j) a[j] = fma(-l, piv[j], a[j]);
#pragma unroll
      for (int j = 0; j < R; ++j) rhs[j] = fma(-l, piv[NT + j], rhs[j]);
    }
    wave_sync();
  }
#pragma unroll 1
  for (int c = NT - 1; c >= 0; --c) {
    if (mystep == c)
#pragma unroll
      for (int j = 0; j < R; ++j) x[c * R + j] = rhs[j] * myinv;
    wave_sync();
    if (mystep >= 0 && mystep < c) {
      double ac = a[0];
#pragma unroll
      for (int q = 1; q < NT; ++q) ac = (q == c) ? a[q] : ac;
#pragma unroll
      for (int j = 0; j < R; ++j) rhs[j] = fma(-ac, x[c * R + j], rhs[j]);
    }
  }
  wave_sync();
}

template <int D, int M>
__global__ __launch_bounds__(64) void predict_tear_kernel(DevGeom g, double dt, const double* __restrict__ Q,
                                                          double* __restrict__ W, PlanTables t,
                                                          const PlanRec* __restrict__ plans,
                                                          const int32_t* __restrict__ elems, int64_t n_elems) {
  using C = PlanCfg<D, M>;
  if constexpr (C::NT <= 64) {
  constexpr int NT = C::NT, NB = C::NB, LB = C::LB, R = 1 + NT;
  __shared__ double s_w[NB][NT][R];  // [alpha | B] of every eliminated block
  __shared__ double s_piv[2 * (NT + R + 1)];
  __shared__ double s_x[NT];
  const int64_t item = blockIdx.x;
  if (item >= n_elems) return;
  const int lane = threadIdx.x & 63;
  const bool idle = lane >= NT;
  const int k = idle ? 0 : lane;
  int addr[LB > 0 ? LB : 1];
#pragma unroll
  for (int r = 0; r < LB; ++r) addr[r] = 4 * (idle ? lane : (k + (1 << r)) % NT);
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  const int32_t e = elems[item];
  int base[3];
  elem_idx(g, e, base);
  const PlanRec* pr = plans + item;
  const int nb = pr->nb;
  const int centre = pr->pad[1];
  const int ccl = t.cc_idx[k];
  const double ccv = t.cc_val[k];
  // blocks in elimination order; block 0 (the tear block) last
  for (int bb = 1; bb <= nb; ++bb) {
    const int b = bb < nb ? bb : 0;
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
    double a[NT];
    {
      const double* a0 = t.A0 + ((size_t)mask * NT + k) * NT;
#pragma unroll
      for (int l = 0; l < NT; ++l) a[l] = a0[l];
    }
#pragma unroll 1
    for (int i = 0; i < D; ++i) {
      const double vi = sel<D>(V0, i);
      const double* kk = t.K + (((size_t)i * 4 + ((mask >> (2 * i)) & 3)) * NT + k) * NT;
#pragma unroll
      for (int l = 0; l < NT; ++l) a[l] = fma(vi, kk[l], a[l]);
    }
    double rhs[R];
#pragma unroll
    for (int j = 0; j < R; ++j) rhs[j] = 0.0;
    rhs[0] = ccv * Q[(int64_t)ccl * nel + ge];
#pragma unroll 1
    for (int i = 0; i < D; ++i) {
      const double vi = sel<D>(V0, i);
#pragma unroll 1
      for (int sd = 0; sd < 2; ++sd) {
        const int src = blk.src[2 * i + sd];
        if (src == kOwn) continue;
        const double* f0 = t.Fn0 + (((size_t)i * 2 + sd) * NT + k) * NT;
        const double* fc = t.FnC + (((size_t)i * 2 + sd) * NT + k) * NT;
        if (src == 0) {  // coupling to the tear unknowns: -A_{b,0} x
#pragma unroll
          for (int l = 0; l < NT; ++l) rhs[1 + l] -= fma(vi, f0[l], fc[l]);
        } else if (b != 0) {  // -A_{b,s} (alpha_s + B_s x)
#pragma unroll 1
          for (int l = 0; l < NT; ++l) {
            const double cl = fma(vi, f0[l], fc[l]);
#pragma unroll
            for (int j = 0; j < R; ++j) rhs[j] = fma(-cl, s_w[src][l][j], rhs[j]);
          }
        } else {  // tear equation: A_00 x + A_{0,s} (alpha_s + B_s x) = b_0
#pragma unroll 1
          for (int l = 0; l < NT; ++l) {
            const double cl = fma(vi, f0[l], fc[l]);
            rhs[0] = fma(-cl, s_w[src][l][0], rhs[0]);
#pragma unroll
            for (int j = 0; j < NT; ++j) a[j] = fma(cl, s_w[src][l][1 + j], a[j]);
          }
        }
      }
    }
    if (b != 0) {
      seg_solve_multi<NT, LB, C::POW2, R>(a, rhs, k, idle, addr, s_piv, &s_w[b][0][0]);
    } else {
      double r0 = rhs[0];
      seg_solve<NT, LB, C::POW2>(a, r0, k, idle, addr, s_piv, s_x);
    }
  }
  if (!idle) {
    double w;
    if (centre == 0) {
      w = s_x[k];
    } else {
      w = s_w[centre][k][0];
#pragma unroll
      for (int j = 0; j < NT; ++j) w = fma(s_w[centre][k][1 + j], s_x[j], w);
    }
    W[(int64_t)k * nel + e] = w;
  }
  }  // theta_T <= 64
}

// ---------------------------------------------------------------- dense region solve
// One workgroup per region: the whole 3^d theta_T system (eq. pred_full_system) assembled in a
// scratch matrix and solved by Gaussian elimination with partial pivoting.
template <int D, int M, int THREADS>
__global__ __launch_bounds__(THREADS) void predict_dense_kernel(DevGeom g, double dt, const double* __restrict__ Q,
                                                            double* __restrict__ W, DevTensors t,
                                                            const int32_t* __restrict__ elems,
                                                            int64_t first, int64_t count,
                                                            double* __restrict__ scratch) {
  constexpr int NS = n_space(D, M), NT = n_spacetime(D, M), NP = D + 1, NB = pow3(D);
  constexpr int N = NB * NT, LD = N + 1;
  const int64_t slot = blockIdx.x;
  if (first + slot >= count) return;
  const int32_t e = elems[first + slot];
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  double* A = scratch + (size_t)slot * N * LD;  // [N][N+1]: matrix | rhs
  __shared__ int s_red_i[THREADS / 64];
  __shared__ double s_x[N];
  __shared__ double s_l[N];
  __shared__ double s_piv[LD];
  int base[3];
  elem_idx(g, e, base);
  for (int R = threadIdx.x; R < N; R += blockDim.x) {
    const int r = R / NT, k = R % NT;
    int o[3] = {0, 0, 0};
    {
      int c = r;
      for (int i = D - 1; i >= 0; --i) {
        o[i] = c % 3 - 1;
        c /= 3;
      }
    }
    int gi[3] = {wrap(base[0] + o[0], g.n0), wrap(base[1] + o[1], g.n1), wrap(base[2] + o[2], g.n2)};
    const int64_t ge = (int64_t)gi[0] + (int64_t)g.n0 * ((int64_t)gi[1] + (int64_t)g.n1 * gi[2]);
    double V[D][D + 1];
    vel_modes<D>(g, gi, dt, V);
    double* row = A + (size_t)R * LD;
    for (int j = 0; j < N; ++j) row[j] = 0.0;
    double* diag = row + r * NT;
    for (int l = 0; l < NT; ++l) diag[l] = t.Tt[k * NT + l];
    for (int i = 0; i < D; ++i) {
      for (int p = 0; p < NP; ++p) {
        if (p == 1 + i || V[i][p] == 0.0) continue;
        const double* bv = t.Bv + (((size_t)i * NP + p) * NT + k) * NT;
        for (int l = 0; l < NT; ++l) diag[l] = fma(-V[i][p], bv[l], diag[l]);
      }
      for (int sd = 0; sd < 2; ++sd) {
        const int s = sd ? 1 : -1;
        int o2 = o[i] + s;
        const bool boundary = (o2 < -1 || o2 > 1);
        const int side = boundary ? 0 : face_side<D>(g, gi, i, s);
        double* dst = diag;
        const double* tens = t.Fo;
        if (side == 1) {
          int oo[3] = {o[0], o[1], o[2]};
          oo[i] = o2;
          int q = 0;
          for (int m = 0; m < D; ++m) q = q * 3 + (oo[m] + 1);
          dst = row + q * NT;
          tens = t.Fn;
        }
        for (int p = 0; p < NP; ++p) {
          if (p == 1 + i || V[i][p] == 0.0) continue;
          const double* f = tens + ((((size_t)i * 2 + sd) * NP + p) * NT + k) * NT;
          for (int l = 0; l < NT; ++l) dst[l] = fma(V[i][p], f[l], dst[l]);
        }
      }
    }
    double rhs = 0.0;
    for (int l = 0; l < NS; ++l) rhs = fma(t.Cc[k * NS + l], Q[(int64_t)l * nel + ge], rhs);
    row[N] = rhs;
  }
  __syncthreads();
  // Gaussian elimination with partial pivoting on [A | b]. Pivot: the row of largest |A[r][c]|,
  // compared on a 32-bit key (FP32 image of |A[r][c]| with the low bits replaced by the row,
  // ties to the lowest row) reduced within each wavefront by DPP and across wavefronts in LDS.
  // The pivot row and the column of multipliers are staged in LDS for the rank-1 update.
  constexpr unsigned RB = N <= 256 ? 8 : (N <= 512 ? 9 : (N <= 1024 ? 10 : 11));
  constexpr unsigned RMASK = (1u << RB) - 1u;
  const int nwaves = blockDim.x >> 6;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int c = 0; c < N; ++c) {
    unsigned key = 0u;
    for (int R = c + threadIdx.x; R < N; R += blockDim.x) {
      const unsigned kk = (__float_as_uint((float)fabs(A[(size_t)R * LD + c])) & ~RMASK) | (RMASK - (unsigned)R);
      key = max(key, kk);
    }
    key = seg_max_pow2<64>(key);
    if (lane == 0) s_red_i[wid] = (int)key;
    __syncthreads();
    unsigned best = 0u;
    for (int w = 0; w < nwaves; ++w) best = max(best, (unsigned)s_red_i[w]);
    const int p = (int)(RMASK - (best & RMASK));
    // swap rows c and p (columns c..N) and stage the pivot row
    for (int j = c + threadIdx.x; j < LD; j += blockDim.x) {
      const double vc = A[(size_t)c * LD + j], vp = A[(size_t)p * LD + j];
      if (p != c) {
        A[(size_t)c * LD + j] = vp;
        A[(size_t)p * LD + j] = vc;
      }
      s_piv[j] = vp;
    }
    __syncthreads();
    const double inv = 1.0 / s_piv[c];
    for (int R = c + 1 + threadIdx.x; R < N; R += blockDim.x) s_l[R] = A[(size_t)R * LD + c] * inv;
    __syncthreads();
    const int rows = N - c - 1, cols = LD - c - 1;
    for (int q = threadIdx.x; q < rows * cols; q += blockDim.x) {
      const int R = c + 1 + q / cols, j = c + 1 + q % cols;
      A[(size_t)R * LD + j] = fma(-s_l[R], s_piv[j], A[(size_t)R * LD + j]);
    }
    __syncthreads();
  }
  // back substitution
  for (int c = N - 1; c >= 0; --c) {
    if (threadIdx.x == 0) s_x[c] = A[(size_t)c * LD + N] / A[(size_t)c * LD + c];
    __syncthreads();
    const double xc = s_x[c];
    for (int R = threadIdx.x; R < c; R += blockDim.x) A[(size_t)R * LD + N] = fma(-A[(size_t)R * LD + c], xc, A[(size_t)R * LD + N]);
    __syncthreads();
  }
  const int centre = (NB - 1) / 2;
  for (int k = threadIdx.x; k < NT; k += blockDim.x) W[(int64_t)k * nel + e] = s_x[centre * NT + k];
}

// ---------------------------------------------------------------- dispatch
template <template <int, int> class F, typename... Args>
static int dispatch_dm(int d, int M, Args... args) {
#define RIDG_CASE(DD, MM) \
  if (d == DD && M == MM) return F<DD, MM>::run(args...);
  RIDG_CASE(1, 1) RIDG_CASE(1, 2) RIDG_CASE(1, 3) RIDG_CASE(1, 4) RIDG_CASE(1, 5)
  RIDG_CASE(2, 1) RIDG_CASE(2, 2) RIDG_CASE(2, 3) RIDG_CASE(2, 4) RIDG_CASE(2, 5)
  RIDG_CASE(3, 1) RIDG_CASE(3, 2) RIDG_CASE(3, 3) RIDG_CASE(3, 4) RIDG_CASE(3, 5)
#undef RIDG_CASE
  return (int)hipErrorInvalidValue;
}

static inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

int launch_aos_to_soa(const double* src, double* dst, int64_t nel, int nmodes, void* stream) {
  int64_t n = nel * nmodes;
  if (n == 0) return 0;
  hipLaunchKernelGGL(aos_to_soa_kernel, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, src, dst, nel, nmodes);
  return (int)hipGetLastError();
}

int launch_soa_to_aos(const double* src, double* dst, int64_t nel, int nmodes, void* stream) {
  int64_t n = nel * nmodes;
  if (n == 0) return 0;
  hipLaunchKernelGGL(soa_to_aos_kernel, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, src, dst, nel, nmodes);
  return (int)hipGetLastError();
}

int launch_check_finite(const double* x, int64_t n, int32_t* flag, void* stream) {
  if (n == 0) return 0;
  hipLaunchKernelGGL(check_finite_kernel, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream, x, n, flag);
  return (int)hipGetLastError();
}

template <int D, int M>
struct PrefactoredL {
  static int run(const DevGeom& g, const double* Q, double* W, const double* G, const int32_t* taps, int ntaps,
                 void* stream) {
    Taps tp;
    for (int t = 0; t < kMaxBlocks; ++t)
      for (int i = 0; i < 3; ++i) tp.off[t][i] = (t < ntaps) ? (int8_t)taps[3 * t + i] : 0;
    const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
    hipLaunchKernelGGL((predict_prefactored_kernel<D, M>), dim3(grid_for(nel, 256)), dim3(256), 0,
                       (hipStream_t)stream, g, Q, W, G, tp, ntaps);
    return (int)hipGetLastError();
  }
};

int launch_predict_prefactored(int d, int M, const DevGeom& g, const double* Q, double* W, const double* G,
                               const int32_t* taps, int ntaps, void* stream) {
  return dispatch_dm<PrefactoredL>(d, M, g, Q, W, G, taps, ntaps, stream);
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

// Segment layout of the plan kernel: packed theta_T-lane segments (default) or power-of-two
// segments with DPP reductions (RIDG_PLAN_PADDED=1), chosen once per process.
static bool plan_padded() {
  static bool v = [] {
    const char* e = getenv("RIDG_PLAN_PADDED");
    return e && atoi(e) == 1;
  }();
  return v;
}

template <int D, int M>
struct IpwL {
  static int run() { return plan_padded() ? PlanCfg<D, M, true>::S : PlanCfg<D, M, false>::S; }
};
int items_per_wave(int d, int M) { return dispatch_dm<IpwL>(d, M); }

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
  static int run(int precision, int refine, const DevGeom& g, double dt, const double* Q, double* W,
                 const PlanTables& t, const PlanRec* plans, const int32_t* items, const int32_t* item_plan,
                 int64_t n_items, void* stream) {
    if (n_spacetime(D, M) > 64) return (int)hipErrorInvalidValue;
    if (plan_padded())
      return launch_plans<D, M, true>(precision, refine, g, dt, Q, W, t, plans, items, item_plan, n_items, stream);
    return launch_plans<D, M, false>(precision, refine, g, dt, Q, W, t, plans, items, item_plan, n_items, stream);
  }
};

int launch_predict_plans(int d, int M, int precision, int refine, const DevGeom& g, double dt, const double* Q,
                         double* W, const PlanTables& t, const PlanRec* plans, const int32_t* items,
                         const int32_t* item_plan, int64_t n_items, void* stream) {
  return dispatch_dm<PlansL>(d, M, precision, refine, g, dt, Q, W, t, plans, items, item_plan, n_items, stream);
}

template <int D, int M>
struct TearL {
  static int run(const DevGeom& g, double dt, const double* Q, double* W, const PlanTables& t, const PlanRec* plans,
                 const int32_t* elems, int64_t n_elems, void* stream) {
    if (n_spacetime(D, M) > 64) return (int)hipErrorInvalidValue;
    if (n_elems == 0) return 0;
    hipLaunchKernelGGL((predict_tear_kernel<D, M>), dim3((unsigned)n_elems), dim3(64), 0, (hipStream_t)stream, g, dt,
                       Q, W, t, plans, elems, n_elems);
    return (int)hipGetLastError();
  }
};

int launch_predict_tear(int d, int M, const DevGeom& g, double dt, const double* Q, double* W, const PlanTables& t,
                        const PlanRec* plans, const int32_t* elems, int64_t n_elems, void* stream) {
  return dispatch_dm<TearL>(d, M, g, dt, Q, W, t, plans, elems, n_elems, stream);
}

// Threads per dense region: RIDG_DENSE_THREADS (256, 512 or 1024) overrides the default 256.
static int dense_threads() {
  static int t = [] {
    const char* v = getenv("RIDG_DENSE_THREADS");
    int x = v ? atoi(v) : 256;
    return (x == 512 || x == 1024) ? x : 256;
  }();
  return t;
}

template <int D, int M>
struct DenseL {
  template <int T>
  static int go(const DevGeom& g, double dt, const double* Q, double* W, const DevTensors& t, const int32_t* elems,
                int64_t n_elems, double* scratch, int64_t scratch_elems, void* stream) {
    for (int64_t first = 0; first < n_elems; first += scratch_elems) {
      const int64_t chunk = (n_elems - first < scratch_elems) ? n_elems - first : scratch_elems;
      hipLaunchKernelGGL((predict_dense_kernel<D, M, T>), dim3((unsigned)chunk), dim3(T), 0, (hipStream_t)stream, g,
                         dt, Q, W, t, elems, first, n_elems, scratch);
      int err = (int)hipGetLastError();
      if (err) return err;
    }
    return 0;
  }
  static int run(const DevGeom& g, double dt, const double* Q, double* W, const DevTensors& t,
                 const int32_t* elems, int64_t n_elems, double* scratch, int64_t scratch_elems, void* stream) {
    switch (dense_threads()) {
      case 1024: return go<1024>(g, dt, Q, W, t, elems, n_elems, scratch, scratch_elems, stream);
      case 512: return go<512>(g, dt, Q, W, t, elems, n_elems, scratch, scratch_elems, stream);
      default: return go<256>(g, dt, Q, W, t, elems, n_elems, scratch, scratch_elems, stream);
    }
  }
};

int launch_predict_dense(int d, int M, const DevGeom& g, double dt, const double* Q, double* W,
                         const DevTensors& t, const int32_t* elems, int64_t n_elems, double* scratch,
                         int64_t scratch_elems, void* stream) {
  return dispatch_dm<DenseL>(d, M, g, dt, Q, W, t, elems, n_elems, scratch, scratch_elems, stream);
}

}  // namespace ridg

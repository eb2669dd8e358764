#pragma once
// Device helpers shared by the HIP kernels of libridg (gfx950 / MI355X): sizes, geometry,
// velocity projection, segment-wide reductions and the per-lane-row block solvers of the
// RIDG prediction (Sec. 2.2 of arXiv 2101.01231).
//
// State and prediction arrays are coefficient-major in HBM (Q[k * nel + e],
// W[k * nel + e]) so that neighbouring threads/elements read neighbouring
// addresses. Element e = i0 + n0 (i1 + n1 i2).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <type_traits>

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
// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b on XCD b % 8), each XCD with
// its own L2. This bijection of [0, n) gives XCD x the contiguous logical range
// [x q + min(x, r), ...) (q = n / 8, r = n % 8), so neighbouring elements, whose data the stencils
// and region gathers share, are processed under one L2.
__device__ inline int64_t xcd_block(int64_t b, int64_t n) {
  constexpr int64_t X = 8;
  const int64_t q = n / X, r = n % X, x = b % X;
  return x * q + (x < r ? x : r) + b / X;
}

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

// element i of a small register array without dynamic indexing (a select chain). Each element
// passes through an empty asm operand (no instruction): otherwise the compiler may fold the
// selects of loads into one indexed load and keep the array in scratch memory.
template <int D>
__device__ inline double sel(const double (&v)[D], int i) {
  double r = v[0];
#pragma unroll
  for (int j = 1; j < D; ++j) {
    double vj = v[j];
    asm("" : "+v"(vj));
    r = (i == j) ? vj : r;
  }
  return r;
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
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
  // register budget hint (waves per SIMD): 2D order 4 (theta_T = 20) fits 128 VGPRs, i.e. four
  // waves, with a few bytes of spill; elsewhere the compiler's own choice is kept
  static constexpr int MIN_WAVES = (D == 2 && M == 4) ? 4 : 1;
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

// 1/x in FP32: hardware reciprocal estimate and one Newton step (FP32 eliminations only).
__device__ inline float recipf(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Compile-time loop: f(std::integral_constant<int, I>) for I = B..E-1.
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

__device__ __forceinline__ unsigned lds_addr(const double* p) {
  return (unsigned)(size_t)(const __attribute__((address_space(3))) double*)p;
}

// LDS stores at compile-time double offsets from a per-lane base. Two values per ds_write2_b64,
// each from its own register pair, so nothing is copied into consecutive registers first (the
// compiler would pair them into ds_write_b128 and insert the copies).
template <int O0, int O1>
__device__ __forceinline__ void lds_store2(unsigned base, double x, double y) {
  asm volatile("ds_write2_b64 %0, %1, %2 offset0:%3 offset1:%4" : : "v"(base), "v"(x), "v"(y), "i"(O0), "i"(O1)
               : "memory");
}
template <int O>
__device__ __forceinline__ void lds_store1(unsigned base, double x) {
  asm volatile("ds_write_b64 %0, %1 offset:%2" : : "v"(base), "v"(x), "i"(O * 8) : "memory");
}

// Publish a[J0..NT-1], rhs and inv at doubles OFF + J0 .. OFF + NT + 1 of the buffer at base.
template <int J, int NT>
__device__ __forceinline__ double row_val(const double (&a)[NT], double rhs, double inv) {
  if constexpr (J < NT)
    return a[J];
  else if constexpr (J == NT)
    return rhs;
  else
    return inv;
}
template <int OFF, int J0, int NT>
__device__ __forceinline__ void publish_row(unsigned base, const double (&a)[NT], double rhs, double inv) {
  constexpr int E = NT + 2;
  constexpr int NP = (E - J0) / 2;
  static_for<0, NP>([&](auto P) {
    constexpr int j = J0 + 2 * decltype(P)::value;
    lds_store2<OFF + j, OFF + j + 1>(base, row_val<j, NT>(a, rhs, inv), row_val<j + 1, NT>(a, rhs, inv));
  });
  if constexpr ((E - J0) & 1) lds_store1<OFF + E - 1>(base, row_val<E - 1, NT>(a, rhs, inv));
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
  static_assert(2 * PS <= 256, "ds_write2_b64 offsets are 8-bit");
  bool used = idle;
  int mystep = -1;
  double myinv = 0.0;
  const unsigned pbase = lds_addr(piv);
  static_for<0, NT>([&](auto C) {
    constexpr int c = decltype(C)::value;
    constexpr int off = (c & 1) * PS;
    const double* pv = piv + off;
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
      publish_row<off, c + 1, NT>(pbase, a, rhs, myinv);
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
  });
  if (mystep >= 0) x[mystep] = rhs * myinv;
  wave_sync();
}

__host__ __device__ constexpr int log2_ceil(int n) {
  return n <= 1 ? 0 : n <= 2 ? 1 : n <= 4 ? 2 : n <= 8 ? 3 : n <= 16 ? 4 : n <= 32 ? 5 : 6;
}

// Several rows per lane: rows k + SEGW u (u = 0 .. RPL-1) of a theta_T-row block system live in lane k
// of a SEGW-lane segment (rows >= theta_T are idle). Row numbers, hence pivot keys (whose low bits
// hold the row with the one-row layout's width), are those of the one-row layout, so every layout
// eliminates in the same order with the same arithmetic. Power-of-two segments of at most 16
// lanes reduce the pivot key with DPP row operations, other widths with ds_bpermute rotations.
template <int D, int M, int RPL_, int SEGW_>
struct PlanCfgNR {
  static constexpr int NS = n_space(D, M);
  static constexpr int NT = n_spacetime(D, M);
  static constexpr int RPL = RPL_;
  static constexpr int SEGW = SEGW_;
  static_assert(RPL * SEGW >= NT, "segment too small");
  static constexpr int S = 64 / SEGW;
  static constexpr bool POW2 = (SEGW & (SEGW - 1)) == 0 && SEGW <= 16;
  static constexpr int LB = log2_ceil(SEGW);   // rotation rounds (non-power-of-two segments)
  static constexpr int LBK = log2_ceil(NT);    // row bits of the pivot key
  static constexpr int NB = D == 3 ? 8 : pow3(D);
  // one wavefront per workgroup: the waves of a workgroup never synchronise with each other, and
  // single-wave workgroups let every SIMD take new work as soon as one of its regions' waves ends
  // (2D order 4: 1.30 ms per step at four waves, 1.19 at two, 1.13 at one)
  static constexpr int WAVES = 1;
  // register budget hint: two rows per lane at 2D order 4 run best at three waves per SIMD
  // (168 VGPRs, a few spilled); elsewhere the compiler's own choice is kept
  static constexpr int MIN_WAVES = (RPL == 2 && D == 2 && M == 4) ? 3 : 1;
};
// layout 3: two rows per lane, ceil(theta_T / 2)-lane segments
template <int D, int M>
using PlanCfg2R = PlanCfgNR<D, M, 2, (n_spacetime(D, M) + 1) / 2>;
// layout 4: power-of-two segments of SEGW >= theta_T / 3 lanes, ceil(theta_T / SEGW) rows per lane
__host__ __device__ constexpr int seg_width_nr(int nt) { return seg_width((nt + 2) / 3); }
template <int D, int M>
using PlanCfgDpp = PlanCfgNR<D, M, (n_spacetime(D, M) + seg_width_nr(n_spacetime(D, M)) - 1) / seg_width_nr(n_spacetime(D, M)),
                             seg_width_nr(n_spacetime(D, M))>;

// Gauss-Jordan with partial pivoting as seg_solve, each lane holding RPL rows: one read of the
// published pivot row updates all of them (1/RPL of the LDS traffic of one row per lane).
template <class C>
__device__ __forceinline__ void seg_solve_nr(double (&a)[C::RPL][C::NT], double (&rhs)[C::RPL], int k,
                                    const bool (&idle)[C::RPL], const int (&addr)[C::LB > 0 ? C::LB : 1], double* piv,
                                    double* x) {
  constexpr int NT = C::NT, RPL = C::RPL, SEGW = C::SEGW;
  constexpr unsigned LMASK = (1u << C::LBK) - 1u;
  constexpr int PS = NT + 2;
  static_assert(2 * PS <= 256, "ds_write2_b64 offsets are 8-bit");
  bool used[RPL];
  int step[RPL];
  double inv[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    used[u] = idle[u];
    step[u] = -1;
    inv[u] = 0.0;
  }
  const unsigned pbase = lds_addr(piv);
  static_for<0, NT>([&](auto CC) {
    constexpr int c = decltype(CC)::value;
    constexpr int off = (c & 1) * PS;
    const double* pv = piv + off;
    unsigned key = 0u;
#pragma unroll
    for (int u = 0; u < RPL; ++u)
      if (!used[u])
        key = max(key, (__float_as_uint((float)fabs(a[u][c])) & ~LMASK) | (LMASK - (unsigned)(k + u * SEGW)));
    if constexpr (C::POW2)
      key = seg_max_pow2<SEGW>(key);
    else
      key = seg_max_rot<SEGW, C::LB>(key, addr);
    const int p = (int)(LMASK - (key & LMASK));
    bool pivu[RPL];
    bool anyp = false;
    double pval = a[0][c];
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      pivu[u] = (p == k + u * SEGW) && !idle[u];
      anyp = anyp || pivu[u];
      if (u > 0) pval = pivu[u] ? a[u][c] : pval;
    }
    // one reciprocal for whichever row of the lane holds the pivot (the row branches below then
    // only store, instead of each running its own reciprocal chain one after the other)
    double pinv = 0.0;
    if (anyp) pinv = recip(pval);
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      if (pivu[u]) {
        inv[u] = pinv;
        publish_row<off, c + 1, NT>(pbase, a[u], rhs[u], pinv);
        used[u] = true;
        step[u] = c;
      }
    }
    wave_sync();
    // every row but the pivot row (and idle rows) is reduced; a zero multiplier leaves a row as is
    const double ip = pv[NT + 1];
    double l[RPL];
#pragma unroll
    for (int u = 0; u < RPL; ++u) l[u] = (pivu[u] || idle[u]) ? 0.0 : a[u][c] * ip;
#pragma unroll
    for (int j = c + 1; j < NT; ++j) {
      const double v = pv[j];
#pragma unroll
      for (int u = 0; u < RPL; ++u) a[u][j] = fma(-l[u], v, a[u][j]);
    }
    const double pr = pv[NT];
#pragma unroll
    for (int u = 0; u < RPL; ++u) rhs[u] = fma(-l[u], pr, rhs[u]);
  });
#pragma unroll
  for (int u = 0; u < RPL; ++u)
    if (step[u] >= 0) x[step[u]] = rhs[u] * inv[u];
  wave_sync();
}

// Two independent systems per segment (row k of each in lane k): the pivot searches, publishes
// and updates of the two eliminations are interleaved so that the latency of one hides behind
// the other's work; one wave-level sync per column serves both.
template <int NT, int LB, bool POW2, int SEGW>
__device__ inline void seg_solve2(double (&a)[2][NT], double (&rhs)[2], int k, bool idle,
                                  const int (&addr)[LB > 0 ? LB : 1], double* piv, double* x0, double* x1) {
  constexpr unsigned LMASK = (1u << LB) - 1u;
  constexpr int PS = NT + 2;
  bool used0 = idle, used1 = idle;
  int step0 = -1, step1 = -1;
  double inv0 = 0.0, inv1 = 0.0;
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    double* pv0 = piv + ((c & 1) * 2 + 0) * PS;
    double* pv1 = piv + ((c & 1) * 2 + 1) * PS;
    unsigned k0 = 0u, k1 = 0u;
    if (!used0) k0 = (__float_as_uint((float)fabs(a[0][c])) & ~LMASK) | (LMASK - (unsigned)k);
    if (!used1) k1 = (__float_as_uint((float)fabs(a[1][c])) & ~LMASK) | (LMASK - (unsigned)k);
    if constexpr (POW2) {
      k0 = seg_max_pow2<SEGW>(k0);
      k1 = seg_max_pow2<SEGW>(k1);
    } else {
#pragma unroll
      for (int r = 0; r < LB; ++r) {
        const unsigned o0 = (unsigned)__builtin_amdgcn_ds_bpermute(addr[r], (int)k0);
        const unsigned o1 = (unsigned)__builtin_amdgcn_ds_bpermute(addr[r], (int)k1);
        k0 = max(k0, o0);
        k1 = max(k1, o1);
      }
    }
    const bool p0 = (k == (int)(LMASK - (k0 & LMASK))) && !idle;
    const bool p1 = (k == (int)(LMASK - (k1 & LMASK))) && !idle;
    if (p0) {
      inv0 = recip(a[0][c]);
      volatile __attribute__((address_space(3))) double* vp = (volatile __attribute__((address_space(3))) double*)pv0;
#pragma unroll
      for (int j = c + 1; j < NT; ++j) vp[j] = a[0][j];
      vp[NT] = rhs[0];
      vp[NT + 1] = inv0;
      used0 = true;
      step0 = c;
    }
    if (p1) {
      inv1 = recip(a[1][c]);
      volatile __attribute__((address_space(3))) double* vp = (volatile __attribute__((address_space(3))) double*)pv1;
#pragma unroll
      for (int j = c + 1; j < NT; ++j) vp[j] = a[1][j];
      vp[NT] = rhs[1];
      vp[NT + 1] = inv1;
      used1 = true;
      step1 = c;
    }
    wave_sync();
    if (!p0 && !idle) {
      const double l = a[0][c] * pv0[NT + 1];
#pragma unroll
      for (int j = c + 1; j < NT; ++j) a[0][j] = fma(-l, pv0[j], a[0][j]);
      rhs[0] = fma(-l, pv0[NT], rhs[0]);
    }
    if (!p1 && !idle) {
      const double l = a[1][c] * pv1[NT + 1];
#pragma unroll
      for (int j = c + 1; j < NT; ++j) a[1][j] = fma(-l, pv1[j], a[1][j]);
      rhs[1] = fma(-l, pv1[NT], rhs[1]);
    }
  }
  if (step0 >= 0) x0[step0] = rhs[0] * inv0;
  if (step1 >= 0) x1[step1] = rhs[1] * inv1;
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

// ---------------------------------------------------------------- correction (per element)
// acc += sum_p V_ip Cown[i][p][bits] w (volume minus own-trace faces of direction i)
template <int D, int M, bool AFFINE>
__device__ inline void own_term(const double* cown, int i, int bits, const double (&V)[D][D + 1],
                                const double (&w)[n_spacetime(D, M)], double (&acc)[n_space(D, M)]) {
  constexpr int NS = n_space(D, M), NT = n_spacetime(D, M), NP = D + 1;
#pragma unroll 1
  for (int p = 0; p < NP; ++p) {
    if (p == 1 + i || (!AFFINE && p > 0)) continue;
    const double vp = V[i][p];
    const double* cv = cown + (((size_t)i * NP + p) * 4 + bits) * NS * NT;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < NT; ++l) s = fma(cv[k * NT + l], w[l], s);
      acc[k] = fma(vp, s, acc[k]);
    }
  }
}

// acc -= sum_p V_ip tens[i][sd][p] w (the face term of direction i, side sd)
template <int D, int M, bool AFFINE>
__device__ inline void face_term(const double* tens, int i, int sd, const double (&V)[D][D + 1],
                                 const double (&w)[n_spacetime(D, M)], double (&acc)[n_space(D, M)]) {
  constexpr int NS = n_space(D, M), NT = n_spacetime(D, M), NP = D + 1;
#pragma unroll 1
  for (int p = 0; p < NP; ++p) {
    if (p == 1 + i || (!AFFINE && p > 0)) continue;
    const double vp = V[i][p];
    const double* cf = tens + (((size_t)i * 2 + sd) * NP + p) * NS * NT;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      double s2 = 0.0;
#pragma unroll
      for (int l = 0; l < NT; ++l) s2 = fma(cf[k * NT + l], w[l], s2);
      acc[k] = fma(-vp, s2, acc[k]);
    }
  }
}

// Q'_e = Q_e + 2^-d [ sum_i sum_p V_ip Cv_ip W_e - sum_faces sum_p V_ip (CFo W_e | CFn W_nbr) ]
template <int D, int M, bool AFFINE>
__device__ inline void correct_elem(const DevGeom& g, double dt, const double* Q, const double* W, double* Qout,
                                    const DevTensors& t, int64_t e, int64_t nel) {
  constexpr int NS = n_space(D, M), NT = n_spacetime(D, M);
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
    const int side_m = face_side<D>(g, idx, i, -1), side_p = face_side<D>(g, idx, i, 1);
    const int bits = (side_m == 0 ? 1 : 0) | (side_p == 0 ? 2 : 0);
    // volume term and the faces that take the element's own trace: one precombined tensor per
    // (velocity mode, own-face set); one branch per set keeps the tensor pointer wave-uniform
    // (scalar loads), and a wavefront whose elements differ runs each set on its own lanes
#pragma unroll 1
    for (int b = 0; b < 4; ++b)
      if (bits == b) own_term<D, M, AFFINE>(t.Cown, i, b, V, we, acc);
    // faces that take the upwind neighbour's trace
#pragma unroll 1
    for (int sd = 0; sd < 2; ++sd) {
      if ((sd ? side_p : side_m) == 0) continue;
      int j[3] = {idx[0], idx[1], idx[2]};
      j[i] += sd ? 1 : -1;
      const int64_t en = elem_lin(g, j[0], j[1], j[2]);
      double wn[NT];
#pragma unroll
      for (int l = 0; l < NT; ++l) wn[l] = W[(int64_t)l * nel + en];
      face_term<D, M, AFFINE>(t.CFn, i, sd, V, wn, acc);
    }
  }
  constexpr double scale = 1.0 / (double)(1 << D);
#pragma unroll
  for (int k = 0; k < NS; ++k) Qout[(int64_t)k * nel + e] = fma(acc[k], scale, Q[(int64_t)k * nel + e]);
}



// Constant velocity: W_e = sum_tap G_tap Q_{e + off_tap} (the Sec. 2.2 system solved once on the host).
struct Taps {
  int8_t off[kMaxBlocks][3];
};

template <int D, int M>
__device__ inline void predict_prefactored_elem(const DevGeom& g, const double* Q, double* W, const double* G,
                                                const Taps& taps, int ntaps, int64_t e, int64_t nel) {
  constexpr int NS = n_space(D, M), NT = n_spacetime(D, M);
  int idx[3];
  elem_idx(g, e, idx);
  double w[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) w[k] = 0.0;
  for (int tp = 0; tp < ntaps; ++tp) {
    const int64_t src = elem_lin(g, idx[0] + taps.off[tp][0], idx[1] + taps.off[tp][1], idx[2] + taps.off[tp][2]);
    double q[NS];
#pragma unroll
    for (int l = 0; l < NS; ++l) q[l] = Q[(int64_t)l * nel + src];
    const double* Gt = G + (size_t)tp * NT * NS;
#pragma unroll
    for (int k = 0; k < NT; ++k)
#pragma unroll
      for (int l = 0; l < NS; ++l) w[k] = fma(Gt[k * NS + l], q[l], w[k]);
  }
#pragma unroll
  for (int k = 0; k < NT; ++k) W[(int64_t)k * nel + e] = w[k];
}

// out_e = base_e + sum_t A_t in_{e + off_t} (constant-velocity operators in tap form; A uniform).
struct TapsN {
  int8_t off[kMaxTapUpdate][3];
};

template <int R, int C, class TAPS>
__device__ inline void tap_update_elem(const DevGeom& g, const double* in, const double* base, double* out,
                                       const double* A, const TAPS& taps, int ntaps, int64_t e, int64_t nel) {
  int idx[3];
  elem_idx(g, e, idx);
  double acc[R];
#pragma unroll
  for (int k = 0; k < R; ++k) acc[k] = 0.0;
  for (int tp = 0; tp < ntaps; ++tp) {
    const int64_t src = elem_lin(g, idx[0] + taps.off[tp][0], idx[1] + taps.off[tp][1], idx[2] + taps.off[tp][2]);
    double x[C];
#pragma unroll
    for (int l = 0; l < C; ++l) x[l] = in[(int64_t)l * nel + src];
    const double* At = A + (size_t)tp * R * C;
#pragma unroll
    for (int k = 0; k < R; ++k)
#pragma unroll
      for (int l = 0; l < C; ++l) acc[k] = fma(At[k * C + l], x[l], acc[k]);
  }
#pragma unroll
  for (int k = 0; k < R; ++k) out[(int64_t)k * nel + e] = base[(int64_t)k * nel + e] + acc[k];
}

}  // namespace ridg

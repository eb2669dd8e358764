// Burgers equation q_t + sum_i (q^2/2)_{x_i} = 0 (eq. burger2d): Newton prediction on each region
// (Sec. 3) and the nonlinear flux-form correction (Sec. 2.3).
//
// Prediction: one workgroup per region of 3^d elements keeps the iterate W (3^d theta_T unknowns) in
// LDS. Each Newton iteration
//   1. evaluates w = Psi^T W_r at the volume and face Gauss points of every region element,
//   2. projects F'(w) = w on the space-time basis (eq. Jacproj; quadrature once per mode),
//   3. assembles one row of [J | R] per pair of lanes in the workgroup's LDS: time term and
//      causal source from the exact tensors, volume flux residual by quadrature, volume Jacobian
//      quasi-quadrature-free (sum_p beta^i_{k l p} F'_p with the exact triple products, eq.
//      Jacobian2), face terms (Rusanov inside the region, own-trace physical flux on its boundary)
//      and their Jacobian blocks by face quadrature,
//   4. solves J delta = R by Gaussian elimination with partial pivoting in LDS (FP64 for the systems of
//      up to 48 KB, FP32 above: 2D orders 3-4, 3D order 2; two threads per row above 64 unknowns,
//      the update's 4-entry chunks spread over the workgroup below) and updates W <- W - delta,
//      until max|delta| <= 1e-13 max(1, max|W|) or the iteration limit.
// Only the centre's W is written. The Rusanov wave speed of a face is max(|mean q_a|, |mean q_b|)
// from the two elements' states at t^n (fixed during the iteration).
//
// Correction: one thread per element, volume term and face fluxes by quadrature from the element's
// own prediction and its face neighbours' predictions.
#include <type_traits>

#include "kernels_common.hpp"

namespace ridg {

namespace {

constexpr double kNewtonTol = 1e-13;


__host__ __device__ constexpr int ipow(int b, int e) { return e == 0 ? 1 : b * ipow(b, e - 1); }

// The elimination keeps each row with two threads of its own for systems above this size
// (newton_solve_rows) and spreads the 4-entry chunks of the rank-1 update over the workgroup below
// it (newton_solve). Measured per Burgers step at 128^2: N = 90 (2D order 3), 9.6 against 10.4 ms;
// N = 36 (2D order 2), 2.6 against 2.3 ms.
constexpr int kRowsSolveMin = 64;
// Threads of a region's workgroup: 512 above this size, where the region system's LDS leaves room
// for one workgroup per CU (two wavefronts per SIMD), 256 below (several workgroups per CU).
// Measured per Burgers step at 128^2: order 4 (N = 180) 79.4 ms at 512 threads against 89.5 ms at
// 256 (one thread per row); at 512 threads, order 3 (N = 90) took 18.3 against 10.5 ms.
constexpr int kWideMin = 128;
__host__ __device__ constexpr int burgers_threads(int n) { return n > kWideMin ? 512 : 256; }

// Row stride of the augmented matrix in LDS: a multiple of 4 entries (the updates move 4-entry
// chunks); for the one-row-per-thread elimination also an odd number of chunks, so that the 16-byte
// chunks of consecutive rows fall in distinct banks.
__host__ __device__ constexpr int burgers_ldp(int n) {
  return (n > kRowsSolveMin && (((n + 4) & ~3) / 4) % 2 == 0) ? ((n + 4) & ~3) + 4 : ((n + 4) & ~3);
}

template <int D, int M>
struct BCfg {
  static constexpr int NS = n_space(D, M), NT = n_spacetime(D, M), NB = pow3(D), N = NB * NT;
  static constexpr int Q = burgers_q(M), NQ = ipow(Q, D + 1), NQF = ipow(Q, D), NF = 2 * D;
};

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

}  // namespace

// Point values of every region element's iterate at the volume and face points, then the projection
// of F'(w) = w on Psi (eq. Jacproj).
template <int D, int M>
__device__ __noinline__ void newton_points(const BurgersDev& t, const double* s_W, double* s_wv, double* s_wf,
                                           double* s_fp) {
  using C = BCfg<D, M>;
  constexpr int NT = C::NT, NB = C::NB, NQ = C::NQ, NQF = C::NQF, NF = C::NF, TH = burgers_threads(C::N);
  const int tid = threadIdx.x;
  for (int x = tid; x < NB * NQ; x += TH) {
    const int r = x / NQ, pt = x % NQ;
    double v = 0.0;
    for (int l = 0; l < NT; ++l) v = fma(t.psiv[l * NQ + pt], s_W[r * NT + l], v);
    s_wv[x] = v;
  }
  for (int x = tid; x < NB * NF * NQF; x += TH) {
    const int r = x / (NF * NQF), f = (x / NQF) % NF, pf = x % NQF;
    double v = 0.0;
    for (int l = 0; l < NT; ++l) v = fma(t.psif[(f * NT + l) * NQF + pf], s_W[r * NT + l], v);
    s_wf[x] = v;
  }
  __syncthreads();
  for (int x = tid; x < NB * NT; x += TH) {
    const int r = x / NT, p = x % NT;
    double v = 0.0;
    for (int pt = 0; pt < NQ; ++pt) v = fma(t.projw[p * NQ + pt], s_wv[r * NQ + pt], v);
    s_fp[x] = v;
  }
  __syncthreads();
}

// Row R = (r, k) of [J | R], by two neighbouring lanes (h = 0, 1): time term and causal source
// (h = 0), volume flux residual by quadrature and volume Jacobian from the triple products (eq.
// Jacobian2) for the directions i = h, h + 2, ..., face terms and their Jacobian blocks by face
// quadrature for the faces on side h of every direction. The two lanes' sums for the diagonal block
// and the residual are added by a lane exchange and stored by lane h = 0; each lane stores the
// neighbour blocks of its own faces.
template <int D, int M, class TS>
__device__ __forceinline__ void newton_row(const BurgersDev& t, double c0, double c1, double c2, int R, int h,
                                        const double* s_W, const double* s_q, const double* s_wv,
                                        const double* s_wf, const double* s_fp, TS* __restrict__ row) {
  using C = BCfg<D, M>;
  constexpr int NS = C::NS, NT = C::NT, N = C::N, NQ = C::NQ, NQF = C::NQF, NF = C::NF;
  const int r = R / NT, k = R % NT;
  // (both lanes' zero stores precede every store of the row's values in their wavefront's order)
  for (int j = h; j < burgers_ldp(N); j += 2) row[j] = (TS)0;
  double dg[NT];
  double res = 0.0;
#pragma unroll
  for (int l = 0; l < NT; ++l) {
    dg[l] = h == 0 ? t.Tt[k * NT + l] : 0.0;
    res = fma(dg[l], s_W[r * NT + l], res);
  }
  if (h == 0)
    for (int j = 0; j < NS; ++j) res = fma(-t.Cc[k * NS + j], s_q[r * NS + j], res);
#pragma unroll 1
  for (int i = h; i < D; i += 2) {
    const double cc = i == 0 ? c0 : (i == 1 ? c1 : c2);
    double v = 0.0;  // int int d_xi_i Psi_k F(w)
    const double* dw = t.dpsivw + ((size_t)i * NT + k) * NQ;
#pragma unroll 4
    for (int pt = 0; pt < NQ; ++pt) {
      const double w = s_wv[r * NQ + pt];
      v = fma(dw[pt], 0.5 * w * w, v);
    }
    res = fma(-cc, v, res);
    const int32_t* bptr = t.bptr + ((size_t)i * NT + k) * NT;
#pragma unroll
    for (int l = 0; l < NT; ++l) {
      double sm = 0.0;
      for (int q = bptr[l]; q < bptr[l + 1]; ++q) sm = fma(t.bval[q], s_fp[r * NT + t.bp[q]], sm);
      dg[l] = fma(-cc, sm, dg[l]);
    }
  }
  // region offset digits of r (o_0 slowest)
  const int d0 = (D == 1) ? r : (D == 2 ? r / 3 : r / 9);
  const int d1 = (D == 2) ? r % 3 : (r / 3) % 3;
  const int d2 = r % 3;
#pragma unroll 1
  for (int f = h; f < NF; f += 2) {
    const int i = f >> 1, fo = f ^ 1;
    const double cc = i == 0 ? c0 : (i == 1 ? c1 : c2);
    const double s = (f & 1) ? 1.0 : -1.0;
    const int oi = (i == 0 ? d0 : (i == 1 ? d1 : d2)) + ((f & 1) ? 1 : -1);
    const bool inside = oi >= 0 && oi <= 2;
    const int stride = (i == D - 1) ? 1 : (i == D - 2 ? 3 : 9);
    const int r2 = inside ? r + ((f & 1) ? stride : -stride) : r;
    const double al = inside ? fmax(fabs(s_q[r * NS]), fabs(s_q[r2 * NS])) : 0.0;
    double nb[NT];
#pragma unroll
    for (int l = 0; l < NT; ++l) nb[l] = 0.0;
    const double* wk = t.psifw + ((size_t)f * NT + k) * NQF;
#pragma unroll 1
    for (int pf = 0; pf < NQF; ++pf) {
      const double a = s_wf[(r * NF + f) * NQF + pf];
      double H, da, db = 0.0;
      if (inside) {
        const double b = s_wf[(r2 * NF + fo) * NQF + pf];
        H = 0.5 * s * (0.5 * a * a + 0.5 * b * b) - 0.5 * al * (b - a);
        da = 0.5 * s * a + 0.5 * al;
        db = 0.5 * s * b - 0.5 * al;
      } else {
        H = 0.5 * s * a * a;
        da = s * a;
      }
      const double cw = cc * wk[pf];
      res = fma(cw, H, res);
      const double* pown = t.psif + (size_t)f * NT * NQF + pf;
      const double* pnbr = t.psif + (size_t)fo * NT * NQF + pf;
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        dg[l] = fma(cw * da, pown[l * NQF], dg[l]);
        nb[l] = fma(cw * db, pnbr[l * NQF], nb[l]);
      }
    }
    if (inside) {
#pragma unroll
      for (int l = 0; l < NT; ++l) row[r2 * NT + l] = (TS)nb[l];
    }
  }
#pragma unroll
  for (int l = 0; l < NT; ++l) dg[l] += __shfl_xor(dg[l], 1, 64);
  res += __shfl_xor(res, 1, 64);
  if (h == 0) {
#pragma unroll
    for (int l = 0; l < NT; ++l) row[r * NT + l] = (TS)dg[l];
    row[N] = (TS)res;
  }
}

// Gaussian elimination with partial pivoting on the augmented N x (N + 1) matrix A held in LDS (rows
// padded to LDP = a multiple of 4 entries), then back substitution; the solution goes to s_x in FP64.
// Pivot: the row of largest |A[r][c]|, compared on a 32-bit key (FP32 image of |A[r][c]| with the low
// bits replaced by the row, ties to the lowest row), reduced within each wavefront and then across
// wavefronts. The rank-1 update runs on 4-entry chunks from the 4-aligned column at or below c:
// entries left of c are dead (the factor L is not kept) and may take any value.
template <int N, class TS>
__device__ __noinline__ void newton_solve(TS* A, double* s_x, TS* s_l, TS* s_piv, int* s_key) {
  constexpr int LDP = burgers_ldp(N), TH = burgers_threads(N), NW = TH / 64;
  constexpr unsigned RB = N <= 256 ? 8 : (N <= 512 ? 9 : 10);
  constexpr unsigned RMASK = (1u << RB) - 1u;
  typedef TS v4 __attribute__((ext_vector_type(4)));
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int c = 0; c < N; ++c) {
    unsigned key = 0u;
    for (int Rr = c + tid; Rr < N; Rr += TH) {
      const unsigned kk = (__float_as_uint((float)fabs((double)A[Rr * LDP + c])) & ~RMASK) | (RMASK - (unsigned)Rr);
      key = max(key, kk);
    }
    key = seg_max_pow2<64>(key);
    if (lane == 0) s_key[wid] = (int)key;
    __syncthreads();
    unsigned best = 0u;
    for (int w = 0; w < NW; ++w) best = max(best, (unsigned)s_key[w]);
    const int p = (int)(RMASK - (best & RMASK));
    const int j0 = c & ~3;
    for (int j = j0 + tid; j < LDP; j += TH) {
      const TS vc = A[c * LDP + j], vp = A[p * LDP + j];
      if (p != c && j >= c) {
        A[c * LDP + j] = vp;
        A[p * LDP + j] = vc;
      }
      s_piv[j] = vp;
    }
    __syncthreads();
    const TS inv = (TS)1 / s_piv[c];
    for (int Rr = c + 1 + tid; Rr < N; Rr += TH) s_l[Rr] = A[Rr * LDP + c] * inv;
    __syncthreads();
    const int nch = (LDP - j0) >> 2, items = (N - c - 1) * nch;
#pragma unroll 4
    for (int q = tid; q < items; q += TH) {
      const int rr = q / nch, ch = q - rr * nch;
      const int Rr = c + 1 + rr;
      v4* a = (v4*)(A + Rr * LDP + j0) + ch;
      const v4 pv = *((const v4*)(s_piv + j0) + ch);
      const TS l = s_l[Rr];
      v4 x = *a;
      x.x = fma(-l, pv.x, x.x);
      x.y = fma(-l, pv.y, x.y);
      x.z = fma(-l, pv.z, x.z);
      x.w = fma(-l, pv.w, x.w);
      *a = x;
    }
    __syncthreads();
  }
  for (int c = N - 1; c >= 0; --c) {
    if (tid == 0) s_x[c] = (double)A[c * LDP + N] / (double)A[c * LDP + c];
    __syncthreads();
    const TS xc = (TS)s_x[c];
    for (int Rr = tid; Rr < c; Rr += TH) A[Rr * LDP + N] = fma(-A[Rr * LDP + c], xc, A[Rr * LDP + N]);
    __syncthreads();
  }
}

// Gaussian elimination with partial pivoting on the augmented N x (N + 1) matrix A in LDS, two
// threads per row and no row exchanges: row p_c, the unused row of largest |A[r][c]| (the same 32-bit
// key as newton_solve), pivots column c, and every unused row r subtracts (A[r][c] / A[p_c][c]) times
// it from the 4-aligned column at or below c on (entries left of c are dead). Each thread forms its
// row's key for the next column right after its update, so a column costs one workgroup barrier.
// Back substitution runs over the pivot rows, x_c = (b_{p_c} - sum_{j>c} A[p_c][j] x_j) / A[p_c][c],
// one barrier per column; the solution goes to s_x in FP64.
template <int N, class TS>
__device__ __noinline__ void newton_solve_rows(TS* A, double* s_x, TS* s_pv, int* s_perm, int* s_key) {
  constexpr int LDP = burgers_ldp(N), TH = burgers_threads(N), NW = TH / 64;
  static_assert(2 * N <= TH, "two threads per row");
  constexpr unsigned RB = N <= 256 ? 8 : (N <= 512 ? 9 : 10);
  constexpr unsigned RMASK = (1u << RB) - 1u;
  typedef TS v4 __attribute__((ext_vector_type(4)));
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int row = tid >> 1, h = tid & 1;  // the two threads of a row take alternate 4-entry chunks
  const bool has_row = row < N;
  bool used = !has_row;
  int mycol = N;  // the column this row pivots
  TS* Ar = A + (has_row ? row : 0) * LDP;
  // the key of column c comes from the thread that last updated the chunk holding it
  auto publish_key = [&](int c, int owner) {
    unsigned k = 0u;
    if (!used && h == owner) k = (__float_as_uint((float)fabs((double)Ar[c])) & ~RMASK) | (RMASK - (unsigned)row);
    k = seg_max_pow2<64>(k);
    if (lane == 0) s_key[(c & 1) * NW + wid] = (int)k;
  };
  publish_key(0, 0);
  __syncthreads();
  for (int c = 0; c < N; ++c) {
    unsigned best = 0u;
#pragma unroll
    for (int w = 0; w < NW; ++w) best = max(best, (unsigned)s_key[(c & 1) * NW + w]);
    const int p = (int)(RMASK - (best & RMASK));
    const TS* Ap = A + p * LDP;
    const TS pvc = Ap[c];
    if (tid == 0) {
      s_perm[c] = p;
      s_pv[c] = pvc;
    }
    if (row == p) {
      used = true;
      mycol = c;
    }
    const int j0 = c & ~3;
    if (!used) {
      // both threads of the row read a_rc before either stores: they are neighbouring lanes of one
      // wavefront, and the load precedes the stores in program order
      const TS l = Ar[c] * ((TS)1 / pvc);
#pragma unroll 4
      for (int j = j0 + 4 * h; j < LDP; j += 8) {
        v4* a = (v4*)(Ar + j);
        const v4 pv = *(const v4*)(Ap + j);
        v4 x = *a;
        x.x = fma(-l, pv.x, x.x);
        x.y = fma(-l, pv.y, x.y);
        x.z = fma(-l, pv.z, x.z);
        x.w = fma(-l, pv.w, x.w);
        *a = x;
      }
    }
    if (c + 1 < N) publish_key(c + 1, (((c + 1) & ~3) - j0) >> 2);
    __syncthreads();
  }
  for (int c = N - 1; c >= 0; --c) {
    const double xc = (double)A[s_perm[c] * LDP + N] / (double)s_pv[c];
    if (tid == 0) s_x[c] = xc;
    if (h == 0 && mycol < c) Ar[N] = fma(-Ar[c], (TS)xc, Ar[N]);
    __syncthreads();
  }
}

// Arithmetic of the region Jacobian's elimination: FP64 for the small systems (up to 48 KB), FP32
// otherwise, which halves the LDS of a workgroup and so raises the workgroups resident per CU (the
// residual stays FP64, so Newton converges to the same FP64 root; an FP32 step only makes the
// convergence linear with a rate of about the FP32 rounding times the condition number).
template <int N>
using NewtonScalar =
    typename std::conditional<(size_t)N * ((N + 4) & ~3) * 8 <= 48 * 1024, double, float>::type;

template <int D, int M>
__global__ __launch_bounds__(burgers_threads(BCfg<D, M>::N)) void burgers_predict_kernel(DevGeom g, double dt,
                                                                          const double* __restrict__ Qs,
                                                                          double* __restrict__ W, BurgersDev t,
                                                                          int64_t first, int64_t nel, int max_iter,
                                                                          int32_t* __restrict__ stats) {
  using C = BCfg<D, M>;
  constexpr int TH = burgers_threads(C::N);
  constexpr int NS = C::NS, NT = C::NT, NB = C::NB, N = C::N, NQ = C::NQ, NQF = C::NQF, NF = C::NF;
  const int64_t e = first + blockIdx.x;
  if (e >= nel) return;
  using TS = NewtonScalar<N>;
  constexpr int LDP = burgers_ldp(N);
  __shared__ __align__(16) TS s_A[N * LDP];  // [N][LDP]: Jacobian | residual | padding
  __shared__ double s_W[N];
  __shared__ double s_q[NB * NS];
  __shared__ double s_wv[NB * NQ];
  __shared__ double s_wf[NB * NF * NQF];
  __shared__ double s_fp[NB * NT];
  __shared__ double s_x[N];
  __shared__ __align__(16) TS s_piv[LDP];
  __shared__ TS s_l[N];
  __shared__ int s_key[2 * (TH / 64)];
  __shared__ int s_perm[N];
  __shared__ double s_red[2][TH / 64];
  __shared__ int64_t s_ge[NB];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  constexpr int NW = TH / 64;
  if (tid < NB) {
    int base[3];
    elem_idx(g, e, base);
    int o[3] = {0, 0, 0}, c = tid;
    for (int i = D - 1; i >= 0; --i) {
      o[i] = c % 3 - 1;
      c /= 3;
    }
    s_ge[tid] = elem_lin(g, base[0] + o[0], base[1] + o[1], base[2] + o[2]);
  }
  __syncthreads();
  for (int x = tid; x < NB * NS; x += TH) {
    const int r = x / NS, j = x % NS;
    s_q[x] = Qs[(int64_t)j * nel + s_ge[r]];
  }
  for (int x = tid; x < N; x += TH) s_W[x] = 0.0;
  __syncthreads();
  for (int x = tid; x < NB * NS; x += TH) {  // W^(0): the state held constant in time
    const int r = x / NS, j = x % NS;
    s_W[r * NT + t.lift[j]] = s_q[x];
  }
  __syncthreads();
  const double c0 = dt / g.h0, c1 = dt / g.h1, c2 = dt / g.h2;
  int it = 0;
  bool converged = false;
  while (it < max_iter && !converged) {
    ++it;
    newton_points<D, M>(t, s_W, s_wv, s_wf, s_fp);
    for (int R = tid >> 1; R < N; R += TH / 2)  // the two lanes of a row stay together
      newton_row<D, M, TS>(t, c0, c1, c2, R, tid & 1, s_W, s_q, s_wv, s_wf, s_fp, s_A + R * LDP);
    __syncthreads();
    if constexpr (N > kRowsSolveMin)
      newton_solve_rows<N, TS>(s_A, s_x, s_l, s_perm, s_key);
    else
      newton_solve<N, TS>(s_A, s_x, s_l, s_piv, s_key);
    // update and convergence test (uniform across the workgroup)
    double md = 0.0, mw = 0.0;
    for (int x = tid; x < N; x += TH) {
      const double w = s_W[x] - s_x[x];
      s_W[x] = w;
      md = fmax(md, fabs(s_x[x]));
      mw = fmax(mw, fabs(w));
    }
    md = wave_max(md);
    mw = wave_max(mw);
    if (lane == 0) {
      s_red[0][wid] = md;
      s_red[1][wid] = mw;
    }
    __syncthreads();
    md = 0.0;
    mw = 0.0;
    for (int w = 0; w < NW; ++w) {
      md = fmax(md, s_red[0][w]);
      mw = fmax(mw, s_red[1][w]);
    }
    converged = md <= kNewtonTol * fmax(1.0, mw);
    __syncthreads();
  }
  const int centre = (NB - 1) / 2;
  for (int k = tid; k < NT; k += TH) W[(int64_t)k * nel + e] = s_W[centre * NT + k];
  if (tid == 0) {
    atomicMax(stats, it);
    if (!converged) atomicAdd(stats + 1, 1);
    atomicAdd((unsigned long long*)(stats + 2), (unsigned long long)it);
    atomicAdd((unsigned long long*)(stats + 4), 1ull);
  }
}

template <int D, int M>
__global__ __launch_bounds__(256) void burgers_correct_kernel(DevGeom g, double dt, const double* __restrict__ Qs,
                                                              const double* __restrict__ W, double* __restrict__ Qout,
                                                              BurgersDev t) {
  using C = BCfg<D, M>;
  constexpr int NS = C::NS, NT = C::NT, NQ = C::NQ, NQF = C::NQF, NF = C::NF;
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nel) return;
  const double ci[3] = {dt / g.h0, dt / g.h1, dt / g.h2};
  double we[NT], acc[NS];
#pragma unroll
  for (int l = 0; l < NT; ++l) we[l] = W[(int64_t)l * nel + e];
#pragma unroll
  for (int k = 0; k < NS; ++k) acc[k] = 0.0;
  // volume: sum_i c_i int int d_xi_i Phi_k F(w_e)
  for (int pt = 0; pt < NQ; ++pt) {
    double w = 0.0;
#pragma unroll
    for (int l = 0; l < NT; ++l) w = fma(t.psiv[l * NQ + pt], we[l], w);
    const double F = 0.5 * w * w;
    for (int i = 0; i < D; ++i) {
      const double cf = ci[i] * F;
#pragma unroll
      for (int k = 0; k < NS; ++k) acc[k] = fma(cf, t.dphivw[((size_t)i * NS + k) * NQ + pt], acc[k]);
    }
  }
  // faces: - sum_f c_i int int Phi_k|_f H(w_e, w_nbr)
  int idx[3];
  elem_idx(g, e, idx);
  const double qe0 = Qs[e];
  for (int f = 0; f < NF; ++f) {
    const int i = f >> 1, fo = f ^ 1;
    const double s = (f & 1) ? 1.0 : -1.0;
    int j[3] = {idx[0], idx[1], idx[2]};
    j[i] += (f & 1) ? 1 : -1;
    const int64_t en = elem_lin(g, j[0], j[1], j[2]);
    double wn[NT];
#pragma unroll
    for (int l = 0; l < NT; ++l) wn[l] = W[(int64_t)l * nel + en];
    const double al = fmax(fabs(qe0), fabs(Qs[en]));
    for (int pf = 0; pf < NQF; ++pf) {
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int l = 0; l < NT; ++l) {
        a = fma(t.psif[((size_t)f * NT + l) * NQF + pf], we[l], a);
        b = fma(t.psif[((size_t)fo * NT + l) * NQF + pf], wn[l], b);
      }
      const double H = 0.5 * s * (0.5 * a * a + 0.5 * b * b) - 0.5 * al * (b - a);
      const double ch = -ci[i] * H;
#pragma unroll
      for (int k = 0; k < NS; ++k) acc[k] = fma(ch, t.phifw[((size_t)f * NS + k) * NQF + pf], acc[k]);
    }
  }
  const double sc = 1.0 / (double)(1 << D);
#pragma unroll
  for (int k = 0; k < NS; ++k) Qout[(int64_t)k * nel + e] = fma(acc[k], sc, Qs[(int64_t)k * nel + e]);
}

namespace {

template <int D, int M>
int burgers_predict_dm(const DevGeom& g, double dt, const double* Q, double* W, const BurgersDev& t, int64_t nel,
                       int max_iter, int32_t* stats, void* stream) {
  constexpr int64_t kChunk = (int64_t)1 << 30;  // workgroups per launch at most
  for (int64_t first = 0; first < nel; first += kChunk) {
    const int64_t chunk = (nel - first < kChunk) ? nel - first : kChunk;
    hipLaunchKernelGGL((burgers_predict_kernel<D, M>), dim3((unsigned)chunk), dim3(burgers_threads(BCfg<D, M>::N)), 0,
                       (hipStream_t)stream, g, dt, Q, W, t, first, nel, max_iter, stats);
    const int err = (int)hipGetLastError();
    if (err) return err;
  }
  return 0;
}

template <int D, int M>
int burgers_correct_dm(const DevGeom& g, double dt, const double* Q, const double* W, double* Qout,
                       const BurgersDev& t, void* stream) {
  const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
  hipLaunchKernelGGL((burgers_correct_kernel<D, M>), dim3(grid_for(nel, 256)), dim3(256), 0, (hipStream_t)stream, g,
                     dt, Q, W, Qout, t);
  return (int)hipGetLastError();
}

}  // namespace

#define RIDG_BURGERS_CASES(X) X(1, 1) X(1, 2) X(1, 3) X(1, 4) X(1, 5) X(2, 1) X(2, 2) X(2, 3) X(2, 4) X(3, 1) X(3, 2)

int launch_burgers_predict(int d, int M, const DevGeom& g, double dt, const double* Q, double* W,
                           const BurgersDev& t, int64_t nel, int max_iter, int32_t* stats, void* stream) {
  if (max_iter < 1) return (int)hipErrorInvalidValue;
#define RIDG_BP(DD, MM) \
  if (d == DD && M == MM) return burgers_predict_dm<DD, MM>(g, dt, Q, W, t, nel, max_iter, stats, stream);
  RIDG_BURGERS_CASES(RIDG_BP)
#undef RIDG_BP
  return (int)hipErrorInvalidValue;
}

int launch_burgers_correct(int d, int M, const DevGeom& g, double dt, const double* Q, const double* W,
                           double* Qout, const BurgersDev& t, void* stream) {
#define RIDG_BC(DD, MM) \
  if (d == DD && M == MM) return burgers_correct_dm<DD, MM>(g, dt, Q, W, Qout, t, stream);
  RIDG_BURGERS_CASES(RIDG_BC)
#undef RIDG_BC
  return (int)hipErrorInvalidValue;
}

}  // namespace ridg

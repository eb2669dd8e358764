// Cyclic regions (tearing) and whole-region dense solves (Sec. 2.2).
#include "kernels_common.hpp"

namespace ridg {

// ---------------------------------------------------------------- cyclic regions by tearing
// Regions whose centre lies on a dependency cycle (around a point where the flow circulates) are
// solved on the same block structure: block 0 of the plan is a tear block whose unknowns x break
// every cycle. The other ancestor blocks are eliminated in upwind order with 1 + theta_T
// right-hand sides, giving W_r = alpha_r + B_r x; the tear block's own equations then form one
// theta_T x theta_T system for x, and W_centre = alpha_c + B_c x. This solves exactly the region
// system of eq. (pred_full_system) restricted to the centre's ancestors.
//
// One workgroup of kTearWaves wavefronts per region. Every wavefront assembles and eliminates the
// same block matrices (identical arithmetic, hence identical pivots) and carries its own slice of
// the right-hand-side columns [alpha | B], so the registers hold theta_T + ceil((1 + theta_T) /
// kTearWaves) values per row and every index into them is static. A block's columns depend only
// on the same columns of its upwind sources, so the wavefronts run independently until the tear
// equation, which needs every column.
constexpr int kTearWaves = 4;

template <int NT>
struct TearCfg {
  static constexpr int R = 1 + NT;                            // right-hand sides: alpha and B
  static constexpr int RW = (R + kTearWaves - 1) / kTearWaves;  // columns per wavefront
  static constexpr int SEGW = seg_width(NT);                  // rows in a power-of-two lane segment
  static constexpr int LB = log2_ceil(SEGW);
};

// Gauss-Jordan elimination with partial pivoting (the pivot rule of seg_solve) of [A | rhs] with
// RW right-hand sides; row k of A in lane k. Columns r < ncols of the solution go to
// x[step * ldx + r] (LDS).
template <int NT, int SEGW, int RW>
__device__ inline void seg_solve_gj_rhs(double (&a)[NT], double (&rhs)[RW], int k, bool idle, double* piv,
                                        double* x, int ldx, int ncols) {
  constexpr int LB = log2_ceil(SEGW);
  constexpr unsigned LMASK = (1u << LB) - 1u;
  constexpr int PS = NT + RW + 1;  // published row: a[c+1..NT-1], rhs, 1/pivot
  bool used = idle;
  int mystep = -1;
  double myinv = 0.0;
  static_for<0, NT>([&](auto C) {
    constexpr int c = decltype(C)::value;
    double* pv = piv + (c & 1) * PS;
    unsigned key = 0u;
    if (!used) key = (__float_as_uint((float)fabs(a[c])) & ~LMASK) | (LMASK - (unsigned)k);
    key = seg_max_pow2<SEGW>(key);
    const int p = (int)(LMASK - (key & LMASK));
    const bool is_piv = (k == p) && !idle;
    if (is_piv) {
      myinv = recip(a[c]);
#pragma unroll
      for (int j = c + 1; j < NT; ++j) pv[j] = a[j];
#pragma unroll
      for (int r = 0; r < RW; ++r) pv[NT + r] = rhs[r];
      pv[NT + RW] = myinv;
      used = true;
      mystep = c;
    }
    wave_sync();
    if (!is_piv && !idle) {
      const double l = a[c] * pv[NT + RW];
#pragma unroll
      for (int j = c + 1; j < NT; ++j) a[j] = fma(-l, pv[j], a[j]);
#pragma unroll
      for (int r = 0; r < RW; ++r) rhs[r] = fma(-l, pv[NT + r], rhs[r]);
    }
  });
  if (mystep >= 0) {
#pragma unroll
    for (int r = 0; r < RW; ++r)
      if (r < ncols) x[mystep * ldx + r] = rhs[r] * myinv;
  }
  wave_sync();
}

template <int D, int M>
__global__ __launch_bounds__(64 * kTearWaves) void predict_tear_kernel(DevGeom g, double dt,
                                                                       const double* __restrict__ Q,
                                                                       double* __restrict__ W, PlanTables t,
                                                                       const PlanRec* __restrict__ plans,
                                                                       const int32_t* __restrict__ elems,
                                                                       int64_t n_elems) {
  constexpr int NT = n_spacetime(D, M);
  if constexpr (NT <= 64) {
    using C = TearCfg<NT>;
    constexpr int NB = PlanCfg<D, M>::NB, R = C::R, RW = C::RW, SEGW = C::SEGW;
    __shared__ double s_w[NB][NT][R];  // [alpha | B] of every eliminated block
    __shared__ double s_piv[kTearWaves][2 * (NT + RW + 1)];
    __shared__ double s_x[NT];
    const int64_t item = blockIdx.x;
    if (item >= n_elems) return;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const bool idle = lane >= NT;
    const int k = idle ? 0 : lane;
    const int j0 = wave * RW;                             // first right-hand-side column of this wavefront
    const int ncols = R - j0 < RW ? (R - j0 > 0 ? R - j0 : 0) : RW;
    const int64_t nel = (int64_t)g.n0 * g.n1 * g.n2;
    const int32_t e = elems[item];
    int base[3];
    elem_idx(g, e, base);
    const PlanRec* pr = plans + item;
    const int nb = pr->nb;
    const int centre = pr->pad[1];
    const int ccl = t.cc_idx[k];
    const double ccv = t.cc_val[k];
    double* piv = &s_piv[wave][0];
    // assembled row k of the diagonal block of plan block b, its causal source, and V0
    // (plan records are read in place: a copied record indexed by face would live in scratch memory)
    auto assemble = [&](int b, double (&a)[NT], double& src0, double (&V0)[D]) {
      const PlanBlock* blk = &pr->blk[b];
      int mask = 0;
#pragma unroll
      for (int i = 0; i < D; ++i)
        mask |= ((blk->src[2 * i] == kOwn ? 1 : 0) | (blk->src[2 * i + 1] == kOwn ? 2 : 0)) << (2 * i);
      const int gi[3] = {wrap(base[0] + blk->off[0], g.n0), wrap(base[1] + blk->off[1], g.n1),
                         wrap(base[2] + blk->off[2], g.n2)};
      const int64_t ge = (int64_t)gi[0] + (int64_t)g.n0 * ((int64_t)gi[1] + (int64_t)g.n1 * gi[2]);
#pragma unroll
      for (int i = 0; i < D; ++i) {
        double v = g.a[i];
#pragma unroll
        for (int j = 0; j < D; ++j) v += g.g[i][j] * ((gi[j] + 0.5) * geom_h(g, j));
        V0[i] = v * dt / geom_h(g, i);
      }
      const double* a0 = t.A0 + ((size_t)mask * NT + k) * NT;
#pragma unroll
      for (int l = 0; l < NT; ++l) a[l] = a0[l];
#pragma unroll 1
      for (int i = 0; i < D; ++i) {
        const double vi = sel<D>(V0, i);
        const double* kk = t.K + (((size_t)i * 4 + ((mask >> (2 * i)) & 3)) * NT + k) * NT;
#pragma unroll
        for (int l = 0; l < NT; ++l) a[l] = fma(vi, kk[l], a[l]);
      }
      src0 = ccv * Q[(int64_t)ccl * nel + ge];
    };
    // eliminated blocks in plan order (block 0, the tear block, comes last)
    for (int b = 1; b < nb; ++b) {
      const uint8_t* bsrc = pr->blk[b].src;
      double a[NT], V0[D], src0;
      assemble(b, a, src0, V0);
      double rhs[RW];
#pragma unroll
      for (int r = 0; r < RW; ++r) rhs[r] = (j0 + r == 0) ? src0 : 0.0;
#pragma unroll 1
      for (int i = 0; i < D; ++i) {
        const double vi = sel<D>(V0, i);
#pragma unroll 1
        for (int sd = 0; sd < 2; ++sd) {
          const int src = bsrc[2 * i + sd];
          if (src == kOwn) continue;
          const double* f0 = t.Fn0 + (((size_t)i * 2 + sd) * NT + k) * NT;
          const double* fc = t.FnC + (((size_t)i * 2 + sd) * NT + k) * NT;
          if (src == 0) {  // coupling to the tear unknowns: column 1 + l of B gets -A_{b,0}[k][l]
#pragma unroll
            for (int r = 0; r < RW; ++r) {
              const int l = j0 + r - 1;
              if (l >= 0 && l < NT) rhs[r] -= fma(vi, f0[l], fc[l]);
            }
          } else {  // -A_{b,s} (alpha_s + B_s x), this wavefront's columns
            const double* ws = &s_w[src][0][0] + j0;
#pragma unroll
            for (int l = 0; l < NT; ++l) {
              const double cl = fma(vi, f0[l], fc[l]);
#pragma unroll
              for (int r = 0; r < RW; ++r)
                if (r < ncols) rhs[r] = fma(-cl, ws[l * R + r], rhs[r]);
            }
          }
        }
      }
      seg_solve_gj_rhs<NT, SEGW, RW>(a, rhs, k, idle, piv, &s_w[b][0][0] + j0, R, ncols);
    }
    __syncthreads();  // every column of every eliminated block is in LDS
    if (wave != 0) return;
    {  // tear equation: A_00 x + sum_s A_{0,s} (alpha_s + B_s x) = b_0
      double a[NT], V0[D], r0;
      assemble(0, a, r0, V0);
      const uint8_t* bsrc = pr->blk[0].src;
#pragma unroll 1
      for (int i = 0; i < D; ++i) {
        const double vi = sel<D>(V0, i);
#pragma unroll 1
        for (int sd = 0; sd < 2; ++sd) {
          const int src = bsrc[2 * i + sd];
          if (src == kOwn) continue;
          const double* f0 = t.Fn0 + (((size_t)i * 2 + sd) * NT + k) * NT;
          const double* fc = t.FnC + (((size_t)i * 2 + sd) * NT + k) * NT;
#pragma unroll
          for (int l = 0; l < NT; ++l) {
            const double cl = fma(vi, f0[l], fc[l]);
            r0 = fma(-cl, s_w[src][l][0], r0);
#pragma unroll
            for (int j = 0; j < NT; ++j) a[j] = fma(cl, s_w[src][l][1 + j], a[j]);
          }
        }
      }
      double rr[1] = {r0};
      seg_solve_gj_rhs<NT, SEGW, 1>(a, rr, k, idle, piv, s_x, 1, 1);
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

template <int D, int M>
struct TearL {
  static int run(const DevGeom& g, double dt, const double* Q, double* W, const PlanTables& t, const PlanRec* plans,
                 const int32_t* elems, int64_t n_elems, void* stream) {
    if (n_spacetime(D, M) > 64) return (int)hipErrorInvalidValue;
    if (n_elems == 0) return 0;
    hipLaunchKernelGGL((predict_tear_kernel<D, M>), dim3((unsigned)n_elems), dim3(64 * kTearWaves), 0,
                       (hipStream_t)stream, g, dt, Q, W, t, plans, elems, n_elems);
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

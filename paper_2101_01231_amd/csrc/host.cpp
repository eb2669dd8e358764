// Host FP64 precompute of libridg: exact Legendre tensors (quasi-quadrature-free
// assembly, Sec. 3 of arXiv 2101.01231), velocity projection, face upwinding,
// upwind elimination plans of the regions (Sec. 2.2), region assembly and the
// prefactored constant-velocity prediction operator.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <limits>
#include <map>

#include "ridg_internal.hpp"

namespace ridg {

// ---------------------------------------------------------------- basis
static std::vector<std::array<int, 4>> graded_indices(int nvar, int M, bool tensor) {
  std::vector<std::array<int, 4>> out;
  int e[4] = {0, 0, 0, 0};
  // enumerate all tuples in [0, M)^nvar with sum <= M-1
  int total = 1;
  for (int i = 0; i < nvar; ++i) total *= M;
  for (int code = 0; code < total; ++code) {
    int c = code, s = 0;
    for (int i = nvar - 1; i >= 0; --i) {
      e[i] = c % M;
      c /= M;
      s += e[i];
    }
    if (!tensor && s > M - 1) continue;  // total degree <= M - 1 (P); tensor degree <= M - 1 per variable (Q)
    out.push_back({e[0], e[1], e[2], e[3]});
  }
  std::sort(out.begin(), out.end(), [nvar](const std::array<int, 4>& x, const std::array<int, 4>& y) {
    int sx = 0, sy = 0;
    for (int i = 0; i < nvar; ++i) {
      sx += x[i];
      sy += y[i];
    }
    if (sx != sy) return sx < sy;
    for (int i = 0; i < nvar; ++i)
      if (x[i] != y[i]) return x[i] > y[i];  // descending lexicographic
    return false;
  });
  return out;
}

Basis make_basis(int d, int M, int family) {
  Basis b;
  b.d = d;
  b.M = M;
  b.family = family;
  b.sidx = graded_indices(d, M, family == RIDG_BASIS_Q);
  b.tidx = graded_indices(d + 1, M, family == RIDG_BASIS_Q);
  b.theta = (int)b.sidx.size();
  b.theta_t = (int)b.tidx.size();
  return b;
}

// ---------------------------------------------------------------- exact 1D integrals
// Linearisation of Legendre products (Adams-Neumann):
//   P_m P_n = sum_k A(m,n,k) P_{m+n-2k},
//   A = a(m-k) a(k) a(n-k) / a(m+n-k) * (2m+2n-4k+1) / (2m+2n-2k+1),  a(r) = (2r-1)!! / r!.
static long double lin_a(int r) {
  long double v = 1.0L;
  for (int j = 1; j <= r; ++j) v *= (long double)(2 * j - 1) / (long double)j;
  return v;
}

static long double leg_triple_unnormalised(int a, int b, int c) {
  // int P_a P_b P_c over [-1, 1]
  if ((a + b + c) % 2) return 0.0L;
  if (c > a + b || c < std::abs(a - b)) return 0.0L;
  int k = (a + b - c) / 2;
  long double A = lin_a(a - k) * lin_a(k) * lin_a(b - k) / lin_a(a + b - k) *
                  (long double)(2 * a + 2 * b - 4 * k + 1) / (long double)(2 * a + 2 * b - 2 * k + 1);
  return A * 2.0L / (long double)(2 * c + 1);
}

double leg_t3(int a, int b, int c) {
  long double nrm = sqrtl((long double)(2 * a + 1) * (2 * b + 1) * (2 * c + 1));
  return (double)(nrm * leg_triple_unnormalised(a, b, c));
}

double leg_d3(int a, int b, int c) {
  // P_a' = sum_{j < a, a - j odd} (2j + 1) P_j
  long double s = 0.0L;
  for (int j = a - 1; j >= 0; j -= 2) s += (long double)(2 * j + 1) * leg_triple_unnormalised(j, b, c);
  long double nrm = sqrtl((long double)(2 * a + 1) * (2 * b + 1) * (2 * c + 1));
  return (double)(nrm * s);
}

double leg_dm(int a, int b) {
  if (b < a && ((a + b) % 2) == 1) return 2.0 * std::sqrt((double)(2 * a + 1) * (2 * b + 1));
  return 0.0;
}

double leg_end(int m, int s) {
  double v = std::sqrt((double)(2 * m + 1));
  return (s < 0 && (m % 2)) ? -v : v;
}

// ---------------------------------------------------------------- reference tensors
RefTensors make_tensors(const Basis& B) {
  RefTensors T;
  const int d = B.d, nt = B.theta_t, ns = B.theta, np = d + 1;
  T.d = d;
  T.nt = nt;
  T.ns = ns;
  T.np = np;
  const double vol = std::ldexp(1.0, d);  // int over [-1,1]^d of 1
  T.Tt.assign((size_t)nt * nt, 0.0);
  T.Cc.assign((size_t)nt * ns, 0.0);
  for (int k = 0; k < nt; ++k) {
    const auto& bk = B.tidx[k];
    for (int l = 0; l < nt; ++l) {
      const auto& bl = B.tidx[l];
      bool same_space = true;
      for (int i = 1; i <= d; ++i) same_space &= (bk[i] == bl[i]);
      if (!same_space) continue;
      // int Psi_k(1) Psi_l(1) dxi - int int d_tau Psi_k Psi_l = 2^d [psi(1) psi(1) - int psi_k' psi_l]
      T.Tt[(size_t)k * nt + l] = vol * (leg_end(bk[0], 1) * leg_end(bl[0], 1) - leg_dm(bk[0], bl[0]));
    }
    for (int l = 0; l < ns; ++l) {
      const auto& al = B.sidx[l];
      bool same = true;
      for (int i = 0; i < d; ++i) same &= (bk[i + 1] == al[i]);
      if (same) T.Cc[(size_t)k * ns + l] = vol * leg_end(bk[0], -1);
    }
  }
  // p-mode exponent on spatial axis m
  auto pexp = [](int p, int m) { return (p == 1 + m) ? 1 : 0; };
  T.Bv.assign((size_t)d * np * nt * nt, 0.0);
  T.Fo.assign((size_t)d * 2 * np * nt * nt, 0.0);
  T.Fn.assign((size_t)d * 2 * np * nt * nt, 0.0);
  T.Cv.assign((size_t)d * np * ns * nt, 0.0);
  T.CFo.assign((size_t)d * 2 * np * ns * nt, 0.0);
  T.CFn.assign((size_t)d * 2 * np * ns * nt, 0.0);
  for (int i = 0; i < d; ++i) {
    for (int p = 0; p < np; ++p) {
      if (p == 1 + i) continue;  // nu_i does not depend on xi_i
      for (int k = 0; k < nt; ++k) {
        const auto& bk = B.tidx[k];
        for (int l = 0; l < nt; ++l) {
          const auto& bl = B.tidx[l];
          // time axis: int psi_k0 psi_0 psi_l0 = 2 delta
          double tt = leg_t3(bk[0], 0, bl[0]);
          if (tt == 0.0) continue;
          double v = tt, fo[2] = {tt, tt}, fn[2] = {tt, tt};
          for (int m = 0; m < d; ++m) {
            int a = bk[m + 1], c = bl[m + 1], q = pexp(p, m);
            if (m == i) {
              v *= leg_d3(a, q, c);
              for (int s = 0; s < 2; ++s) {
                int sg = s ? 1 : -1;
                fo[s] *= sg * leg_end(a, sg) * leg_end(c, sg);
                fn[s] *= sg * leg_end(a, sg) * leg_end(c, -sg);
              }
            } else {
              double t3 = leg_t3(a, q, c);
              v *= t3;
              fo[0] *= t3;
              fo[1] *= t3;
              fn[0] *= t3;
              fn[1] *= t3;
            }
          }
          T.Bv[T.bv(i, p) + (size_t)k * nt + l] = v;
          for (int s = 0; s < 2; ++s) {
            int sg = s ? 1 : -1;
            T.Fo[T.f(i, sg, p) + (size_t)k * nt + l] = fo[s];
            T.Fn[T.f(i, sg, p) + (size_t)k * nt + l] = fn[s];
          }
        }
      }
      for (int k = 0; k < ns; ++k) {
        const auto& ak = B.sidx[k];
        for (int l = 0; l < nt; ++l) {
          const auto& bl = B.tidx[l];
          double tt = leg_t3(0, 0, bl[0]);  // Phi has no time dependence
          if (tt == 0.0) continue;
          double v = tt, fo[2] = {tt, tt}, fn[2] = {tt, tt};
          for (int m = 0; m < d; ++m) {
            int a = ak[m], c = bl[m + 1], q = pexp(p, m);
            if (m == i) {
              v *= leg_d3(a, q, c);
              for (int s = 0; s < 2; ++s) {
                int sg = s ? 1 : -1;
                fo[s] *= sg * leg_end(a, sg) * leg_end(c, sg);
                fn[s] *= sg * leg_end(a, sg) * leg_end(c, -sg);
              }
            } else {
              double t3 = leg_t3(a, q, c);
              v *= t3;
              fo[0] *= t3;
              fo[1] *= t3;
              fn[0] *= t3;
              fn[1] *= t3;
            }
          }
          T.Cv[T.cv(i, p) + (size_t)k * nt + l] = v;
          for (int s = 0; s < 2; ++s) {
            int sg = s ? 1 : -1;
            T.CFo[T.cf(i, sg, p) + (size_t)k * nt + l] = fo[s];
            T.CFn[T.cf(i, sg, p) + (size_t)k * nt + l] = fn[s];
          }
        }
      }
    }
  }
  // volume term minus the faces that take the element's own trace, per set of such faces
  T.Cown.assign((size_t)d * np * 4 * ns * nt, 0.0);
  for (int i = 0; i < d; ++i)
    for (int p = 0; p < np; ++p)
      for (int bits = 0; bits < 4; ++bits) {
        double* C = &T.Cown[T.cown(i, p, bits)];
        for (size_t q = 0; q < (size_t)ns * nt; ++q) {
          double v = T.Cv[T.cv(i, p) + q];
          if (bits & 1) v -= T.CFo[T.cf(i, -1, p) + q];
          if (bits & 2) v -= T.CFo[T.cf(i, 1, p) + q];
          C[q] = v;
        }
      }
  return T;
}

// ---------------------------------------------------------------- problem / velocity
int resolve_problem(const ridg_problem* p, Problem* out, std::string* msg) {
  if (!p) {
    *msg = "problem is NULL";
    return RIDG_E_INVAL;
  }
  Problem P;
  P.d = p->dim;
  if (P.d < 1 || P.d > 3) {
    *msg = "dim must be 1, 2 or 3";
    return RIDG_E_INVAL;
  }
  if (p->basis != RIDG_BASIS_P && p->basis != RIDG_BASIS_Q) {
    *msg = "unknown basis";
    return RIDG_E_INVAL;
  }
  P.basis = p->basis;
  P.nel = 1;
  for (int i = 0; i < 3; ++i) {
    if (i < P.d) {
      if (p->n[i] < 3) {
        *msg = "n[i] must be >= 3 (the 3^d region elements must be distinct)";
        return RIDG_E_INVAL;
      }
      if (p->n[i] > (1 << 20)) {
        *msg = "n[i] too large";
        return RIDG_E_INVAL;
      }
      const double L = p->length[i] == 0.0 ? 1.0 : p->length[i];
      if (!(L > 0.0) || !std::isfinite(L)) {
        *msg = "length[i] must be positive and finite (0 stands for 1)";
        return RIDG_E_INVAL;
      }
      P.n[i] = p->n[i];
      P.L[i] = L;
      P.h[i] = L / p->n[i];
      P.nel *= p->n[i];
    } else {
      P.n[i] = 1;
      P.L[i] = 1.0;
      P.h[i] = 1.0;
    }
  }
  if (P.nel > (int64_t)1 << 31) {
    *msg = "more than 2^31 elements";
    return RIDG_E_INVAL;
  }
  P.M = p->order;
  if (P.M < 1) {
    *msg = "order must be >= 1";
    return RIDG_E_INVAL;
  }
  const int max_order = (P.basis == RIDG_BASIS_Q && P.d == 1) ? kMaxOrderQ1 : kMaxOrder;
  if (P.M > max_order) {
    *msg = P.basis == RIDG_BASIS_Q && P.d == 1 ? "order above 12 is not implemented for the 1D tensor basis"
                                               : "order above 5 is not implemented";
    return RIDG_E_UNSUPPORTED;
  }
  if (p->reserved != 0) {
    *msg = "reserved must be 0";
    return RIDG_E_INVAL;
  }
  P.flux = p->flux;
  Affine& v = P.vel;
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(p->velocity[i])) {
      *msg = "velocity not finite";
      return RIDG_E_INVAL;
    }
  if (P.flux == RIDG_FLUX_CONST) {
    for (int i = 0; i < P.d; ++i) v.a[i] = p->velocity[i];
  } else if (P.flux == RIDG_FLUX_ROTATION) {
    if (P.d != 2) {
      *msg = "RIDG_FLUX_ROTATION needs dim == 2";
      return RIDG_E_INVAL;
    }
    double cx = p->rot_center[0], cy = p->rot_center[1];
    if (!std::isfinite(cx) || !std::isfinite(cy)) {
      *msg = "rot_center not finite";
      return RIDG_E_INVAL;
    }
    // v = (-(y - cy), x - cx) = (cy, -cx) + [[0, -1], [1, 0]] x
    v.a[0] = cy;
    v.a[1] = -cx;
    v.g[0][1] = -1.0;
    v.g[1][0] = 1.0;
  } else if (P.flux == RIDG_FLUX_BURGERS) {
    // nonlinear flux q^2 / 2 along every axis: the velocity fields are not used
  } else if (P.flux == RIDG_FLUX_AFFINE) {
    for (int i = 0; i < P.d; ++i) {
      v.a[i] = p->velocity[i];
      for (int j = 0; j < P.d; ++j) {
        double gij = p->vel_grad[3 * i + j];
        if (!std::isfinite(gij)) {
          *msg = "vel_grad not finite";
          return RIDG_E_INVAL;
        }
        if (i == j && gij != 0.0) {
          *msg = "vel_grad diagonal must be zero (v_i independent of x_i)";
          return RIDG_E_INVAL;
        }
        v.g[i][j] = gij;
      }
    }
  } else {
    *msg = "unknown flux kind";
    return RIDG_E_INVAL;
  }
  P.precision = p->precision;
  if (P.precision != RIDG_FP64 && P.precision != RIDG_FP32_REFINE) {
    *msg = "unknown precision";
    return RIDG_E_INVAL;
  }
  P.refine = p->refine_steps;
  if (P.refine < 0 || P.refine > 3) {
    *msg = "refine_steps must be in 0..3";
    return RIDG_E_INVAL;
  }
  int solver = p->solver;
  if (solver == RIDG_SOLVER_AUTO)
    solver = (P.flux == RIDG_FLUX_CONST) ? RIDG_SOLVER_PREFACTORED
                                         : (P.flux == RIDG_FLUX_BURGERS ? RIDG_SOLVER_NEWTON : RIDG_SOLVER_REGION);
  if (solver < RIDG_SOLVER_PREFACTORED || solver > RIDG_SOLVER_NEWTON) {
    *msg = "unknown solver";
    return RIDG_E_INVAL;
  }
  if ((solver == RIDG_SOLVER_NEWTON) != (P.flux == RIDG_FLUX_BURGERS)) {
    *msg = "RIDG_FLUX_BURGERS is solved by (and only by) RIDG_SOLVER_NEWTON";
    return RIDG_E_INVAL;
  }
  if (P.flux == RIDG_FLUX_BURGERS) {
    if (p->newton_max_iter < 0 || p->newton_max_iter > 100) {
      *msg = "newton_max_iter must be in 0..100";
      return RIDG_E_INVAL;
    }
    P.newton_max = p->newton_max_iter ? p->newton_max_iter : 20;
    if (P.precision != RIDG_FP64) {
      *msg = "RIDG_FLUX_BURGERS runs in FP64";
      return RIDG_E_UNSUPPORTED;
    }
    if (!burgers_supported(P.d, P.M)) {
      *msg = "RIDG_FLUX_BURGERS is implemented for orders 1-5 in 1D, 1-4 in 2D and 1-2 in 3D";
      return RIDG_E_UNSUPPORTED;
    }
  } else if (p->newton_max_iter != 0) {
    *msg = "newton_max_iter must be 0 for the linear fluxes";
    return RIDG_E_INVAL;
  }
  if (solver == RIDG_SOLVER_PREFACTORED && P.flux != RIDG_FLUX_CONST) {
    *msg = "RIDG_SOLVER_PREFACTORED needs a constant velocity";
    return RIDG_E_INVAL;
  }
  if (P.precision == RIDG_FP32_REFINE && solver != RIDG_SOLVER_REGION &&
      !(solver == RIDG_SOLVER_PREFACTORED && brick_supported(P.d, P.M, P.n, true))) {
    *msg = "RIDG_FP32_REFINE is implemented for RIDG_SOLVER_REGION, and for RIDG_SOLVER_PREFACTORED in 3D at "
           "orders 2-3 on meshes with n[0] % 16 == 0, n[1] % 4 == 0, n[2] % 4 == 0";
    return RIDG_E_UNSUPPORTED;
  }
  if (P.basis == RIDG_BASIS_Q &&
      (P.d > 2 || P.flux != RIDG_FLUX_CONST || solver != RIDG_SOLVER_PREFACTORED || P.precision != RIDG_FP64)) {
    *msg = "the tensor (Q) basis is implemented for constant-velocity FP64 problems in 1D and 2D (RIDG_SOLVER_AUTO or "
           "RIDG_SOLVER_PREFACTORED, composite stencil)";
    return RIDG_E_UNSUPPORTED;
  }
  P.solver = solver;
  // every face must have one upwind side
  int idx[3] = {0, 0, 0};
  if (P.flux != RIDG_FLUX_CONST && P.flux != RIDG_FLUX_BURGERS) {
    // v_i depends on x_j (j != i) only through element rows: scan each axis line once
    for (int i = 0; i < P.d; ++i) {
      int64_t lines = P.nel / P.n[i];
      for (int64_t t = 0; t < lines; ++t) {
        int64_t r = t;
        for (int j = 0; j < P.d; ++j) {
          if (j == i) {
            idx[j] = 0;
            continue;
          }
          idx[j] = (int)(r % P.n[j]);
          r /= P.n[j];
        }
        if (face_side(P, idx, i, 1) < 0) {
          *msg = "the normal velocity changes sign inside a face; put the zero line of v on element boundaries";
          return RIDG_E_INVAL;
        }
      }
    }
  }
  *out = P;
  return RIDG_OK;
}

void nu_coeffs(const Problem& P, const int idx[3], double dt, double c0[3], double c[3][3]) {
  for (int i = 0; i < 3; ++i) {
    c0[i] = 0.0;
    for (int j = 0; j < 3; ++j) c[i][j] = 0.0;
  }
  for (int i = 0; i < P.d; ++i) {
    double v = P.vel.a[i];
    for (int j = 0; j < P.d; ++j) v += P.vel.g[i][j] * ((idx[j] + 0.5) * P.h[j]);
    c0[i] = v * dt / P.h[i];
    for (int j = 0; j < P.d; ++j) c[i][j] = P.vel.g[i][j] * (0.5 * P.h[j]) * dt / P.h[i];
  }
}

int face_side(const Problem& P, const int idx[3], int i, int s) {
  double c0[3], c[3][3];
  nu_coeffs(P, idx, 1.0, c0, c);
  double spread = 0.0;
  for (int j = 0; j < P.d; ++j) spread += std::fabs(c[i][j]);
  double mid = s * c0[i];
  double tol = 1e-12 * (std::fabs(c0[i]) + spread);
  double mn = mid - spread, mx = mid + spread;
  if (mn >= -tol) return 0;  // outflow (or no flow): own trace
  if (mx <= tol) return 1;   // inflow: neighbour trace
  return -1;
}

// ---------------------------------------------------------------- geometry and plans
std::vector<std::array<int, 3>> region_offsets(int d) {
  std::vector<std::array<int, 3>> out;
  int nb = 1;
  for (int i = 0; i < d; ++i) nb *= 3;
  for (int code = 0; code < nb; ++code) {
    std::array<int, 3> o = {0, 0, 0};
    int c = code;
    for (int i = d - 1; i >= 0; --i) {  // o_1 slowest
      o[i] = c % 3 - 1;
      c /= 3;
    }
    out.push_back(o);
  }
  return out;
}

void element_index(const Problem& P, int64_t e, int idx[3]) {
  for (int i = 0; i < 3; ++i) {
    if (i < P.d) {
      idx[i] = (int)(e % P.n[i]);
      e /= P.n[i];
    } else {
      idx[i] = 0;
    }
  }
}

int64_t element_linear(const Problem& P, const int idx[3]) {
  int64_t e = 0;
  for (int i = P.d - 1; i >= 0; --i) {
    int k = ((idx[i] % P.n[i]) + P.n[i]) % P.n[i];
    e = e * P.n[i] + k;
  }
  return e;
}

// periodic image of base + off (element positions always lie in the unit box)
static void wrapped(const Problem& P, const int base[3], const int off[3], int out[3]) {
  for (int i = 0; i < 3; ++i) {
    int k = base[i] + off[i];
    out[i] = (i < P.d) ? ((k % P.n[i]) + P.n[i]) % P.n[i] : 0;
  }
}

static int offset_code(int d, const int o[3]) {
  int c = 0;
  for (int i = 0; i < d; ++i) c = c * 3 + (o[i] + 1);
  return c;
}

// Region dependency graph of element e: pred[r] has bit r' set when block r takes the upwind trace
// of block r' on some face inside the region (src_of[r][face] = r', -1 for own-trace faces).
static void region_graph(const Problem& P, int64_t e, const std::vector<std::array<int, 3>>& offs,
                         uint32_t pred[kMaxBlocks], int src_of[kMaxBlocks][6]) {
  const int d = P.d, nb = (int)offs.size();
  int base[3];
  element_index(P, e, base);
  for (int r = 0; r < nb; ++r) {
    pred[r] = 0;
    int g[3];
    wrapped(P, base, offs[r].data(), g);
    for (int f = 0; f < 6; ++f) src_of[r][f] = -1;
    for (int i = 0; i < d; ++i) {
      for (int s = -1; s <= 1; s += 2) {
        int o2[3] = {offs[r][0], offs[r][1], offs[r][2]};
        o2[i] += s;
        if (o2[i] < -1 || o2[i] > 1) continue;  // region boundary: own trace
        if (face_side(P, g, i, s) == 1) {
          int r2 = offset_code(d, o2);
          pred[r] |= 1u << r2;
          src_of[r][2 * i + (s > 0)] = r2;
        }
      }
    }
  }
}

static uint32_t ancestors(const uint32_t pred[kMaxBlocks], int nb, int root) {
  uint32_t anc = 1u << root, frontier = anc;
  while (frontier) {
    uint32_t nxt = 0;
    for (int r = 0; r < nb; ++r)
      if (frontier & (1u << r)) nxt |= pred[r];
    nxt &= ~anc;
    anc |= nxt;
    frontier = nxt;
  }
  return anc;
}

// Topological order of the blocks in `set` (Kahn, lowest index first), blocks in `known` being
// already available; false on a cycle.
static bool topo_order(const uint32_t pred[kMaxBlocks], int nb, uint32_t set, uint32_t known, int* order,
                       int* count) {
  uint32_t done = known;
  int placed = 0;
  const int want = __builtin_popcount(set);
  while (placed < want) {
    int pick = -1;
    for (int r = 0; r < nb; ++r) {
      if (!(set & (1u << r)) || (done & (1u << r))) continue;
      if ((pred[r] & (set | known) & ~done) == 0) {
        pick = r;
        break;
      }
    }
    if (pick < 0) return false;
    order[placed++] = pick;
    done |= 1u << pick;
  }
  *count = placed;
  return true;
}

static void fill_plan(const std::vector<std::array<int, 3>>& offs, int d, const int* order, int count,
                      const int src_of[kMaxBlocks][6], PlanRec* out) {
  int pos[kMaxBlocks];
  for (int q = 0; q < count; ++q) pos[order[q]] = q;
  std::memset(out, 0, sizeof(*out));
  out->nb = count;
  for (int q = 0; q < count; ++q) {
    int r = order[q];
    PlanBlock& b = out->blk[q];
    for (int i = 0; i < 3; ++i) b.off[i] = (int8_t)offs[r][i];
    for (int f = 0; f < 6; ++f) b.src[f] = kOwn;
    for (int f = 0; f < 2 * d; ++f)
      if (src_of[r][f] >= 0) b.src[f] = (uint8_t)pos[src_of[r][f]];
  }
}

bool element_plan(const Problem& P, int64_t e, PlanRec* out) {
  const int d = P.d;
  auto offs = region_offsets(d);
  const int nb = (int)offs.size();
  uint32_t pred[kMaxBlocks];
  int src_of[kMaxBlocks][6];
  region_graph(P, e, offs, pred, src_of);
  const int centre = (nb - 1) / 2;
  const uint32_t anc = ancestors(pred, nb, centre);
  int order[kMaxBlocks], count = 0;
  if (!topo_order(pred, nb, anc, 0u, order, &count)) return false;  // dependency cycle among the ancestors
  fill_plan(offs, d, order, count, src_of, out);  // the centre comes last: every other block is its ancestor
  return true;
}

bool element_tear_plan(const Problem& P, int64_t e, PlanRec* out) {
  const int d = P.d;
  auto offs = region_offsets(d);
  const int nb = (int)offs.size();
  uint32_t pred[kMaxBlocks];
  int src_of[kMaxBlocks][6];
  region_graph(P, e, offs, pred, src_of);
  const int centre = (nb - 1) / 2;
  const uint32_t anc = ancestors(pred, nb, centre);
  for (int t = 0; t < nb; ++t) {
    if (!(anc & (1u << t))) continue;
    int order[kMaxBlocks], count = 0;
    if (!topo_order(pred, nb, anc & ~(1u << t), 1u << t, order + 1, &count)) continue;
    order[0] = t;  // the tear block is position 0; the others follow in elimination order
    fill_plan(offs, d, order, count + 1, src_of, out);
    out->pad[0] = 1;  // one tear block
    for (int q = 0; q <= count; ++q)
      if (order[q] == centre) out->pad[1] = q;
    return true;
  }
  return false;
}

static int n_spacetime_host(int d, int M) {
  int r = 1;
  for (int i = 1; i <= d + 1; ++i) r = r * (M + d - (d + 1) + i) / i;
  return r;
}

int plan_max_blocks(int d) { return d == 3 ? 8 : (d == 2 ? 9 : 3); }

HostPlanTables build_plan_tables(const Problem& P, const RefTensors& T, double dt) {
  const int d = P.d, nt = T.nt, ns = T.ns, np = T.np;
  const size_t nn = (size_t)nt * nt;
  HostPlanTables H;
  // transverse slopes of nu_i (identical on every element)
  double Vs[3][4] = {{0}};
  {
    int idx[3] = {0, 0, 0};
    double c0[3], c[3][3];
    nu_coeffs(P, idx, dt, c0, c);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Vs[i][1 + j] = c[i][j] / std::sqrt(3.0);
  }
  const int nmask = 1 << (2 * d);
  H.A0.assign((size_t)nmask * nn, 0.0);
  for (int m = 0; m < nmask; ++m) {
    double* A = &H.A0[(size_t)m * nn];
    for (size_t q = 0; q < nn; ++q) A[q] = T.Tt[q];
    for (int i = 0; i < d; ++i) {
      const int bits = (m >> (2 * i)) & 3;
      for (int p = 1; p < np; ++p) {
        const double v = Vs[i][p];
        if (v == 0.0 || p == 1 + i) continue;
        const double* bv = &T.Bv[T.bv(i, p)];
        for (size_t q = 0; q < nn; ++q) A[q] -= v * bv[q];
        for (int sd = 0; sd < 2; ++sd) {
          if (!((bits >> sd) & 1)) continue;
          const double* fo = &T.Fo[T.f(i, sd ? 1 : -1, p)];
          for (size_t q = 0; q < nn; ++q) A[q] += v * fo[q];
        }
      }
    }
  }
  H.K.assign((size_t)d * 4 * nn, 0.0);
  for (int i = 0; i < d; ++i)
    for (int bits = 0; bits < 4; ++bits) {
      double* K = &H.K[((size_t)i * 4 + bits) * nn];
      const double* bv = &T.Bv[T.bv(i, 0)];
      for (size_t q = 0; q < nn; ++q) K[q] = -bv[q];
      for (int sd = 0; sd < 2; ++sd) {
        if (!((bits >> sd) & 1)) continue;
        const double* fo = &T.Fo[T.f(i, sd ? 1 : -1, 0)];
        for (size_t q = 0; q < nn; ++q) K[q] += fo[q];
      }
    }
  H.Fn0.assign((size_t)d * 2 * nn, 0.0);
  H.FnC.assign((size_t)d * 2 * nn, 0.0);
  for (int i = 0; i < d; ++i)
    for (int sd = 0; sd < 2; ++sd) {
      const int s = sd ? 1 : -1;
      const double* f0 = &T.Fn[T.f(i, s, 0)];
      double* F0 = &H.Fn0[((size_t)i * 2 + sd) * nn];
      double* FC = &H.FnC[((size_t)i * 2 + sd) * nn];
      for (size_t q = 0; q < nn; ++q) F0[q] = f0[q];
      for (int p = 1; p < np; ++p) {
        const double v = Vs[i][p];
        if (v == 0.0 || p == 1 + i) continue;
        const double* fp = &T.Fn[T.f(i, s, p)];
        for (size_t q = 0; q < nn; ++q) FC[q] += v * fp[q];
      }
    }
  H.cc_idx.assign(nt, 0);
  H.cc_val.assign(nt, 0.0);
  for (int k = 0; k < nt; ++k)
    for (int l = 0; l < ns; ++l)
      if (T.Cc[(size_t)k * ns + l] != 0.0) {
        H.cc_idx[k] = l;
        H.cc_val[k] = T.Cc[(size_t)k * ns + l];
      }
  return H;
}

// Growth of elimination without row exchanges on the diagonal region blocks. V_i0 is affine in
// the element centre, so its range over the mesh is spanned by the box corners; the grid samples
// that range (5 points per axis in 1D/2D, 3 in 3D) for every face mask.
double static_pivot_growth(const Problem& P, const HostPlanTables& H, int nt, double dt) {
  const int d = P.d;
  const size_t nn = (size_t)nt * nt;
  double vmin[3] = {0, 0, 0}, vmax[3] = {0, 0, 0};
  for (int i = 0; i < d; ++i) {
    vmin[i] = 1e300;
    vmax[i] = -1e300;
    for (int c = 0; c < (1 << d); ++c) {
      double v = P.vel.a[i];
      for (int j = 0; j < d; ++j) {
        const double x = ((c >> j) & 1) ? P.L[j] - 0.5 * P.h[j] : 0.5 * P.h[j];
        v += P.vel.g[i][j] * x;
      }
      v *= dt / P.h[i];
      vmin[i] = std::min(vmin[i], v);
      vmax[i] = std::max(vmax[i], v);
    }
  }
  const int per = d == 3 ? 3 : 5;
  int npts = 1;
  for (int i = 0; i < d; ++i) npts *= per;
  double worst = 1.0;
  std::vector<double> A(nn);
  for (int mask = 0; mask < (1 << (2 * d)); ++mask) {
    for (int q = 0; q < npts; ++q) {
      double V[3] = {0, 0, 0};
      int r = q;
      for (int i = 0; i < d; ++i) {
        const int s = r % per;
        r /= per;
        V[i] = vmin[i] + (vmax[i] - vmin[i]) * s / (per - 1);
      }
      // only the face masks that occur at this velocity: the outflow face of every axis (s v_i > 0)
      // takes the block's own trace, so its bit is set
      bool occurs = true;
      for (int i = 0; i < d; ++i) {
        const int bits = (mask >> (2 * i)) & 3;
        if (V[i] > 0.0 && !(bits & 2)) occurs = false;
        if (V[i] < 0.0 && !(bits & 1)) occurs = false;
      }
      if (!occurs) continue;
      for (size_t z = 0; z < nn; ++z) A[z] = H.A0[(size_t)mask * nn + z];
      for (int i = 0; i < d; ++i) {
        const double* K = &H.K[((size_t)i * 4 + ((mask >> (2 * i)) & 3)) * nn];
        for (size_t z = 0; z < nn; ++z) A[z] = std::fma(V[i], K[z], A[z]);
      }
      double amax = 0.0;
      for (size_t z = 0; z < nn; ++z) amax = std::max(amax, std::fabs(A[z]));
      double gmax = amax;
      for (int c = 0; c < nt; ++c) {
        const double p = A[(size_t)c * nt + c];
        if (!(std::fabs(p) > 0.0)) return std::numeric_limits<double>::infinity();
        for (int rr = c + 1; rr < nt; ++rr) {
          const double l = A[(size_t)rr * nt + c] / p;
          if (l == 0.0) continue;
          for (int j = c + 1; j < nt; ++j) {
            A[(size_t)rr * nt + j] -= l * A[(size_t)c * nt + j];
            gmax = std::max(gmax, std::fabs(A[(size_t)rr * nt + j]));
          }
        }
      }
      worst = std::max(worst, amax > 0.0 ? gmax / amax : std::numeric_limits<double>::infinity());
    }
  }
  return worst;
}

RegionPlans build_plans(const Problem& P) {
  RegionPlans R;
  R.elem_plan.assign((size_t)P.nel, -1);
  std::map<std::string, int> ids;
  PlanRec rec;
  // For affine fields the plan depends on the element through its axis lines only; a cache
  // keyed by the face-side pattern keeps this linear in the element count.
  for (int64_t e = 0; e < P.nel; ++e) {
    if (!element_plan(P, e, &rec) || rec.nb > plan_max_blocks(P.d)) {
      PlanRec tr;
      if (n_spacetime_host(P.d, P.M) <= 64 && element_tear_plan(P, e, &tr) && tr.nb <= plan_max_blocks(P.d)) {
        R.tear_elems.push_back((int32_t)e);
        R.tear_plans.push_back(tr);
      } else {
        R.dense_elems.push_back((int32_t)e);
      }
      continue;
    }
    std::string key((const char*)&rec, sizeof(rec));
    auto it = ids.find(key);
    int id;
    if (it == ids.end()) {
      id = (int)R.plans.size();
      ids.emplace(key, id);
      R.plans.push_back(rec);
    } else {
      id = it->second;
    }
    R.elem_plan[(size_t)e] = id;
  }
  return R;
}

// ---------------------------------------------------------------- host assembly
static void velocity_modes(const Problem& P, const int idx[3], double dt, double V[3][4]) {
  double c0[3], c[3][3];
  nu_coeffs(P, idx, dt, c0, c);
  const double inv_sqrt3 = 1.0 / std::sqrt(3.0);
  for (int i = 0; i < 3; ++i) {
    V[i][0] = c0[i];
    for (int j = 0; j < 3; ++j) V[i][1 + j] = c[i][j] * inv_sqrt3;
  }
}

void assemble_region(const Problem& P, const RefTensors& T, int64_t e, double dt,
                     const std::vector<std::array<int, 3>>& offs, std::vector<double>* Aout) {
  const int d = P.d, nt = T.nt, np = T.np;
  const int nb = (int)offs.size();
  const int n = nb * nt;
  std::vector<double>& A = *Aout;
  A.assign((size_t)n * n, 0.0);
  int base[3];
  element_index(P, e, base);
  auto find = [&](const int o[3]) {
    for (int q = 0; q < nb; ++q)
      if (offs[q][0] == o[0] && offs[q][1] == o[1] && offs[q][2] == o[2]) return q;
    return -1;
  };
  for (int r = 0; r < nb; ++r) {
    int g[3];
    wrapped(P, base, offs[r].data(), g);
    double V[3][4];
    velocity_modes(P, g, dt, V);
    double* D = &A[(size_t)r * nt * n + (size_t)r * nt];
    for (int k = 0; k < nt; ++k)
      for (int l = 0; l < nt; ++l) D[(size_t)k * n + l] += T.Tt[(size_t)k * nt + l];
    for (int i = 0; i < d; ++i) {
      for (int p = 0; p < np; ++p) {
        double vp = V[i][p];
        if (vp == 0.0) continue;
        const double* bv = &T.Bv[T.bv(i, p)];
        for (int k = 0; k < nt; ++k)
          for (int l = 0; l < nt; ++l) D[(size_t)k * n + l] -= vp * bv[(size_t)k * nt + l];
      }
      for (int s = -1; s <= 1; s += 2) {
        int o2[3] = {offs[r][0], offs[r][1], offs[r][2]};
        o2[i] += s;
        bool boundary = (o2[i] < -1 || o2[i] > 1);
        int side = boundary ? 0 : face_side(P, g, i, s);
        int q = boundary ? -1 : find(o2);
        if (side == 1 && q < 0) continue;  // source outside the listed blocks (not an ancestor)
        double* Bk = (side == 0) ? D : &A[(size_t)r * nt * n + (size_t)q * nt];
        for (int p = 0; p < np; ++p) {
          double vp = V[i][p];
          if (vp == 0.0) continue;
          const double* f = side == 0 ? &T.Fo[T.f(i, s, p)] : &T.Fn[T.f(i, s, p)];
          for (int k = 0; k < nt; ++k)
            for (int l = 0; l < nt; ++l) Bk[(size_t)k * n + l] += vp * f[(size_t)k * nt + l];
        }
      }
    }
  }
}

bool lu_factor(int n, double* a, int* piv) {
  for (int c = 0; c < n; ++c) {
    int p = c;
    double best = std::fabs(a[(size_t)c * n + c]);
    for (int r = c + 1; r < n; ++r) {
      double v = std::fabs(a[(size_t)r * n + c]);
      if (v > best) {
        best = v;
        p = r;
      }
    }
    piv[c] = p;
    if (best == 0.0) return false;
    if (p != c)
      for (int j = 0; j < n; ++j) std::swap(a[(size_t)c * n + j], a[(size_t)p * n + j]);
    double inv = 1.0 / a[(size_t)c * n + c];
    for (int r = c + 1; r < n; ++r) {
      double l = a[(size_t)r * n + c] * inv;
      a[(size_t)r * n + c] = l;
      if (l == 0.0) continue;
      for (int j = c + 1; j < n; ++j) a[(size_t)r * n + j] -= l * a[(size_t)c * n + j];
    }
  }
  return true;
}

void lu_solve(int n, const double* lu, const int* piv, double* b, int nrhs) {
  for (int c = 0; c < n; ++c)
    if (piv[c] != c)
      for (int j = 0; j < nrhs; ++j) std::swap(b[(size_t)c * nrhs + j], b[(size_t)piv[c] * nrhs + j]);
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < r; ++c) {
      double l = lu[(size_t)r * n + c];
      if (l == 0.0) continue;
      for (int j = 0; j < nrhs; ++j) b[(size_t)r * nrhs + j] -= l * b[(size_t)c * nrhs + j];
    }
  for (int r = n - 1; r >= 0; --r) {
    for (int c = r + 1; c < n; ++c) {
      double u = lu[(size_t)r * n + c];
      if (u == 0.0) continue;
      for (int j = 0; j < nrhs; ++j) b[(size_t)r * nrhs + j] -= u * b[(size_t)c * nrhs + j];
    }
    double inv = 1.0 / lu[(size_t)r * n + r];
    for (int j = 0; j < nrhs; ++j) b[(size_t)r * nrhs + j] *= inv;
  }
}

int build_prefactored(const Problem& P, const RefTensors& T, double dt, Prefactored* out, std::string* msg) {
  PlanRec rec;
  if (!element_plan(P, 0, &rec)) {
    *msg = "constant velocity plan has a cycle";
    return RIDG_E_INVAL;
  }
  const int nt = T.nt, ns = T.ns, nb = rec.nb;
  std::vector<std::array<int, 3>> offs(nb);
  for (int q = 0; q < nb; ++q) offs[q] = {rec.blk[q].off[0], rec.blk[q].off[1], rec.blk[q].off[2]};
  std::vector<double> A;
  assemble_region(P, T, 0, dt, offs, &A);
  const int n = nb * nt;
  std::vector<int> piv(n);
  if (!lu_factor(n, A.data(), piv.data())) {
    *msg = "zero pivot in the region matrix";
    return RIDG_E_SINGULAR;
  }
  // right-hand sides: blockdiag(Cc), n x (nb ns)
  const int nr = nb * ns;
  std::vector<double> B((size_t)n * nr, 0.0);
  for (int q = 0; q < nb; ++q)
    for (int k = 0; k < nt; ++k)
      for (int l = 0; l < ns; ++l) B[(size_t)(q * nt + k) * nr + q * ns + l] = T.Cc[(size_t)k * ns + l];
  lu_solve(n, A.data(), piv.data(), B.data(), nr);
  // the centre is the last block of the plan
  out->offs = offs;
  out->G.assign((size_t)nb * nt * ns, 0.0);
  const int c = nb - 1;
  for (int q = 0; q < nb; ++q)
    for (int k = 0; k < nt; ++k)
      for (int l = 0; l < ns; ++l)
        out->G[((size_t)q * nt + k) * ns + l] = B[(size_t)(c * nt + k) * nr + q * ns + l];
  return RIDG_OK;
}

void build_correction_taps(const Problem& P, const RefTensors& T, double dt, TapOperator* out) {
  const int d = P.d, ns = T.ns, nt = T.nt;
  const double scale = std::ldexp(1.0, -d);
  out->rows = ns;
  out->cols = nt;
  out->offs.assign(1, {0, 0, 0});
  out->A.assign((size_t)ns * nt, 0.0);
  int idx[3] = {0, 0, 0};
  double c0[3], c[3][3];
  nu_coeffs(P, idx, dt, c0, c);
  auto add = [&](const std::array<int, 3>& o, const double* M, double f) {
    size_t t = 0;
    while (t < out->offs.size() && out->offs[t] != o) ++t;
    if (t == out->offs.size()) {
      out->offs.push_back(o);
      out->A.resize(out->offs.size() * (size_t)ns * nt, 0.0);
    }
    double* A = &out->A[t * (size_t)ns * nt];
    for (size_t q = 0; q < (size_t)ns * nt; ++q) A[q] += f * M[q];
  };
  for (int i = 0; i < d; ++i) {
    const double vi = c0[i];
    if (vi == 0.0) continue;
    add({0, 0, 0}, &T.Cv[T.cv(i, 0)], scale * vi);
    for (int s = -1; s <= 1; s += 2) {
      if (face_side(P, idx, i, s) == 0) {
        add({0, 0, 0}, &T.CFo[T.cf(i, s, 0)], -scale * vi);
      } else {
        std::array<int, 3> o = {0, 0, 0};
        o[i] = s;
        add(o, &T.CFn[T.cf(i, s, 0)], -scale * vi);
      }
    }
  }
}

std::vector<double> mfma_fragments(const double* A, int ntaps, int rows, int cols) {
  const int mt_n = (rows + 15) / 16, cq_n = (cols + 3) / 4;
  std::vector<double> f(mfma_fragment_doubles(ntaps, rows, cols), 0.0);
  size_t at = 0;
  for (int mt = 0; mt < mt_n; ++mt)
    for (int t = 0; t < ntaps; ++t)
      for (int q = 0; q < cq_n; ++q)
        for (int lane = 0; lane < 64; ++lane, ++at) {
          const int r = 16 * mt + lane % 16, c = 4 * q + lane / 16;
          if (r < rows && c < cols) f[at] = A[((size_t)t * rows + r) * cols + c];
        }
  return f;
}

void build_composite(const Problem& P, const Prefactored& G, const TapOperator& Dc, TapOperator* out) {
  (void)P;
  const int ns = Dc.rows, nt = Dc.cols;
  out->rows = ns;
  out->cols = ns;
  out->offs.clear();
  out->A.clear();
  for (size_t t = 0; t < Dc.offs.size(); ++t)
    for (size_t g = 0; g < G.offs.size(); ++g) {
      std::array<int, 3> o = {Dc.offs[t][0] + G.offs[g][0], Dc.offs[t][1] + G.offs[g][1], Dc.offs[t][2] + G.offs[g][2]};
      size_t q = 0;
      while (q < out->offs.size() && out->offs[q] != o) ++q;
      if (q == out->offs.size()) {
        out->offs.push_back(o);
        out->A.resize(out->offs.size() * (size_t)ns * ns, 0.0);
      }
      double* K = &out->A[q * (size_t)ns * ns];
      const double* D = &Dc.A[t * (size_t)ns * nt];
      const double* Gs = &G.G[g * (size_t)nt * ns];
      for (int r = 0; r < ns; ++r)
        for (int k = 0; k < nt; ++k) {
          const double dv = D[(size_t)r * nt + k];
          if (dv == 0.0) continue;
          for (int c = 0; c < ns; ++c) K[(size_t)r * ns + c] += dv * Gs[(size_t)k * ns + c];
        }
    }
  // column order: offsets sorted by (x, y, z), so the taps of one (x, y) column follow each other
  // with increasing z (the 3D kernel that advances two z-neighbours per thread reuses one element's
  // load for the other's next tap); every composite kernel sums its taps in this order
  std::vector<size_t> perm(out->offs.size());
  for (size_t q = 0; q < perm.size(); ++q) perm[q] = q;
  std::sort(perm.begin(), perm.end(), [&](size_t a, size_t b) { return out->offs[a] < out->offs[b]; });
  std::vector<std::array<int, 3>> offs(perm.size());
  std::vector<double> A(out->A.size());
  for (size_t q = 0; q < perm.size(); ++q) {
    offs[q] = out->offs[perm[q]];
    std::copy_n(&out->A[perm[q] * (size_t)ns * ns], (size_t)ns * ns, &A[q * (size_t)ns * ns]);
  }
  out->offs.swap(offs);
  out->A.swap(A);
}


// ---------------------------------------------------------------- von Neumann analysis (constant v)
// Eigenvalues of a complex n x n matrix (row-major): Householder reduction to Hessenberg form, then
// explicitly shifted QR steps (Givens rotations, Wilkinson shifts) with deflation.
static void eig_complex(int n, std::vector<std::complex<double>> A, std::vector<std::complex<double>>* ev) {
  using cd = std::complex<double>;
  auto at = [&](int r, int c) -> cd& { return A[(size_t)r * n + c]; };
  for (int k = 0; k + 2 < n; ++k) {  // Householder: zero column k below row k + 1
    double xn = 0.0;
    for (int i = k + 1; i < n; ++i) xn += std::norm(at(i, k));
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const cd x0 = at(k + 1, k);
    const cd ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cd(1.0, 0.0);
    std::vector<cd> v(n, 0.0);
    v[k + 1] = x0 + ph * xn;
    for (int i = k + 2; i < n; ++i) v[i] = at(i, k);
    double vn = 0.0;
    for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
    if (vn == 0.0) continue;
    for (int j = 0; j < n; ++j) {  // A = (I - 2 v v^H / |v|^2) A
      cd s = 0.0;
      for (int i = k + 1; i < n; ++i) s += std::conj(v[i]) * at(i, j);
      s *= 2.0 / vn;
      for (int i = k + 1; i < n; ++i) at(i, j) -= v[i] * s;
    }
    for (int i = 0; i < n; ++i) {  // A = A (I - 2 v v^H / |v|^2)
      cd s = 0.0;
      for (int j = k + 1; j < n; ++j) s += at(i, j) * v[j];
      s *= 2.0 / vn;
      for (int j = k + 1; j < n; ++j) at(i, j) -= s * std::conj(v[j]);
    }
  }
  ev->clear();
  int hi = n - 1, iter = 0;
  std::vector<double> gc(n);
  std::vector<cd> gs(n);
  while (hi >= 0) {
    if (hi == 0) {
      ev->push_back(at(0, 0));
      break;
    }
    int lo = hi;
    while (lo > 0) {
      const double scale = std::abs(at(lo, lo)) + std::abs(at(lo - 1, lo - 1));
      if (std::abs(at(lo, lo - 1)) <= 1e-15 * (scale > 0.0 ? scale : 1.0)) break;
      --lo;
    }
    if (lo == hi || iter > 300) {  // deflate (or give up on this eigenvalue after many steps)
      ev->push_back(at(hi, hi));
      if (hi > 0) at(hi, hi - 1) = 0.0;
      --hi;
      iter = 0;
      continue;
    }
    ++iter;
    const cd a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
    const cd tr = a + d, det = a * d - b * c;
    const cd disc = std::sqrt(tr * tr / 4.0 - det);
    cd mu = (std::abs(tr / 2.0 + disc - d) < std::abs(tr / 2.0 - disc - d)) ? tr / 2.0 + disc : tr / 2.0 - disc;
    if (iter % 11 == 10) mu = d + std::abs(at(hi, hi - 1));  // exceptional shift
    for (int k = lo; k <= hi; ++k) at(k, k) -= mu;
    for (int k = lo; k < hi; ++k) {  // QR of the active block by Givens rotations
      const cd x = at(k, k), y = at(k + 1, k);
      const double r = std::sqrt(std::norm(x) + std::norm(y));
      double cc = 1.0;
      cd ss = 0.0;
      if (r > 0.0) {
        if (std::abs(x) == 0.0) {
          cc = 0.0;
          ss = std::conj(y) / std::abs(y);
        } else {
          cc = std::abs(x) / r;
          ss = (x / std::abs(x)) * std::conj(y) / r;
        }
      }
      gc[k] = cc;
      gs[k] = ss;
      for (int j = k; j < n; ++j) {
        const cd p = at(k, j), q = at(k + 1, j);
        at(k, j) = cc * p + ss * q;
        at(k + 1, j) = -std::conj(ss) * p + cc * q;
      }
    }
    for (int k = lo; k < hi; ++k) {  // R Q
      const double cc = gc[k];
      const cd ss = gs[k];
      const int rmax = std::min(k + 2, hi);
      for (int i = 0; i <= rmax; ++i) {
        const cd p = at(i, k), q = at(i, k + 1);
        at(i, k) = p * cc + q * std::conj(ss);
        at(i, k + 1) = -p * ss + q * cc;
      }
    }
    for (int k = lo; k <= hi; ++k) at(k, k) += mu;
  }
}

double spectral_radius(const TapOperator& K, int d, int nk) {
  using cd = std::complex<double>;
  const int ns = K.rows;
  int npts = 1;
  for (int i = 0; i < d; ++i) npts *= nk;
  double worst = 0.0;
  std::vector<cd> G((size_t)ns * ns);
  std::vector<cd> ev;
  const double two_pi = 6.283185307179586476925;
  for (int q = 0; q < npts; ++q) {
    double kap[3] = {0, 0, 0};
    int r = q;
    for (int i = 0; i < d; ++i) {
      kap[i] = two_pi * (r % nk) / nk;
      r /= nk;
    }
    for (int z = 0; z < ns * ns; ++z) G[z] = 0.0;
    for (int z = 0; z < ns; ++z) G[(size_t)z * ns + z] = 1.0;  // the identity of Q' = Q + ...
    for (size_t t = 0; t < K.offs.size(); ++t) {
      double ph = 0.0;
      for (int i = 0; i < d; ++i) ph += kap[i] * K.offs[t][i];
      const cd e(std::cos(ph), std::sin(ph));
      const double* A = &K.A[t * (size_t)ns * ns];
      for (int z = 0; z < ns * ns; ++z) G[z] += e * A[z];
    }
    eig_complex(ns, G, &ev);
    for (const cd& x : ev) worst = std::max(worst, std::abs(x));
  }
  return worst;
}

int von_neumann_radius(const Problem& P, const RefTensors& T, double dt, double* rho, std::string* msg) {
  if (P.flux != RIDG_FLUX_CONST) {
    *msg = "the von Neumann analysis needs a constant velocity";
    return RIDG_E_INVAL;
  }
  Prefactored pf;
  int rc = build_prefactored(P, T, dt, &pf, msg);
  if (rc) return rc;
  TapOperator dc, kc;
  build_correction_taps(P, T, dt, &dc);
  build_composite(P, pf, dc, &kc);
  const int nk = P.d == 1 ? 256 : (P.d == 2 ? 48 : 12);
  *rho = spectral_radius(kc, P.d, nk);
  return RIDG_OK;
}

}  // namespace ridg

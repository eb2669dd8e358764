// Host FP64 tables of the Burgers path (Newton prediction, Sec. 3; nonlinear correction, Sec. 2.3):
// basis values at tensor Gauss-Legendre points of the space-time element and of its faces, and the
// exact triple products beta^i_{k l p} = int int d_xi_i Psi_k Psi_p Psi_l of the quasi-quadrature-free
// Jacobian (eq. Jacobian2), which factor into one-dimensional Legendre integrals.
#include <cmath>

#include "ridg_internal.hpp"

namespace ridg {

namespace {

// P_m(x) and P_m'(x) by the three-term recurrence.
void legendre(int m, double x, double* p, double* dp) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (m == 0) {
    *p = 1.0;
    *dp = 0.0;
    return;
  }
  for (int k = 2; k <= m; ++k) {
    const double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    const double d2 = d0 + (2 * k - 1) * p1;  // P_k' = P_{k-2}' + (2k - 1) P_{k-1}
    p0 = p1;
    p1 = p2;
    d0 = d1;
    d1 = d2;
  }
  *p = p1;
  *dp = d1;
}

// psi_m = sqrt(2m+1) P_m and its derivative.
double psi(int m, double x) {
  double p, dp;
  legendre(m, x, &p, &dp);
  return std::sqrt(2.0 * m + 1.0) * p;
}
double dpsi(int m, double x) {
  double p, dp;
  legendre(m, x, &p, &dp);
  return std::sqrt(2.0 * m + 1.0) * dp;
}

// q-point Gauss-Legendre rule: the roots of P_q by Newton's method from the Chebyshev-like guesses
// cos(pi (j + 3/4) / (q + 1/2)), weights 2 / ((1 - x^2) P_q'(x)^2).
void gauss_rule(int q, std::vector<double>* x, std::vector<double>* w) {
  x->assign(q, 0.0);
  w->assign(q, 0.0);
  for (int j = 0; j < q; ++j) {
    double r = std::cos(M_PI * (j + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(q, r, &p, &dp);
      const double step = p / dp;
      r -= step;
      if (std::fabs(step) < 1e-17) break;
    }
    double p, dp;
    legendre(q, r, &p, &dp);
    (*x)[j] = r;
    (*w)[j] = 2.0 / ((1.0 - r * r) * dp * dp);
  }
}

}  // namespace

bool burgers_supported(int d, int M) {
  if (M < 1) return false;
  if (d == 1) return M <= 5;
  if (d == 2) return M <= 4;
  if (d == 3) return M <= 2;
  return false;
}

int build_burgers_tables(const Problem& P, const Basis& B, BurgersHost* out, std::string* msg) {
  const int d = P.d, M = P.M, nt = B.theta_t, ns = B.theta, nv = d + 1;
  if (!burgers_supported(d, M)) {
    *msg = "RIDG_FLUX_BURGERS is implemented for orders 1-5 in 1D, 1-4 in 2D and 1-2 in 3D";
    return RIDG_E_UNSUPPORTED;
  }
  BurgersHost& H = *out;
  H.q = burgers_q(M);
  std::vector<double> gx, gw;
  gauss_rule(H.q, &gx, &gw);
  H.nq = 1;
  for (int a = 0; a < nv; ++a) H.nq *= H.q;
  H.nqf = H.nq / H.q;
  // volume points: variable a (0 = tau, 1.. = xi) of point pt is digit a of pt in base q
  auto vcoord = [&](int pt, int a) {
    for (int b = 0; b < a; ++b) pt /= H.q;
    return pt % H.q;
  };
  const double pscale = std::ldexp(1.0, -(d + 1));
  H.psiv.assign((size_t)nt * H.nq, 0.0);
  H.projw.assign((size_t)nt * H.nq, 0.0);
  H.dpsivw.assign((size_t)d * nt * H.nq, 0.0);
  H.dphivw.assign((size_t)d * ns * H.nq, 0.0);
  for (int pt = 0; pt < H.nq; ++pt) {
    double wt = 1.0, x[4];
    for (int a = 0; a < nv; ++a) {
      x[a] = gx[vcoord(pt, a)];
      wt *= gw[vcoord(pt, a)];
    }
    for (int l = 0; l < nt; ++l) {
      const auto& b = B.tidx[l];
      double v = 1.0;
      for (int a = 0; a < nv; ++a) v *= psi(b[a], x[a]);
      H.psiv[(size_t)l * H.nq + pt] = v;
      H.projw[(size_t)l * H.nq + pt] = wt * v * pscale;
      for (int i = 0; i < d; ++i) {
        double dv = 1.0;
        for (int a = 0; a < nv; ++a) dv *= (a == i + 1) ? dpsi(b[a], x[a]) : psi(b[a], x[a]);
        H.dpsivw[((size_t)i * nt + l) * H.nq + pt] = wt * dv;
      }
    }
    for (int k = 0; k < ns; ++k) {
      const auto& al = B.sidx[k];
      for (int i = 0; i < d; ++i) {
        double dv = 1.0;
        for (int a = 0; a < d; ++a) dv *= (a == i) ? dpsi(al[a], x[a + 1]) : psi(al[a], x[a + 1]);
        H.dphivw[((size_t)i * ns + k) * H.nq + pt] = wt * dv;
      }
    }
  }
  // face points: (tau, xi_perp) in base q, xi_i = s on face f = 2 i + (s > 0)
  const int nf = 2 * d;
  H.psif.assign((size_t)nf * nt * H.nqf, 0.0);
  H.psifw.assign((size_t)nf * nt * H.nqf, 0.0);
  H.phifw.assign((size_t)nf * ns * H.nqf, 0.0);
  for (int f = 0; f < nf; ++f) {
    const int i = f / 2;
    const double s = (f % 2) ? 1.0 : -1.0;
    for (int pf = 0; pf < H.nqf; ++pf) {
      double x[4], wt = 1.0;
      int c = pf;
      for (int a = 0; a < nv; ++a) {
        if (a == i + 1) {
          x[a] = s;
          continue;
        }
        x[a] = gx[c % H.q];
        wt *= gw[c % H.q];
        c /= H.q;
      }
      for (int l = 0; l < nt; ++l) {
        const auto& b = B.tidx[l];
        double v = 1.0;
        for (int a = 0; a < nv; ++a) v *= psi(b[a], x[a]);
        H.psif[((size_t)f * nt + l) * H.nqf + pf] = v;
        H.psifw[((size_t)f * nt + l) * H.nqf + pf] = wt * v;
      }
      for (int k = 0; k < ns; ++k) {
        const auto& al = B.sidx[k];
        double v = 1.0;
        for (int a = 0; a < d; ++a) v *= psi(al[a], x[a + 1]);
        H.phifw[((size_t)f * ns + k) * H.nqf + pf] = wt * v;
      }
    }
  }
  // exact triple products, stored sparsely per (i, k, l)
  H.bptr.assign((size_t)d * nt * nt + 1, 0);
  H.bp.clear();
  H.bval.clear();
  for (int i = 0; i < d; ++i)
    for (int k = 0; k < nt; ++k)
      for (int l = 0; l < nt; ++l) {
        H.bptr[((size_t)i * nt + k) * nt + l] = (int32_t)H.bp.size();
        for (int p = 0; p < nt; ++p) {
          double v = 1.0;
          for (int a = 0; a < nv && v != 0.0; ++a) {
            const int kk = B.tidx[k][a], pp = B.tidx[p][a], ll = B.tidx[l][a];
            v *= (a == i + 1) ? leg_d3(kk, pp, ll) : leg_t3(kk, pp, ll);
          }
          if (std::fabs(v) > 1e-13) {
            H.bp.push_back(p);
            H.bval.push_back(v);
          }
        }
      }
  H.bptr[(size_t)d * nt * nt] = (int32_t)H.bp.size();
  H.lift.assign(ns, -1);
  for (int j = 0; j < ns; ++j)
    for (int l = 0; l < nt; ++l) {
      bool same = B.tidx[l][0] == 0;
      for (int a = 0; a < d; ++a) same &= B.tidx[l][a + 1] == B.sidx[j][a];
      if (same) H.lift[j] = l;
    }
  return RIDG_OK;
}

}  // namespace ridg

namespace ridg {

// Tables of the Jacobian-assembly comparison (any dimension, orders 1..6): the same point sets and
// exact triple products as the Burgers tables, with the directions summed (uniform dt / h).
int build_assembly_tables(int d, int M, AsmHost* out, std::string* msg) {
  if (d < 1 || d > 3 || M < 1 || M > 6) {
    *msg = "assembly comparison: dim 1..3, order 1..6";
    return RIDG_E_INVAL;
  }
  const Basis B = make_basis(d, M);
  const int nt = B.theta_t, nv = d + 1;
  AsmHost& H = *out;
  H.nt = nt;
  H.q = burgers_q(M);
  std::vector<double> gx, gw;
  gauss_rule(H.q, &gx, &gw);
  H.nq = 1;
  for (int a = 0; a < nv; ++a) H.nq *= H.q;
  const double pscale = std::ldexp(1.0, -(d + 1));
  H.psiv.assign((size_t)nt * H.nq, 0.0);
  H.projw.assign((size_t)nt * H.nq, 0.0);
  H.dsum.assign((size_t)nt * H.nq, 0.0);
  for (int pt = 0; pt < H.nq; ++pt) {
    double x[4], wt = 1.0;
    int c = pt;
    for (int a = 0; a < nv; ++a) {
      x[a] = gx[c % H.q];
      wt *= gw[c % H.q];
      c /= H.q;
    }
    for (int l = 0; l < nt; ++l) {
      const auto& b = B.tidx[l];
      double v = 1.0, dv = 0.0;
      for (int a = 0; a < nv; ++a) v *= psi(b[a], x[a]);
      for (int i = 0; i < d; ++i) {
        double t = 1.0;
        for (int a = 0; a < nv; ++a) t *= (a == i + 1) ? dpsi(b[a], x[a]) : psi(b[a], x[a]);
        dv += t;
      }
      H.psiv[(size_t)l * H.nq + pt] = v;
      H.projw[(size_t)l * H.nq + pt] = wt * v * pscale;
      H.dsum[(size_t)l * H.nq + pt] = wt * dv;
    }
  }
  H.rptr.assign((size_t)nt * nt + 1, 0);
  H.bp.clear();
  H.bval.clear();
  for (int k = 0; k < nt; ++k)
    for (int l = 0; l < nt; ++l) {
      H.rptr[(size_t)k * nt + l] = (int32_t)H.bp.size();
      for (int p = 0; p < nt; ++p) {
        double sum = 0.0;
        for (int i = 0; i < d; ++i) {
          double v = 1.0;
          for (int a = 0; a < nv && v != 0.0; ++a) {
            const int kk = B.tidx[k][a], pp = B.tidx[p][a], ll = B.tidx[l][a];
            v *= (a == i + 1) ? leg_d3(kk, pp, ll) : leg_t3(kk, pp, ll);
          }
          sum += v;
        }
        if (std::fabs(sum) > 1e-13) {
          H.bp.push_back(p);
          H.bval.push_back(sum);
        }
      }
    }
  H.rptr[(size_t)nt * nt] = (int32_t)H.bp.size();
  return RIDG_OK;
}

}  // namespace ridg

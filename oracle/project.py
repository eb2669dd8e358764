"""Projections, exact solutions and the paper's error measure (test infrastructure).

* ``project``: element-wise L2 projection X_e = (1/|T|) int_T Phi q (Sec. 4, the
  "exact projection" behind the error definition), by tensor Gauss quadrature.
* ``exact_translate`` / ``exact_rotation``: the exact solutions of constant
  advection (q0(x - v t), periodic) and of the solid-body rotation
  (q0 rotated by -t about the centre).
* ``l2rel_paper``: the approximate relative L2 error of eq. (l2relerror):
  coefficient error on the basis plus the next-degree truncation terms.
"""

import itertools

import numpy as np

from .basis import gauss, psi, spatial_indices


def _elem_points(prob_d, n, h, q):
    g, w = gauss(q)
    xi = np.array(list(itertools.product(g, repeat=prob_d))).T  # (d, P)
    wt = np.prod(np.array(list(itertools.product(w, repeat=prob_d))), axis=1)
    return xi, wt


def project(f, d, n, M, q=None, family="P", length=None):
    """(N_el, theta) coefficients of f on every element of the n-mesh.

    f takes points of shape (d, P) and returns values of shape (P,).
    Elements are numbered x fastest.
    """
    n = tuple(n)
    if length is None:
        length = (1.0,) * d
    h = np.array([L / k for L, k in zip(length, n)])
    if q is None:
        q = M + 8
    sidx = spatial_indices(d, M, family)
    xi, wt = _elem_points(d, n, h, q)
    basis = np.array([np.prod([psi(a[j], xi[j]) for j in range(d)], axis=0) for a in sidx])
    bw = basis * wt / (2.0 ** d)  # (theta, P): (1/2^d) sum w Phi
    n_el = int(np.prod(n))
    out = np.empty((n_el, len(sidx)))
    # iterate over elements (x fastest)
    grids = [np.arange(k) for k in n]
    for e, idx in enumerate(itertools.product(*reversed(grids))):
        idx = tuple(reversed(idx))
        xc = np.array([(i + 0.5) * hh for i, hh in zip(idx, h)])
        X = xc[:, None] + 0.5 * h[:, None] * xi
        out[e] = bw @ f(X)
    return out


def periodic_translate(f, v, t, length=None):
    """x -> f(x - v t) wrapped into the periodic box."""
    v = np.asarray(v, dtype=np.float64)

    def g(X):
        L = np.ones(X.shape[0]) if length is None else np.asarray(length)
        Y = np.mod(X - v[:, None] * t, L[:, None])
        return f(Y)

    return g


def exact_translate(f0, d, n, M, v, t, q=None, family="P"):
    """Projection of the exact solution of q_t + v.grad q = 0 at time t."""
    return project(periodic_translate(f0, v, t), d, n, M, q=q, family=family)


def exact_rotation(f0, n, M, centre, t, q=None):
    """Projection of q0 rotated by angle t about ``centre`` (v = (-(y-c_y), x-c_x))."""
    c = np.asarray(centre, dtype=np.float64)

    def g(X):
        dx, dy = X[0] - c[0], X[1] - c[1]
        ct, st = np.cos(t), np.sin(t)
        # the value at x came from R(-t)(x - c) + c
        x0 = c[0] + ct * dx + st * dy
        y0 = c[1] - st * dx + ct * dy
        return f0(np.array([x0, y0]))

    return project(g, 2, n, M, q=q)


def l2rel_paper(Q, f_exact, d, n, M, family="P", q=None):
    """Approximate relative L2 error of eq. (l2relerror).

    X are the exact projections onto the next-larger basis (order M+1); the
    error is the coefficient error on the first theta modes plus the norm of
    the modes theta+1..theta^+, relative to the norm of all theta^+ modes.
    """
    Xp = project(f_exact, d, n, M + 1, q=q, family=family)
    sidx = spatial_indices(d, M, family)
    sidx_p = spatial_indices(d, M + 1, family)
    pos = [sidx_p.index(a) for a in sidx]
    rest = [j for j in range(len(sidx_p)) if j not in pos]
    err = np.sum((Xp[:, pos] - Q) ** 2) + np.sum(Xp[:, rest] ** 2)
    return float(np.sqrt(err / np.sum(Xp ** 2)))

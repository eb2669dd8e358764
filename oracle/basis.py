"""Orthonormal Legendre bases and Gauss quadrature for the oracle (test infrastructure).

Sec. 2.1 of the paper asks for a spatial basis that is orthonormal with respect
to the element average, (1/|T|) int_T Phi_k Phi_l = delta_kl, and Sec. 2.2 asks
the same of the space-time basis on the space-time element. On the reference
interval [-1, 1] the scaled Legendre polynomials psi_m = sqrt(2m+1) P_m satisfy
(1/2) int psi_m psi_n = delta_mn, so tensor products of them are orthonormal on
the reference cube in exactly that sense.

Basis family: total degree (the P space). The paper's tensor (Q) space is
available too (``family='Q'``) for the one-dimensional comparison with the
printed convergence table.

Ordering (part of the library's data contract):
  * spatial index alpha = (a_1..a_d): by total degree, then lexicographically
    descending in (a_1, ..., a_d)  ("descending x-degree, then y-degree ...");
  * space-time index beta = (b_t, b_1..b_d): by total degree, then
    lexicographically descending in (b_t, b_1, ..., b_d).
"""

import itertools

import numpy as np
from numpy.polynomial import legendre as _leg


def _indices(nvar, M, family):
    out = []
    for idx in itertools.product(range(M), repeat=nvar):
        if family == "P" and sum(idx) > M - 1:
            continue
        out.append(idx)
    # total degree ascending, then lexicographically descending
    out.sort(key=lambda a: (sum(a), tuple(-x for x in a)))
    return out


def spatial_indices(d, M, family="P"):
    """Multi-indices of the spatial basis Phi on a d-cube, order M (= degree + 1)."""
    return _indices(d, M, family)


def spacetime_indices(d, M, family="P"):
    """Multi-indices (b_t, b_1..b_d) of the space-time basis Psi."""
    return _indices(d + 1, M, family)


def psi(m, s):
    """psi_m(s) = sqrt(2m+1) P_m(s): orthonormal w.r.t. (1/2) int_{-1}^{1}."""
    c = np.zeros(m + 1)
    c[m] = 1.0
    return np.sqrt(2 * m + 1) * _leg.legval(np.asarray(s, dtype=np.float64), c)


def dpsi(m, s):
    """Derivative of psi_m."""
    c = np.zeros(m + 1)
    c[m] = 1.0
    dc = _leg.legder(c) if m > 0 else np.zeros(1)
    return np.sqrt(2 * m + 1) * _leg.legval(np.asarray(s, dtype=np.float64), dc)


def gauss(q):
    """q-point Gauss-Legendre rule on [-1, 1] (exact for degree <= 2q-1)."""
    x, w = _leg.leggauss(q)
    return x.astype(np.float64), w.astype(np.float64)

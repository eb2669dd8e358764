"""Von Neumann analysis of the constant-velocity RIDG step (test infrastructure).

For constant v the whole step is a linear, translation-invariant map
Q'_e = sum_o K_o Q_{e+o}, with offsets o in {-2..2}^d (the region radius plus
the face neighbours used by the correction). The oracle's own step applied to
unit impulses on a periodic 5^d mesh yields every K_o; the amplification
matrix of the Fourier mode exp(i kappa.e) is G(kappa) = sum_o K_o exp(i kappa.o).
The paper's stability claim (Sec. 1 and Sec. 6.1: the largest stable CFL of
RIDG does not shrink with the order) is checked on max spectral radius.
"""

import itertools

import numpy as np

from .scheme import Problem, step


def stencil(d, M, v, nu, family="P"):
    """K_o (dict offset -> theta x theta) for velocity v and CFL nu = dt max|v_i| / h."""
    n = (5,) * d
    prob = Problem(d=d, n=n, M=M, velocity=("const", tuple(v)), family=family)
    dt = nu * prob.h[0] / max(abs(x) for x in v)
    th = prob.theta
    K = {}
    for o in itertools.product(range(-2, 3), repeat=d):
        K[o] = np.zeros((th, th))
    for ell in range(th):
        Q = np.zeros((prob.n_el, th))
        Q[0, ell] = 1.0
        Qn = step(prob, Q, dt, 1)
        for e in range(prob.n_el):
            idx = prob.multi(e)
            o = tuple(((-i + 2) % 5) - 2 for i in idx)
            K[o][:, ell] = Qn[e]
    return K


def spectral_radius(K, d, nk=64):
    """max over a kappa grid of the spectral radius of G(kappa)."""
    ks = 2 * np.pi * np.arange(nk) / nk
    offs = list(K)
    Ks = np.array([K[o] for o in offs])  # (O, th, th)
    O = np.array(offs, dtype=np.float64)  # (O, d)
    rmax = 0.0
    for kap in itertools.product(ks, repeat=d):
        ph = np.exp(1j * (O @ np.array(kap)))
        G = np.tensordot(ph, Ks, axes=(0, 0))
        rmax = max(rmax, float(np.max(np.abs(np.linalg.eigvals(G)))))
    return rmax


def nu_max(d, M, v, family="P", lo=0.05, hi=3.0, tol=1e-3, nk=32):
    """Largest CFL with max spectral radius <= 1 + 1e-12 (bisection)."""
    def stable(nu):
        return spectral_radius(stencil(d, M, v, nu, family), d, nk) <= 1 + 1e-12

    if not stable(lo):
        return 0.0
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if stable(mid):
            lo = mid
        else:
            hi = mid
    return lo

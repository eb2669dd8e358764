"""RIDG for the scalar Burgers equation with Newton iterations on the region system, written out
plainly in FP64 (test infrastructure).

The conservation law is q_t + sum_i (q^2 / 2)_{x_i} = 0 on a periodic box (eq. (burger2d) in two
dimensions; the same flux along every axis in one and three). In reference coordinates, with
c_i = dt / h_i and F(q) = q^2 / 2, the prediction residual of region element r is (Sec. 2.2 with
the nonlinear flux, the residual of Sec. 3)

    R_r = T W_r - sum_i c_i int int d_xi_i Psi F(w_r)
        + sum_faces c_i int int Psi|_face H(w_r, w_nbr; s e_i) - C Q^n_r,

w_r = Psi^T W_r. Inside the region H is the Rusanov flux
H(a, b; s e_i) = s (F(a) + F(b)) / 2 - alpha (b - a) / 2; on the region boundary it is the physical
flux of the element's own trace, s F(a). The correction (Sec. 2.3) is

    Q_e <- Q_e + 2^-d [ sum_i c_i int int d_xi_i Phi F(w_e) - sum_faces c_i int int Phi|_face H(w_e, w_nbr) ].

Readings where the paper leaves the choice open:
  * wave speed of the Rusanov flux: alpha = max(|Qbar_a|, |Qbar_b|) per face, from the averages
    (coefficient 0) of the two elements' states at t^n (|F'(q)| = |q|), in the prediction and in
    the correction alike. It is known before the prediction, so the region residual is a quadratic
    polynomial in W;
  * Newton (Sec. 3): W^(0) = Q^n held constant in time on every region element; the Jacobian is
    the exact derivative of the residual; iterate W <- W - J^-1 R until
    max|delta| <= tol * max(1, max|W|) (tol = 1e-13) or max_iter iterations.

Three ways to form the volume part of the Jacobian (Sec. 3): ``jacobian_volume_quadrature``
(quadrature of every entry), ``jacobian_volume_qqf`` (projection of F'(w) onto Psi, then the
precomputed triple products beta), and ``jacobian_perturbation`` (differences of the residual,
one column per unknown). All integrals here are tensor Gauss-Legendre sums with q = M + 2 points per
axis, exact for every polynomial integrand that occurs for M <= 6.
"""

import itertools
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

from .scheme import _reference
from .basis import spatial_indices, spacetime_indices

NEWTON_TOL = 1e-13


class NewtonFailure(RuntimeError):
    """The region system had no root within reach: too large a time step for the local compression."""


@dataclass
class BurgersProblem:
    d: int
    n: tuple
    M: int
    length: tuple = None
    family: str = "P"
    max_iter: int = 20
    tol: float = NEWTON_TOL
    _cache: dict = field(default_factory=dict, repr=False, compare=False)

    def __post_init__(self):
        self.n = tuple(int(x) for x in self.n)
        assert len(self.n) == self.d
        if self.length is None:
            self.length = (1.0,) * self.d
        self.length = tuple(float(x) for x in self.length)
        self.h = np.array([L / k for L, k in zip(self.length, self.n)])
        self.sidx = spatial_indices(self.d, self.M, self.family)
        self.tidx = spacetime_indices(self.d, self.M, self.family)
        self.theta = len(self.sidx)
        self.theta_t = len(self.tidx)
        self.n_el = int(np.prod(self.n))
        self.ref = _reference(self.d, self.M, self.family, self.M + 2)
        ref = self.ref
        self.T = (ref.Psi_top * ref.sw) @ ref.Psi_top.T - (ref.dPsi[0] * ref.vw) @ ref.Psi.T
        self.C = (ref.Psi_bot * ref.sw) @ ref.Phi_s.T
        # space-time coefficients of a spatial state held constant in time (b_t = 0)
        self.lift = np.zeros((self.theta_t, self.theta))
        for j, a in enumerate(self.sidx):
            self.lift[self.tidx.index((0,) + tuple(a)), j] = 1.0

    def multi(self, e):
        out = []
        for k in self.n:
            out.append(e % k)
            e //= k
        return tuple(out)

    def linear(self, idx):
        e = 0
        for k, i in zip(reversed(self.n), reversed(idx)):
            e = e * k + (i % k)
        return e


def flux(q):
    return 0.5 * q * q


def dflux(q):
    return q


def rusanov(a, b, s, alpha):
    """Rusanov flux through a face with outward normal s e_i (a own trace, b neighbour trace)."""
    return 0.5 * s * (flux(a) + flux(b)) - 0.5 * alpha * (b - a)


def _region(prob, e):
    offs = list(itertools.product((-1, 0, 1), repeat=prob.d))
    base = prob.multi(e)
    elems = [prob.linear(tuple(b + o for b, o in zip(base, oo))) for oo in offs]
    return offs, elems


def _faces(prob):
    return [(i, s) for i in range(prob.d) for s in (-1, 1)]


def wave_speed(qa, qb):
    """Rusanov wave speed of a face from the two elements' states at t^n."""
    return max(abs(qa[0]), abs(qb[0]))


def residual(prob, offs, Wr, Qr, dt):
    """Region residual (nb, theta_T) for region iterate Wr (nb, theta_T) and states Qr (nb, theta)."""
    ref, d = prob.ref, prob.d
    pos = {o: j for j, o in enumerate(offs)}
    c = dt / prob.h
    R = np.zeros_like(Wr)
    for j, o in enumerate(offs):
        w = ref.Psi.T @ Wr[j]
        r = prob.T @ Wr[j] - prob.C @ Qr[j]
        for i in range(d):
            r -= c[i] * ((ref.dPsi[i + 1] * ref.vw) @ flux(w))
        for (i, s) in _faces(prob):
            F = ref.face[(i, s)]
            a = F["Psi_own"].T @ Wr[j]
            o2 = list(o)
            o2[i] += s
            o2 = tuple(o2)
            if o2 in pos:
                k = pos[o2]
                b = F["Psi_nbr"].T @ Wr[k]
                H = rusanov(a, b, s, wave_speed(Qr[j], Qr[k]))
            else:
                H = s * flux(a)
            r += c[i] * ((F["Psi_own"] * ref.fw) @ H)
        R[j] = r
    return R


def jacobian_volume_quadrature(prob, w_coef, dt):
    """-sum_i c_i int int d_xi_i Psi_k F'(w) Psi_l, every entry by quadrature (Sec. 3, eq. (Jacobian))."""
    ref = prob.ref
    c = dt / prob.h
    fp = dflux(ref.Psi.T @ w_coef)
    J = np.zeros((prob.theta_t, prob.theta_t))
    for i in range(prob.d):
        J -= c[i] * ((ref.dPsi[i + 1] * (ref.vw * fp)) @ ref.Psi.T)
    return J


def qqf_tensors(prob):
    """beta^i_{k l p} = int int d_xi_i Psi_k Psi_p Psi_l (Sec. 3, the precomputed integrals)."""
    if "beta" not in prob._cache:
        ref = prob.ref
        B = []
        for i in range(prob.d):
            B.append(np.einsum("kq,pq,lq,q->klp", ref.dPsi[i + 1], ref.Psi, ref.Psi, ref.vw))
        prob._cache["beta"] = B
    return prob._cache["beta"]


def project_spacetime(prob, values):
    """Coefficients of point values on Psi (eq. (Jacproj)): int Psi_p f / int Psi_p^2."""
    ref = prob.ref
    return (ref.Psi * ref.vw) @ values / (2.0 ** (prob.d + 1))


def jacobian_volume_qqf(prob, w_coef, dt):
    """The same block from the projection F'_p of F'(w) and the triple products (eq. (Jacobian2))."""
    c = dt / prob.h
    Fp = project_spacetime(prob, dflux(prob.ref.Psi.T @ w_coef))
    J = np.zeros((prob.theta_t, prob.theta_t))
    for i, B in enumerate(qqf_tensors(prob)):
        J -= c[i] * (B @ Fp)
    return J


def jacobian(prob, offs, Wr, Qr, dt):
    """Region Jacobian (n x n) of ``residual``."""
    ref, d, nt = prob.ref, prob.d, prob.theta_t
    pos = {o: j for j, o in enumerate(offs)}
    c = dt / prob.h
    nb = len(offs)
    J = np.zeros((nb * nt, nb * nt))
    for j, o in enumerate(offs):
        sl = slice(j * nt, (j + 1) * nt)
        J[sl, sl] += prob.T + jacobian_volume_quadrature(prob, Wr[j], dt)
        for (i, s) in _faces(prob):
            F = ref.face[(i, s)]
            a = F["Psi_own"].T @ Wr[j]
            o2 = list(o)
            o2[i] += s
            o2 = tuple(o2)
            if o2 in pos:
                k = pos[o2]
                b = F["Psi_nbr"].T @ Wr[k]
                al = wave_speed(Qr[j], Qr[k])
                da = 0.5 * s * dflux(a) + 0.5 * al
                db = 0.5 * s * dflux(b) - 0.5 * al
                J[sl, sl] += c[i] * ((F["Psi_own"] * (ref.fw * da)) @ F["Psi_own"].T)
                J[sl, k * nt:(k + 1) * nt] += c[i] * ((F["Psi_own"] * (ref.fw * db)) @ F["Psi_nbr"].T)
            else:
                J[sl, sl] += c[i] * ((F["Psi_own"] * (ref.fw * (s * dflux(a)))) @ F["Psi_own"].T)
    return J


def jacobian_perturbation(prob, offs, Wr, Qr, dt, eps=1e-3):
    """The Jacobian by central differences of the residual, one column per unknown (Sec. 3's
    perturbation method). The residual is quadratic in W, so the differences are exact up to
    rounding."""
    nb, nt = Wr.shape
    J = np.zeros((nb * nt, nb * nt))
    for col in range(nb * nt):
        Wp, Wm = Wr.copy(), Wr.copy()
        Wp.flat[col] += eps
        Wm.flat[col] -= eps
        J[:, col] = (residual(prob, offs, Wp, Qr, dt) - residual(prob, offs, Wm, Qr, dt)).ravel() / (2 * eps)
    return J


def newton_region(prob, e, Q, dt, history=None):
    """Newton iterations on the region system of element e; returns (offsets, W of the whole region,
    iterations). Raises NewtonFailure when the iteration has not converged after max_iter steps."""
    offs, elems = _region(prob, e)
    Qr = np.array([Q[g] for g in elems])
    Wr = Qr @ prob.lift.T
    for it in range(1, prob.max_iter + 1):
        R = residual(prob, offs, Wr, Qr, dt)
        J = jacobian(prob, offs, Wr, Qr, dt)
        delta = scipy.linalg.solve(J, R.ravel()).reshape(Wr.shape)
        Wr = Wr - delta
        if history is not None:
            history.append(float(np.max(np.abs(delta))))
        if np.max(np.abs(delta)) <= prob.tol * max(1.0, float(np.max(np.abs(Wr)))):
            return offs, Wr, it
    raise NewtonFailure(f"Newton on the region of element {e} did not converge in {prob.max_iter} iterations")


def predict(prob, Q, dt, elements=None, iterations=None):
    """Centre predictions W_e (theta_T) for the given elements (default: all)."""
    if elements is None:
        elements = range(prob.n_el)
    centre = (0,) * prob.d
    W = {}
    for e in elements:
        offs, Wr, it = newton_region(prob, e, Q, dt)
        W[e] = Wr[offs.index(centre)]
        if iterations is not None:
            iterations[e] = it
    return W


def correct(prob, Q, W, dt, elements=None):
    """Corrected states for the given elements from the predictions W (dict or array)."""
    ref, d = prob.ref, prob.d
    c = dt / prob.h
    if elements is None:
        elements = range(prob.n_el)
    out = {}
    for e in elements:
        base = prob.multi(e)
        w = ref.Psi.T @ W[e]
        acc = np.zeros(prob.theta)
        for i in range(d):
            acc += c[i] * ((ref.dPhi[i] * ref.vw) @ flux(w))
        for (i, s) in _faces(prob):
            F = ref.face[(i, s)]
            nb = list(base)
            nb[i] += s
            g = prob.linear(tuple(nb))
            a = F["Psi_own"].T @ W[e]
            b = F["Psi_nbr"].T @ W[g]
            acc -= c[i] * ((F["Phi_own"] * ref.fw) @ rusanov(a, b, s, wave_speed(Q[e], Q[g])))
        out[e] = Q[e] + acc / (2.0 ** d)
    return out


def step(prob, Q, dt, n_steps=1):
    """n_steps full RIDG steps (Newton prediction on every region, then the correction)."""
    Q = np.array(Q, dtype=np.float64, copy=True)
    for _ in range(n_steps):
        W = predict(prob, Q, dt)
        Qn = correct(prob, Q, W, dt)
        Q = np.array([Qn[e] for e in range(prob.n_el)])
    return Q


def _dilate(prob, elements):
    out = set()
    for e in elements:
        base = prob.multi(e)
        for o in itertools.product(range(-2, 3), repeat=prob.d):
            out.add(prob.linear(tuple(b + x for b, x in zip(base, o))))
    return sorted(out)


def step_sampled(prob, Q, dt, elements, n_steps=1):
    """n_steps steps evaluated only where the listed elements need them (see scheme.step_sampled)."""
    elements = sorted(set(int(e) for e in elements))
    sets = [elements]
    for _ in range(n_steps - 1):
        sets.insert(0, _dilate(prob, sets[0]))
    Q = np.array(Q, dtype=np.float64, copy=True)
    out = None
    for S in sets:
        need = set()
        for e in S:
            need.add(e)
            base = prob.multi(e)
            for i in range(prob.d):
                for s in (-1, 1):
                    nb = list(base)
                    nb[i] += s
                    need.add(prob.linear(tuple(nb)))
        W = predict(prob, Q, dt, sorted(need))
        out = correct(prob, Q, W, dt, S)
        for e, q in out.items():
            Q[e] = q
    return out


def exact_solution(q0, t, d):
    """Pointwise exact solution q(x, t) = q0(x - q t (1,..,1)) of the smooth (pre-shock) problem,
    by Newton on the characteristic equation; q0 must be periodic with period 1 and C^1."""

    def f(X):
        q = q0(X)
        shift = np.full((d, 1), 1e-6)
        for _ in range(100):
            Y = X - t * q[None, :]
            g = q - q0(Y)
            # d/dq [q - q0(x - q t (1,..,1))] = 1 + t (directional derivative of q0 along (1,..,1))
            dq0 = (q0(Y + shift) - q0(Y - shift)) / 2e-6
            upd = g / (1.0 + t * dq0)
            q = q - upd
            if np.max(np.abs(upd)) < 1e-15:
                break
        return q

    return f


def cosine_bump(d):
    """The initial state of eq. (burger2d), read as periodic on the unit box:
    q0 = 2^-d prod_i (1 - cos 2 pi x_i) (max 1)."""

    def f(X):
        v = np.ones(X.shape[1])
        for i in range(d):
            v = v * 0.5 * (1.0 - np.cos(2.0 * np.pi * X[i]))
        return v

    return f

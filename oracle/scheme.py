"""RIDG prediction and correction, written out plainly in FP64 (test infrastructure).

Every integral is taken by tensor Gauss-Legendre quadrature on the reference
space-time element (tau, xi_1..xi_d) in [-1, 1]^(d+1). With
x = x_e + (h/2) xi and t = t^n + (tau + 1) dt/2, dividing the prediction
equations of eq. (pred_full_system) by prod(h_i/2) gives, for every region
element r and test function Psi_k,

    [int Psi_k(1,.) Psi(1,.)^T - int int d_tau Psi_k Psi^T] W_r           (time term)
  - sum_i int int d_xi_i Psi_k nu_i Psi^T W_r                            (internal flux)
  + sum_faces int int Psi_k|_face (s nu_i) w_hat                         (surface flux)
  - [int Psi_k(-1,.) Phi^T] Q^n_r = 0                                    (causal source)

with nu_i(x) = v_i(x) dt / h_i and s = +-1 the side of the face. On faces
strictly inside the region w_hat is the upwind trace (Rusanov flux with the
local wave speed |v.n|, which for linear advection is exact upwinding); on the
region boundary w_hat is the trace of the region element itself (Sec. 2.2 text
and the "interior flux" markers of Fig. 1). Only the centre's W is kept.

The correction (Sec. 2.3), divided by |T| = 2^d prod(h_i/2), is

    Q_e <- Q_e + 2^-d [ sum_i int int d_xi_i Phi nu_i Psi^T W_e
                        - sum_faces int int Phi|_face (s nu_i) w_hat ]

with w_hat the upwind trace of the neighbours' own predictions.

Elements are numbered x fastest: e = i_0 + n_0 (i_1 + n_1 i_2). State arrays
are (N_el, theta) and predictions (N_el, theta_T), coefficients in the order of
``basis.spatial_indices`` / ``basis.spacetime_indices``.
"""

import itertools
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

from .basis import dpsi, gauss, psi, spacetime_indices, spatial_indices


@dataclass
class Problem:
    """A scalar linear advection problem q_t + div(v q) = 0 on a periodic box.

    velocity: ('const', (v_1..v_d)) or ('rotation', (c_x, c_y)) for the
    solid-body rotation v = (-(y - c_y), x - c_x) (2D only).
    region_radius: 1 for RIDG (3^d vertex neighbours); 0 reduces the
    predictor to a single element with interior traces on all faces
    (the locally implicit ADER-type predictor the paper starts from).
    """

    d: int
    n: tuple
    M: int
    velocity: tuple
    length: tuple = None
    family: str = "P"
    region_radius: int = 1
    quad_extra: int = 2
    _cache: dict = field(default_factory=dict, repr=False, compare=False)

    def __post_init__(self):
        self.n = tuple(int(x) for x in self.n)
        assert len(self.n) == self.d
        if self.length is None:
            self.length = (1.0,) * self.d
        self.length = tuple(float(x) for x in self.length)
        self.h = np.array([L / n for L, n in zip(self.length, self.n)])
        self.sidx = spatial_indices(self.d, self.M, self.family)
        self.tidx = spacetime_indices(self.d, self.M, self.family)
        self.theta = len(self.sidx)
        self.theta_t = len(self.tidx)
        self.n_el = int(np.prod(self.n))
        self._ref = _reference(self.d, self.M, self.family, self.M + self.quad_extra)

    # ---- geometry -------------------------------------------------------
    def multi(self, e):
        out = []
        for n in self.n:
            out.append(e % n)
            e //= n
        return tuple(out)

    def linear(self, idx):
        e = 0
        for n, i in zip(reversed(self.n), reversed(idx)):
            e = e * n + (i % n)
        return e

    def centre(self, idx):
        return np.array([(i + 0.5) * h for i, h in zip(idx, self.h)])

    def vel(self, x):
        """Velocity at points x of shape (d, npts)."""
        kind, par = self.velocity
        if kind == "const":
            return np.array([np.full(x.shape[1], float(v)) for v in par])
        if kind == "rotation":
            cx, cy = par
            return np.array([-(x[1] - cy), x[0] - cx])
        raise ValueError(kind)


class _Ref:
    pass


def _reference(d, M, family, q):
    """Basis values at tensor Gauss points of the reference space-time element."""
    r = _Ref()
    sidx = spatial_indices(d, M, family)
    tidx = spacetime_indices(d, M, family)
    g, w = gauss(q)
    r.g, r.w = g, w
    # volume points: (tau, xi_1..xi_d)
    pts = np.array(list(itertools.product(g, repeat=d + 1))).T  # (d+1, Q)
    wts = np.prod(np.array(list(itertools.product(w, repeat=d + 1))), axis=1)
    r.vpts, r.vw = pts, wts

    def st_vals(P, deriv=None):
        # P: (d+1, npts) space-time points; deriv: None or axis index (0 = tau)
        out = np.empty((len(tidx), P.shape[1]))
        for k, b in enumerate(tidx):
            v = np.ones(P.shape[1])
            for a in range(d + 1):
                v = v * (dpsi(b[a], P[a]) if deriv == a else psi(b[a], P[a]))
            out[k] = v
        return out

    def sp_vals(X, deriv=None):
        # X: (d, npts) spatial points
        out = np.empty((len(sidx), X.shape[1]))
        for k, a_ in enumerate(sidx):
            v = np.ones(X.shape[1])
            for a in range(d):
                v = v * (dpsi(a_[a], X[a]) if deriv == a else psi(a_[a], X[a]))
            out[k] = v
        return out

    r.st_vals, r.sp_vals = st_vals, sp_vals
    r.Psi = st_vals(pts)
    r.dPsi = [st_vals(pts, a) for a in range(d + 1)]  # [0] = d/dtau
    r.Phi = sp_vals(pts[1:])
    r.dPhi = [sp_vals(pts[1:], a) for a in range(d)]

    # spatial-only points (for the t = t^n and t = t^{n+1} traces)
    spts = np.array(list(itertools.product(g, repeat=d))).T if d > 0 else np.zeros((0, 1))
    sw = np.prod(np.array(list(itertools.product(w, repeat=d))), axis=1)
    r.spts, r.sw = spts, sw
    top = np.vstack([np.ones((1, spts.shape[1])), spts])
    bot = np.vstack([-np.ones((1, spts.shape[1])), spts])
    r.Psi_top = st_vals(top)
    r.Psi_bot = st_vals(bot)
    r.Phi_s = sp_vals(spts)

    # face points: for face (i, s) the points (tau, xi_perp) with xi_i = s
    fpts = np.array(list(itertools.product(g, repeat=d))).T  # (d, F): tau + (d-1) spatial
    fw = np.prod(np.array(list(itertools.product(w, repeat=d))), axis=1)
    r.fw = fw
    r.face = {}
    for i in range(d):
        for s in (-1, 1):
            def at(side):
                P = np.empty((d + 1, fpts.shape[1]))
                P[0] = fpts[0]
                j = 1
                for a in range(d):
                    if a == i:
                        P[a + 1] = side
                    else:
                        P[a + 1] = fpts[j]
                        j += 1
                return P
            Pown, Pnbr = at(s), at(-s)
            r.face[(i, s)] = dict(
                pts=Pown,
                Psi_own=st_vals(Pown),
                Psi_nbr=st_vals(Pnbr),
                Phi_own=sp_vals(Pown[1:]),
            )
    return r


def element_blocks(prob, e, dt):
    """All per-element matrices of the prediction and correction for element e.

    Returned dict (rows = test functions):
      T      time term  int Psi(1)Psi(1)^T - int int d_tau Psi Psi^T      (theta_T x theta_T)
      Vol    sum_i int int d_xi_i Psi nu_i Psi^T                           (theta_T x theta_T)
      C      causal source int Psi(-1) Phi^T                               (theta_T x theta)
      own_up[(i,s)], nbr_up[(i,s)], own_all[(i,s)]   surface flux blocks
      VolPhi sum_i int int d_xi_i Phi nu_i Psi^T                           (theta x theta_T)
      fown_phi[(i,s)], fnbr_phi[(i,s)]                                     (theta x theta_T)
    """
    ref = prob._ref
    d = prob.d
    idx = prob.multi(e)
    xc = prob.centre(idx)
    h = prob.h
    # nu_i at volume points
    X = xc[:, None] + 0.5 * h[:, None] * ref.vpts[1:]
    nu = prob.vel(X) * dt / h[:, None]
    key_parts = [nu.tobytes()]
    faces_nu = {}
    for (i, s), F in ref.face.items():
        Xf = xc[:, None] + 0.5 * h[:, None] * F["pts"][1:]
        nf = prob.vel(Xf)[i] * dt / h[i]
        faces_nu[(i, s)] = nf
        key_parts.append(nf.tobytes())
    key = ("blk", b"".join(key_parts))
    cache = prob._cache
    if key in cache:
        return cache[key]

    w = ref.vw
    out = {}
    out["T"] = (ref.Psi_top * ref.sw) @ ref.Psi_top.T - (ref.dPsi[0] * w) @ ref.Psi.T
    Vol = np.zeros((prob.theta_t, prob.theta_t))
    VolPhi = np.zeros((prob.theta, prob.theta_t))
    for i in range(d):
        Vol += (ref.dPsi[i + 1] * (w * nu[i])) @ ref.Psi.T
        VolPhi += (ref.dPhi[i] * (w * nu[i])) @ ref.Psi.T
    out["Vol"] = Vol
    out["VolPhi"] = VolPhi
    out["C"] = (ref.Psi_bot * ref.sw) @ ref.Phi_s.T
    own_up, nbr_up, own_all, fown, fnbr = {}, {}, {}, {}, {}
    for (i, s), F in ref.face.items():
        snu = s * faces_nu[(i, s)]
        if np.any(snu > 0) and np.any(snu < 0):
            raise ValueError(
                "v.n changes sign inside a face; the oracle (like the library) "
                "only treats faces with one upwind side"
            )
        up = (snu >= 0).astype(np.float64)
        wf = ref.fw * snu
        own_up[(i, s)] = (F["Psi_own"] * (wf * up)) @ F["Psi_own"].T
        nbr_up[(i, s)] = (F["Psi_own"] * (wf * (1 - up))) @ F["Psi_nbr"].T
        own_all[(i, s)] = (F["Psi_own"] * wf) @ F["Psi_own"].T
        fown[(i, s)] = (F["Phi_own"] * (wf * up)) @ F["Psi_own"].T
        fnbr[(i, s)] = (F["Phi_own"] * (wf * (1 - up))) @ F["Psi_nbr"].T
    out.update(own_up=own_up, nbr_up=nbr_up, own_all=own_all, fown_phi=fown, fnbr_phi=fnbr)
    out["key"] = key
    if len(cache) > 4096:  # variable coefficients: every element differs; keep memory bounded
        for k in [k for k in cache if isinstance(k, tuple) and k and k[0] == "blk"]:
            del cache[k]
    cache[key] = out
    return out


def _offsets(d, R):
    return list(itertools.product(range(-R, R + 1), repeat=d))


def _region_elements(prob, e):
    d, R = prob.d, prob.region_radius
    offs = _offsets(d, R)
    base = prob.multi(e)
    return offs, [prob.linear(tuple(bi + oi for bi, oi in zip(base, o))) for o in offs]


def region_system(prob, e, Q, dt, build_matrix=True):
    """Dense region matrix A, right-hand side b, the centre block index and a key.

    Block r (offset in {-R..R}^d, lexicographic) holds the theta_T unknowns of
    the region element e + r (periodic). The key identifies A: regions whose
    elements have identical blocks (constant coefficients) share one matrix.
    """
    d = prob.d
    offs, elems = _region_elements(prob, e)
    pos = {o: j for j, o in enumerate(offs)}
    nt = prob.theta_t
    nb = len(offs)
    blocks = [element_blocks(prob, g, dt) for g in elems]
    keys = tuple(B["key"] for B in blocks)
    b = np.zeros(nb * nt)
    for j, (g, B) in enumerate(zip(elems, blocks)):
        b[j * nt:(j + 1) * nt] = B["C"] @ Q[g]
    if not build_matrix:
        return None, b, pos[(0,) * d], keys
    A = np.zeros((nb * nt, nb * nt))
    for j, (o, B) in enumerate(zip(offs, blocks)):
        sl = slice(j * nt, (j + 1) * nt)
        A[sl, sl] += B["T"] - B["Vol"]
        for i in range(d):
            for s in (-1, 1):
                o2 = list(o)
                o2[i] += s
                o2 = tuple(o2)
                if o2 in pos:  # face strictly inside the region: upwind
                    A[sl, sl] += B["own_up"][(i, s)]
                    k = pos[o2]
                    A[sl, k * nt:(k + 1) * nt] += B["nbr_up"][(i, s)]
                else:  # region boundary: interior trace
                    A[sl, sl] += B["own_all"][(i, s)]
    return A, b, pos[(0,) * d], keys


def predict(prob, Q, dt, elements=None):
    """Centre predictions W_e (theta_T) for the given elements (default: all)."""
    if elements is None:
        elements = range(prob.n_el)
    nt = prob.theta_t
    W = {}
    lu_cache = prob._cache.setdefault("lu", {})
    for e in elements:
        _, b, c, keys = region_system(prob, e, Q, dt, build_matrix=False)
        lu = lu_cache.get(keys)
        if lu is None:
            A, b, c, keys = region_system(prob, e, Q, dt)
            lu = scipy.linalg.lu_factor(A)
            if len(lu_cache) < 64:  # same region matrix (constant coefficients): reuse the factors
                lu_cache[keys] = lu
        x = scipy.linalg.lu_solve(lu, b)
        W[e] = x[c * nt:(c + 1) * nt]
    return W


def correct(prob, Q, W, dt, elements=None):
    """Corrected states for the given elements from the predictions W (dict or array)."""
    d = prob.d
    if elements is None:
        elements = range(prob.n_el)
    out = {}
    for e in elements:
        B = element_blocks(prob, e, dt)
        base = prob.multi(e)
        acc = B["VolPhi"] @ W[e]
        for i in range(d):
            for s in (-1, 1):
                nbr = list(base)
                nbr[i] += s
                g = prob.linear(tuple(nbr))
                acc = acc - B["fown_phi"][(i, s)] @ W[e] - B["fnbr_phi"][(i, s)] @ W[g]
        out[e] = Q[e] + acc / (2.0 ** d)
    return out


def step(prob, Q, dt, n_steps=1):
    """n_steps full RIDG steps (prediction on every region, then correction)."""
    Q = np.array(Q, dtype=np.float64, copy=True)
    for _ in range(n_steps):
        W = predict(prob, Q, dt)
        Qn = correct(prob, Q, W, dt)
        Q = np.array([Qn[e] for e in range(prob.n_el)])
    return Q


def _dilate(prob, elements):
    """The elements within two elements (in every axis) of the given ones: everything one step at
    them reads (region radius 1, plus 1 for the face neighbours' predictions), periodic."""
    out = set()
    for e in elements:
        base = prob.multi(e)
        for o in itertools.product(range(-2, 3), repeat=prob.d):
            out.add(prob.linear(tuple(b + x for b, x in zip(base, o))))
    return sorted(out)


def step_sampled(prob, Q, dt, elements, n_steps=1):
    """n_steps full steps evaluated only where they are needed for the listed elements.

    Step j updates only the elements that steps j+1..n_steps read (each step reads the state within
    two elements of where it is evaluated); the last step updates the listed elements. Returns a
    dict element -> state after n_steps.
    """
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
                    nbr = list(base)
                    nbr[i] += s
                    need.add(prob.linear(tuple(nbr)))
        W = predict(prob, Q, dt, sorted(need))
        out = correct(prob, Q, W, dt, S)
        for e, q in out.items():  # entries outside S are stale and never read again
            Q[e] = q
    return out


def predictions(prob, Q, dt):
    """All predictions as an (N_el, theta_T) array."""
    W = predict(prob, Q, dt)
    return np.array([W[e] for e in range(prob.n_el)])

"""Seeded synthetic inputs: initial modal coefficients for the advection workloads.

This module prepares inputs only; it contains no part of the prediction or the
correction. It draws the random parameters of each workload from a seeded
``numpy.random.default_rng`` and projects the resulting initial condition onto
the modal basis the library expects:

    Q_e^k = (1/|T_e|) int_{T_e} Phi_k q0 dx,   Phi_alpha = prod_i sqrt(2 a_i + 1) P_{a_i}(xi_i),

multi-indices alpha of total degree <= M-1, ordered by total degree and then
lexicographically descending (the library's documented state layout,
element e = i_0 + n_0 (i_1 + n_1 i_2), coefficient-fastest).

Projections use Gauss-Legendre quadrature with M + 8 points per axis per
element. Sums of separable terms (Gaussians, Fourier modes) are projected one
axis at a time; the compact C-infinity bumps of the rotation workload use the
full tensor rule on the elements inside their support.

The paper measures only analytic bumps on periodic boxes (no datasets); the
workloads here follow its problem shapes with the sizes of the benchmark
configurations.
"""

import itertools
import math
from dataclasses import dataclass, field

import numpy as np
from numpy.polynomial import legendre as _leg


def basis_indices(d, M):
    out = [a for a in itertools.product(range(M), repeat=d) if sum(a) <= M - 1]
    out.sort(key=lambda a: (sum(a), tuple(-x for x in a)))
    return out


def _psi_table(M, x):
    """(M, len(x)) values of sqrt(2m+1) P_m(x)."""
    out = np.empty((M, len(x)))
    for m in range(M):
        c = np.zeros(m + 1)
        c[m] = 1.0
        out[m] = math.sqrt(2 * m + 1) * _leg.legval(x, c)
    return out


def project_1d(f, n, M, length=1.0, q=None):
    """(n, M) coefficients (1/h) int f psi_m over each of n cells of [0, length)."""
    q = q or M + 8
    g, w = _leg.leggauss(q)
    h = length / n
    centres = (np.arange(n) + 0.5) * h
    X = centres[:, None] + 0.5 * h * g[None, :]
    F = f(X)
    P = _psi_table(M, g)
    return 0.5 * (F * w[None, :]) @ P.T


def project_separable(terms, d, n, M):
    """Sum over terms (coef, [f_1..f_d]) of prod_i f_i(x_i), projected on the P basis."""
    idx = basis_indices(d, M)
    n_el = int(np.prod(n))
    out = np.zeros((n_el, len(idx)))
    for coef, fs in terms:
        c1 = [project_1d(f, n[i], M) for i, f in enumerate(fs)]  # each (n_i, M), maybe complex
        for k, a in enumerate(idx):
            # outer product over axes, x fastest in the flattened element index
            t = c1[0][:, a[0]]
            for i in range(1, d):
                t = np.multiply.outer(c1[i][:, a[i]], t)  # axis i slower
            out[:, k] += np.real(coef * t.reshape(-1))
    return out


def project_tensor(f, d, n, M, elements=None):
    """Full tensor-rule projection of f on the listed elements (default: all)."""
    q = M + 8
    g, w = _leg.leggauss(q)
    idx = basis_indices(d, M)
    xi = np.array(list(itertools.product(g, repeat=d))).T
    wt = np.prod(np.array(list(itertools.product(w, repeat=d))), axis=1)
    P = _psi_table(M, g)
    # basis at the tensor points
    ipts = np.array(list(itertools.product(range(q), repeat=d))).T
    B = np.array([np.prod([P[a[i]][ipts[i]] for i in range(d)], axis=0) for a in idx])
    BW = B * wt / 2.0 ** d
    h = np.array([1.0 / k for k in n])
    n_el = int(np.prod(n))
    out = np.zeros((n_el, len(idx)))
    if elements is None:
        elements = range(n_el)
    elements = np.asarray(list(elements), dtype=np.int64)
    if elements.size == 0:
        return out
    mi = []
    rem = elements.copy()
    for k in n:
        mi.append(rem % k)
        rem //= k
    mi = np.array(mi)  # (d, E)
    xc = (mi + 0.5) * h[:, None]
    X = xc[:, :, None] + 0.5 * h[:, None, None] * xi[:, None, :]  # (d, E, P)
    F = f(X)  # (E, P)
    out[elements] = F @ BW.T
    return out


# ---------------------------------------------------------------- workloads

@dataclass
class Workload:
    name: str
    d: int
    n: tuple
    M: int
    velocity: tuple           # ('const', v) or ('rotation', centre)
    dt: float
    steps: int
    q0: np.ndarray            # (N_el, theta) initial coefficients
    exact: callable = field(default=None, repr=False)  # t -> (N_el, theta) exact projection
    params: dict = field(default_factory=dict, repr=False)


def _periodic_gauss_1d(c, s2):
    """x -> sum over images k in {-1,0,1} of exp(-(x - c - k)^2 / s2)."""
    def f(x):
        return sum(np.exp(-((x - c - k) ** 2) / s2) for k in (-1, 0, 1))
    return f


def _cexp_1d(k, shift=0.0):
    return lambda x: np.exp(2j * np.pi * k * (x - shift))


def sine_1d(n=64, M=3, cfl=0.5, steps=200):
    """Workload: 1D u_t + u_x = 0, u0 = sin(2 pi x), periodic [0,1]."""
    dt = cfl / n

    def ex(t):
        return project_1d(lambda x: np.sin(2 * np.pi * (x - t)), n, M)
    return Workload("1d-sine", 1, (n,), M, ("const", (1.0,)), dt, steps, ex(0.0), ex)


def advection_2d(n=256, M=3, seed=2102, cfl=0.5, steps=100):
    """Workload: 2D advection, v = (1, 0.5), Gaussian bump + random Fourier modes |k| <= 8."""
    rng = np.random.default_rng(seed)
    v = np.array([1.0, 0.5])
    ks = [(kx, ky) for kx in range(-8, 9) for ky in range(-8, 9)
          if 0 < kx * kx + ky * ky <= 64 and (kx > 0 or (kx == 0 and ky > 0))]
    A = rng.normal(0.0, 0.1, len(ks))
    B = rng.normal(0.0, 0.1, len(ks))
    sigma = 0.1

    def terms(t):
        sx, sy = v * t
        out = [(1.0, [_periodic_gauss_1d(0.5 + sx, sigma ** 2), _periodic_gauss_1d(0.5 + sy, sigma ** 2)])]
        for (kx, ky), a, b in zip(ks, A, B):
            # a cos(2 pi k.x') + b sin(2 pi k.x') = Re((a - i b) e^{2 pi i k.x'})
            out.append((complex(a, -b), [_cexp_1d(kx, sx), _cexp_1d(ky, sy)]))
        return out

    def ex(t):
        return project_separable(terms(t), 2, (n, n), M)
    dt = cfl / n  # max |v_i| = 1
    return Workload("2d-advection", 2, (n, n), M, ("const", tuple(v)), dt, steps, ex(0.0), ex,
                    dict(ks=ks, A=A, B=B))


def bump(r):
    """C-infinity bump exp(1 - 1/(1 - r^2)) for r < 1, else 0 (peak 1)."""
    out = np.zeros_like(r)
    m = r < 1.0
    out[m] = np.exp(1.0 - 1.0 / (1.0 - r[m] ** 2))
    return out


def rotation_2d(n=512, M=4, seed=2103, cfl=0.5, steps=20):
    """Workload: solid-body rotation v = (-(y-1/2), x-1/2), three compact bumps."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 1.0, 3)
    om = rng.uniform(0.08, 0.15, 3)
    ang = rng.uniform(0.0, 2 * np.pi, 3)
    rad = 0.25 * np.sqrt(rng.uniform(0.0, 1.0, 3))
    cen = np.stack([0.5 + rad * np.cos(ang), 0.5 + rad * np.sin(ang)], axis=1)

    def ex(t):
        ct, st = math.cos(t), math.sin(t)
        cs = np.stack([0.5 + ct * (cen[:, 0] - 0.5) - st * (cen[:, 1] - 0.5),
                       0.5 + st * (cen[:, 0] - 0.5) + ct * (cen[:, 1] - 0.5)], axis=1)

        def f(X):
            out = 0.0
            for m in range(3):
                r = np.sqrt((X[0] - cs[m, 0]) ** 2 + (X[1] - cs[m, 1]) ** 2) / om[m]
                out = out + a[m] * bump(r)
            return out
        # only elements that can touch a support
        h = 1.0 / n
        ii = np.arange(n)
        sel = np.zeros((n, n), dtype=bool)
        for m in range(3):
            mx = np.abs((ii + 0.5) * h - cs[m, 0]) <= om[m] + h
            my = np.abs((ii + 0.5) * h - cs[m, 1]) <= om[m] + h
            sel |= np.outer(my, mx)
        return project_tensor(f, 2, (n, n), M, np.flatnonzero(sel.reshape(-1)))
    vmax = 0.5
    dt = cfl / (n * vmax)
    return Workload("2d-rotation", 2, (n, n), M, ("rotation", (0.5, 0.5)), dt, steps, ex(0.0), ex,
                    dict(a=a, om=om, cen=cen))


def advection_3d(n=128, M=3, seed=2104, cfl=0.5, steps=20, shape=None):
    """Workload: 3D advection, v = (1,1,1), sum of 5 periodised Gaussians (on an n^3 mesh, or on a
    mesh of the given shape with the step size of its finest axis)."""
    rng = np.random.default_rng(seed)
    mesh = tuple(shape) if shape is not None else (n, n, n)
    cen = rng.uniform(0.0, 1.0, (5, 3))
    sig = rng.uniform(0.05, 0.15, 5)
    v = np.array([1.0, 1.0, 1.0])

    def ex(t):
        terms = []
        for m in range(5):
            s2 = 2 * sig[m] ** 2
            terms.append((1.0, [_periodic_gauss_1d(cen[m, i] + v[i] * t, s2) for i in range(3)]))
        return project_separable(terms, 3, mesh, M)
    dt = cfl / max(mesh)
    return Workload("3d-advection", 3, mesh, M, ("const", tuple(v)), dt, steps, ex(0.0), ex,
                    dict(cen=cen, sig=sig))


def burgers(d=2, n=128, M=4, cfl=0.1, steps=20):
    """Workload: Burgers q_t + sum_i (q^2/2)_{x_i} = 0 from the initial state of eq. (burger2d), read as
    periodic on the unit box, q0 = 2^-d prod_i (1 - cos 2 pi x_i) (values in [0, 1], so the largest
    wave speed is 1 and dt = cfl h). Smooth until t ~ 0.245 in 2D (1/pi in 1D); at cfl = 0.1 the
    region systems stay solvable well past t = 0.2."""
    mesh = (n,) * d

    def half_one_minus_cos(x):
        return 0.5 * (1.0 - np.cos(2.0 * np.pi * x))

    q0 = project_separable([(1.0, [half_one_minus_cos] * d)], d, mesh, M)

    def q0_at(X):
        v = np.ones(X.shape[1:])
        for i in range(d):
            v = v * half_one_minus_cos(X[i])
        return v

    def grad_sum(X):  # sum_i d q0 / d x_i
        tot = np.zeros(X.shape[1:])
        for i in range(d):
            g = np.pi * np.sin(2.0 * np.pi * X[i])
            for j in range(d):
                if j != i:
                    g = g * half_one_minus_cos(X[j])
            tot = tot + g
        return tot

    def ex(t):
        """Projection of the exact pre-shock solution: q = q0(x - q t (1,..,1)) at every quadrature
        point (characteristics), solved by Newton's method."""
        def f(X):
            q = q0_at(X)
            for _ in range(100):
                Y = X - t * q[None]
                upd = (q - q0_at(Y)) / (1.0 + t * grad_sum(Y))
                q = q - upd
                if np.max(np.abs(upd)) < 1e-15:
                    break
            return q
        return project_tensor(f, d, mesh, M)

    return Workload(f"{d}d-burgers", d, mesh, M, ("burgers", ()), cfl / n, steps, q0, ex)


def random_state(d, n, M, seed):
    """Seeded random coefficients with a decaying modal spectrum (parity inputs)."""
    rng = np.random.default_rng(seed)
    idx = basis_indices(d, M)
    deg = np.array([sum(a) for a in idx], dtype=np.float64)
    n_el = int(np.prod(n))
    return rng.standard_normal((n_el, len(idx))) * (0.5 ** deg)[None, :]


def serving_requests(count=200, seed=2201, rate=20.0):
    """Poisson arrivals of independent periodic advection runs (mixed d, N, M)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(count):
        t += rng.exponential(1.0 / rate)
        d = int(rng.choice([2, 1, 3], p=[0.6, 0.3, 0.1]))
        if d == 1:
            side = int(rng.integers(64, 2049))
        elif d == 2:
            side = int(rng.integers(64, 513))
        else:
            side = int(rng.integers(32, 97))
        M = int(rng.integers(1, 6))
        steps = int(rng.integers(50, 501))
        while True:
            v = rng.uniform(-1.0, 1.0, d)
            if np.max(np.abs(v)) >= 1e-3:
                break
        dt = 0.5 / (side * np.max(np.abs(v)))
        out.append(dict(id=r, arrival=t, d=d, n=(side,) * d, M=M, steps=steps,
                        velocity=tuple(float(x) for x in v), dt=float(dt),
                        seed=int(rng.integers(0, 2 ** 31 - 1))))
    return out


def gaussian_bump_state(d, n, M, seed, sigma=0.1):
    """Periodised Gaussian bump with a seeded centre (initial data of a serving request)."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.3, 0.7, d)
    terms = [(1.0, [_periodic_gauss_1d(c[i], sigma ** 2) for i in range(d)])]
    return project_separable(terms, d, tuple(n), M)

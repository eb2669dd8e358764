"""Pins of the oracle's RIDG step against what the paper and the mathematics fix.

Each test names the passage or fact it pins:
  * QQF == quadrature for a flux Jacobian inside the span (Sec. 3): the
    internal-flux and surface blocks of a variable-velocity element equal the
    closed-form triple-product sums sum_p beta_p F'_p;
  * the single-element special case (Sec. 2: RIDG generalises the locally
    implicit ADER predictor) is exact on polynomial data;
  * exactness of the full step on global polynomials away from the periodic
    wrap (a consequence of the interior-trace region boundary of Sec. 2.2;
    a planted "drop the boundary faces" mistake fails it);
  * design order of accuracy on refinement (eq. Mratio, Sec. 6.1);
  * conservation of the element-average sum (flux form of Sec. 2.3);
  * von Neumann stability at the configured CFL, and the paper's CFL 0.9 for
    the tensor basis in 1D (Sec. 6.1);
  * symmetries: translation, mirror, axis swap, 90-degree rotation of the
    rotation field, linearity, dt = 0;
  * dimension reduction 2D -> 1D for data constant in y;
  * rigid rotation of a compact bump converges at the design order.
"""

import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle.scheme as S
from oracle import basis
from oracle.project import project, l2rel_paper, periodic_translate, exact_rotation
from oracle.stability import nu_max, spectral_radius, stencil

from test_oracle_basis import leg_dint_rational, triple_closed


# ------------------------------------------------------------ 1D closed forms
def t3(a, b, c):
    """int psi_a psi_b psi_c (exact)."""
    return math.sqrt((2 * a + 1) * (2 * b + 1) * (2 * c + 1)) * float(triple_closed(a, b, c))


def d3(a, b, c):
    """int psi_a' psi_b psi_c, with P_a' = sum_{j<a, a-j odd} (2j+1) P_j."""
    tot = Fraction(0)
    for j in range(a):
        if (a - j) % 2 == 1:
            tot += (2 * j + 1) * triple_closed(j, b, c)
    return math.sqrt((2 * a + 1) * (2 * b + 1) * (2 * c + 1)) * float(tot)


def rot_nu(prob, e, dt):
    """nu_i = c0_i + sum_j c_ij xi_j for the rotation field on element e."""
    idx = prob.multi(e)
    xc = prob.centre(idx)
    h = prob.h
    cx, cy = prob.velocity[1]
    # v_x = -(y - cy), v_y = x - cx ; y = yc + h_y xi_y / 2
    c0 = np.array([-(xc[1] - cy) * dt / h[0], (xc[0] - cx) * dt / h[1]])
    cl = {(0, 1): -(h[1] / 2) * dt / h[0], (1, 0): (h[0] / 2) * dt / h[1]}
    return c0, cl


@pytest.mark.parametrize("M", [2, 3, 4])
def test_qqf_equals_quadrature_rotation(M):
    """Sec. 3: J = time - sum_p beta_p F'_p + surface; exact when F' is in the span."""
    prob = S.Problem(d=2, n=(8, 8), M=M, velocity=("rotation", (0.5, 0.5)))
    dt = 0.01
    tid = prob.tidx
    for e in (0, 19, 45):
        B = S.element_blocks(prob, e, dt)
        c0, cl = rot_nu(prob, e, dt)
        # projection of nu_i on Psi: V_0 = c0, V_(xi_j) = c_ij / sqrt(3) (psi_1 = sqrt(3) xi)
        Vol = np.zeros((len(tid), len(tid)))
        for i in range(2):
            terms = [((0, 0, 0), c0[i])]
            for (ii, j), c in cl.items():
                if ii == i:
                    p = [0, 0, 0]
                    p[1 + j] = 1
                    terms.append((tuple(p), c / math.sqrt(3)))
            for k, bk in enumerate(tid):
                for l, bl in enumerate(tid):
                    acc = 0.0
                    for p, V in terms:
                        val = 1.0
                        for ax in range(3):
                            if ax == 1 + i:
                                val *= d3(bk[ax], p[ax], bl[ax])
                            else:
                                val *= t3(bk[ax], p[ax], bl[ax])
                        acc += V * val
                    Vol[k, l] += acc
        np.testing.assert_allclose(B["Vol"], Vol, atol=1e-13)
        # surface block on the region boundary: s sum_p V_p psi(s) psi(s) prod t3
        for i in range(2):
            for s in (-1, 1):
                terms = [((0, 0, 0), c0[i])]
                for (ii, j), c in cl.items():
                    if ii == i:
                        p = [0, 0, 0]
                        p[1 + j] = 1
                        terms.append((tuple(p), c / math.sqrt(3)))
                F = np.zeros((len(tid), len(tid)))
                for k, bk in enumerate(tid):
                    for l, bl in enumerate(tid):
                        acc = 0.0
                        for p, V in terms:
                            val = s * math.sqrt((2 * bk[1 + i] + 1) * (2 * bl[1 + i] + 1)) * s ** (bk[1 + i] + bl[1 + i])
                            for ax in range(3):
                                if ax != 1 + i:
                                    val *= t3(bk[ax], p[ax], bl[ax])
                            acc += V * val
                        F[k, l] = acc
                np.testing.assert_allclose(B["own_all"][(i, s)], F, atol=1e-13)


def _poly(coeffs):
    """Global polynomial sum c * x^a y^b ... ; coeffs: dict exponent-tuple -> c."""
    def f(X):
        out = np.zeros(X.shape[1:])
        for ex, c in coeffs.items():
            term = np.full(X.shape[1:], float(c))
            for i, a in enumerate(ex):
                term = term * X[i] ** a
            out = out + term
        return out
    return f


def _rand_poly(d, deg, rng):
    co = {}
    for ex in itertools.product(range(deg + 1), repeat=d):
        if sum(ex) <= deg:
            co[ex] = rng.uniform(-1, 1)
    return co


@pytest.mark.parametrize("d,M", [(1, 3), (2, 2), (2, 3)])
def test_single_element_predictor_exact(d, M):
    """Region of one element with interior traces everywhere: W is the exact space-time
    projection of p(x - v (t - t^n)) for polynomial data of degree <= M-1."""
    rng = np.random.default_rng(7)
    v = (0.7, -0.4)[:d]
    prob = S.Problem(d=d, n=(5,) * d, M=M, velocity=("const", v), region_radius=0)
    co = _rand_poly(d, M - 1, rng)
    f = _poly(co)
    Q = project(f, d, prob.n, M, q=M + 4)
    dt = 0.3 * prob.h[0]
    W = S.predict(prob, Q, dt)
    g, w = basis.gauss(M + 4)
    pts = np.array(list(itertools.product(g, repeat=d + 1))).T
    wts = np.prod(np.array(list(itertools.product(w, repeat=d + 1))), axis=1)
    Psi = np.array([np.prod([basis.psi(b[a], pts[a]) for a in range(d + 1)], axis=0) for b in prob.tidx])
    for e in range(prob.n_el):
        xc = prob.centre(prob.multi(e))
        t = (pts[0] + 1) * dt / 2
        X = xc[:, None] + 0.5 * prob.h[:, None] * pts[1:] - np.array(v)[:, None] * t[None, :]
        exact = (Psi * wts) @ f(X) / 2.0 ** (d + 1)
        np.testing.assert_allclose(W[e], exact, atol=1e-12)


def _interior_elements(prob, margin):
    out = []
    for e in range(prob.n_el):
        idx = prob.multi(e)
        if all(margin <= i <= n - 1 - margin for i, n in zip(idx, prob.n)):
            out.append(e)
    return out


@pytest.mark.parametrize("d,M,v", [(1, 3, (0.9,)), (2, 3, (0.8, -0.5)), (2, 2, (-0.6, 0.0))])
def test_polynomial_reproduction(d, M, v):
    """Global polynomial data: after one step every element whose 2-neighbourhood does
    not cross the periodic wrap holds the exact projection of p(x - v dt)."""
    rng = np.random.default_rng(11)
    prob = S.Problem(d=d, n=(8,) * d, M=M, velocity=("const", v))
    f = _poly(_rand_poly(d, M - 1, rng))
    Q = project(f, d, prob.n, M, q=M + 4)
    dt = 0.45 * prob.h[0] / max(abs(x) for x in v)
    Q1 = S.step(prob, Q, dt, 1)
    ex = project(lambda X: f(X - np.array(v)[:, None] * dt), d, prob.n, M, q=M + 4)
    el = _interior_elements(prob, 2)
    np.testing.assert_allclose(Q1[el], ex[el], atol=1e-12)


def test_polynomial_reproduction_rejects_dropped_boundary_faces(monkeypatch):
    """Planted mistake in the oracle: dropping the region-boundary surface terms (the other
    reading of eq. pred_full_system) breaks polynomial reproduction."""
    orig = S.element_blocks

    def dropped(prob, e, dt):
        B = dict(orig(prob, e, dt))
        B["own_all"] = {k: 0 * x for k, x in B["own_all"].items()}
        return B

    monkeypatch.setattr(S, "element_blocks", dropped)
    rng = np.random.default_rng(11)
    prob = S.Problem(d=1, n=(8,), M=3, velocity=("const", (0.9,)))
    f = _poly(_rand_poly(1, 2, rng))
    Q = project(f, 1, prob.n, 3, q=7)
    dt = 0.45 * prob.h[0] / 0.9
    Q1 = S.step(prob, Q, dt, 1)
    ex = project(lambda X: f(X - 0.9 * dt), 1, prob.n, 3, q=7)
    el = _interior_elements(prob, 2)
    assert np.max(np.abs(Q1[el] - ex[el])) > 1e-6


@pytest.mark.parametrize("M", [1, 2, 3, 4])
def test_convergence_order_1d(M):
    """eq. (Mratio): observed order ~ M (degree M-1) on sin(2 pi x), CFL 0.5."""
    f0 = lambda X: np.sin(2 * np.pi * X[0])
    errs = []
    for n in (16, 32):
        prob = S.Problem(d=1, n=(n,), M=M, velocity=("const", (1.0,)))
        Q = project(f0, 1, (n,), M)
        dt = 0.5 / n
        steps = n // 2  # T = 0.25
        Q1 = S.step(prob, Q, dt, steps)
        errs.append(l2rel_paper(Q1, periodic_translate(f0, [1.0], dt * steps), 1, (n,), M))
    order = math.log(errs[0] / errs[1]) / math.log(2)
    assert abs(order - M) < 0.35, (errs, order)


@pytest.mark.parametrize("M", [2, 3])
def test_convergence_order_2d(M):
    f0 = lambda X: np.sin(2 * np.pi * X[0]) * np.cos(2 * np.pi * X[1])
    v = (1.0, 0.5)
    errs = []
    for n in ((16, 32) if M == 2 else (8, 16)):
        prob = S.Problem(d=2, n=(n, n), M=M, velocity=("const", v))
        Q = project(f0, 2, (n, n), M)
        dt = 0.5 / n
        steps = n // 4  # T = 0.125
        Q1 = S.step(prob, Q, dt, steps)
        errs.append(l2rel_paper(Q1, periodic_translate(f0, v, dt * steps), 2, (n, n), M))
    order = math.log(errs[0] / errs[1]) / math.log(2)
    assert abs(order - M) < 0.45, (errs, order)


@pytest.mark.parametrize("vel", [("rotation", (0.5, 0.5)), ("const", (0.7, -0.3))])
def test_conservation(vel):
    """Flux form (Sec. 2.3) on a periodic mesh: sum of element averages is invariant."""
    prob = S.Problem(d=2, n=(6, 6), M=3, velocity=vel)
    rng = np.random.default_rng(3)
    Q = rng.standard_normal((prob.n_el, prob.theta))
    Q1 = S.step(prob, Q, 0.04, 3)
    assert abs(Q1[:, 0].sum() - Q[:, 0].sum()) < 1e-13 * np.abs(Q[:, 0]).sum()


def test_constant_preserved_rotation():
    """Divergence-free field: q = const is an exact solution and W = const solves every region."""
    prob = S.Problem(d=2, n=(6, 6), M=4, velocity=("rotation", (0.5, 0.5)))
    Q = np.zeros((prob.n_el, prob.theta))
    Q[:, 0] = 1.7
    np.testing.assert_allclose(S.step(prob, Q, 0.05, 2), Q, atol=1e-13)


@pytest.mark.parametrize("d,M,v", [(1, 3, (1.0,)), (2, 3, (1.0, 0.5)), (2, 4, (1.0, 0.5))])
def test_stable_at_configured_cfl(d, M, v):
    """Von Neumann: spectral radius of the step at CFL 0.5 does not exceed 1."""
    K = stencil(d, M, v, 0.5)
    assert spectral_radius(K, d, 48 if d == 1 else 24) <= 1 + 1e-12


def test_unstable_far_beyond_cfl():
    K = stencil(1, 3, (1.0,), 1.5)
    assert spectral_radius(K, 1, 64) > 1.01


def test_tensor_basis_cfl_matches_paper_1d():
    """Sec. 6.1 runs 1D RIDG (tensor space-time basis) at CFL 0.9 for M_deg = 3; the oracle's
    stability limit for that case sits at 0.899, and growth at 0.9 is below 1e-4 per step."""
    nm = nu_max(1, 4, (1.0,), family="Q", lo=0.5, hi=1.5, nk=96, tol=2e-3)
    assert 0.88 <= nm <= 0.92
    assert spectral_radius(stencil(1, 4, (1.0,), 0.9, "Q"), 1, 128) < 1 + 1e-4


def _rand_state(prob, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((prob.n_el, prob.theta))


def test_translation_and_linearity_and_dt0():
    prob = S.Problem(d=2, n=(6, 5), M=3, velocity=("const", (0.6, -0.8)))
    Q = _rand_state(prob, 1)
    Q2 = _rand_state(prob, 2)
    dt = 0.4 * prob.h[0]
    Q1 = S.step(prob, Q, dt, 2)
    # translation by one element in x
    sh = lambda A: A.reshape(5, 6, -1)[:, np.r_[5, 0:5], :].reshape(30, -1)
    np.testing.assert_allclose(S.step(prob, sh(Q), dt, 2), sh(Q1), atol=1e-12)
    # linearity
    np.testing.assert_allclose(S.step(prob, 2.0 * Q - 3.0 * Q2, dt, 2),
                               2.0 * Q1 - 3.0 * S.step(prob, Q2, dt, 2), atol=1e-11)
    # dt = 0
    np.testing.assert_allclose(S.step(prob, Q, 0.0, 1), Q, atol=1e-14)


def test_mirror_and_axis_swap():
    M = 3
    sid = basis.spatial_indices(2, M)
    n = 6
    Q = _rand_state(S.Problem(d=2, n=(n, n), M=M, velocity=("const", (0.6, -0.3))), 5)
    dt = 0.05
    base = S.step(S.Problem(d=2, n=(n, n), M=M, velocity=("const", (0.6, -0.3))), Q, dt, 1)

    def mirror_x(A):
        B = A.reshape(n, n, -1)[:, ::-1, :].copy()
        sg = np.array([(-1) ** a[0] for a in sid])
        return (B * sg).reshape(n * n, -1)

    got = S.step(S.Problem(d=2, n=(n, n), M=M, velocity=("const", (-0.6, -0.3))), mirror_x(Q), dt, 1)
    np.testing.assert_allclose(got, mirror_x(base), atol=1e-12)

    perm = [sid.index((a[1], a[0])) for a in sid]

    def swap(A):
        B = A.reshape(n, n, -1).transpose(1, 0, 2)
        return B[:, :, perm].reshape(n * n, -1)

    got = S.step(S.Problem(d=2, n=(n, n), M=M, velocity=("const", (-0.3, 0.6))), swap(Q), dt, 1)
    np.testing.assert_allclose(got, swap(base), atol=1e-12)


def test_rotation_field_quarter_turn_symmetry():
    """The rotation field is invariant under a 90-degree turn about its centre, so rotating
    the data commutes with the step: Q'[(i,j),(b,a)] = (-1)^b Q[(j, n-1-i),(a,b)]."""
    M, n = 3, 6
    sid = basis.spatial_indices(2, M)
    prob = S.Problem(d=2, n=(n, n), M=M, velocity=("rotation", (0.5, 0.5)))
    Q = _rand_state(prob, 9)

    def turn(A):
        A = A.reshape(n, n, -1)  # [j, i, k]
        B = np.empty_like(A)
        for i in range(n):
            for j in range(n):
                for k, (a, b) in enumerate(sid):
                    B[j, i, sid.index((b, a))] = (-1) ** b * A[n - 1 - i, j, k]
        return B.reshape(n * n, -1)

    dt = 0.05
    np.testing.assert_allclose(S.step(prob, turn(Q), dt, 1), turn(S.step(prob, Q, dt, 1)), atol=1e-12)


def test_dimension_reduction_2d_to_1d():
    """Data constant in y: the 2D step (any v_y) equals the 1D step with v_x."""
    M, n = 3, 8
    f = lambda X: np.sin(2 * np.pi * X[0]) + 0.3 * np.cos(6 * np.pi * X[0])
    Q1d = project(f, 1, (n,), M)
    Q2d = project(f, 2, (n, n), M)
    dt = 0.04
    r1 = S.step(S.Problem(d=1, n=(n,), M=M, velocity=("const", (0.8,))), Q1d, dt, 2)
    r2 = S.step(S.Problem(d=2, n=(n, n), M=M, velocity=("const", (0.8, -0.55))), Q2d, dt, 2)
    sid = basis.spatial_indices(2, M)
    r2 = r2.reshape(n, n, -1)
    for k, (a, b) in enumerate(sid):
        for j in range(n):
            if b == 0:
                np.testing.assert_allclose(r2[j, :, k], r1[:, a], atol=1e-12)
            else:
                np.testing.assert_allclose(r2[j, :, k], 0.0, atol=1e-12)


def test_rotation_bump_converges():
    """Rigid rotation of a compactly supported smooth profile (support inside r < 0.45 of the
    centre, so the periodic wrap never sees it): the error against the rotated exact solution
    falls at close to the design order (M = 3; pre-asymptotic meshes 8 -> 16)."""
    M = 3
    c, R = np.array([0.55, 0.5]), 0.4

    def f0(X):
        r2 = ((X[0] - c[0]) ** 2 + (X[1] - c[1]) ** 2) / R ** 2
        return np.where(r2 < 1, (1 - np.minimum(r2, 1)) ** 8, 0.0)

    errs = []
    T = 0.25
    for n in (8, 16):
        prob = S.Problem(d=2, n=(n, n), M=M, velocity=("rotation", (0.5, 0.5)))
        Q = project(f0, 2, (n, n), M, q=M + 10)
        steps = int(math.ceil(T / (0.5 / (n * 0.5))))
        dt = T / steps
        Q1 = S.step(prob, Q, dt, steps)
        ex = exact_rotation(f0, (n, n), M, (0.5, 0.5), T, q=M + 10)
        errs.append(np.linalg.norm(Q1 - ex) / np.linalg.norm(ex))
    order = math.log(errs[0] / errs[1]) / math.log(2)
    assert order > M - 0.7, (errs, order)


# ------------------------------------------------------------ the sampled step behind full-size parity
@pytest.mark.parametrize("n_steps", [1, 2])
def test_step_sampled_equals_full_step_rotation(n_steps):
    """step_sampled (the reference of every full-size GPU parity test) gives exactly what the whole
    mesh's step gives on corner, edge, interior and circulation-point elements (8^2, order 4)."""
    prob = S.Problem(d=2, n=(8, 8), M=4, velocity=("rotation", (0.5, 0.5)))
    rng = np.random.default_rng(41)
    Q = rng.standard_normal((prob.n_el, prob.theta)) * 0.5 ** np.array([sum(a) for a in prob.sidx])
    dt = 0.5 / (8 * 0.5)
    el = [prob.linear(ij) for ij in [(0, 0), (7, 7), (0, 7), (7, 0), (0, 3), (3, 0), (3, 4), (4, 4), (3, 3), (5, 6)]]
    full = S.step(prob, Q, dt, n_steps)
    got = S.step_sampled(prob, Q, dt, el, n_steps)
    assert sorted(got) == sorted(el)
    for e in el:
        np.testing.assert_allclose(got[e], full[e], rtol=0, atol=1e-14 * np.abs(full).max())


def test_step_sampled_equals_full_step_3d():
    prob = S.Problem(d=3, n=(5, 4, 4), M=3, velocity=("const", (1.0, -0.5, 0.75)))
    rng = np.random.default_rng(42)
    Q = rng.standard_normal((prob.n_el, prob.theta))
    dt = 0.4 / (5 * 1.0)
    el = [0, prob.n_el - 1, prob.linear((2, 1, 3)), prob.linear((4, 0, 2))]
    for n_steps in (1, 2):
        full = S.step(prob, Q, dt, n_steps)
        got = S.step_sampled(prob, Q, dt, el, n_steps)
        for e in el:
            np.testing.assert_allclose(got[e], full[e], rtol=0, atol=1e-14 * np.abs(full).max())


# ------------------------------------------------------------ eq. (l2relerror)
def _local_mode(d, n, M, axis, c):
    """1 + c psi_M(xi_axis): a constant plus one next-degree mode on every element (local coords)."""
    h = 1.0 / n

    def f(X):
        x = X[axis]
        xc = (np.floor(x / h) + 0.5) * h
        return 1.0 + c * basis.psi(M, 2.0 * (x - xc) / h)
    return f


@pytest.mark.parametrize("d,M", [(1, 2), (1, 4), (2, 3)])
def test_l2rel_paper_closed_forms(d, M):
    """eq. (l2relerror) on data with known coefficients: the constant mode is 1 and the only
    next-degree mode has coefficient c, so the exact projection onto the basis (order M) is the
    constant and the error is the truncation term alone, sqrt(c^2 / (1 + c^2)); an error delta in
    one retained mode adds delta^2 to the numerator; data inside the basis gives 0."""
    n = (6,) * d
    c, delta = 0.3, 0.05
    f = _local_mode(d, 6, M, 0, c)
    Q = np.zeros((6 ** d, len(basis.spatial_indices(d, M))))
    Q[:, 0] = 1.0
    assert abs(l2rel_paper(Q, f, d, n, M) - math.sqrt(c * c / (1 + c * c))) < 1e-13
    Q[:, 1] += delta
    assert abs(l2rel_paper(Q, f, d, n, M) - math.sqrt((c * c + delta * delta) / (1 + c * c))) < 1e-13
    # data inside the basis: a global polynomial of degree M - 1 and its projection
    g = lambda X: 0.5 + X[0] ** (M - 1) - 0.25 * X[-1]
    assert l2rel_paper(project(g, d, n, M), g, d, n, M) < 1e-13

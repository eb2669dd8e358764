"""CPU pins of the Burgers oracle (Newton on the region system, Sec. 3; eq. (burger2d)).

Each pin ties the oracle to something other than itself:
  * the analytic Jacobian against central differences of the residual (the perturbation method),
  * the quasi-quadrature-free Jacobian (projection of F'(w) and triple products, eq. (Jacobian2))
    against quadrature of every entry (eq. (Jacobian)),
  * Newton's quadratic convergence on the region system,
  * the small-amplitude limit: about a constant state c the Burgers step linearises to the
    constant-velocity advection step with v = c (1,..,1) of the linear oracle (independently pinned),
  * constant states preserved, element averages conserved,
  * the design order of accuracy against the exact pre-shock solution (method of characteristics).
"""

import numpy as np
import pytest

import oracle.burgers as B
import oracle.scheme as S
from oracle.project import project


def _random_region(p, seed, amp=0.1):
    rng = np.random.default_rng(seed)
    Q = 0.5 + amp * rng.standard_normal((p.n_el, p.theta))
    e = p.n_el // 2
    offs, elems = B._region(p, e)
    Qr = np.array([Q[g] for g in elems])
    Wr = Qr @ p.lift.T + 0.05 * rng.standard_normal((len(offs), p.theta_t))
    return Q, e, offs, Qr, Wr


@pytest.mark.parametrize("d,n,M", [(1, (5,), 4), (2, (4, 3), 3), (2, (3, 3), 2), (3, (3, 3, 3), 2)])
def test_jacobian_matches_perturbation(d, n, M):
    p = B.BurgersProblem(d=d, n=n, M=M)
    Q, e, offs, Qr, Wr = _random_region(p, 11 + d + M)
    dt = 0.3 / max(n)
    J = B.jacobian(p, offs, Wr, Qr, dt)
    Jfd = B.jacobian_perturbation(p, offs, Wr, Qr, dt)
    assert np.max(np.abs(J - Jfd)) <= 1e-9 * np.max(np.abs(J))
    # a planted mistake (a dropped neighbour block) is caught by the same comparison
    Jbad = J.copy()
    nt = p.theta_t
    Jbad[:nt, nt:2 * nt] = 0.0
    assert np.max(np.abs(Jbad - Jfd)) > 1e-6 * np.max(np.abs(J))


@pytest.mark.parametrize("d,M", [(1, 2), (1, 5), (2, 3), (2, 4), (3, 3)])
def test_qqf_jacobian_equals_quadrature(d, M):
    p = B.BurgersProblem(d=d, n=(3,) * d, M=M)
    rng = np.random.default_rng(3 + M)
    for _ in range(3):
        w = rng.standard_normal(p.theta_t)
        Jq = B.jacobian_volume_quadrature(p, w, 0.07)
        Jf = B.jacobian_volume_qqf(p, w, 0.07)
        assert np.max(np.abs(Jq - Jf)) <= 1e-13 * max(1.0, np.max(np.abs(Jq)))


def test_projection_reproduces_basis_functions():
    p = B.BurgersProblem(d=2, n=(3, 3), M=3)
    for k in range(p.theta_t):
        e = np.zeros(p.theta_t)
        e[k] = 1.0
        got = B.project_spacetime(p, p.ref.Psi.T @ e)
        assert np.max(np.abs(got - e)) <= 1e-14


def test_newton_converges_quadratically():
    p = B.BurgersProblem(d=2, n=(6, 6), M=3)
    Q = project(B.cosine_bump(2), 2, (6, 6), 3)
    hist = []
    B.newton_region(p, 8, Q, 0.1 / 6, hist)
    assert hist[-1] <= 1e-13
    # quadratic: each update at most C times the square of the previous one once in the basin
    for a, b in zip(hist[1:-1], hist[2:]):
        if a < 1e-3 and b > 1e-15:
            assert b <= 50.0 * a * a


@pytest.mark.parametrize("d,n,M", [(1, (6,), 3), (2, (4, 3), 2), (2, (3, 4), 3)])
def test_small_amplitude_limit_is_linear_advection(d, n, M):
    """Q = c e_0 + eps q1: the Burgers step is c e_0 + eps (advection step of q1 with v = c 1) + O(eps^2)."""
    c, eps = 0.6, 1e-6
    p = B.BurgersProblem(d=d, n=n, M=M)
    rng = np.random.default_rng(5 + d + M)
    q1 = rng.standard_normal((p.n_el, p.theta))
    Q = eps * q1
    Q[:, 0] += c
    dt = 0.4 / max(n)
    got = (B.step(p, Q, dt, 2) - np.eye(p.theta)[0] * c) / eps
    lin = S.step(S.Problem(d=d, n=n, M=M, velocity=("const", (c,) * d)), q1, dt, 2)
    assert np.linalg.norm(got - lin) <= 1e-4 * np.linalg.norm(lin)
    # the same comparison with the wrong advection speed fails
    wrong = S.step(S.Problem(d=d, n=n, M=M, velocity=("const", (0.5 * c,) * d)), q1, dt, 2)
    assert np.linalg.norm(got - wrong) > 1e-2 * np.linalg.norm(lin)


def test_constant_state_and_conservation():
    p = B.BurgersProblem(d=2, n=(4, 5), M=3)
    Q = np.zeros((p.n_el, p.theta))
    Q[:, 0] = 0.7
    assert np.max(np.abs(B.step(p, Q, 0.02, 2) - Q)) <= 1e-14
    Q = project(B.cosine_bump(2), 2, (4, 5), 3)
    Q1 = B.step(p, Q, 0.1 / 5, 2)
    assert abs(Q1[:, 0].sum() - Q[:, 0].sum()) <= 1e-14 * Q[:, 0].sum()


def test_step_sampled_matches_step():
    p = B.BurgersProblem(d=2, n=(5, 5), M=2)
    Q = project(B.cosine_bump(2), 2, (5, 5), 2)
    dt = 0.1 / 5
    full = B.step(p, Q, dt, 2)
    els = [0, 7, 24]
    got = B.step_sampled(p, Q, dt, els, n_steps=2)
    for e in els:
        assert np.max(np.abs(got[e] - full[e])) <= 1e-14


def test_exact_solution_satisfies_characteristics():
    q0 = B.cosine_bump(2)
    f = B.exact_solution(q0, 0.15, 2)
    X = np.random.default_rng(1).random((2, 50))
    q = f(X)
    assert np.max(np.abs(q - q0(X - 0.15 * q[None, :]))) <= 1e-13
    assert np.max(np.abs(B.exact_solution(q0, 0.0, 2)(X) - q0(X))) <= 1e-15


@pytest.mark.parametrize("M", [2, 3])
def test_order_of_accuracy_1d(M):
    """Smooth 1D solution at t = 0.15 (breaking at 1/pi): the error ratio between n and 2n is 2^M."""
    T = 0.15
    errs = []
    for n in (16, 32):
        p = B.BurgersProblem(d=1, n=(n,), M=M)
        Q = project(B.cosine_bump(1), 1, (n,), M)
        steps = int(round(T / (0.3 / n)))
        Q = B.step(p, Q, T / steps, steps)
        ex = project(B.exact_solution(B.cosine_bump(1), T, 1), 1, (n,), M)
        errs.append(np.sqrt(np.sum((Q - ex) ** 2) / n))
    order = np.log2(errs[0] / errs[1])
    assert order >= M - 0.35, (errs, order)


def test_newton_failure_is_reported():
    """Past the solvable range (steep compression at a large step) the oracle raises, never returns."""
    p = B.BurgersProblem(d=2, n=(8, 8), M=3, max_iter=8)
    Q = project(B.cosine_bump(2), 2, (8, 8), 3)
    with pytest.raises(B.NewtonFailure):
        B.newton_region(p, 54, Q, 0.5 / 8)

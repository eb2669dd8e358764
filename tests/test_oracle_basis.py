"""Pins of the oracle's basis, quadrature and element matrices against closed forms.

Nothing here re-runs the oracle's own formulas: the expected values are exact
rationals (Python ``fractions``), the Wigner-3j closed form of the Legendre
triple product (the finite-p property the paper relies on in Sec. 3), and the
spherical-Bessel closed form of Legendre moments of Fourier modes.
"""

import itertools
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import spherical_jn

from oracle import basis
from oracle.scheme import Problem, element_blocks
from oracle.project import project


def leg_int_rational(m, n):
    """int_{-1}^{1} P_m P_n = 2/(2m+1) delta_mn."""
    return Fraction(2, 2 * m + 1) if m == n else Fraction(0)


def leg_dint_rational(m, n):
    """int_{-1}^{1} P_m' P_n = 2 if n < m and m + n odd, else 0."""
    return Fraction(2) if (n < m and (m + n) % 2 == 1) else Fraction(0)


def triple_closed(a, b, c):
    """int_{-1}^{1} P_a P_b P_c = 2 (a b c; 0 0 0)^2 (Wigner 3j), exact rational."""
    s2 = a + b + c
    if s2 % 2 or c > a + b or a > b + c or b > a + c:
        return Fraction(0)
    s = s2 // 2
    f = math.factorial
    three_j_sq = Fraction(f(2 * s - 2 * a) * f(2 * s - 2 * b) * f(2 * s - 2 * c), f(2 * s + 1)) * \
        Fraction(f(s), f(s - a) * f(s - b) * f(s - c)) ** 2
    return 2 * three_j_sq


def quad(fn, q=20):
    x, w = basis.gauss(q)
    return float(np.sum(w * fn(x)))


@pytest.mark.parametrize("m", range(8))
def test_psi_mass_derivative_endpoints(m):
    for n in range(8):
        norm = math.sqrt((2 * m + 1) * (2 * n + 1))
        got = quad(lambda x: basis.psi(m, x) * basis.psi(n, x))
        assert got == pytest.approx(norm * float(leg_int_rational(m, n)), abs=1e-13)
        got = quad(lambda x: basis.dpsi(m, x) * basis.psi(n, x))
        assert got == pytest.approx(norm * float(leg_dint_rational(m, n)), abs=1e-12)
    for s in (-1.0, 1.0):
        assert float(basis.psi(m, np.array([s]))[0]) == pytest.approx(math.sqrt(2 * m + 1) * s ** m, abs=1e-13)


def test_triple_products_closed_form():
    for a, b, c in itertools.product(range(7), repeat=3):
        got = quad(lambda x: basis.psi(a, x) * basis.psi(b, x) * basis.psi(c, x))
        want = math.sqrt((2 * a + 1) * (2 * b + 1) * (2 * c + 1)) * float(triple_closed(a, b, c))
        assert got == pytest.approx(want, abs=1e-12)


def test_index_sets_and_order():
    assert basis.spatial_indices(2, 3) == [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]
    assert basis.spacetime_indices(1, 2) == [(0, 0), (1, 0), (0, 1)]
    # counts: theta = C(M-1+d, d), theta_T = C(M+d, d+1)
    for d in (1, 2, 3):
        for M in range(1, 6):
            assert len(basis.spatial_indices(d, M)) == math.comb(M - 1 + d, d)
            assert len(basis.spacetime_indices(d, M)) == math.comb(M + d, d + 1)
    assert len(basis.spacetime_indices(2, 4, "Q")) == 64  # the paper's tensor space, (M_deg+1)^(d+1)


@pytest.mark.parametrize("d,M", [(1, 3), (2, 3), (2, 4)])
def test_time_term_and_causal_source_exact(d, M):
    """Time term and causal matrix against exact rationals (eq. pred_full_system).

    T[k,l] = 2^d delta(space) [psi_k0(1) psi_l0(1) - int psi_k0' psi_l0],
    C[k,l] = 2^d psi_k0(-1) delta(spatial part of k = l).
    """
    prob = Problem(d=d, n=(4,) * d, M=M, velocity=("const", (0.3,) * d))
    B = element_blocks(prob, 0, 0.01)
    tid, sid = prob.tidx, prob.sidx
    T = np.zeros((len(tid), len(tid)))
    C = np.zeros((len(tid), len(sid)))
    for k, bk in enumerate(tid):
        for l, bl in enumerate(tid):
            if bk[1:] != bl[1:]:
                continue
            a, b = bk[0], bl[0]
            norm = math.sqrt((2 * a + 1) * (2 * b + 1))
            T[k, l] = 2 ** d * norm * (1.0 - float(leg_dint_rational(a, b)))
        for l, al in enumerate(sid):
            if bk[1:] == al:
                C[k, l] = 2 ** d * math.sqrt(2 * bk[0] + 1) * (-1) ** bk[0]
    np.testing.assert_allclose(B["T"], T, atol=1e-12)
    np.testing.assert_allclose(B["C"], C, atol=1e-12)


@pytest.mark.parametrize("k", [1, 2, 5])
@pytest.mark.parametrize("M", [2, 4])
def test_projection_spherical_bessel(k, M):
    """int_{-1}^{1} e^{i w s} P_n(s) ds = 2 i^n j_n(w): exact moments of Fourier modes."""
    n = 8
    Q = project(lambda X: np.cos(2 * np.pi * k * X[0]), 1, (n,), M, q=M + 14)
    h = 1.0 / n
    w = 2 * np.pi * k * h / 2
    for e in range(n):
        xc = (e + 0.5) * h
        for m in range(M):
            # (1/2) int cos(2 pi k (xc + h s/2)) psi_m(s) ds
            mom = 2 * (1j ** m) * spherical_jn(m, w)  # int e^{i w s} P_m
            val = 0.5 * math.sqrt(2 * m + 1) * np.real(np.exp(1j * 2 * np.pi * k * xc) * mom)
            assert Q[e, m] == pytest.approx(val, abs=1e-13)

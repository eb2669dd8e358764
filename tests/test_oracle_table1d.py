"""The oracle against the errors the paper prints for 1D advection (Sec. 6.1, Table 1D; fixture
tests/golden/table1d_printed.json), tensor (Q) space-time basis, CFL 0.9, T = 1, error of eq. (l2relerror).

Reading (recorded with the other readings of the paper): with the bump of eq. (adv1d) as printed,
exp(1 / ((x - c)^2 - omega^2)) with omega = 1/3, every printed error is 100-300x above the oracle's,
with the same convergence orders; the final time, an interpolated instead of projected initial state
and the error formula do not account for it. A bump with omega = 1/5 reproduces the printed rows:
within 0.6-1.3x for M_deg = 3 and 5 (and within 3-11x for M_deg = 7 and 9). The test pins the oracle
to the printed values under that reading and records the factor under the printed one.
"""

import json
import os

import numpy as np
import pytest

import oracle.scheme as S
from oracle.project import l2rel_paper, periodic_translate, project

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = json.load(open(os.path.join(HERE, "golden", "table1d_printed.json")))


def bump(omega, c=0.5):
    def f(X):
        r2 = (X[0] - c) ** 2
        out = np.zeros_like(X[0])
        m = r2 < omega ** 2
        out[m] = np.exp(1.0 / (r2[m] - omega ** 2))
        return out
    return f


def run(N, Mdeg, omega):
    M = Mdeg + 1
    q0 = bump(omega)
    p = S.Problem(d=1, n=(N,), M=M, velocity=("const", (1.0,)), family="Q")
    Q = project(q0, 1, (N,), M, family="Q")
    steps = int(round(TABLE["final_time"] / (TABLE["cfl"] / N)))
    Q = S.step(p, Q, TABLE["final_time"] / steps, steps)
    return l2rel_paper(Q, periodic_translate(q0, (1.0,), TABLE["final_time"]), 1, (N,), M, family="Q")


@pytest.mark.parametrize("mdeg", ["3", "5"])
def test_printed_errors_reproduced_with_narrower_bump(mdeg):
    for N, printed in TABLE["rows"][mdeg][:3]:
        err = run(N, int(mdeg), 0.2)
        assert 0.5 <= printed / err <= 2.0, (N, err, printed)


def test_printed_bump_gives_errors_two_orders_lower():
    N, printed = TABLE["rows"]["3"][0]
    err = run(N, 3, 1.0 / 3.0)
    assert 50.0 <= printed / err <= 300.0

"""GPU: the temporally blocked 2D composite stencil (RIDG_OPT_COMPOSITE = 3; Sec. 2.2-2.3 composed into
taps on the state, four steps per launch) bitwise against the one-step composite kernel (the same
fused multiply-adds in the same order) for step counts that are and are not multiples of four,
against the FP64 oracle, and on the 256^2 order-3 workload."""

import numpy as np
import pytest

import oracle.scheme as S
from paper_2101_01231_amd import inputs as I
from paper_2101_01231_amd import ridg

pytestmark = pytest.mark.gpu


def _run(n, M, v, q0, dt, steps, composite):
    sim = ridg.Simulation(ridg.make_problem(2, n, M, velocity=v))
    sim.set_option(ridg.OPT_COMPOSITE, composite)
    sim.set_state(q0)
    sim.step(steps, dt)
    out = sim.get_state()
    sim.close()
    return out


CASES = [((32, 48), 3, (1.0, 0.5)), ((16, 16), 4, (-0.6, 0.8)), ((32, 16), 5, (0.3, -0.9)),
         ((16, 32), 1, (0.7, 0.0)), ((48, 16), 2, (-0.2, -0.9))]


@pytest.mark.parametrize("n,M,v", CASES)
def test_tblock_bitwise_and_oracle(n, M, v):
    q0 = I.random_state(2, n, M, seed=140 + M)
    dt = 0.4 / max(n) / max(abs(x) for x in v)
    for steps in (4, 7, 9):
        print(f"[gpu] tblock n={n} M={M} v={v} steps={steps}", flush=True)
        got = _run(n, M, v, q0, dt, steps, 3)
        assert np.array_equal(got, _run(n, M, v, q0, dt, steps, 1)), steps
    if np.prod(n) <= 768:
        ref = S.step(S.Problem(d=2, n=n, M=M, velocity=("const", v)), q0, dt, 9)
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_tblock_full_size_bitwise():
    wl = I.advection_2d()
    print("[gpu] tblock 256^2, 100 steps", flush=True)
    a = _run(wl.n, wl.M, wl.velocity[1], wl.q0, wl.dt, wl.steps, 3)
    b = _run(wl.n, wl.M, wl.velocity[1], wl.q0, wl.dt, wl.steps, 1)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("d,n,kw", [(2, (24, 16), {}), (3, (16, 16, 16), {}), (2, (16, 16), {"solver": ridg.SOLVER_REGION})])
def test_tblock_rejected_where_not_applicable(d, n, kw):
    sim = ridg.Simulation(ridg.make_problem(d, n, 3, velocity=(1.0,) * d, **kw))
    with pytest.raises(ridg.RidgError) as ei:
        sim.set_option(ridg.OPT_COMPOSITE, 3)
    assert ei.value.code == ridg.RIDG_E_UNSUPPORTED
    sim.close()

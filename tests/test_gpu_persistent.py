"""GPU: persistent multi-step launches (RIDG_OPT_FUSED = 2: every step of a ridg_step call in one
cooperative launch, a grid-wide barrier between steps) against the composite stencil launched step by
step (bitwise: the same fused multiply-adds) and against the stored FP64 oracle run of the 2D
advection workload (32^2, order 3, 100 steps)."""

import os

import numpy as np
import pytest

from paper_2101_01231_amd import inputs as I
from paper_2101_01231_amd import ridg

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _run(d, n, M, v, q0, dt, steps, fused):
    sim = ridg.Simulation(ridg.make_problem(d, n, M, velocity=v))
    sim.set_option(ridg.OPT_COMPOSITE, 1)
    sim.set_option(ridg.OPT_FUSED, fused)
    sim.set_state(q0)
    sim.step(steps, dt)
    out = sim.get_state()
    sim.close()
    return out


@pytest.mark.parametrize("d,n,M,v,steps", [(2, (256, 256), 3, (1.0, 0.5), 7), (2, (256, 256), 3, (1.0, 0.5), 100),
                                           (1, (64,), 3, (1.0,), 13), (3, (20, 12, 16), 2, (0.6, -0.9, 0.2), 4)])
def test_persistent_equals_stepwise(d, n, M, v, steps):
    q0 = I.random_state(d, n, M, seed=200 + steps)
    dt = 0.4 / max(n) / max(abs(x) for x in v)
    print(f"[gpu] persistent d={d} n={n} M={M} steps={steps}", flush=True)
    a = _run(d, n, M, v, q0, dt, steps, 2)
    b = _run(d, n, M, v, q0, dt, steps, 0)
    assert np.array_equal(a, b)


def test_persistent_against_stored_oracle():
    z = np.load(os.path.join(GOLDEN, "adv2d32_m3_100steps.npz"))
    n, M = tuple(int(x) for x in z["n"]), int(z["M"])
    v = tuple(float(x) for x in z["velocity"])
    got = _run(2, n, M, v, z["q0"], float(z["dt"]), int(z["steps"]), 2)
    ref = z["ref"]
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.max(np.linalg.norm(got - ref, axis=1)) <= 1e-11 * np.max(np.linalg.norm(ref, axis=1))

"""GPU: the z-marched composite stencil (RIDG_OPT_COMPOSITE = 2; Sec. 2.2-2.3 composed into taps on the
state) against the FP64 oracle, and bitwise against the one-element-per-thread composite kernel (the
same fused multiply-adds in the same order), including the 128^3 order-3 workload."""

import numpy as np
import pytest

import oracle.scheme as S
from paper_2101_01231_amd import inputs as I
from paper_2101_01231_amd import ridg

pytestmark = pytest.mark.gpu


def _run(n, M, v, q0, dt, steps, composite):
    sim = ridg.Simulation(ridg.make_problem(3, n, M, velocity=v))
    sim.set_option(ridg.OPT_COMPOSITE, composite)
    sim.set_state(q0)
    sim.step(steps, dt)
    out = sim.get_state()
    sim.close()
    return out


@pytest.mark.parametrize("n,M,v", [((16, 16, 8), 3, (1.0, 1.0, 1.0)), ((16, 16, 8), 2, (-0.7, 0.4, 0.0)),
                                   ((32, 16, 16), 3, (0.5, -0.8, 0.3))])
def test_zmarch_against_oracle_and_composite(n, M, v):
    q0 = I.random_state(3, n, M, seed=120 + M)
    dt = 0.45 / max(n) / max(abs(x) for x in v)
    print(f"[gpu] zmarch n={n} M={M} v={v}", flush=True)
    got = _run(n, M, v, q0, dt, 2, 2)
    assert np.array_equal(got, _run(n, M, v, q0, dt, 2, 1))
    if np.prod(n) <= 2048:
        ref = S.step(S.Problem(d=3, n=n, M=M, velocity=("const", v)), q0, dt, 2)
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_zmarch_full_size_bitwise():
    wl = I.advection_3d()
    print("[gpu] zmarch 128^3", flush=True)
    a = _run(wl.n, wl.M, wl.velocity[1], wl.q0, wl.dt, 2, 2)
    b = _run(wl.n, wl.M, wl.velocity[1], wl.q0, wl.dt, 2, 1)
    assert np.array_equal(a, b)


def test_zmarch_rejected_where_not_applicable():
    sim = ridg.Simulation(ridg.make_problem(3, (12, 16, 8), 3, velocity=(1.0, 1.0, 1.0)))
    with pytest.raises(ridg.RidgError):
        sim.set_option(ridg.OPT_COMPOSITE, 2)
    sim.close()


def test_banded_two_plane_kernel_small_mesh():
    """On a mesh whose y-bands hold whole workgroups (64 x 32 x 4) the composite step runs two
    z-neighbours per thread with the XCD band mapping: bitwise the z-marched kernel's result (same
    taps, same order), and the prediction + correction path's to rounding."""
    n, M, v = (64, 32, 4), 3, (0.8, -0.6, 0.4)
    q0 = I.random_state(3, n, M, seed=131)
    dt = 0.45 / max(n) / max(abs(x) for x in v)
    print(f"[gpu] banded z2 n={n}", flush=True)
    got = _run(n, M, v, q0, dt, 3, 1)
    assert np.array_equal(got, _run(n, M, v, q0, dt, 3, 2))
    ref = _run(n, M, v, q0, dt, 3, 0)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)

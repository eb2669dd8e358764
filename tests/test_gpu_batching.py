"""GPU: execution options of the batching row - graph replay, segment layouts, fused small-mesh
steps and the autotuner - leave the results unchanged (bitwise where the arithmetic is the same)."""

import numpy as np
import pytest

import oracle.scheme as S
from paper_2101_01231_amd import inputs as I
from paper_2101_01231_amd import ridg

pytestmark = pytest.mark.gpu


def _rot(n, M, **kw):
    return ridg.make_problem(2, (n, n), M, flux=ridg.FLUX_ROTATION, rot_center=(0.5, 0.5), **kw)


def _max_elem_rel(a, b):
    """Largest per-element error relative to the state's largest element norm."""
    return float(np.max(np.linalg.norm(a - b, axis=1)) / np.max(np.linalg.norm(b, axis=1)))


def _run(problem, q0, dt, steps, options=(), chunks=None):
    sim = ridg.Simulation(problem)
    for opt, val in options:
        sim.set_option(opt, val)
    sim.set_state(q0)
    for c in (chunks or [steps]):
        sim.step(c, dt)
    out = sim.get_state()
    sim.close()
    return out


@pytest.mark.parametrize("problem_kind", ["rotation", "constant2d", "constant3d"])
def test_graph_replay_matches_direct(problem_kind):
    if problem_kind == "rotation":
        p, q0, dt = _rot(32, 4), I.random_state(2, (32, 32), 4, seed=1), 1.0 / 32
    elif problem_kind == "constant2d":
        p, q0, dt = ridg.make_problem(2, (24, 20), 3, velocity=(1.0, 0.5)), I.random_state(2, (24, 20), 3, seed=2), 0.02
    else:
        p, q0, dt = ridg.make_problem(3, (6, 5, 4), 3, velocity=(1.0, 1.0, 1.0)), I.random_state(3, (6, 5, 4), 3, 3), 0.05
    print(f"[gpu] graph {problem_kind}", flush=True)
    direct = _run(p, q0, dt, 9)
    # graph replays: several launches of the same graph with eager work (odd steps) in between
    graph = _run(p, q0, dt, 9, options=[(ridg.OPT_GRAPH, 1)], chunks=[4, 1, 2, 2])
    assert np.array_equal(direct, graph)


@pytest.mark.parametrize("case", ["rotation", "const3d", "const1d"])
def test_plan_layouts_agree(case):
    """Every segment layout of the region-solve kernel gives bitwise the same steps (same arithmetic)."""
    if case == "rotation":
        p, q0, dt = _rot(24, 4), I.random_state(2, (24, 24), 4, seed=4), 1.0 / 24
        ref_prob = S.Problem(d=2, n=(24, 24), M=4, velocity=("rotation", (0.5, 0.5)))
    elif case == "const3d":
        v = (1.0, -0.5, 0.25)
        p = ridg.make_problem(3, (5, 6, 7), 3, velocity=v, solver=ridg.SOLVER_REGION)
        q0, dt = I.random_state(3, (5, 6, 7), 3, seed=9), 0.05
        ref_prob = S.Problem(d=3, n=(5, 6, 7), M=3, velocity=("const", v))
    else:
        p = ridg.make_problem(1, (29,), 5, velocity=(-0.7,), solver=ridg.SOLVER_REGION)
        q0, dt = I.random_state(1, (29,), 5, seed=10), 0.4 / 29 / 0.7
        ref_prob = S.Problem(d=1, n=(29,), M=5, velocity=("const", (-0.7,)))
    print(f"[gpu] plan layouts {case}", flush=True)
    a = _run(p, q0, dt, 3)
    for lay in (1, 2, 3, 4):
        b = _run(p, q0, dt, 3, options=[(ridg.OPT_PLAN_LAYOUT, lay)])
        assert np.array_equal(a, b), lay
    ref = S.step(ref_prob, q0, dt, 3)
    assert np.linalg.norm(a - ref) / np.linalg.norm(ref) <= 1e-12
    # static pivots: a different elimination, the same solution to rounding
    sim = ridg.Simulation(p)
    sim.set_option(ridg.OPT_PLAN_LAYOUT, 5)
    sim.set_state(q0)
    sim.step(3, dt)
    sp = sim.get_state()
    assert sim.get_info().static_pivot_growth <= 64.0  # static pivots ran (no fallback)
    sim.close()
    assert np.linalg.norm(sp - ref) / np.linalg.norm(ref) <= 1e-12
    assert _max_elem_rel(sp, ref) <= 1e-11


def test_two_region_layout_rejected_for_fp32():
    p = ridg.make_problem(2, (16, 16), 3, flux=ridg.FLUX_ROTATION, rot_center=(0.5, 0.5),
                          precision=ridg.FP32_REFINE, refine_steps=2)
    sim = ridg.Simulation(p)
    with pytest.raises(ridg.RidgError):
        sim.set_option(ridg.OPT_PLAN_LAYOUT, 2)
    with pytest.raises(ridg.RidgError):
        sim.set_option(ridg.OPT_PLAN_LAYOUT, 3)
    with pytest.raises(ridg.RidgError):
        sim.set_option(ridg.OPT_PLAN_LAYOUT, 6)
    sim.set_option(ridg.OPT_PLAN_LAYOUT, 5)  # static pivots take FP32 with refinement
    sim.close()


@pytest.mark.parametrize("d,n,M,v", [(1, (64,), 3, (1.0,)), (1, (37,), 5, (-0.6,)), (2, (12, 10), 3, (0.8, -0.4))])
def test_fused_small_mesh_matches_direct(d, n, M, v):
    p = ridg.make_problem(d, n, M, velocity=v)
    q0 = I.random_state(d, n, M, seed=5)
    dt = 0.45 / max(n) / max(abs(x) for x in v)
    direct = _run(p, q0, dt, 25)
    fused = _run(p, q0, dt, 25, options=[(ridg.OPT_FUSED, 1)], chunks=[10, 15])
    # the fused kernel applies the correction term by term, the default step in precombined tap form
    assert np.linalg.norm(fused - direct) / np.linalg.norm(direct) <= 1e-13


def test_fused_rejected_when_not_applicable():
    sim = ridg.Simulation(_rot(16, 3))
    with pytest.raises(ridg.RidgError):
        sim.set_option(ridg.OPT_FUSED, 1)
    big = ridg.Simulation(ridg.make_problem(2, (256, 256), 3, velocity=(1.0, 0.5)))
    with pytest.raises(ridg.RidgError):
        big.set_option(ridg.OPT_FUSED, 1)
    sim.close()
    big.close()


@pytest.mark.parametrize("kind", ["rotation", "sine"])
def test_autotune_keeps_state_and_results(kind):
    if kind == "rotation":
        p, q0, dt = _rot(32, 4), I.random_state(2, (32, 32), 4, seed=6), 1.0 / 32
    else:
        wl = I.sine_1d()
        p, q0, dt = ridg.make_problem(1, wl.n, wl.M, velocity=(1.0,)), wl.q0, wl.dt
    ref = _run(p, q0, dt, 7)
    sim = ridg.Simulation(p)
    sim.set_state(q0)
    ms = sim.autotune(dt, steps=6)
    assert ms > 0 or ms == -1.0
    np.testing.assert_array_equal(sim.get_state(), q0)  # tuning restored the state
    sim.step(7, dt)
    got = sim.get_state()
    sim.close()
    # the tuner may pick a composed or fused variant: same scheme, different rounding order
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-13


@pytest.mark.parametrize("d,n,M,v", [(3, (6, 5, 4), 3, (1.0, 1.0, 1.0)), (2, (24, 20), 4, (1.0, 0.5)),
                                     (1, (40,), 5, (-0.8,)), (2, (9, 8), 2, (0.0, -0.6)),
                                     (3, (4, 3, 5), 4, (0.6, -0.8, 0.3)), (3, (3, 4, 3), 5, (-0.5, 0.7, 0.9)),
                                     (2, (17, 19), 5, (0.3, 0.9))])
def test_composite_and_tap_correction_match_oracle(d, n, M, v):
    """Constant velocity: the tap-form correction (default) and the composite stencil against the oracle."""
    p = ridg.make_problem(d, n, M, velocity=v)
    q0 = I.random_state(d, n, M, seed=8)
    dt = 0.45 * min(1.0 / k for k in n) / max(abs(x) for x in v)
    ref = S.step(S.Problem(d=d, n=n, M=M, velocity=("const", v)), q0, dt, 3)
    for opts in ([], [(ridg.OPT_COMPOSITE, 1)], [(ridg.OPT_MFMA, 1)], [(ridg.OPT_MFMA, 1), (ridg.OPT_COMPOSITE, 1)]):
        print(f"[gpu] taps d={d} n={n} M={M} {opts}", flush=True)
        got = _run(p, q0, dt, 3, options=opts)
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-12, opts


@pytest.mark.parametrize("d,n,M,v", [(3, (16, 9, 5), 3, (1.0, -0.7, 0.4)), (2, (33, 17), 4, (-1.0, 0.5)),
                                     (2, (40, 40), 5, (0.3, 0.9)), (1, (50,), 4, (0.8,)), (3, (5, 4, 6), 4, (0.2, 0.3, -0.9)),
                                     (3, (6, 5, 7), 5, (0.5, -1.0, 0.3)), (2, (384, 384), 3, (1.0, 0.5))])
def test_mfma_tap_kernels_match_vector_kernels(d, n, M, v):
    """FP64 MFMA tap kernels (prediction, correction, composite) against the vector kernels: ragged
    tile tails (element counts not multiples of 16), several row tiles (theta_T > 16), operators
    too large for LDS (3D order 5, read through the caches), and a 384^2 mesh of 2304 workgroups."""
    p = ridg.make_problem(d, n, M, velocity=v)
    q0 = I.random_state(d, n, M, seed=11)
    dt = 0.4 * min(1.0 / k for k in n) / max(abs(x) for x in v)
    print(f"[gpu] mfma d={d} n={n} M={M}", flush=True)
    for comp in (0, 1):
        ref = _run(p, q0, dt, 4, options=[(ridg.OPT_COMPOSITE, comp)])
        got = _run(p, q0, dt, 4, options=[(ridg.OPT_COMPOSITE, comp), (ridg.OPT_MFMA, 1)])
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-13, comp


def test_mfma_option_needs_prefactored():
    sim = ridg.Simulation(_rot(16, 3))
    with pytest.raises(ridg.RidgError):
        sim.set_option(ridg.OPT_MFMA, 1)
    sim.close()

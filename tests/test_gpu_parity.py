"""GPU parity: libridg (HIP, gfx950) against the FP64 oracle on the same seeded inputs.

Bar: relative L2 over all coefficients <= 1e-12 for the FP64 paths (the tolerance the
method's FP64 results are held to), on small meshes for several steps (several thread
blocks and a ragged tail) and on sampled elements at the benchmark sizes for one step.
"""

import math
import os

import numpy as np
import pytest

import oracle.scheme as S
from paper_2101_01231_amd import inputs as I
from paper_2101_01231_amd import ridg

pytestmark = pytest.mark.gpu

TOL = 1e-12


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def max_elem_rel(a, b):
    """Largest per-element error, relative to the largest element norm of the reference."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.linalg.norm(a - b, axis=1)) / np.max(np.linalg.norm(b, axis=1)))


def oracle_problem(d, n, M, velocity):
    return S.Problem(d=d, n=tuple(n), M=M, velocity=velocity)


def lib_problem(d, n, M, velocity, solver=ridg.SOLVER_AUTO, precision=ridg.FP64, refine=0):
    if velocity[0] == "const":
        return ridg.make_problem(d, n, M, velocity=velocity[1], solver=solver, precision=precision,
                                 refine_steps=refine)
    return ridg.make_problem(d, n, M, flux=ridg.FLUX_ROTATION, rot_center=velocity[1], solver=solver,
                             precision=precision, refine_steps=refine)


def run_gpu(d, n, M, velocity, q0, dt, steps, solver=ridg.SOLVER_AUTO, **kw):
    print(f"[gpu] d={d} n={n} M={M} vel={velocity} solver={solver} steps={steps}", flush=True)
    sim = ridg.Simulation(lib_problem(d, n, M, velocity, solver, **kw))
    sim.set_state(q0)
    sim.step(steps, dt)
    out = sim.get_state()
    sim.close()
    return out


def test_config_sine_1d_full():
    """1D, 64 elements, order 3, v = 1, sin(2 pi x), CFL 0.5, 200 steps: both solvers, and the
    timed paths (all steps in one fused launch, graph replay) against the oracle."""
    wl = I.sine_1d()
    prob = oracle_problem(1, wl.n, wl.M, wl.velocity)
    ref = S.step(prob, wl.q0, wl.dt, wl.steps)
    for solver in (ridg.SOLVER_PREFACTORED, ridg.SOLVER_REGION):
        got = run_gpu(1, wl.n, wl.M, wl.velocity, wl.q0, wl.dt, wl.steps, solver)
        assert rel_l2(got, ref) <= TOL
        assert max_elem_rel(got, ref) <= 1e-11
    for opts in ([(ridg.OPT_FUSED, 1)], [(ridg.OPT_GRAPH, 1)], [(ridg.OPT_GRAPH, 1), (ridg.OPT_COMPOSITE, 1)]):
        sim = ridg.Simulation(lib_problem(1, wl.n, wl.M, wl.velocity))
        for o in opts:
            sim.set_option(*o)
        sim.set_state(wl.q0)
        sim.step(wl.steps, wl.dt)
        got = sim.get_state()
        sim.close()
        assert rel_l2(got, ref) <= TOL, opts
        assert max_elem_rel(got, ref) <= 1e-11, opts


CONST_CASES = [
    (1, (37,), 1, ("const", (0.9,))),
    (1, (29,), 5, ("const", (-0.7,))),
    (2, (24, 20), 3, ("const", (1.0, 0.5))),
    (2, (17, 9), 2, ("const", (-0.4, 0.8))),
    (2, (6, 5), 5, ("const", (0.3, 0.0))),
    (3, (6, 5, 4), 3, ("const", (1.0, 1.0, 1.0))),
    (3, (4, 3, 5), 2, ("const", (-0.5, 0.25, 0.75))),
    (3, (4, 3, 5), 4, ("const", (0.6, -0.8, 0.3))),
    (3, (3, 4, 3), 5, ("const", (-0.5, 0.7, 0.9))),
]


@pytest.mark.parametrize("d,n,M,vel", CONST_CASES)
@pytest.mark.parametrize("solver", [ridg.SOLVER_PREFACTORED, ridg.SOLVER_REGION, ridg.SOLVER_DENSE])
def test_constant_velocity_small(d, n, M, vel, solver):
    if solver == ridg.SOLVER_REGION and math.comb(M + d, d + 1) > 64:
        # 3D order 5 (theta_T = 70) has no block-elimination kernel: a clear error, not a wrong result
        sim = ridg.Simulation(lib_problem(d, n, M, vel, solver))
        with pytest.raises(ridg.RidgError) as ei:
            sim.step(1, 0.01)
        sim.close()
        assert ei.value.code == ridg.RIDG_E_UNSUPPORTED
        return
    prob = oracle_problem(d, n, M, vel)
    q0 = I.random_state(d, n, M, seed=17 + d + M)
    vmax = max(abs(x) for x in vel[1])
    dt = 0.45 * min(prob.h) / vmax
    steps = 3
    ref = S.step(prob, q0, dt, steps)
    got = run_gpu(d, n, M, vel, q0, dt, steps, solver)
    assert rel_l2(got, ref) <= TOL


ROT_CASES = [(16, 4), (12, 3), (8, 5), (10, 2), (6, 1)]


@pytest.mark.parametrize("n,M", ROT_CASES)
@pytest.mark.parametrize("solver", [ridg.SOLVER_REGION, ridg.SOLVER_DENSE])
def test_rotation_small(n, M, solver):
    vel = ("rotation", (0.5, 0.5))
    prob = oracle_problem(2, (n, n), M, vel)
    q0 = I.random_state(2, (n, n), M, seed=5 + M)
    dt = 0.5 / (n * 0.5)
    steps = 2
    ref = S.step(prob, q0, dt, steps)
    got = run_gpu(2, (n, n), M, vel, q0, dt, steps, solver)
    assert rel_l2(got, ref) <= TOL
    assert max_elem_rel(got, ref) <= 1e-11


@pytest.mark.parametrize("n,M", [(16, 4), (12, 3), (8, 5), (10, 2)])
def test_rotation_static_pivots_and_cyclic_regions(n, M):
    """Static-pivot region solves (layout 5) against the oracle, and every cyclic (torn) region's
    prediction checked on its own against the oracle's region solve."""
    vel = ("rotation", (0.5, 0.5))
    prob = oracle_problem(2, (n, n), M, vel)
    q0 = I.random_state(2, (n, n), M, seed=7 + M)
    dt = 0.5 / (n * 0.5)
    ref = S.step(prob, q0, dt, 2)
    sim = ridg.Simulation(lib_problem(2, (n, n), M, vel, ridg.SOLVER_REGION))
    sim.set_option(ridg.OPT_PLAN_LAYOUT, 5)
    sim.set_state(q0)
    sim.step(2, dt)
    got = sim.get_state()
    assert 1.0 <= sim.get_info().static_pivot_growth <= 64.0  # layout 5 ran (no fallback)
    assert rel_l2(got, ref) <= TOL
    assert max_elem_rel(got, ref) <= 1e-11
    # predictions of the regions around the two circulation points (centre and periodic corner)
    c = n // 2
    torn = [prob.linear((i, j)) for i in (c - 1, c) for j in (c - 1, c)]
    torn += [prob.linear((i, j)) for i in (n - 1, 0) for j in (n - 1, 0)]
    W = sim.get_prediction(dt)  # from the state after the two steps
    sim.close()
    Wref = S.predict(prob, got, dt, torn)
    for e in torn:
        assert np.linalg.norm(W[e] - Wref[e]) <= 1e-12 * np.linalg.norm(Wref[e]), e


@pytest.mark.parametrize("d,n,M,vel", [
    (2, (16, 16), 4, ("rotation", (0.5, 0.5))),
    (2, (10, 7), 3, ("const", (0.6, -0.9))),
    (3, (4, 5, 3), 2, ("const", (0.5, 1.0, -0.5))),
])
def test_prediction_parity(d, n, M, vel):
    """The prediction alone: the centre predictions W against the oracle's region solves."""
    prob = oracle_problem(d, n, M, vel)
    q0 = I.random_state(d, n, M, seed=99)
    dt = 0.4 * min(prob.h) / (0.5 if vel[0] == "rotation" else max(abs(x) for x in vel[1]))
    ref = S.predictions(prob, q0, dt)
    solvers = [ridg.SOLVER_REGION, ridg.SOLVER_DENSE] + ([ridg.SOLVER_PREFACTORED] if vel[0] == "const" else [])
    for solver in solvers:
        sim = ridg.Simulation(lib_problem(d, n, M, vel, solver))
        sim.set_state(q0)
        w = sim.get_prediction(dt)
        sim.close()
        assert rel_l2(w, ref) <= TOL, solver


def _sample(prob, rng, count, extra=()):
    el = set(int(x) for x in rng.integers(0, prob.n_el, count))
    el.update(extra)
    return sorted(el)


def test_rotation_full_size_sampled():
    """512x512, order 4, rotation about (1/2, 1/2): two steps on sampled elements (including the
    cyclic regions around the rotation centre and the periodic corner, solved by tearing) against
    the oracle, per element and in rel-L2."""
    wl = I.rotation_2d()
    n = wl.n[0]
    prob = oracle_problem(2, wl.n, wl.M, wl.velocity)
    rng = np.random.default_rng(4)
    q0 = wl.q0 + 0.01 * I.random_state(2, wl.n, wl.M, seed=3)  # every element non-trivial
    c = n // 2
    torn = [prob.linear((i, j)) for i in (c - 1, c) for j in (c - 1, c)]
    torn += [prob.linear((i, j)) for i in (n - 1, 0) for j in (n - 1, 0)]
    special = [prob.linear((i, j)) for i in (c - 2, c - 1, c, c + 1) for j in (c - 2, c - 1, c, c + 1)]
    special += [prob.linear((0, 0)), prob.linear((n - 1, n - 1)), prob.linear((c, 0)), prob.linear((0, c))]
    el = _sample(prob, rng, 16, special + torn)
    ref = S.step_sampled(prob, q0, wl.dt, el, n_steps=2)
    sim = ridg.Simulation(lib_problem(2, wl.n, wl.M, wl.velocity))
    # the rotation centre and the periodic corner are the two circulation points: 4 cyclic regions each
    assert sim.info.n_tear_elements == 8 and sim.info.n_dense_elements == 0
    refs = np.array([ref[e] for e in el])
    it = [el.index(e) for e in torn]
    # every segment layout of the region-solve kernel, then the autotuned configuration bench.py times
    for lay in range(6):
        print(f"[gpu] rotation 512^2 layout {lay}", flush=True)
        sim.set_option(ridg.OPT_PLAN_LAYOUT, lay)
        sim.set_state(q0)
        sim.step(2, wl.dt)
        got = sim.get_state()[el]
        if lay == 5:
            assert sim.get_info().static_pivot_growth <= 64.0  # static pivots ran (no fallback)
        assert rel_l2(got, refs) <= TOL, lay
        assert max_elem_rel(got, refs) <= 1e-11, lay
        assert max_elem_rel(got[it], refs[it]) <= 1e-11, lay  # the torn regions on their own
    sim.set_state(q0)
    sim.autotune(wl.dt, steps=4)
    print(f"[gpu] rotation 512^2 autotuned layout {sim.get_option(ridg.OPT_PLAN_LAYOUT)}", flush=True)
    sim.step(2, wl.dt)  # the timed path: graph replay when the tuner picked it
    got = sim.get_state()
    sim.close()
    assert rel_l2(got[el], refs) <= TOL
    assert max_elem_rel(got[el], refs) <= 1e-11


def _const_full_size(d, wl, el, ref, steps):
    """`steps` steps in each constant-velocity kernel configuration, and autotuned as bench.py runs
    it (graph replay or fused launches included when the tuner picks them)."""
    refs = np.array([ref[e] for e in el])
    sim = ridg.Simulation(lib_problem(d, wl.n, wl.M, wl.velocity))
    for comp in (0, 1):
        for mfma in (0, 1):
            print(f"[gpu] {wl.name} composite={comp} mfma={mfma}", flush=True)
            sim.set_option(ridg.OPT_COMPOSITE, comp)
            sim.set_option(ridg.OPT_MFMA, mfma)
            sim.set_state(wl.q0)
            sim.step(steps, wl.dt)
            got = sim.get_state()[el]
            assert rel_l2(got, refs) <= TOL, (comp, mfma)
            assert max_elem_rel(got, refs) <= 1e-11, (comp, mfma)
    sim.set_state(wl.q0)
    sim.autotune(wl.dt, steps=4)
    sim.step(steps, wl.dt)
    got = sim.get_state()
    sim.close()
    assert rel_l2(got[el], refs) <= TOL
    assert max_elem_rel(got[el], refs) <= 1e-11


def test_advection_3d_full_size_sampled():
    wl = I.advection_3d()
    prob = oracle_problem(3, wl.n, wl.M, wl.velocity)
    rng = np.random.default_rng(5)
    el = _sample(prob, rng, 6, [0, prob.n_el - 1])
    ref = S.step_sampled(prob, wl.q0, wl.dt, el, n_steps=2)
    _const_full_size(3, wl, el, ref, 2)


def test_advection_2d_full_size_sampled():
    wl = I.advection_2d()
    prob = oracle_problem(2, wl.n, wl.M, wl.velocity)
    rng = np.random.default_rng(6)
    el = _sample(prob, rng, 24, [0, prob.n_el - 1])
    ref = S.step_sampled(prob, wl.q0, wl.dt, el, n_steps=2)
    _const_full_size(2, wl, el, ref, 2)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("name", ["rotation64_m4_20steps", "adv3d12_m3_20steps", "adv2d32_m3_100steps"])
def test_full_step_counts_against_stored_oracle(name):
    """Reduced meshes of the benchmark workloads run for their configurations' full step counts
    (20, 20 and 100) against oracle results stored by tests/golden/make_refs.py: every element,
    in the default configuration, the autotuned timed path, and the other kernel variants."""
    z = np.load(os.path.join(GOLDEN, name + ".npz"))
    d, n, M = int(z["d"]), tuple(int(x) for x in z["n"]), int(z["M"])
    vel = (str(z["velocity_kind"]), tuple(float(x) for x in z["velocity"]))
    q0, ref, dt, steps = z["q0"], z["ref"], float(z["dt"]), int(z["steps"])
    variants = [[], ["tune"]]
    if vel[0] == "rotation":
        variants += [[(ridg.OPT_PLAN_LAYOUT, 4)], [(ridg.OPT_PLAN_LAYOUT, 5)], [(ridg.OPT_PLAN_LAYOUT, 0)]]
    else:
        variants += [[(ridg.OPT_COMPOSITE, 1)], [(ridg.OPT_MFMA, 1)], [(ridg.OPT_GRAPH, 1)]]
        if d == 2 and all(x % 16 == 0 for x in n):
            variants.append([(ridg.OPT_COMPOSITE, 3)])  # four steps per launch
    for opts in variants:
        print(f"[gpu] {name} {opts}", flush=True)
        sim = ridg.Simulation(lib_problem(d, n, M, vel))
        sim.set_state(q0)
        for o in opts:
            if o == "tune":
                sim.autotune(dt, steps=4)
            else:
                sim.set_option(*o)
        sim.step(steps, dt)
        got = sim.get_state()
        sim.close()
        assert rel_l2(got, ref) <= TOL, opts
        assert max_elem_rel(got, ref) <= 1e-11, opts


def test_conservation_determinism_checkpoint():
    wl = I.rotation_2d(n=64, M=4)
    p = lib_problem(2, wl.n, wl.M, wl.velocity)
    sim = ridg.Simulation(p)
    sim.set_state(wl.q0)
    sim.step(10, wl.dt)
    a = sim.get_state()
    sim.set_state(wl.q0)
    sim.step(5, wl.dt)
    mid = sim.get_state()
    sim.set_state(mid)
    sim.step(5, wl.dt)
    b = sim.get_state()
    sim.close()
    assert np.array_equal(a, b)  # bitwise: deterministic, and get/set is a lossless checkpoint
    assert abs(a[:, 0].sum() - wl.q0[:, 0].sum()) <= 1e-13 * np.abs(wl.q0[:, 0]).sum() + 1e-15


def test_error_paths():
    p = ridg.make_problem(2, (8, 8), 3, velocity=(1.0, 0.5))
    sim = ridg.Simulation(p)
    q = np.zeros((64, 6))
    q[3, 2] = np.nan
    with pytest.raises(ridg.RidgError) as ei:
        sim.set_state(q)
    assert ei.value.code == ridg.RIDG_E_NONFINITE
    with pytest.raises(ridg.RidgError) as ei:
        sim.set_state(np.zeros((63, 6)))
    assert ei.value.code == ridg.RIDG_E_INVAL
    sim.set_state(np.ones((64, 6)))
    assert sim.step(0, 0.01) == 0
    for bad_dt in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(ridg.RidgError):
            sim.step(1, bad_dt)
    with pytest.raises(ridg.RidgError):
        sim.step(-1, 0.01)
    assert sim.step(1, 1.0) == ridg.RIDG_W_UNSTABLE
    sim.close()


def test_unstable_warning_is_the_von_neumann_limit():
    """ridg_step warns from the step's von Neumann amplification (2D order 4, v = (1, 0.5): the limit
    lies between CFL 0.5 and 0.8), and keeps the CFL rule for the rotation field."""
    n = 16
    sim = ridg.Simulation(ridg.make_problem(2, (n, n), 4, velocity=(1.0, 0.5)))
    sim.set_state(I.random_state(2, (n, n), 4, seed=3))
    assert sim.step(1, 0.5 / n) == ridg.RIDG_OK
    assert 1.0 - 1e-12 <= sim.get_info().spectral_radius <= 1.0 + 1e-10
    assert sim.step(1, 0.8 / n) == ridg.RIDG_W_UNSTABLE
    assert sim.get_info().spectral_radius > 1.0 + 1e-10
    sim.close()
    rot = ridg.Simulation(ridg.make_problem(2, (n, n), 3, flux=ridg.FLUX_ROTATION))
    rot.set_state(I.random_state(2, (n, n), 3, seed=4))
    assert rot.step(1, 1.0 / n) == ridg.RIDG_OK       # CFL 0.5 (max |v| = 1/2)
    assert rot.step(1, 2.5 / n) == ridg.RIDG_W_UNSTABLE  # CFL 1.25
    rot.close()


@pytest.mark.parametrize("refine,tol", [(0, 1e-5), (1, 1e-9), (2, 1e-12)])
def test_fp32_refine_rotation(refine, tol):
    """Reduced precision (FP32 block factorisations + FP64-residual refinement) against the FP64
    oracle: the stated bound per number of refinement sweeps."""
    n, M = 16, 4
    vel = ("rotation", (0.5, 0.5))
    prob = oracle_problem(2, (n, n), M, vel)
    q0 = I.random_state(2, (n, n), M, seed=21)
    dt = 1.0 / n
    ref = S.step(prob, q0, dt, 3)
    got = run_gpu(2, (n, n), M, vel, q0, dt, 3, ridg.SOLVER_REGION, precision=ridg.FP32_REFINE, refine=refine)
    err = rel_l2(got, ref)
    print(f"[fp32] refine={refine} rel-L2 {err:.3e}")
    assert err <= tol


def test_fp32_refine_constant_velocity_region():
    d, n, M, vel = 2, (12, 10), 3, ("const", (0.7, -0.4))
    prob = oracle_problem(d, n, M, vel)
    q0 = I.random_state(d, n, M, seed=22)
    dt = 0.45 * min(prob.h) / 0.7
    ref = S.step(prob, q0, dt, 3)
    got = run_gpu(d, n, M, vel, q0, dt, 3, ridg.SOLVER_REGION, precision=ridg.FP32_REFINE, refine=2)
    assert rel_l2(got, ref) <= 1e-12

"""The seeded input generators agree with the oracle's own projection (two independent
implementations of the element-average-orthonormal modal projection)."""

import numpy as np

from oracle.project import project
from paper_2101_01231_amd import inputs as I


def test_separable_projection_matches_oracle():
    wl = I.advection_2d(n=12, M=3)
    ks, A, B = wl.params["ks"], wl.params["A"], wl.params["B"]

    def f(X):
        out = sum(np.exp(-((X[0] - 0.5 - a) ** 2 + (X[1] - 0.5 - b) ** 2) / 0.01)
                  for a in (-1, 0, 1) for b in (-1, 0, 1))
        for (kx, ky), a, b in zip(ks, A, B):
            ph = 2 * np.pi * (kx * X[0] + ky * X[1])
            out = out + a * np.cos(ph) + b * np.sin(ph)
        return out

    np.testing.assert_allclose(wl.q0, project(f, 2, (12, 12), 3, q=12), atol=1e-12)


def test_rotation_and_3d_inputs_match_oracle():
    wl = I.rotation_2d(n=24, M=4)
    p = wl.params

    def g(X):
        out = 0.0
        for m in range(3):
            r = np.hypot(X[0] - p["cen"][m, 0], X[1] - p["cen"][m, 1]) / p["om"][m]
            out = out + p["a"][m] * I.bump(r)
        return out

    np.testing.assert_allclose(wl.q0, project(g, 2, (24, 24), 4, q=12), atol=1e-13)
    wl = I.advection_3d(n=6, M=2)
    p = wl.params

    def h(X):
        out = 0.0
        for m in range(5):
            s2 = 2 * p["sig"][m] ** 2
            prod = 1.0
            for i in range(3):
                prod = prod * sum(np.exp(-((X[i] - p["cen"][m, i] - k) ** 2) / s2) for k in (-1, 0, 1))
            out = out + prod
        return out

    np.testing.assert_allclose(wl.q0, project(h, 3, (6, 6, 6), 2, q=10), atol=1e-12)


def test_workload_seeds_are_deterministic():
    a = I.rotation_2d(n=16, M=2).q0
    b = I.rotation_2d(n=16, M=2).q0
    assert np.array_equal(a, b)
    r1 = I.serving_requests(20)
    r2 = I.serving_requests(20)
    assert r1 == r2
    assert all(0 < r["dt"] for r in r1)

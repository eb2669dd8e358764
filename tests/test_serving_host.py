"""Serving requests (host side, no GPU): the seeded Poisson mix and its admission sizes."""

from paper_2101_01231_amd import inputs, ridg, serve


def test_mix_is_seeded_and_admissible():
    specs = inputs.serving_requests(50)
    assert specs == inputs.serving_requests(50)
    reqs = serve.requests_from_mix(specs)
    assert all(b.arrival >= a.arrival for a, b in zip(reqs, reqs[1:]))
    for r in reqs[:10]:
        assert ridg.workspace_bytes(r.problem()) > 0
        assert 1 <= r.M <= 5 and r.d in (1, 2, 3)


def test_serving_kernel_policy():
    """Requests with theta_T >= 30 (2D order 5, 3D orders 4-5) are served on the matrix cores."""
    from paper_2101_01231_amd import serve
    mk = lambda d, M: serve.Request(0, 0.0, d, (8,) * d, M, 1, (1.0,) * d, 0.01, 0)
    assert [mk(2, M).theta_t for M in (3, 4, 5)] == [10, 20, 35]
    assert [mk(3, M).theta_t for M in (3, 4, 5)] == [15, 35, 70]
    big = [(d, M) for d in (1, 2, 3) for M in range(1, 6) if mk(d, M).theta_t >= serve.MFMA_MIN_THETA_T]
    assert big == [(2, 5), (3, 4), (3, 5)]

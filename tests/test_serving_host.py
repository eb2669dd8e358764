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

"""Host-side parts of the serving loop: the request generator."""
import numpy as np

from paper_2012_05348_amd import serve


def test_random_walk_steps_are_bounded():
    rng = np.random.default_rng(3)
    req = serve.make_requests(20, np.inf, 4, rng, batch_max=64)
    for r in range(len(req)):
        P = req.poses[req.first[r]:req.first[r] + req.count[r]].astype(np.float64)
        for a, b in zip(P[:-1], P[1:]):
            rel = a[:, :3].T @ b[:, :3]
            ang = np.arccos(np.clip((np.trace(rel) - 1) / 2, -1, 1))
            assert ang <= 0.05 + 1e-5
            assert np.linalg.norm(b[:, 3] - a[:, 3]) <= 0.02 + 1e-6


def test_requests_follow_the_stated_distributions():
    rng = np.random.default_rng(4)
    req = serve.make_requests(3000, 500.0, 32, rng)
    assert req.count.min() >= 1 and req.count.max() <= 4096
    assert abs((req.kind == serve.COLLIDE).mean() - 0.7) < 0.03
    assert set(np.unique(req.obstacle)) == set(range(32))
    gaps = np.diff(req.arrival)
    assert abs(gaps.mean() * 500.0 - 1.0) < 0.08          # Poisson arrivals at 500/s
    assert abs(np.median(np.log(req.count)) - np.log(4097) / 2) < 0.25  # log-uniform sizes
    assert np.array_equal(req.first[1:], np.cumsum(req.count)[:-1])

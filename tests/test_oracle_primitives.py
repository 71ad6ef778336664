"""Pins of the oracle's triangle-level geometry against things other than itself.

- intersection: three independent formulations must agree (separating axes,
  edge-pierces-triangle, intervals on the planes' intersection line), plus
  hand-built touching / coplanar / disjoint cases;
- distance: closed forms (tests/golden/closed_forms.txt) and a numerical QP
  (scipy SLSQP over barycentric coordinates) on random pairs;
- penetration depth: a hand-built piercing pair with a known answer.
"""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle

A0 = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], dtype=np.float64)


def _rand_tri(rng, scale=1.0):
    return rng.normal(size=(3, 3)) * scale


def _random_pairs(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        a = _rand_tri(rng)
        b = _rand_tri(rng) * rng.uniform(0.3, 1.5) + rng.normal(size=3) * rng.uniform(0.0, 1.5)
        out.append((a, b))
    return out


def test_three_formulations_agree_random():
    pairs = _random_pairs(4000, 1)
    res = np.array([[oracle.tt_sat(a, b), oracle.tt_segtri(a, b), oracle.tt_interval(a, b)] for a, b in pairs])
    assert (res[:, 0] == res[:, 1]).all()
    assert (res[:, 0] == res[:, 2]).all()
    # the sample exercises both outcomes
    assert 0.1 < res[:, 0].mean() < 0.9


def test_three_formulations_agree_coplanar():
    rng = np.random.default_rng(2)
    n_hit = 0
    for _ in range(1500):
        a = rng.normal(size=(3, 3)); a[:, 2] = 0.0
        b = rng.normal(size=(3, 3)) * 0.7 + np.r_[rng.normal(size=2), 0.0]; b[:, 2] = 0.0
        r = (oracle.tt_sat(a, b), oracle.tt_segtri(a, b), oracle.tt_interval(a, b))
        assert r[0] == r[1] == r[2], (a, b, r)
        n_hit += r[0]
    assert 100 < n_hit < 1400


@pytest.mark.parametrize(
    "b, expect",
    [
        (A0 + [0, 0, 0.1], False),                                        # parallel, apart
        (np.array([[0.2, 0.2, -0.5], [0.2, 0.2, 0.5], [0.3, 0.5, 0.5]]), True),   # pierces interior
        (np.array([[1, 0, 0], [2, 0, 1], [2, 1, -1]]), True),              # shares a vertex: touching
        (np.array([[0.5, 0.5, 0], [1, 1, 1], [1, 1, -1]]), True),          # vertex on A's edge
        (np.array([[0.6, 0.6, -1], [0.6, 0.6, 1], [2, 2, 0]]), False),     # passes outside the hypotenuse
        (np.array([[0.25, 0.25, 0], [0.5, 0.25, 0], [0.25, 0.5, 0]]), True),  # coplanar, inside
        (np.array([[2, 2, 0], [3, 2, 0], [2, 3, 0]]), False),              # coplanar, outside
    ],
)
def test_hand_built_cases(b, expect):
    b = np.asarray(b, dtype=np.float64)
    for f in (oracle.tt_sat, oracle.tt_segtri, oracle.tt_interval):
        assert f(A0, b) == expect, f.__name__
        assert f(b, A0) == expect, f.__name__


def _golden():
    import os
    rows = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                name, val, _ = [s.strip() for s in line.split("|")]
                rows[name] = val
    return rows


@pytest.mark.parametrize("h", [1e-4, 0.01, 0.3, 2.0])
def test_distance_closed_forms(h):
    g = _golden()
    assert g["tri_parallel_h"] == "h"
    assert oracle.tt_dist(A0, A0 + [0, 0, h]) == pytest.approx(h, rel=1e-12)
    b = np.array([[0.2, 0.2, h], [0.2, 0.3, h + 1], [0.3, 0.2, h + 1]])
    assert oracle.tt_dist(A0, b) == pytest.approx(h, rel=1e-12)
    a2 = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0]], dtype=np.float64)
    b2 = np.array([[0, -1, h], [0, 1, h], [0, 0, h + 1]], dtype=np.float64)
    assert oracle.tt_dist(a2, b2) == pytest.approx(h, rel=1e-12)
    assert oracle.tt_dist(b2, a2) == pytest.approx(h, rel=1e-12)


def _qp_dist(a, b):
    """min |sum l_i a_i - sum m_j b_j| over two probability simplices (SLSQP)."""
    def f(x):
        d = x[:3] @ a - x[3:] @ b
        return d @ d

    def grad(x):
        d = x[:3] @ a - x[3:] @ b
        return np.concatenate([2 * a @ d, -2 * b @ d])

    best = np.inf
    for x0 in (np.full(6, 1 / 3), np.r_[1, 0, 0, 1, 0, 0], np.r_[0, 1, 0, 0, 0, 1], np.r_[0, 0, 1, 0, 1, 0]):
        r = minimize(f, x0.astype(float), jac=grad, method="SLSQP", bounds=[(0, 1)] * 6,
                     constraints=[{"type": "eq", "fun": lambda x: x[:3].sum() - 1},
                                  {"type": "eq", "fun": lambda x: x[3:].sum() - 1}],
                     options={"ftol": 1e-16, "maxiter": 500})
        best = min(best, np.sqrt(max(r.fun, 0.0)))
    return best


def test_distance_matches_qp_random():
    pairs = _random_pairs(300, 3)
    n = 0
    for a, b in pairs:
        d = oracle.tt_dist(a, b)
        q = _qp_dist(a, b)
        if oracle.tt_sat(a, b):
            assert d == 0.0
            assert q < 1e-6
        else:
            n += 1
            assert d == pytest.approx(q, rel=1e-6, abs=1e-9)
    assert n > 50


def test_point_triangle_and_segments_match_qp():
    rng = np.random.default_rng(4)
    for _ in range(200):
        t = rng.normal(size=(3, 3))
        p = rng.normal(size=3) * 2
        # point-triangle as a QP over the simplex
        r = minimize(lambda l: np.sum((l @ t - p) ** 2), np.full(3, 1 / 3), method="SLSQP", bounds=[(0, 1)] * 3,
                     constraints=[{"type": "eq", "fun": lambda l: l.sum() - 1}], options={"ftol": 1e-16})
        assert oracle.pt_tri_dist(p, t) == pytest.approx(np.sqrt(r.fun), rel=1e-6, abs=1e-9)
        s = rng.normal(size=(4, 3))
        g = np.linspace(0, 1, 401)
        P = s[0] + g[:, None] * (s[1] - s[0])
        Q = s[2] + g[:, None] * (s[3] - s[2])
        brute = np.sqrt(((P[:, None, :] - Q[None, :, :]) ** 2).sum(-1)).min()
        d = oracle.seg_seg_dist(*s)
        assert d <= brute + 1e-12
        assert d >= brute - 0.01 * np.linalg.norm(s[1] - s[0]) - 0.01 * np.linalg.norm(s[3] - s[2])


def test_parallel_segments():
    # parallel segments offset by 0.5 in y, overlapping in x: distance 0.5
    assert oracle.seg_seg_dist([0, 0, 0], [2, 0, 0], [1, 0.5, 0], [3, 0.5, 0]) == pytest.approx(0.5)
    # parallel, not overlapping in x: distance between closest endpoints
    assert oracle.seg_seg_dist([0, 0, 0], [1, 0, 0], [2, 1, 0], [3, 1, 0]) == pytest.approx(np.sqrt(2))


def test_penetration_depth_hand_built():
    a = np.array([[-10, -10, 0], [10, -10, 0], [0, 10, 0]], dtype=np.float64)
    b = np.array([[0, 0, -0.3], [0.1, 0, 0.5], [-0.1, 0.05, 0.5]], dtype=np.float64)
    assert oracle.tt_sat(a, b)
    assert oracle.tt_pd(a, b) == pytest.approx(0.3, rel=1e-12)
    assert oracle.tt_signed(a, b) == pytest.approx(-0.3, rel=1e-12)
    b2 = b + [0, 0, 0.31]
    assert not oracle.tt_sat(a, b2)
    assert oracle.tt_signed(a, b2) == pytest.approx(0.01, rel=1e-9)


def test_pd_bounded_by_any_axis_overlap():
    # PD is a minimum over axes: never above the overlap along the z axis for a pair crossing z=0
    rng = np.random.default_rng(5)
    for _ in range(300):
        a = rng.normal(size=(3, 3)); a[:, 2] = 0
        b = rng.normal(size=(3, 3)) * 0.5
        if oracle.tt_sat(a, b):
            oz = min(b[:, 2].max(), -b[:, 2].min())
            assert oracle.tt_pd(a, b) <= oz + 1e-12

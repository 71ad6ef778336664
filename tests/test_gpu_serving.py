"""GPU tests of the continuous-batching serving loop: every request's result
is the same alone and in the mix (booleans exactly, distances bitwise)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2012_05348_amd as cb  # noqa: E402
from paper_2012_05348_amd import serve  # noqa: E402
from synth import configs  # noqa: E402

DEV = "cuda:0"
SMALL = configs.BatchedWorkload(index=4, n_obstacles=6, tri_max=20000, min_poses=0)


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def server():
    w = SMALL
    kw = dict(bv=cb.DOP18, branching=w.branching, leaf_size=w.leaf_size, bits=w.bits)
    link = cb.Model.build(*w.link_mesh(), **kw).to(DEV)
    obs = [cb.Model.build(*w.obstacle_mesh(i), **kw).to(DEV) for i in range(w.n_obstacles)]
    # small launches so that requests really mix across several launches and slots
    srv = serve.Server(link, cb.Obstacles(obs, DEV), DEV, slots_per_kind=2, max_poses=600)
    return link, obs, srv


def _alone(link, obs, req, r):
    P = torch.from_numpy(req.poses[req.first[r]:req.first[r] + req.count[r]]).to(DEV)
    m = obs[int(req.obstacle[r])]
    if req.kind[r] == serve.COLLIDE:
        h, st = cb.collide(link, m, P)
        return h.cpu().numpy(), st.cpu().numpy()
    d, st = cb.distance(link, m, P)
    return d.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("realtime", [False, True])
def test_results_are_the_same_alone_and_in_the_mix(server, realtime):
    link, obs, srv = server
    rng = np.random.default_rng(11 + realtime)
    # up to 500 poses: some requests are too large for the small-request slot
    req = serve.make_requests(90, 3000.0 if realtime else np.inf, len(obs), rng, batch_max=500)
    res = srv.run(req, realtime=realtime)
    _log(f"serving realtime={realtime}: {res['launches']} launches, largest {res['largest_launch']}, "
         f"p50 {res['p50_ms']:.2f} ms p99 {res['p99_ms']:.2f} ms, {res['poses_per_sec']:.0f} poses/s")
    assert (res["status"] == 0).all()
    assert np.isfinite(res["latency_s"]).all() and (res["latency_s"] >= 0).all()
    assert res["launches"] >= 4
    for r in range(len(req)):
        sl = slice(req.first[r], req.first[r] + req.count[r])
        got = res["hit"][sl] if req.kind[r] == serve.COLLIDE else res["dist"][sl]
        ref, st = _alone(link, obs, req, r)
        assert (st == 0).all()
        if req.kind[r] == serve.COLLIDE:
            assert np.array_equal(got, ref), r
        else:
            assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), r
    assert (req.kind == serve.COLLIDE).any() and (req.kind == serve.DISTANCE).any()


def test_a_request_larger_than_a_launch_is_rejected(server):
    _, obs, srv = server
    req = serve.make_requests(3, np.inf, len(obs), np.random.default_rng(3), batch_min=700, batch_max=800)
    with pytest.raises(ValueError):
        srv.run(req, realtime=False)

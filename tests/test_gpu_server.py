"""Serving layer on the GPU: every robot's results through the server (queued,
admitted by budget and slots, batched with other robots on several streams)
are bit-identical to the same robot stepped alone through the plain path, in
submission order; the first served step matches the oracle."""
import numpy as np
import pytest

import oracle
from conftest import f32_params
from paper_2504_06437_amd import workloads as W

pytestmark = pytest.mark.gpu


def _robots(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    wls = []
    for i in range(n):
        wl = W.mixed_controller(rng, 500 + i, K=int(round(2 ** rng.uniform(6, 10))), T=int(rng.integers(5, 30)),
                                J=int(rng.integers(0, 60)))
        wls.append(wl)
    return wls


def _requests(wls, steps, seed):
    """Per robot: `steps` start states near its start and their references."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for wl in wls:
        reqs = []
        for _ in range(steps):
            x = wl["x0"].copy()
            x[:2] += rng.uniform(-0.3, 0.3, size=2).astype(np.float32)
            reqs.append((x, W.reference(wl, x)))
        out.append(reqs)
    return out


def _alone(wl):
    from paper_2504_06437_amd.controller import Controller
    c = Controller(wl["params"])
    c.set_obstacles(wl["obstacles"])
    return c


def _scratch_bound(p):
    """Upper bound of one request's scratch bytes (tiles of the smallest
    size; no exported noise)."""
    K, T = p["K"], p["T"]
    Kp = (K + 63) // 64 * 64
    tiles = (K + 15) // 16
    a = lambda b: (b + 255) // 256 * 256  # noqa: E731
    return a(0) + a(8 * Kp) + a(4 * Kp) + 3 * a(8 * tiles) + a(4 * tiles) + a(16 * T * tiles)


def _serve_and_compare(wls, reqs, **server_kw):
    from paper_2504_06437_amd.controller import Server
    srv = Server(**server_kw)
    ids = [srv.add_robot(wl["params"], wl["obstacles"]) for wl in wls]
    steps = len(reqs[0])
    tickets = [[] for _ in wls]
    for s in range(steps):                        # interleaved: every robot's queue holds several requests
        for i in range(len(wls)):
            x, ref = reqs[i][s]
            tickets[i].append(srv.submit(ids[i], x, ref))
    served = [[srv.wait(t) for t in tk] for tk in tickets]
    for i, wl in enumerate(wls):
        a = _alone(wl)
        for s in range(steps):
            x, ref = reqs[i][s]
            a.set_reference(ref)
            u = a.step(x)
            u_srv, lat, st = served[i][s]
            assert st == 0 and lat >= 0.0
            np.testing.assert_array_equal(u, u_srv, err_msg=f"robot {i} step {s}")
        U, counter = srv.robot_state(ids[i])
        np.testing.assert_array_equal(U, a.controls())
        assert counter == a.get_state()["counter"]
        a.close()
    stats = srv.stats()
    srv.close()
    n = len(wls) * steps
    assert stats["submitted"] == n and stats["completed"] == n
    assert 1 <= stats["launches"] <= n
    return stats


def test_server_equals_alone_in_fifo_order():
    wls = _robots(8, seed=31)
    stats = _serve_and_compare(wls, _requests(wls, 3, seed=32), budget_bytes=64 << 20, streams=2, max_batch=8)
    assert stats["deferred_budget"] == 0
    assert stats["mean_batch"] >= 1.0


def test_small_budget_defers_and_serves_identically():
    wls = _robots(6, seed=41)
    budget = max(_scratch_bound(wl["params"]) for wl in wls) + 4096
    stats = _serve_and_compare(wls, _requests(wls, 3, seed=42), budget_bytes=budget, streams=3, max_batch=6)
    assert stats["deferred_budget"] > 0
    assert stats["peak_bytes_in_flight"] <= budget


def test_one_slot_one_stream_serialises():
    wls = _robots(3, seed=51)
    stats = _serve_and_compare(wls, _requests(wls, 2, seed=52), budget_bytes=64 << 20, streams=1, max_slots=1,
                               max_batch=1)
    assert stats["launches"] == 6 and stats["mean_batch"] == 1.0


def test_served_step_matches_oracle():
    from paper_2504_06437_amd.controller import Server
    wl = W.quad_small(K=512)
    srv = Server(budget_bytes=32 << 20)
    rid = srv.add_robot(wl["params"], wl["obstacles"])
    u0, _, st = srv.wait(srv.submit(rid, wl["x0"], wl["x_ref"]))
    assert st == 0
    U, counter = srv.robot_state(rid)
    srv.close()
    p = f32_params(wl["params"])
    ref = oracle.step(p, oracle.World.from_workload(wl), wl["x0"], np.zeros((p["T"], 2)), wl["x_ref"], 1.0, 0)
    scale = np.asarray(p["sigma"])
    assert np.all(np.abs(u0 - ref["u0"]) <= 1e-4 * (np.abs(ref["u0"]) + scale))
    assert np.all(np.abs(U - ref["Unext"]) <= 1e-4 * (np.abs(ref["Unext"]) + scale))
    assert counter == 1


def test_server_rejects_bad_requests():
    from paper_2504_06437_amd import _lib as A
    from paper_2504_06437_amd.controller import Server
    wl = W.quad_small(K=256)
    srv = Server(budget_bytes=1 << 12)                    # too small for this robot's scratch
    with pytest.raises(A.MppiError):
        srv.add_robot(wl["params"], wl["obstacles"])
    srv.close()
    srv = Server(budget_bytes=32 << 20)
    rid = srv.add_robot(wl["params"], wl["obstacles"])
    with pytest.raises(A.MppiError):
        srv.submit(rid + 1, wl["x0"])
    bad = wl["x0"].copy()
    bad[0] = np.nan
    with pytest.raises(A.MppiError):
        srv.submit(rid, bad)
    with pytest.raises(A.MppiError):
        srv.poll(12345)
    t = srv.submit(rid, wl["x0"], wl["x_ref"])
    assert srv.wait(t)[2] == 0
    srv.close()

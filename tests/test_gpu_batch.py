"""Batched persistent launch: each controller's result is the same alone and
in the mixed batch (bit-exact: a controller's tile shape depends only on its
own shape), and matches the oracle."""
import numpy as np
import pytest

import oracle
from conftest import f32_params
from paper_2504_06437_amd import workloads as W

pytestmark = pytest.mark.gpu


def _mix(n=10, seed=21):
    rng = np.random.Generator(np.random.PCG64(seed))
    wls = []
    for i in range(n):
        wl = W.mixed_controller(rng, 100 + i, K=int(round(2 ** rng.uniform(6, 10))), T=int(rng.integers(5, 30)),
                                J=int(rng.integers(0, 60)))
        wl["U0"] = W.random_controls(rng, wl["params"]["T"], 0.2)
        wls.append(wl)
    return wls


def _make(wl):
    from paper_2504_06437_amd.controller import Controller
    c = Controller(wl["params"])
    c.load_workload(wl)
    return c


def test_batch_equals_alone_and_oracle():
    from paper_2504_06437_amd.controller import Batch
    wls = _mix()
    alone = [_make(wl) for wl in wls]
    mixed = [_make(wl) for wl in wls]
    batch = Batch(mixed)
    for step in range(3):
        states = [c.get_state() for c in mixed]
        x0s = [wl["x0"] for wl in wls]
        u_b, sts = batch.step(x0s)
        assert np.all(sts == 0)
        for i, (a, m, wl) in enumerate(zip(alone, mixed, wls)):
            u_a = a.step(wl["x0"])
            np.testing.assert_array_equal(u_a, u_b[i])
            np.testing.assert_array_equal(a.controls(), m.controls())
            np.testing.assert_array_equal(a.costs(), m.costs())
            if step == 0:
                p = f32_params(wl["params"])
                ref = oracle.step(p, oracle.World.from_workload(wl), wl["x0"], states[i]["U"], wl["x_ref"], 1.0,
                                  states[i]["counter"])
                S = m.costs()
                # cost bound of test_gpu_parity: relative 1e-4 plus the barrier's conditioning
                bound = 1e-4 * np.maximum(np.abs(ref["S"]), 1.0) + 1e-5 * ref["sens"]
                assert np.all(np.abs(S - ref["S"]) <= bound)
                scale = np.asarray(p["sigma"])
                assert np.all(np.abs(m.last_optimal() - ref["Ustar"]) <= 1e-4 * (np.abs(ref["Ustar"]) + scale))
    batch.close()
    for c in alone + mixed:
        c.close()


def test_batch_replays_follow_obstacle_changes():
    """Changing a controller's obstacles between graph replays rebuilds the
    batch; results still equal the standalone controller's."""
    from paper_2504_06437_amd.controller import Batch
    wls = _mix(4, seed=5)
    alone = [_make(wl) for wl in wls]
    mixed = [_make(wl) for wl in wls]
    batch = Batch(mixed)
    batch.step([wl["x0"] for wl in wls])
    for a, wl in zip(alone, wls):
        a.step(wl["x0"])
    new_obs = np.array([[1.0, 1.5, 0.3], [2.0, 2.5, 0.4], [3.0, 1.0, 0.5]], dtype=np.float32)
    alone[1].set_obstacles(new_obs)
    mixed[1].set_obstacles(new_obs)
    u_b, _ = batch.step([wl["x0"] for wl in wls])
    for i, (a, wl) in enumerate(zip(alone, wls)):
        np.testing.assert_array_equal(a.step(wl["x0"]), u_b[i])
    batch.close()
    for c in alone + mixed:
        c.close()


@pytest.mark.parametrize("models", [("quad6", "quad5", "car"), ("quad5",), ("car", "car")])
def test_batch_groups_by_model(models):
    """The batched rollout runs one persistent launch per kernel group present
    (model, and for the layout-form tiles the tile size), each with its own
    queue; every controller still equals its standalone run, on
    replays too (each launch's queue is reset by its last workgroup), and a
    shape point count other than the model's default takes the runtime-P tile."""
    from paper_2504_06437_amd.controller import Batch
    rng = np.random.Generator(np.random.PCG64(33))
    wls = []
    for i, m in enumerate(models):
        wl = W.mixed_controller(rng, 300 + i, K=int(rng.integers(100, 900)), T=int(rng.integers(6, 25)),
                                J=int(rng.integers(1, 50)), model=m)
        wl["U0"] = W.random_controls(rng, wl["params"]["T"], 0.2)
        wls.append(wl)
    if models == ("car", "car"):
        shape = np.float32([[-1.0, 0.0], [0.0, 0.0], [1.0, 0.0]])
        wls[1]["params"]["shape"] = shape.tolist()
    alone = [_make(wl) for wl in wls]
    mixed = [_make(wl) for wl in wls]
    batch = Batch(mixed)
    for _ in range(3):
        u_b, sts = batch.step([wl["x0"] for wl in wls])
        assert np.all(sts == 0)
        for i, (a, m, wl) in enumerate(zip(alone, mixed, wls)):
            np.testing.assert_array_equal(a.step(wl["x0"]), u_b[i])
            np.testing.assert_array_equal(a.costs(), m.costs())
    batch.close()
    for c in alone + mixed:
        c.close()


def test_batch_kernels_by_tile_shape():
    """Layout-form tiles without a costmap run in one batched kernel per
    model and tile size, every other tile (a costmap, a runtime-P body) in
    the model's general batched kernel: a batch holding each kind, at tile
    sizes 64, 128, 256 and the tuned ones, equals each controller stepped
    alone."""
    from paper_2504_06437_amd.controller import Batch
    rng = np.random.Generator(np.random.PCG64(41))
    wls = [W.quad_large(K=700, T=12, J=40, cells=64),
           W.mixed_controller(rng, 501, K=900, T=14, J=30, model="quad6"),
           W.mixed_controller(rng, 502, K=400, T=9, J=25, model="car"),
           W.mixed_controller(rng, 503, K=600, T=11, J=33, model="quad6"),
           W.mixed_controller(rng, 504, K=700, T=10, J=28, model="car"),
           W.mixed_controller(rng, 505, K=900, T=13, J=36, model="quad6")]
    wls[3]["params"] = dict(wls[3]["params"], tile_samples=64)
    wls[4]["params"] = dict(wls[4]["params"], tile_samples=128)
    wls[5]["params"] = dict(wls[5]["params"], tile_samples=256)
    wls[2]["params"] = dict(wls[2]["params"], shape=[[-1.0, 0.0], [0.0, 0.0], [1.0, 0.0]])
    alone = [_make(wl) for wl in wls]
    mixed = [_make(wl) for wl in wls]
    batch = Batch(mixed)
    for _ in range(2):
        u_b, sts = batch.step([wl["x0"] for wl in wls])
        assert np.all(sts == 0)
        for i, (a, m, wl) in enumerate(zip(alone, mixed, wls)):
            np.testing.assert_array_equal(a.step(wl["x0"]), u_b[i])
            np.testing.assert_array_equal(a.costs(), m.costs())
    batch.close()
    for c in alone + mixed:
        c.close()


def test_batch_at_full_mixed_sizes_matches_oracle():
    """Controllers of the mixed batch's largest sizes -- both models, K up to
    8192, T up to 80, J up to 400 -- among them 256-sample tiles whose noise
    does not fit in LDS and is drawn again in the batched kernel's epilogue:
    each equals its standalone run bit for bit, on two steps, and matches the
    oracle's iteration at the first (threaded oracle)."""
    from paper_2504_06437_amd.controller import Batch
    rng = np.random.Generator(np.random.PCG64(61))
    shapes = [("quad6", 8192, 80, 400, 256), ("car", 8192, 80, 400, 0), ("car", 6000, 64, 250, 256),
              ("quad6", 3000, 45, 180, 0), ("car", 700, 20, 10, 0), ("quad6", 8100, 77, 399, 128)]
    wls = []
    for i, (m, K, T, J, S) in enumerate(shapes):
        wl = W.mixed_controller(rng, 700 + i, K=K, T=T, J=J, model=m)
        wl["U0"] = W.random_controls(rng, T, 0.2)
        wl["params"]["tile_samples"] = S
        wls.append(wl)
    alone = [_make(wl) for wl in wls]
    mixed = [_make(wl) for wl in wls]
    batch = Batch(mixed)
    redrawn = 0
    for step in range(2):
        states = [c.get_state() for c in mixed]
        u_b, sts = batch.step([wl["x0"] for wl in wls])
        assert np.all(sts == 0)
        for i, (a, m, wl) in enumerate(zip(alone, mixed, wls)):
            np.testing.assert_array_equal(a.step(wl["x0"]), u_b[i])
            np.testing.assert_array_equal(a.costs(), m.costs())
            np.testing.assert_array_equal(a.controls(), m.controls())
            if step == 0:
                p = f32_params(wl["params"])
                ref = oracle.step(p, oracle.World.from_workload(wl), wl["x0"], states[i]["U"], wl["x_ref"], 1.0,
                                  states[i]["counter"])
                assert ref["status"] == 0
                S = m.costs()
                bound = 1e-4 * np.maximum(np.abs(ref["S"]), 1.0) + 1e-5 * ref["sens"]
                assert np.all(np.abs(S - ref["S"]) <= bound), f"controller {i}"
                scale = np.asarray(p["sigma"])
                for key, got in (("Ustar", m.last_optimal()), ("Unext", m.controls())):
                    assert np.all(np.abs(got - ref[key]) <= 1e-4 * (np.abs(ref[key]) + scale)), f"{key} {i}"
                np.testing.assert_allclose(m.weights(), ref["w"], rtol=0, atol=1e-4 * ref["w"].max())
                info = m.info()
                redrawn += int(info["noise_kept"] == 0)
    assert redrawn >= 2
    batch.close()
    for c in alone + mixed:
        c.close()

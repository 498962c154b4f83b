"""The seeded synthetic inputs follow the recipe the design states: sizes,
value ranges, clear start and goal, determinism per seed, and a reference
that runs from the projection of the state towards the goal at v_set."""
import math

import numpy as np

from paper_2504_06437_amd import workloads as W


def _clearance(obs, pt):
    return min(math.hypot(c[0] - pt[0], c[1] - pt[1]) - c[2] for c in obs)


def test_named_workload_sizes_and_ranges():
    for wl, model, K, T, J, lo, hi, rlo, rhi in (
            (W.quad_small(), "quad6", 256, 20, 10, 0.0, 10.0, 0.3, 0.8),
            (W.car(), "car", 4096, 50, 100, 0.0, 20.0, 0.2, 1.0),
            (W.quad_large(), "quad6", 16384, 100, 400, 0.0, 40.0, 0.3, 0.8)):
        p = wl["params"]
        assert (p["model"], p["K"], p["T"]) == (model, K, T)
        obs = np.asarray(wl["obstacles"])
        assert obs.shape == (J, 3) and obs.dtype == np.float32
        assert np.all(obs[:, :2] >= lo) and np.all(obs[:, :2] <= hi)
        assert np.all(obs[:, 2] >= rlo) and np.all(obs[:, 2] <= rhi)
        clear = W.BODY_RADIUS[model] + 0.5
        assert _clearance(obs, wl["start"]) > clear - 1e-5 and _clearance(obs, wl["goal"]) > clear - 1e-5
        assert wl["x_ref"].shape == (T + 1, W.MODEL_DIMS[model])
        assert np.all(wl["U0"] == 0.0)
    m = W.quad_large()["map"]
    assert m["sdf"].shape == (512, 512) and m["sdf"].dtype == np.float32 and abs(m["res"] - 40.0 / 512) < 1e-12
    assert W.quad_large()["params"]["normaliser"] == "on"


def test_workloads_are_deterministic_per_seed():
    a, b = W.car(seed=1), W.car(seed=1)
    np.testing.assert_array_equal(a["obstacles"], b["obstacles"])
    c = W.car(seed=2)
    assert not np.array_equal(a["obstacles"], c["obstacles"])
    ba, bb = W.batch(8, 3), W.batch(8, 3)
    for x, y in zip(ba, bb):
        assert x["params"] == y["params"]
        np.testing.assert_array_equal(x["obstacles"], y["obstacles"])


def test_mixed_batch_recipe():
    wls = W.batch(64, 3)
    Ks = np.array([wl["params"]["K"] for wl in wls])
    Ts = np.array([wl["params"]["T"] for wl in wls])
    Js = np.array([len(wl["obstacles"]) for wl in wls])
    models = {wl["params"]["model"] for wl in wls}
    assert models == {"quad6", "car"}
    assert Ks.min() >= 256 and Ks.max() <= 8192
    assert Ts.min() >= 20 and Ts.max() <= 80
    assert Js.min() >= 10 and Js.max() <= 400
    assert len({wl["params"]["seed"] for wl in wls}) == 64


def test_blob_costmap_is_a_signed_distance():
    """Cells inside a blob are negative, and the field changes by at most one
    cell size between neighbouring cells (a distance function is 1-Lipschitz)."""
    rng = np.random.Generator(np.random.PCG64(11))
    sdf, res = W.blob_sdf(rng, 8, 10.0, 128)
    assert sdf.min() < 0.0 < sdf.max()
    assert np.max(np.abs(np.diff(sdf, axis=0))) <= res * (1 + 1e-5)
    assert np.max(np.abs(np.diff(sdf, axis=1))) <= res * (1 + 1e-5)


def test_reference_starts_at_the_projection_and_moves_at_v_set():
    wl = W.car()
    p = wl["params"]
    x = wl["x0"].copy()
    x[:2] += np.float32([0.7, -0.7])          # off the line, on the normal through the start
    ref = W.reference(wl, x)
    np.testing.assert_allclose(ref[0, :2], wl["start"], atol=1e-5)
    step = np.linalg.norm(np.diff(ref[:, :2], axis=0), axis=1)
    np.testing.assert_allclose(step, wl["v_set"] * p["dt"], rtol=1e-5)
    assert np.all(ref[:, 3] == np.float32(wl["v_set"]))

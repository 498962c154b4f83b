"""The closed-loop mission harness (Sec. VI mission set-up, synthetic
layouts): the layouts carry the paper's mission settings; the collision test
agrees with the oracle's clearance (an independent FP64 implementation of
the same geometry); the path error has its closed form; the loop ends on the
goal or on a collision; and with the FP64 oracle as the controller a vehicle
mission at 8 m/s is completed without collision."""
import math

import numpy as np
import pytest

import oracle
from conftest import f32_params
from paper_2504_06437_amd import mission as M
from paper_2504_06437_amd import workloads as W


@pytest.mark.parametrize("mission", [1, 2, 3])
def test_layouts_carry_the_paper_settings(mission):
    for seed in range(5):
        wl = M.layout(mission, seed)
        p, m = wl["params"], M.MISSIONS[mission]
        assert p["model"] == m["model"] and wl["v_set"] == m["v_set"]
        assert (p["K"], p["T"], p["dt"], p["gamma_u"], p["explore_mu"]) == (1024, 20, 0.02, 2.0, 0.4)
        assert p["adaptive_explore"]
        np.testing.assert_allclose(np.square(p["sigma"]), m["var"], rtol=1e-12)
        obs = np.asarray(wl["obstacles"], dtype=np.float64)
        assert obs.shape == (m["J"], 3) and np.allclose(obs[:, 2], m["radius"])
        # the obstacles flank the path on alternate sides, edge clearance within the gap range
        off = obs[:, 1] - m["height"]
        assert np.all(np.sign(off[1:]) == -np.sign(off[:-1]))
        clear = np.abs(off) - m["radius"] - m["half_width"]
        assert np.all(clear >= m["gap"][0] - 1e-5) and np.all(clear <= m["gap"][1] + 1e-5)
        # a body on the path, aligned with it, touches nothing anywhere along it
        for s in np.linspace(0.0, m["length"], 241):
            x = np.zeros(W.MODEL_DIMS[m["model"]], dtype=np.float64)
            x[0], x[1] = s, m["height"]
            assert not M.collides(p, obs, x)
    # layouts differ by seed and repeat for a seed
    a, b, c = M.layout(2, 0), M.layout(2, 0), M.layout(2, 1)
    np.testing.assert_array_equal(a["obstacles"], b["obstacles"])
    assert not np.array_equal(a["obstacles"], c["obstacles"])


def test_collision_agrees_with_the_oracle_clearance():
    rng = np.random.Generator(np.random.PCG64(3))
    for mission in (1, 2):
        wl = M.layout(mission, 0)
        p = wl["params"]
        pf = f32_params(p)
        world = oracle.World.from_workload(wl)
        obs = np.asarray(wl["obstacles"], dtype=np.float64)
        n = W.MODEL_DIMS[p["model"]]
        hits = 0
        for _ in range(400):
            j = rng.integers(len(obs))
            x = np.zeros(n)
            ang, rad = rng.uniform(0.0, 2 * math.pi), obs[j, 2] * rng.uniform(0.3, 1.8)
            x[0], x[1] = obs[j, 0] + rad * math.cos(ang), obs[j, 1] + rad * math.sin(ang)
            x[2] = rng.uniform(-math.pi, math.pi)
            col = M.collides(p, obs, x)
            assert col == (oracle.clearance(pf, world, x) <= 0.0)
            hits += col
        assert 50 < hits < 350


def test_path_error_closed_form():
    wl = M.layout(2, 0)
    L = M.MISSIONS[2]["length"]
    assert M.path_error(wl, [0.3 * L, 2.5]) == pytest.approx(2.5)
    assert M.path_error(wl, [0.7 * L, -1.0]) == pytest.approx(1.0)
    assert M.path_error(wl, [-3.0, 4.0]) == pytest.approx(5.0)         # before the start: to the end point
    assert M.path_error(wl, [L + 6.0, 8.0]) == pytest.approx(10.0)


class _Cruise:
    """Straight ahead at v_set: no steering, proportional acceleration."""

    def __init__(self, v):
        self.v = v

    def set_reference(self, ref):
        self.ref = ref

    def step(self, x):
        return np.float32([0.0, np.clip(2.0 * (self.v - x[3]), -2.0, 2.0)])


def test_loop_ends_on_goal_or_collision():
    wl = M.layout(2, 0)
    free = dict(wl, obstacles=np.zeros((0, 3), np.float32))
    r = M.run(_Cruise(5.0), free)
    assert r["success"] and r["reached"] and not r["collided"]
    assert r["error"] == pytest.approx(0.0, abs=1e-6)
    assert 3.0 < r["avg_speed"] < 5.0
    assert r["time"] == pytest.approx(r["steps"] * 0.02)
    # an obstacle on the path: the cruise hits it
    blocked = dict(wl, obstacles=np.float32([[60.0, 0.0, 4.3]]))
    r = M.run(_Cruise(5.0), blocked)
    assert r["collided"] and not r["success"]
    s = M.summarize([r, M.run(_Cruise(5.0), free)])
    assert s["runs"] == 2 and s["success_pct"] == 50.0 and s["collisions"] == 1 and s["timeouts"] == 0
    assert M.summarize([r])["error_m"] is None


class _OracleController:
    """The FP64 oracle as the controller: the warm start and the Philox counter
    carried over, and the exploration rate fed back (Alg. 1)."""

    def __init__(self, wl):
        self.p = f32_params(wl["params"])
        self.world = oracle.World.from_workload(wl)
        self.U = np.zeros((self.p["T"], 2))
        self.counter, self.S_e = 0, 1.0

    def set_reference(self, ref):
        self.ref = ref

    def step(self, x):
        r = oracle.step(self.p, self.world, x, self.U, self.ref, self.S_e, self.counter)
        self.counter += 1
        self.S_e, _ = oracle.exploration(self.p, self.world, x, r["Ustar"], r["beta_d"], self.p["explore_mu"])
        self.U = r["Unext"]
        return r["u0"].astype(np.float32)


def test_reference_controller_completes_a_vehicle_mission():
    wl = M.layout(3, 0, samples=256)
    r = M.run(_OracleController(wl), wl)
    assert r["success"], r
    assert 6.0 < r["avg_speed"] < 8.0 and r["error"] < 1.0

"""The comparison controllers of Sec. V on the GPU: Vanilla MPPI (normal
sampling, weighted collision indicator), Log-MPPI (normal x log-normal
sampling, the same indicator) and DBaS-Log-MPPI, as modes of the same
kernels, against the oracle's modes.

The indicator decides an integer from floating point (does some h fall below
0?), and the kernel takes that decision on FP32 positions, the oracle on FP64
ones.  A sample whose every step keeps |h| above a guard (1e-3 m^2, some ten
times the FP32 error of h) has one correct cost, compared to 1e-4.  For a
sample with a step inside the guard both decisions are correct to the
precision of the arithmetic; its GPU cost must then equal the oracle's plus
a whole number of collision weights (at most one per step).  The weights are
checked as the GPU's own costs through the FP64 softmax, and U* as the
oracle's noise averaged with the GPU's weights; where no sample near the
boundary carries weight, weights and U* are compared with the oracle's own.
"""
import math

import numpy as np
import pytest

import oracle
from conftest import f32_params
from parity_checks import TOL_U, check
from paper_2504_06437_amd import mission as M
from paper_2504_06437_amd import workloads as W

pytestmark = pytest.mark.gpu

GUARD = 1e-3


def _ctrl(wl, params):
    from paper_2504_06437_amd.controller import Controller
    p = dict(params, export_noise=True)
    c = Controller(p)
    c.load_workload(wl)
    return c, p


def _gpu(c, u0):
    return {"S": c.costs(), "w": c.weights(), "du": c.noise().astype(np.float64),
            "Ustar": c.last_optimal().astype(np.float64), "Unext": c.controls().astype(np.float64),
            "u0": np.asarray(u0, dtype=np.float64)}


def check_indicator(g, ref, margin, U, p, S_e=1.0, what=""):
    wI, lam = p["collision_weight"], p["lambda"]
    scale = math.sqrt(S_e) * np.asarray(p["sigma"], dtype=np.float64)
    d = np.abs(g["du"] - ref["du"])
    assert np.all(d <= 1e-5 * np.abs(ref["du"]) + 1e-6 * scale + 1e-30), f"{what} noise"
    base = 1e-4 * np.maximum(np.abs(ref["S"]), 1.0)
    dS = g["S"] - ref["S"]
    sure = margin >= GUARD
    assert np.all(np.abs(dS[sure]) <= base[sure]), f"{what} costs {np.max(np.abs(dS[sure]) / base[sure])}"
    n = np.round(dS[~sure] / wI)
    assert np.all(np.abs(n) <= p["T"]), what
    assert np.all(np.abs(dS[~sure] - n * wI) <= base[~sure]), f"{what} near-boundary costs"
    _, w_iso, _, _ = oracle.weights(g["S"], lam)
    big = w_iso >= 1e-8 * w_iso.max()
    assert np.max(np.abs(g["w"][big] - w_iso[big]) / w_iso[big]) <= 1e-5, f"{what} softmax"
    Us_iso = oracle.update(U, ref["du"], g["w"])
    assert np.all(np.abs(g["Ustar"] - Us_iso) <= TOL_U * (np.abs(Us_iso) + scale)), f"{what} U* given the weights"
    if np.all(ref["w"][~sure] < 1e-8 * ref["w"].max()) and np.all(g["w"][~sure] < 1e-8 * g["w"].max()):
        assert np.max(np.abs(g["w"] - ref["w"])) <= 1e-4 * ref["w"].max() + np.expm1(2 * np.max(np.abs(dS[sure])) / lam)
        assert np.all(np.abs(g["Ustar"] - ref["Ustar"]) <= TOL_U * (np.abs(ref["Ustar"]) + scale)), f"{what} U*"
    return float(np.mean(~sure))


def _iteration(wl, name, steps=1, **over):
    params = W.as_controller(wl["params"], name)
    params.update(over)
    c, p = _ctrl(wl, params)
    pf = f32_params(p)
    world = oracle.World.from_workload(wl)
    x = np.asarray(wl["x0"], dtype=np.float32)
    near = []
    for _ in range(steps):
        st = c.get_state()
        u0 = c.step(x)
        g = _gpu(c, u0)
        ref = oracle.step(pf, world, x, st["U"], wl["x_ref"], float(np.float32(st["S_e"])), st["counter"])
        assert ref["status"] == 0
        if p["cost_mode"] == "indicator":
            margin = oracle.margins(pf, world, x, st["U"], ref["du"])
            near.append(check_indicator(g, ref, margin, st["U"], p, st["S_e"], what=f"{name}"))
            assert c.info()["beta0"] == 0.0 and c.info()["beta_d"] == 0.0
        else:
            check(g, ref, p, S_e=st["S_e"], what=name)
    c.close()
    return near


@pytest.mark.parametrize("name", ["vanilla", "log", "dbas"])
@pytest.mark.parametrize("make", [lambda: W.quad_small(K=600, T=20, J=25), lambda: W.car(K=1000, T=24, J=60),
                                  lambda: W.quad_large(K=1500, T=30, J=150, cells=128)],
                         ids=["quad6", "car", "quad6_costmap"])
def test_controller_modes_match_oracle(name, make):
    wl = make()
    rng = np.random.Generator(np.random.PCG64(9))
    wl["U0"] = W.random_controls(rng, wl["params"]["T"], 0.3)
    near = _iteration(wl, name, steps=2)
    assert all(f < 0.2 for f in near), near


@pytest.mark.parametrize("mission", [1, 2])
@pytest.mark.parametrize("name", ["vanilla", "log", "dbas"])
def test_paper_settings_match_oracle(mission, name):
    """The missions' controller settings (M = 1024, N = 20, dt = 0.02 s, the
    paper's Sigma_u, gamma = 2), each controller, three steps."""
    wl = M.layout(mission, seed=3)
    _iteration(wl, name, steps=3)


def test_indicator_tile_shapes_and_batch():
    """Every tile size of the indicator kernel, and indicator controllers in a
    batch with barrier-state ones: each equals its standalone run."""
    from paper_2504_06437_amd.controller import Batch, Controller
    wl = W.car(K=300, T=11, J=21)
    for S in (16, 64, 256):
        _iteration(wl, "log", tile_samples=S)
    rng = np.random.Generator(np.random.PCG64(17))
    wls, names = [], []
    for i, name in enumerate(["vanilla", "dbas", "log", "vanilla", "dbas"]):
        m = "car" if i % 2 else "quad6"
        w = W.mixed_controller(rng, 900 + i, K=int(rng.integers(200, 1500)), T=int(rng.integers(8, 30)),
                               J=int(rng.integers(5, 80)), model=m)
        w["params"] = W.as_controller(w["params"], name)
        wls.append(w)
        names.append(name)

    def make(w):
        c = Controller(w["params"])
        c.load_workload(w)
        return c
    alone = [make(w) for w in wls]
    mixed = [make(w) for w in wls]
    batch = Batch(mixed)
    for _ in range(2):
        u_b, sts = batch.step([w["x0"] for w in wls])
        assert np.all(sts == 0)
        for i, (a, m, w) in enumerate(zip(alone, mixed, wls)):
            np.testing.assert_array_equal(a.step(w["x0"]), u_b[i], err_msg=names[i])
            np.testing.assert_array_equal(a.costs(), m.costs())
    batch.close()
    for c in alone + mixed:
        c.close()


def test_invalid_mode_settings_are_rejected():
    from paper_2504_06437_amd import _lib as A
    from paper_2504_06437_amd.controller import Controller
    p = W.base_params("car", 64, 10)
    for bad in ({"cost_mode": "indicator", "adaptive_explore": True}, {"collision_weight": -1.0},
                {"collision_weight": float("inf")}):
        with pytest.raises(A.MppiError):
            Controller(dict(p, **bad))

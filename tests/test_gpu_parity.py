"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (stated once, used everywhere below):
  * Philox words: bit-exact.
  * noise du: |d| <= 1e-5 |ref| + 1e-6 sqrt(S_e) sigma_c  (FP32 log/sqrt/sincospi/exp
    of exactly equal uniforms: a few ulp).
  * costs S_k: |d| <= 1e-4 max(|S_ref|, 1) + DP * sens_k.  sens_k (from the
    oracle) bounds |dS_k| per metre of shape-point displacement through the
    barrier for moves of up to DP per coordinate: R_B/(1-gamma_B) sum_t sum
    over terms of |grad h|_1 times the steepest slope of B within the move,
    which grows like 1/h^2 near a boundary (and 1/h_eps^2 at the cap).
    DP = 1e-5 m is the FP32 position-error budget (positions of <= 10 m in the
    iteration's local frame, ulp ~1e-6 m, over <= 100 Euler steps).  Far from
    obstacles the first term governs: the test requires it to govern for most
    samples.
  * weights: normwise |dw| <= 1e-4 max w_ref; elementwise relative 1e-4 plus
    the propagated cost error expm1(2 max|dS| / lambda) over the weighted
    samples; the GPU softmax alone (GPU costs through the FP64 softmax) 1e-5.
  * U*, shifted U, u0: |d| <= 1e-4 (|ref| + sqrt(S_e) sigma_c).
"""
import math

import numpy as np
import pytest

import oracle
from conftest import f32_params
from parity_checks import DP, TOL_S, TOL_U, check as _check, check_costs as _check_costs, gpu_outputs as _gpu_outputs
from paper_2504_06437_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ctrl(wl, **over):
    """A controller on the workload; the noise is exported (for the noise
    checks) unless the caller says otherwise."""
    from paper_2504_06437_amd.controller import Controller
    p = dict(wl["params"])
    p["export_noise"] = True
    p.update(over)
    c = Controller(p)
    c.load_workload(wl)
    return c, p


def _world(wl):
    return oracle.World.from_workload(wl)


def _one_iteration(wl, S_e=1.0, min_governed=0.5, **over):
    c, p = _ctrl(wl, **over)
    if S_e != 1.0:
        c.set_exploration(S_e)
    st = c.get_state()
    u0 = c.step(wl["x0"])
    g = _gpu_outputs(c, u0)
    info = c.info()
    ref = oracle.step(f32_params(p), _world(wl), wl["x0"], st["U"], wl["x_ref"], np.float32(S_e), st["counter"])
    assert ref["status"] == 0 and info["status"] == 0
    _check(g, ref, p, S_e, what=str(over), min_governed=min_governed)
    c.close()
    return g, ref, info


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("counter", [0, 1, 2**32 + 5, 2**63 + 7])
def test_philox_words_bit_exact(counter):
    wl = W.quad_small(K=300, T=7)
    c, p = _ctrl(wl, seed=0x0123456789ABCDEF)
    g = c.philox_words(counter)
    want = oracle.noise_words(f32_params(p), counter)
    assert np.array_equal(g, want)
    c.close()


@pytest.mark.parametrize("name,make", [
    ("tiny_quad6", lambda: W.tiny("quad6")),
    ("tiny_quad5", lambda: W.tiny("quad5")),
    ("tiny_car", lambda: W.tiny("car")),
    ("quad_small", lambda: W.quad_small()),
    ("quad_small_ragged", lambda: W.quad_small(K=300, T=7)),
    ("car_medium", lambda: W.car(K=1000, T=20, J=40)),
    ("quad5_medium", lambda: W.quad_small(K=777, T=15, J=25, model="quad5")),
    ("quad_costmap", lambda: W.quad_large(K=2048, T=30, J=100, cells=128)),
])
def test_iteration_matches_oracle(name, make):
    _one_iteration(make())


def test_both_barrier_forms_match_oracle():
    """The fixed-P tiles use the layout of the paper's bodies (rectangle
    corners and side midpoints; points on the quadrotor's axis, mirrored
    about its centre or not); any other shape runs on the runtime-P tile.
    Every form matches the oracle, and the same point set in another order
    gives the same costs."""
    wl = W.car(K=700, T=17, J=30)
    g_fixed, _, info = _one_iteration(wl)
    assert info["barrier_form"] == 1
    wl_rev = dict(wl, params=dict(wl["params"], shape=wl["params"]["shape"][::-1]))
    g_rev, ref_rev, info = _one_iteration(wl_rev)
    assert info["barrier_form"] == 0
    bound = TOL_S * np.maximum(np.abs(ref_rev["S"]), 1.0) + DP * ref_rev["sens"]
    assert np.all(np.abs(g_rev["S"] - g_fixed["S"]) <= 2.0 * bound)
    wq = W.quad_small(K=500, T=13, J=20, model="quad5")
    g_mirror, _, info = _one_iteration(wq)
    assert info["barrier_form"] == 2
    # the same points with the middle one moved off the end of the list: on
    # the axis, no longer mirrored in the order the mirrored form reads
    sh = wq["params"]["shape"]
    moved = [sh[3]] + sh[:3] + sh[4:]
    g_axis, ref_axis, info = _one_iteration(dict(wq, params=dict(wq["params"], shape=moved)))
    assert info["barrier_form"] == 1
    bound = TOL_S * np.maximum(np.abs(ref_axis["S"]), 1.0) + DP * ref_axis["sens"]
    assert np.all(np.abs(g_axis["S"] - g_mirror["S"]) <= 2.0 * bound)
    off_axis = [[a, 0.01 * (i % 2)] for i, (a, _) in enumerate(sh)]
    assert _one_iteration(dict(wq, params=dict(wq["params"], shape=off_axis)))[2]["barrier_form"] == 0
    # other bodies of the same layouts: a 3.4 m x 1.2 m rectangle, and a
    # mirrored axis whose middle point is off the centre
    a, b = 1.7, 0.6
    rect = [[a, b], [a, -b], [-a, b], [-a, -b], [a, 0.0], [-a, 0.0], [0.0, b], [0.0, -b]]
    assert _one_iteration(dict(wl, params=dict(wl["params"], shape=rect)))[2]["barrier_form"] == 1
    axis = [[-0.3, 0.0], [-0.2, 0.0], [-0.05, 0.0], [0.02, 0.0], [0.05, 0.0], [0.2, 0.0], [0.3, 0.0]]
    assert _one_iteration(dict(wq, params=dict(wq["params"], shape=axis)))[2]["barrier_form"] == 2


def test_far_and_touching_obstacles_match_oracle():
    """The layout forms' two guards.  An obstacle touching the start sends
    some samples into it, where an h falls below h_eps: those waves take the
    clamped per-point form for that obstacle.  An obstacle far from the
    start (240 m for the quadrotor, 120 m for the vehicle, in the
    iteration's local frame) lets the pair fractions' shared term pass its
    cap, so no unit may drop the cap test: the vehicle tests it per
    obstacle, the quadrotor's axis runs the clamped per-point form.  Each
    case matches the oracle.  Every quadrotor sample passes within a few
    centimetres of the touching obstacle, so there the barrier's
    conditioning governs the cost bound for most samples (the case is here
    for the guard's failure branch, not for the 1e-4 bar, which the
    far-only case and the vehicle's cases hold)."""
    q = W.quad_small(K=512, T=20, J=10)
    x, y = float(q["x0"][0]), float(q["x0"][1])
    near_q, far_q = [x + 0.45, y, 0.22], [x + 240.0, y, 0.5]
    c = W.car(K=512, T=20, J=20)
    x, y = float(c["x0"][0]), float(c["x0"][1])
    d = 2.6 / math.sqrt(2.0)          # ahead of the vehicle, along its 45-degree heading
    near_c, far_c = [x + d, y + d, 0.5], [x, y + 120.0, 0.5]
    cases = ((q, [far_q], 2, 0.0, 0.5), (q, [near_q], 2, 0.02, 0.0), (q, [near_q, far_q], 2, 0.02, 0.0),
             (c, [near_c], 1, 0.02, 0.5), (c, [near_c, far_c], 1, 0.02, 0.5))
    for wl, extra, form, least_inside, governed in cases:
        w = dict(wl, obstacles=np.vstack([wl["obstacles"], np.asarray(extra, dtype=np.float32)]))
        _, ref, info = _one_iteration(w, min_governed=governed)
        assert info["barrier_form"] == form
        inside = np.mean(np.asarray(ref["clear"]) < wl["params"]["h_eps"])
        assert least_inside <= inside < 0.5, inside


def test_degenerate_and_largest_sizes_match_oracle():
    """One sample, one step, one obstacle and a one-point body; one step with
    no obstacle; the most obstacles (MPPI_JMAX = 2048); the longest horizon
    (MPPI_TMAX = 1024), whose noise does not fit in LDS and is drawn again in
    the epilogue."""
    wl = W.car(K=1, T=1, J=1)
    _one_iteration(dict(wl, params=dict(wl["params"], shape=[[1.0, 0.5]])))
    _one_iteration(_no_obstacles(W.quad_small(K=64, T=1, J=1)))
    _one_iteration(W.car(K=20, T=2, J=2048))
    _one_iteration(W.car(K=16, T=1024, J=3), tile_samples=16)


def _no_obstacles(wl):
    return dict(wl, obstacles=np.zeros((0, 3), dtype=np.float32))


@pytest.mark.parametrize("S", [16, 32, 64, 128, 256])
def test_every_tile_shape_matches_oracle(S):
    _one_iteration(W.quad_small(K=300, T=11, J=13), tile_samples=S)
    _one_iteration(W.car(K=200, T=9, J=21), tile_samples=S)


def test_long_horizon_spans_several_chunks():
    """T = 300 with 256-sample tiles needs several horizon chunks."""
    _one_iteration(W.car(K=600, T=300, J=20), tile_samples=256)
    _one_iteration(W.quad_small(K=100, T=200, J=12), tile_samples=16)


def test_exploration_rate_scales_noise_and_control_cost():
    wl = W.quad_small(K=512, T=20)
    rng = np.random.Generator(np.random.PCG64(3))
    wl["U0"] = W.random_controls(rng, 20)
    _one_iteration(wl, S_e=2.75)


def test_no_obstacles_and_fp64_normaliser_modes():
    wl = W.quad_small(K=256, T=20, J=10)
    wl["obstacles"] = np.zeros((0, 3), dtype=np.float32)
    _one_iteration(wl, normaliser="on")
    _one_iteration(W.quad_small(K=256, T=20), normaliser="off")


def test_receding_horizon_teacher_forced():
    """Several control steps; each GPU iteration is compared with the oracle
    started from the GPU's own warm start, counter and state."""
    wl = W.quad_small(K=512, T=20)
    c, p = _ctrl(wl)
    pf = f32_params(p)
    x = wl["x0"].astype(np.float32)
    for step in range(6):
        xr = W.reference(wl, x)
        c.set_reference(xr)
        st = c.get_state()
        u0 = c.step(x)
        g = _gpu_outputs(c, u0)
        wl2 = dict(wl, x_ref=xr)
        ref = oracle.step(pf, _world(wl2), x, st["U"], xr, 1.0, st["counter"])
        assert st["counter"] == step
        _check(g, ref, p, what=f"step {step}")
        x = oracle.dynamics(pf, x, u0).astype(np.float32)   # the simulated plant
    c.close()


def test_full_size_vehicle_workload():
    """Ground vehicle, K=4096, T=50, 100 obstacles: every output compared."""
    _, _, info = _one_iteration(W.car())
    assert info["tiles"] >= 1


def test_full_size_quadrotor_with_costmap():
    """Quadrotor at scale, K=16384, T=100, 400 obstacles + 512x512 costmap,
    FP64 normaliser, in the launch configuration the benchmark times (no
    noise export): every sample's cost, the weights, U*, the shifted U and
    u0 against the oracle's own iteration (threaded over samples), and the
    Philox words of sampled (k, t)."""
    wl = W.quad_large()
    c, p = _ctrl(wl, export_noise=False)
    st = c.get_state()
    u0 = c.step(wl["x0"])
    info = c.info()
    assert info["status"] == 0 and info["fp64_tiles"] == info["tiles"]
    g = _gpu_outputs(c, u0, with_noise=False)
    words = c.philox_words(st["counter"])
    for k in (0, 1, 4097, 9999, 16383):
        for t in (0, 57, 99):
            want = oracle.philox([k, t, st["counter"] & 0xFFFFFFFF, st["counter"] >> 32],
                                 [p["seed"] & 0xFFFFFFFF, p["seed"] >> 32])
            assert list(words[k, t]) == want
    ref = oracle.step(f32_params(p), _world(wl), wl["x0"], st["U"], wl["x_ref"], 1.0, st["counter"])
    assert ref["status"] == 0
    _check(g, ref, p, what="full-size quadrotor")
    assert abs(g["w"].sum() - 1.0) < 1e-9
    np.testing.assert_array_equal(g["u0"], g["Ustar"][0])
    c.close()


# --- special cases the paper fixes -------------------------------------------

def test_zero_noise_keeps_the_sequence():
    wl = W.quad_small(K=256, T=20)
    rng = np.random.Generator(np.random.PCG64(4))
    wl["U0"] = W.random_controls(rng, 20)
    c, p = _ctrl(wl, sigma=[0.0, 0.0])
    u0 = c.step(wl["x0"])
    du, S, w, Us, U = c.noise(), c.costs(), c.weights(), c.last_optimal(), c.controls()
    assert np.all(du == 0.0)
    assert np.all(S == S[0])
    np.testing.assert_allclose(w, 1.0 / 256, rtol=1e-12)
    np.testing.assert_array_equal(Us, wl["U0"])
    np.testing.assert_array_equal(U[:-1], wl["U0"][1:])
    np.testing.assert_array_equal(U[-1], wl["U0"][-1])
    np.testing.assert_array_equal(u0, wl["U0"][0])
    ref = oracle.step(f32_params(p), _world(wl), wl["x0"], wl["U0"], wl["x_ref"], 1.0, 0)
    assert abs(S[0] - ref["S"][0]) <= TOL_S * abs(ref["S"][0])
    c.close()


def test_single_sample_returns_that_sample():
    wl = W.quad_small(K=1, T=20)
    c, p = _ctrl(wl)
    c.step(wl["x0"])
    assert c.weights()[0] == 1.0
    np.testing.assert_allclose(c.last_optimal(), wl["U0"] + c.noise()[0], rtol=0, atol=1e-6)
    c.close()


def test_temperature_limits():
    wl = W.quad_small(K=64, T=20)
    c, _ = _ctrl(wl, **{"lambda": 1e-9})
    c.step(wl["x0"])
    k = int(np.argmin(c.costs()))
    np.testing.assert_allclose(c.last_optimal(), wl["U0"] + c.noise()[k], rtol=0, atol=1e-6)
    c.close()
    c, _ = _ctrl(wl, **{"lambda": 1e15})
    c.step(wl["x0"])
    np.testing.assert_allclose(c.last_optimal(), wl["U0"] + c.noise().mean(axis=0), rtol=0, atol=1e-6)
    c.close()


def test_numeric_failure_leaves_state_unchanged():
    from paper_2504_06437_amd import _lib as A
    wl = W.quad_small(K=128, T=20)
    c, _ = _ctrl(wl, Q=[3e38] * 6)
    before = c.get_state()
    st, u0 = c.step_status(wl["x0"] + np.float32(5.0))
    assert st == A.E_NUMERIC
    after = c.get_state()
    assert after["counter"] == before["counter"]
    np.testing.assert_array_equal(after["U"], before["U"])
    np.testing.assert_array_equal(u0, before["U"][0])
    c.close()


def test_invalid_inputs_are_rejected_before_launch():
    from paper_2504_06437_amd import _lib as A
    from paper_2504_06437_amd.controller import Controller
    wl = W.quad_small(K=64, T=20)
    c, _ = _ctrl(wl)
    x = wl["x0"].copy()
    x[2] = np.nan
    st, _ = c.step_status(x)
    assert st == A.E_INVALID
    assert c.get_state()["counter"] == 0
    with pytest.raises(A.MppiError):
        c.set_exploration(-1.0)
    with pytest.raises(A.MppiError):
        c.set_obstacles(np.array([[1.0, 2.0, -0.5]]))
    for bad in ({"lambda": 0.0}, {"gamma_b": 1.0}, {"K": 0}, {"h_eps": 0.0}, {"tile_samples": 3}):
        p = dict(wl["params"])
        p.update(bad)
        with pytest.raises(A.MppiError):
            Controller(p)
    c.close()


def test_checkpoint_resume_is_bit_identical():
    wl = W.car(K=512, T=20, J=30)
    c, _ = _ctrl(wl)
    c.step(wl["x0"])
    saved = c.get_state()
    u_a = c.step(wl["x0"])
    U_a, S_a = c.controls(), c.costs()
    c.set_state(saved)
    u_b = c.step(wl["x0"])
    np.testing.assert_array_equal(u_a, u_b)
    np.testing.assert_array_equal(U_a, c.controls())
    np.testing.assert_array_equal(S_a, c.costs())
    c.close()


def test_async_device_step_matches_sync_step():
    from paper_2504_06437_amd.hip import DeviceArray
    wl = W.quad_small(K=256, T=20)
    a, _ = _ctrl(wl)
    b, _ = _ctrl(wl)
    ua = a.step(wl["x0"])
    ua2 = a.step(wl["x0"] + np.float32(0.01))
    x0 = DeviceArray.from_numpy(np.stack([wl["x0"], wl["x0"] + np.float32(0.01)]))
    u0 = DeviceArray((2, 2))
    b.step_async(x0.at(0), u0.at(0))
    b.step_async(x0.at(1), u0.at(1))
    assert b.synchronize() == 0
    got = u0.numpy()
    np.testing.assert_array_equal(ua, got[0])
    np.testing.assert_array_equal(ua2, got[1])
    np.testing.assert_array_equal(a.controls(), b.controls())
    a.close()
    b.close()


def test_noise_export_changes_nothing_else():
    """Without export the noise is never stored (and cannot be read back);
    every other output is bit-identical to the exporting controller's."""
    from paper_2504_06437_amd import _lib as A
    wl = W.car(K=1000, T=30, J=40)
    a, _ = _ctrl(wl)
    b, _ = _ctrl(wl, export_noise=False)
    for _ in range(2):
        np.testing.assert_array_equal(a.step(wl["x0"]), b.step(wl["x0"]))
        np.testing.assert_array_equal(a.costs(), b.costs())
        np.testing.assert_array_equal(a.weights(), b.weights())
        np.testing.assert_array_equal(a.controls(), b.controls())
    with pytest.raises(A.MppiError):
        b.noise()
    a.close()
    b.close()


def test_synchronous_step_returns_the_iterations_own_u0():
    """mppi_step returns as soon as the update marks completion in pinned
    memory: its u0 must be the iteration's U*[0] and its status final, step
    after step (with adaptive exploration queued behind the update too)."""
    wl = W.car(K=2048, T=30, J=60)
    for over in ({}, {"adaptive_explore": True}):
        c, _ = _ctrl(wl, **over)
        x = wl["x0"].copy()
        for i in range(25):
            u0 = c.step(x)
            np.testing.assert_array_equal(u0, c.last_optimal()[0])
            assert c.info()["status"] == 0 and c.get_state()["counter"] == i + 1
            x = x + np.float32(0.01)
        c.close()

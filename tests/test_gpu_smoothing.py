"""Savitzky-Golay smoothing of the update on the GPU (Algorithm 1's SGF):
U* = U + SGF(sum_k w_k du_k), the filter applied along the horizon to each
tile's partial sums (it is linear).  Parity against the oracle's smoothing
(the local least-squares fit, written from its definition), to the update
tolerance |dU*| <= 1e-4 (|U*| + sigma); in isolation (the GPU's own weights
and noise through the oracle's filter) to 1e-5; batched equals standalone
bit for bit."""
import numpy as np
import pytest

import oracle
from conftest import f32_params
from paper_2504_06437_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ctrl(wl, **over):
    from paper_2504_06437_amd.controller import Controller
    p = dict(wl["params"], export_noise=True)
    p.update(over)
    c = Controller(p)
    c.load_workload(wl)
    return c, p


@pytest.mark.parametrize("case", [("quad_small", 3, 2), ("car", 5, 3), ("single_window", 4, 4)])
def test_smoothed_update_matches_oracle(case):
    name, m, order = case
    if name == "quad_small":
        wl = W.quad_small()
    elif name == "car":
        wl = W.car(K=512, T=40, J=50)
    else:
        wl = W.car(K=300, T=9, J=20)          # T = 2m + 1: one window for every step
    rng = np.random.default_rng(5)
    wl["U0"] = W.random_controls(rng, wl["params"]["T"], 0.2)
    c, p = _ctrl(wl, sgf_half_window=m, sgf_order=order)
    st = c.get_state()
    c.step(wl["x0"])
    Us = c.last_optimal().astype(np.float64)
    pf = f32_params(p)
    ref = oracle.step(pf, oracle.World.from_workload(wl), wl["x0"], st["U"], wl["x_ref"], 1.0, st["counter"])
    scale = np.asarray(pf["sigma"])
    assert np.all(np.abs(Us - ref["Ustar"]) <= 1e-4 * (np.abs(ref["Ustar"]) + scale))
    # isolation: the GPU's weights and noise through the oracle's filter
    w, du = c.weights(), c.noise().astype(np.float64)
    iso = st["U"] + oracle.sgf(np.einsum("k,ktc->tc", w, du), m, order)
    assert np.all(np.abs(Us - iso) <= 1e-5 * (np.abs(iso) + scale))
    # the smoothing changed something (it is not the identity here)
    raw = st["U"] + np.einsum("k,ktc->tc", w, du)
    if order < 2 * m:
        assert np.max(np.abs(raw - Us)) > 1e-6
    c.close()


def test_invalid_smoothing_settings_are_rejected():
    from paper_2504_06437_amd import _lib as A
    from paper_2504_06437_amd.controller import Controller
    wl = W.quad_small(K=256, T=20)
    for bad in ({"sgf_half_window": 10, "sgf_order": 2},      # T < 2m + 1
                {"sgf_half_window": 3, "sgf_order": 7},       # order > 2m
                {"sgf_half_window": 17, "sgf_order": 2}):
        p = dict(wl["params"])
        p.update(bad)
        with pytest.raises(A.MppiError):
            Controller(p)


def test_batched_smoothing_equals_standalone():
    from paper_2504_06437_amd.controller import Batch, Controller
    rng = np.random.Generator(np.random.PCG64(17))
    wls = []
    for i in range(5):
        wl = W.mixed_controller(rng, 900 + i, K=int(round(2 ** rng.uniform(6, 9))), T=int(rng.integers(12, 30)),
                                J=int(rng.integers(5, 40)))
        if i % 2 == 0:
            wl["params"].update(sgf_half_window=3, sgf_order=2)
        wls.append(wl)

    def make(wl):
        c = Controller(wl["params"])
        c.load_workload(wl)
        return c

    alone = [make(wl) for wl in wls]
    mixed = [make(wl) for wl in wls]
    batch = Batch(mixed)
    for _ in range(2):
        u_b, sts = batch.step([wl["x0"] for wl in wls])
        assert np.all(sts == 0)
        for i, (a, wl) in enumerate(zip(alone, wls)):
            np.testing.assert_array_equal(a.step(wl["x0"]), u_b[i])
            np.testing.assert_array_equal(a.last_optimal(), mixed[i].last_optimal())
    batch.close()
    for c in alone + mixed:
        c.close()

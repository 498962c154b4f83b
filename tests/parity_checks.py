"""Parity checks of GPU outputs against the FP64 oracle, shared by the GPU
test modules.  The tolerances are stated in test_gpu_parity's docstring and
derived in the design notes; the cost bound's second term is the oracle's
barrier sensitivity over the FP32 position budget (conftest.SENS_REACH)."""
import math

import numpy as np

import oracle
from conftest import SENS_REACH

TOL_S = 1e-4
TOL_W = 1e-4
TOL_U = 1e-4
DP = SENS_REACH


def check_costs(Sg, Sr, sens, what="", min_governed=0.5):
    """Costs within 1e-4 relative plus the barrier's conditioning; the
    relative term must govern for at least `min_governed` of the samples
    (lower only where every sample passes within centimetres of an
    obstacle, so that the conditioning governs by construction)."""
    base = TOL_S * np.maximum(np.abs(Sr), 1.0)
    cond = DP * sens
    assert np.mean(cond <= base) >= min_governed, f"{what}: the relative bound governs only {np.mean(cond <= base):.2f}"
    d = np.abs(Sg - Sr)
    assert np.all(np.isfinite(Sg))
    assert np.all(d <= base + cond), f"{what} costs {np.max(d / (base + cond))} of the bound"


def check_weights(wg, wr, Sg, Sr, lam, what=""):
    """Weights: normwise relative 1e-4; elementwise relative 1e-4 plus what
    the cost difference itself propagates (w_k ~ exp(-S_k/lambda), so
    |dw_k|/w_k <= expm1(2 max|dS|/lambda) to first order); and the GPU's
    softmax alone (its own costs through the FP64 softmax) to 1e-5."""
    assert np.max(np.abs(wg - wr)) <= TOL_W * wr.max(), f"{what} weights normwise"
    big = wr >= 1e-8 * wr.max()
    dS = np.max(np.abs(Sg - Sr)[big])
    bound = TOL_W + np.expm1(2.0 * dS / lam)
    rel = np.abs(wg[big] - wr[big]) / wr[big]
    assert rel.max() <= bound, f"{what} weights {rel.max()} > {bound}"
    assert np.all(np.abs(wg[~big] - wr[~big]) <= 1e-8 * wr.max()), f"{what} small weights"
    _, w_iso, _, _ = oracle.weights(Sg, lam)
    big = w_iso >= 1e-8 * w_iso.max()
    assert np.max(np.abs(wg[big] - w_iso[big]) / w_iso[big]) <= 1e-5, f"{what} softmax in isolation"


def check(gpu: dict, ref: dict, p: dict, S_e=1.0, what="", min_governed=0.5):
    scale = math.sqrt(S_e) * np.asarray(p["sigma"], dtype=np.float64)
    if "du" in gpu:
        d = np.abs(gpu["du"] - ref["du"])
        assert np.all(d <= 1e-5 * np.abs(ref["du"]) + 1e-6 * scale + 1e-30), f"{what} noise {d.max()}"
    check_costs(gpu["S"], ref["S"], ref["sens"], what, min_governed)
    check_weights(gpu["w"], ref["w"], gpu["S"], ref["S"], p["lambda"], what)
    for key in ("Ustar", "Unext"):
        d = np.abs(gpu[key] - ref[key])
        assert np.all(d <= TOL_U * (np.abs(ref[key]) + scale)), f"{what} {key} {d.max()}"
    d = np.abs(gpu["u0"] - ref["u0"])
    assert np.all(d <= TOL_U * (np.abs(ref["u0"]) + scale)), f"{what} u0"


def gpu_outputs(c, u0, with_noise=True):
    g = {"S": c.costs(), "w": c.weights(), "Ustar": c.last_optimal().astype(np.float64),
         "Unext": c.controls().astype(np.float64), "u0": np.asarray(u0, dtype=np.float64)}
    if with_noise:
        g["du"] = c.noise().astype(np.float64)
    return g

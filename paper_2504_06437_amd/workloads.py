"""Seeded synthetic workloads shared by the GPU path's tests/bench and the oracle.

This module only *generates inputs*: parameter dictionaries, obstacle sets,
costmaps, start/goal states and straight-line reference trajectories.  It holds
none of the controller's arithmetic (no sampling, dynamics, barrier, cost or
weighting), so that the oracle and the HIP path can both be fed from it without
sharing any of the method's code.

Workloads (sizes from the project's target configurations; everything random is
drawn from numpy's PCG64 with the stated seed):

* ``quad_small``  -- planar quadrotor (6 states, 2 rotor thrusts), K=256, T=20,
  dt=0.02 s, 10 circles with centres U([0,10]^2) and radii U[0.3,0.8], seed 0.
* ``car``         -- Ackermann vehicle, K=4096, T=50, dt=0.05 s, 100 circles
  U([0,20]^2) with radii U[0.2,1.0], seed 1.
* ``quad_large``  -- quadrotor, K=16384, T=100, 400 circles in [0,40]^2 plus a
  512x512 signed-distance costmap of 64 random blobs, FP64 normaliser, seed 2.
* ``batch64``     -- 64 controllers, model Bernoulli(1/2), K=round(2^U(8,13)),
  T~U{20..80}, J~U{10..400}, world side 10..40 m growing with J, seed 3.

The noise is N(0, diag(0.5^2)) times a log-normal factor with mu=0, sigma=0.3
and lambda=1 in every workload (the quad5 paper model uses the paper's
Sigma_u = diag(0.4, 0.12) instead).  Parameters the paper does not give
(Q, R_B, gamma_B, h_eps, start, goal) are fixed here; they change values, not
work.
"""
from __future__ import annotations

import copy
import math

import numpy as np

MODEL_DIMS = {"quad6": 6, "quad5": 5, "car": 4}

# Shape points (body frame: along the heading, normal to it).
# Quadrotor: 7 points evenly spaced on the 0.4 m frame, both propellers at the
# ends (written as 0.4 (i - 3) / 6, so the middle point is exactly the centre
# and the pairs are exact mirrors).
QUAD_SHAPE = [[0.4 * (i - 3) / 6.0, 0.0] for i in range(7)]
# Vehicle: corners and side midpoints of a 4 m x 3 m rectangle.
CAR_SHAPE = [[2.0, 1.5], [2.0, -1.5], [-2.0, 1.5], [-2.0, -1.5],
             [2.0, 0.0], [-2.0, 0.0], [0.0, 1.5], [0.0, -1.5]]
BODY_RADIUS = {"quad6": 0.2, "quad5": 0.2, "car": 2.5}


def base_params(model: str, K: int, T: int, seed: int = 0) -> dict:
    """Physical and tuning parameters of one controller (plain dict)."""
    p = {
        "model": model, "K": int(K), "T": int(T), "seed": int(seed),
        "mu_ln": 0.0, "sigma_ln": 0.3, "lambda": 1.0,
        "gamma_u": 2.0, "gamma_b": 0.5, "r_b": 0.1, "h_eps": 1e-4,
        "init_mode": "repeat", "normaliser": "auto", "collision_weight": 1000.0,
        "mass": 0.5, "gravity": 9.81, "arm": 0.2, "inertia": 0.005, "wheelbase": 4.0,
    }
    if model == "quad6":
        half = 0.5 * 0.5 * 9.81          # per-rotor limit: +-m g / 2
        p.update(dt=0.02, u_min=[-half, -half], u_max=[half, half], sigma=[0.5, 0.5],
                 Q=[1.0, 1.0, 0.1, 0.1, 0.1, 0.1], shape=copy.deepcopy(QUAD_SHAPE))
    elif model == "quad5":
        p.update(dt=0.02, u_min=[-4.0, -0.981], u_max=[4.0, 0.981],
                 sigma=[math.sqrt(0.4), math.sqrt(0.12)],
                 Q=[1.0, 1.0, 0.1, 0.1, 0.1], shape=copy.deepcopy(QUAD_SHAPE))
    elif model == "car":
        p.update(dt=0.05, u_min=[-1.013, -2.0], u_max=[1.013, 2.0], sigma=[0.5, 0.5],
                 Q=[1.0, 1.0, 0.1, 0.1], shape=copy.deepcopy(CAR_SHAPE))
    else:
        raise ValueError(model)
    p["Qf"] = [10.0 * q for q in p["Q"]]
    return p


def circles(rng, J, lo, hi, r_lo, r_hi, keep_clear=(), clear_r=0.0):
    """J circles with centres U([lo,hi]^2), radii U[r_lo,r_hi], rejecting any
    that come within clear_r of a keep-clear point."""
    out = []
    while len(out) < J:
        c = rng.uniform(lo, hi, size=2)
        r = rng.uniform(r_lo, r_hi)
        if all(math.hypot(c[0] - q[0], c[1] - q[1]) > r + clear_r for q in keep_clear):
            out.append([c[0], c[1], r])
    return np.asarray(out, dtype=np.float32).reshape(-1, 3)


def blob_sdf(rng, n_blobs, side, cells, keep_clear=(), clear_r=0.0):
    """Signed distance (metres, FP64 then rounded to fp32) of a union of
    random blobs; each blob is 3 discs with radii U[0.3,1.2] whose centres lie
    within 1 m of the blob centre.  Cell (col i, row j) is sampled at its
    centre ((i+1/2) res, (j+1/2) res)."""
    discs = []
    while len(discs) < 3 * n_blobs:
        centre = rng.uniform(0.0, side, size=2)
        blob = []
        for _ in range(3):
            ang = rng.uniform(0.0, 2.0 * math.pi)
            rad = rng.uniform(0.0, 1.0)
            c = centre + rad * np.array([math.cos(ang), math.sin(ang)])
            r = rng.uniform(0.3, 1.2)
            blob.append((c[0], c[1], r))
        if all(math.hypot(b[0] - q[0], b[1] - q[1]) > b[2] + clear_r for b in blob for q in keep_clear):
            discs.extend(blob)
    res = side / cells
    xs = (np.arange(cells) + 0.5) * res
    gx, gy = np.meshgrid(xs, xs)            # gy varies along rows
    d = np.full((cells, cells), np.inf)
    for (cx, cy, r) in discs:
        d = np.minimum(d, np.hypot(gx - cx, gy - cy) - r)
    return d.astype(np.float32), res


def start_state(model: str, start, goal) -> np.ndarray:
    n = MODEL_DIMS[model]
    x = np.zeros(n, dtype=np.float32)
    x[0], x[1] = start[0], start[1]
    if model == "car":
        x[2] = math.atan2(goal[1] - start[1], goal[0] - start[0])
    return x


def reference(wl: dict, x0) -> np.ndarray:
    """Straight start->goal reference at v_set, re-anchored each control step at
    the projection of the current position on the line: x_ref[(T+1), n] fp32."""
    p = wl["params"]
    model, T, dt = p["model"], p["T"], p["dt"]
    n = MODEL_DIMS[model]
    a = np.asarray(wl["start"], dtype=np.float64)
    b = np.asarray(wl["goal"], dtype=np.float64)
    L = float(np.linalg.norm(b - a))
    d = (b - a) / L
    s0 = float(np.clip(np.dot(np.asarray(x0[:2], dtype=np.float64) - a, d), 0.0, L))
    v = wl["v_set"]
    ref = np.zeros((T + 1, n), dtype=np.float64)
    for t in range(T + 1):
        s = min(s0 + v * t * dt, L)
        moving = s < L
        ref[t, 0:2] = a + s * d
        if model == "car":
            ref[t, 2] = math.atan2(d[1], d[0])
            ref[t, 3] = v if moving else 0.0
        else:
            ref[t, 3:5] = (v * d) if moving else 0.0
    return ref.astype(np.float32)


def _finish(params, obstacles, start, goal, v_set, steps, sdf=None, res=None):
    wl = {"params": params, "obstacles": obstacles, "start": list(start), "goal": list(goal),
          "v_set": v_set, "steps": steps, "map": None}
    if sdf is not None:
        wl["map"] = {"sdf": sdf, "origin": (0.0, 0.0), "res": res}
    wl["x0"] = start_state(params["model"], start, goal)
    wl["U0"] = np.zeros((params["T"], 2), dtype=np.float32)
    wl["x_ref"] = reference(wl, wl["x0"])
    return wl


def quad_small(K=256, T=20, J=10, seed=0, model="quad6") -> dict:
    rng = np.random.Generator(np.random.PCG64(seed))
    start, goal = (1.0, 1.0), (9.0, 9.0)
    obs = circles(rng, J, 0.0, 10.0, 0.3, 0.8, (start, goal), BODY_RADIUS[model] + 0.5)
    return _finish(base_params(model, K, T, seed), obs, start, goal, 1.0, 50)


def car(K=4096, T=50, J=100, seed=1) -> dict:
    rng = np.random.Generator(np.random.PCG64(seed))
    start, goal = (2.0, 2.0), (18.0, 18.0)
    obs = circles(rng, J, 0.0, 20.0, 0.2, 1.0, (start, goal), BODY_RADIUS["car"] + 0.5)
    return _finish(base_params("car", K, T, seed), obs, start, goal, 5.0, 200)


def quad_large(K=16384, T=100, J=400, seed=2, cells=512, with_map=True) -> dict:
    rng = np.random.Generator(np.random.PCG64(seed))
    start, goal = (2.0, 2.0), (38.0, 38.0)
    clear = BODY_RADIUS["quad6"] + 0.5
    obs = circles(rng, J, 0.0, 40.0, 0.3, 0.8, (start, goal), clear)
    sdf = res = None
    if with_map:
        sdf, res = blob_sdf(rng, 64, 40.0, cells, (start, goal), clear)
    p = base_params("quad6", K, T, seed)
    p["normaliser"] = "on"
    return _finish(p, obs, start, goal, 1.0, 100, sdf, res)


def mixed_controller(rng, seed, K=None, T=None, J=None, model=None) -> dict:
    """One controller of the mixed batch: model Bernoulli(1/2), K log-uniform
    in [256, 8192], T uniform in {20..80}, J uniform in {10..400}."""
    model = model or ("quad6" if rng.uniform() < 0.5 else "car")
    K = K or int(round(2.0 ** rng.uniform(8.0, 13.0)))
    T = T or int(rng.integers(20, 81))
    J = J or int(rng.integers(10, 401))
    side = 10.0 + 30.0 * (J - 10) / 390.0
    start, goal = (0.1 * side, 0.1 * side), (0.9 * side, 0.9 * side)
    clear = BODY_RADIUS[model] + 0.5
    if model == "car":
        obs = circles(rng, J, 0.0, side, 0.2, 1.0, (start, goal), clear)
        v = 5.0
    else:
        obs = circles(rng, J, 0.0, side, 0.3, 0.8, (start, goal), clear)
        v = 1.0
    return _finish(base_params(model, K, T, seed), obs, start, goal, v, 100)


def batch(n=64, seed=3) -> list:
    rng = np.random.Generator(np.random.PCG64(seed))
    return [mixed_controller(rng, seed * 1000 + i) for i in range(n)]


def tiny(model="quad6", K=4, T=3, J=2, seed=7) -> dict:
    """A tiny case for brute-force cross-checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if model == "car":
        start, goal = (2.0, 2.0), (12.0, 12.0)
        obs = circles(rng, J, 4.0, 10.0, 0.2, 1.0, (start, goal), 3.0)
        v = 5.0
    else:
        start, goal = (1.0, 1.0), (5.0, 5.0)
        obs = circles(rng, J, 1.5, 4.5, 0.3, 0.8, (start, goal), 0.7)
        v = 1.0
    return _finish(base_params(model, K, T, seed), obs, start, goal, v, 5)


def random_controls(rng, T, scale=0.3) -> np.ndarray:
    return (scale * rng.standard_normal((T, 2))).astype(np.float32)


# The paper's controller and its two baselines (Sec. V, the mission table) as
# settings of the same iteration: Vanilla MPPI samples the normal law and
# pays a weighted collision indicator, Log-MPPI samples the normal x
# log-normal mixture with the same indicator, DBaS-Log-MPPI samples the
# mixture, carries the barrier state and adapts its exploration rate.
CONTROLLERS = {
    "vanilla": {"sampling": "normal", "cost_mode": "indicator", "adaptive_explore": False},
    "log": {"sampling": "nln", "cost_mode": "indicator", "adaptive_explore": False},
    "dbas": {"sampling": "nln", "cost_mode": "dbas", "adaptive_explore": True},
}


def as_controller(params: dict, name: str) -> dict:
    """The parameters with the sampling law, collision cost and exploration
    setting of controller `name` ("vanilla", "log" or "dbas")."""
    out = dict(params)
    out.update(CONTROLLERS[name])
    return out


NAMED = {"quad_small": quad_small, "car": car, "quad_large": quad_large}

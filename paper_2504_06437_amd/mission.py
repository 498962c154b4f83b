"""Closed-loop navigation missions on synthetic layouts (Sec. VI).

The paper's three simulated missions, with its controller settings
(M = 1024 samples, N = 20 steps, dt = 0.02 s, its Sigma_u per vehicle,
gamma = 2, coarseness mu = 0.4 with the exploration feedback on):
  1. the planar quadrotor (Sec. V-A) at v_set = 1 m/s among three obstacles
     of radius 0.8 m;
  2. the ground vehicle (Sec. V-B) at v_set = 5 m/s among five obstacles of
     radius 4.3 m;
  3. the same vehicle at v_set = 8 m/s.
The indicators are those of the paper's mission table: collision-free
success, path tracking error and average speed.

The paper's layouts and cost weights are not published.  These layouts are
drawn from a seed: the obstacles flank the straight start-goal reference
path at even spacing on alternate sides, each with its edge a narrow,
passable clearance from the robot's body on the path.  The tracking weights
(a speed weight high enough to reach v_set within the 0.4 s horizon) and
the barrier weight R_B (0.3 for the quadrotor, 5 for the vehicle) are this
harness's choice, made with the FP64 reference controller on the CPU.  The numbers this harness gives are therefore its own,
not the paper's table.

This is the environment side of the loop.  It drives any controller that has
set_reference(x_ref) and step(x) -> u0 (the HIP Controller among them)
through the host plant, and never enters the controller's arithmetic.
"""
from __future__ import annotations

import math

import numpy as np

from . import plant
from . import workloads as W

# mission -> model, reference speed, obstacle count and radius, Sigma_u
# (variances, Sec. VI), the path length, where the goal counts as reached,
# the body's half-width across the path, the clearance range of the gaps, the
# tracking weights Q (state order of the model; Qf = 10 Q) and the barrier
# weight R_B
MISSIONS = {
    1: dict(model="quad5", v_set=1.0, J=3, radius=0.8, var=(0.4, 0.12), length=12.0, goal_tol=0.5,
            height=5.0, half_width=0.1, gap=(0.15, 0.5), Q=[0.5, 2.0, 1.0, 4.0, 4.0], r_b=0.3),
    2: dict(model="car", v_set=5.0, J=5, radius=4.3, var=(0.075, 2.0), length=120.0, goal_tol=3.0,
            height=0.0, half_width=1.5, gap=(0.3, 1.0), Q=[1.0, 1.0, 0.1, 5.0], r_b=5.0),
    3: dict(model="car", v_set=8.0, J=5, radius=4.3, var=(0.075, 2.0), length=120.0, goal_tol=3.0,
            height=0.0, half_width=1.5, gap=(0.3, 1.0), Q=[1.0, 1.0, 0.1, 5.0], r_b=5.0),
}


def layout(mission: int, seed: int = 0, samples: int = 1024, horizon: int = 20) -> dict:
    """The workload of one experiment: controller parameters, obstacles, start
    and goal.  `seed` draws the layout and seeds the controller's noise."""
    m = MISSIONS[mission]
    rng = np.random.Generator(np.random.PCG64(1000 * mission + seed))
    p = W.base_params(m["model"], samples, horizon, seed)
    p.update(dt=0.02, sigma=[math.sqrt(m["var"][0]), math.sqrt(m["var"][1])], gamma_u=2.0,
             adaptive_explore=True, explore_mu=0.4, Q=list(m["Q"]), Qf=[10.0 * q for q in m["Q"]],
             r_b=m["r_b"])
    L, r, J = m["length"], m["radius"], m["J"]
    start, goal = (0.0, m["height"]), (L, m["height"])
    side = 1.0 if rng.uniform() < 0.5 else -1.0
    obs = []
    for i in range(J):
        s = L * (i + 1) / (J + 1)
        off = side * (r + m["half_width"] + rng.uniform(*m["gap"]))
        obs.append([s, m["height"] + off, r])
        side = -side
    wl = W._finish(p, np.asarray(obs, dtype=np.float32), start, goal, m["v_set"], 0)
    wl["mission"] = mission
    wl["goal_tol"] = m["goal_tol"]
    # long enough to cover the path at half the reference speed
    wl["max_time"] = 2.0 * L / m["v_set"]
    return wl


def shape_points(params: dict, x) -> np.ndarray:
    """World positions [P, 2] of the body's shape points at state x (FP64)."""
    c, s = math.cos(float(x[2])), math.sin(float(x[2]))
    sh = np.asarray(params["shape"], dtype=np.float64).reshape(-1, 2)
    return np.stack([x[0] + sh[:, 0] * c - sh[:, 1] * s, x[1] + sh[:, 0] * s + sh[:, 1] * c], axis=1)


def collides(params: dict, obstacles, x) -> bool:
    """Does any shape point lie inside (or on) an obstacle circle?"""
    pts = shape_points(params, x)
    o = np.asarray(obstacles, dtype=np.float64).reshape(-1, 3)
    if o.size == 0:
        return False
    d2 = (pts[:, None, 0] - o[None, :, 0]) ** 2 + (pts[:, None, 1] - o[None, :, 1]) ** 2
    return bool(np.any(d2 <= o[None, :, 2] ** 2))


def path_error(wl: dict, x) -> float:
    """Distance from the robot's position to the start-goal reference segment."""
    a = np.asarray(wl["start"], dtype=np.float64)
    b = np.asarray(wl["goal"], dtype=np.float64)
    q = np.asarray(x[:2], dtype=np.float64)
    d = b - a
    t = float(np.clip(np.dot(q - a, d) / np.dot(d, d), 0.0, 1.0))
    return float(np.linalg.norm(q - (a + t * d)))


def run(controller, wl: dict) -> dict:
    """One closed-loop experiment: every period, re-anchor the reference at
    the robot's projection on the path, ask the controller for u0, and
    advance the true state by the plant.  It ends on reaching the goal, on a
    collision, or at the time limit."""
    p = wl["params"]
    x = np.asarray(wl["x0"], dtype=np.float32).copy()
    goal = np.asarray(wl["goal"], dtype=np.float64)
    steps = int(round(wl["max_time"] / p["dt"]))
    errs, dist = [], 0.0
    collided = reached = False
    k = 0
    for k in range(1, steps + 1):
        controller.set_reference(W.reference(wl, x))
        u = controller.step(x)
        xn = plant.advance(p, x, u)
        if not np.all(np.isfinite(xn)):
            collided = True
            break
        dist += float(np.linalg.norm(np.asarray(xn[:2], np.float64) - np.asarray(x[:2], np.float64)))
        x = xn
        errs.append(path_error(wl, x))
        if collides(p, wl["obstacles"], x):
            collided = True
            break
        if np.linalg.norm(np.asarray(x[:2], np.float64) - goal) <= wl["goal_tol"]:
            reached = True
            break
    t = k * p["dt"]
    return {"success": reached and not collided, "collided": collided, "reached": reached, "steps": k,
            "time": t, "error": float(np.mean(errs)) if errs else 0.0, "avg_speed": dist / t if t > 0 else 0.0}


def summarize(results: list) -> dict:
    """Success rate over all runs; tracking error and average speed over the
    successful ones (the paper leaves them blank when none succeeds)."""
    ok = [r for r in results if r["success"]]
    return {"runs": len(results), "success_pct": 100.0 * len(ok) / max(len(results), 1),
            "error_m": float(np.mean([r["error"] for r in ok])) if ok else None,
            "avg_speed": float(np.mean([r["avg_speed"] for r in ok])) if ok else None,
            "collisions": sum(1 for r in results if r["collided"]),
            "timeouts": sum(1 for r in results if not r["reached"] and not r["collided"])}


def run_mission(mission: int, runs: int = 10, first_seed: int = 0, device: int = 0, controller: str = "dbas") -> dict:
    """`runs` experiments of one mission with the HIP controller, as the
    paper's controller ("dbas") or one of its baselines ("vanilla", "log")."""
    from .controller import Controller
    results = []
    for sd in range(first_seed, first_seed + runs):
        wl = layout(mission, sd)
        c = Controller(W.as_controller(wl["params"], controller), device=device)
        try:
            c.load_workload(wl)
            results.append(run(c, wl))
        finally:
            c.close()
    out = summarize(results)
    out["mission"] = mission
    out["controller"] = controller
    return out


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="closed-loop missions on synthetic layouts")
    ap.add_argument("--mission", type=int, nargs="+", default=[1, 2, 3])
    ap.add_argument("--runs", type=int, default=10)
    args = ap.parse_args()
    for m in args.mission:
        print(json.dumps(run_mission(m, args.runs)), flush=True)

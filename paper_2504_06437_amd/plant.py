"""Simulated robots for closed-loop runs (the "GetStateEstimate" side of the
control loop): apply the controller's u0 to the true state for one period.

This is the environment, not the controller: the HIP library never calls it.
Explicit Euler of the same vehicle models (Sec. V-A/V-B), inputs saturated.
"""
from __future__ import annotations

import math

import numpy as np


def advance(params: dict, x, u) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    u0 = min(max(float(u[0]), params["u_min"][0]), params["u_max"][0])
    u1 = min(max(float(u[1]), params["u_min"][1]), params["u_max"][1])
    dt, m, g = params["dt"], params.get("mass", 0.5), params.get("gravity", 9.81)
    xn = x.copy()
    if params["model"] == "quad6":
        F = m * g + u0 + u1
        xn[0:3] = x[0:3] + x[3:6] * dt
        xn[3] = x[3] - F / m * math.sin(x[2]) * dt
        xn[4] = x[4] + (F / m * math.cos(x[2]) - g) * dt
        xn[5] = x[5] + (u1 - u0) * params.get("arm", 0.2) / params.get("inertia", 0.005) * dt
    elif params["model"] == "quad5":
        acc = (m * g + u1) / m
        xn[0:2] = x[0:2] + x[3:5] * dt
        xn[2] = x[2] + u0 * dt
        xn[3] = x[3] - acc * math.sin(x[2]) * dt
        xn[4] = x[4] + (acc * math.cos(x[2]) - g) * dt
    else:
        xn[0] = x[0] + x[3] * math.cos(x[2]) * dt
        xn[1] = x[1] + x[3] * math.sin(x[2]) * dt
        xn[2] = x[2] + x[3] * math.tan(u0) / params.get("wheelbase", 4.0) * dt
        xn[3] = x[3] + u1 * dt
    return xn.astype(np.float32)

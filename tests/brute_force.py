"""An independent brute-force evaluation of one DBaS-Log-MPPI iteration, in
pure Python floats (binary64), for tiny problems (K <= 4, T <= 3, J <= 2).

It exists only to pin the C oracle: it is written from the paper's
definitions, not from the oracle's code, and shares nothing with it (no
import, no helper, no table).  Where the paper leaves a choice open it takes
the reading the whole project states (the form of B, the 6-state quadrotor,
the costmap lookup, the noise counter map, the collision indicator of the
comparison controllers).

  * Philox4x32-10 (Salmon et al., SC'11) on Python integers.
  * Uniforms from the top 23 bits of a word, centred in their cell.
  * Sec. IV-C: du = sqrt(S_e) sigma n exp(mu_ln + sigma_ln z) (n, z standard
    normals by Box-Muller); Vanilla sampling drops the log-normal factor.
  * Sec. V-A/V-B dynamics as explicit Euler x + dt f(x, sat(u)).
  * Sec. III-B/IV-A: beta_t = sum B(h(x_t)) - gamma_B (beta_d - beta_{t-1}),
    B(h) = 1/max(h, h_eps); cost per Algorithm 1: sum over t = 1..T of
    q(x_t) + gamma_u U_t . v_t / (S_e sigma^2) + R_B beta_t, plus phi(x_T);
    or, for the comparison controllers, w_I 1[some h(x_t) < 0] in place of
    R_B beta_t.
  * Sec. III-A eq. control_update: softmax of -(S - min S)/lambda and the
    weighted average of the noise; Algorithm 1's shift.
"""
from __future__ import annotations

import math

MASK32 = 0xFFFFFFFF
STATE_DIM = {"quad6": 6, "quad5": 5, "car": 4}


# --- the generator -----------------------------------------------------------

def philox4x32_10(counter, key):
    """Ten Philox rounds: two 32x32 -> 64-bit products per round, the high
    halves xor-ed with the other words and the round key, the key bumped by
    the Weyl increments after every round."""
    x = [int(v) & MASK32 for v in counter]
    k = [int(v) & MASK32 for v in key]
    M0, M1 = 0xD2511F53, 0xCD9E8D57
    W0, W1 = 0x9E3779B9, 0xBB67AE85
    for _ in range(10):
        prod0 = M0 * x[0]
        prod1 = M1 * x[2]
        x = [((prod1 >> 32) ^ x[1] ^ k[0]) & MASK32, prod1 & MASK32,
             ((prod0 >> 32) ^ x[3] ^ k[1]) & MASK32, prod0 & MASK32]
        k = [(k[0] + W0) & MASK32, (k[1] + W1) & MASK32]
    return x


def to_uniform(word):
    return ((word >> 9) + 0.5) / float(1 << 23)


def noise(p, counter, S_e):
    """du[k][t][c]."""
    K, T = p["K"], p["T"]
    seed = int(p["seed"]) & 0xFFFFFFFFFFFFFFFF
    key = (seed & MASK32, seed >> 32)
    out = []
    for k in range(K):
        rows = []
        for t in range(T):
            w = philox4x32_10((k, t, counter & MASK32, counter >> 32), key)
            u = [to_uniform(v) for v in w]
            radius_n = math.sqrt(-2.0 * math.log(u[0]))
            radius_z = math.sqrt(-2.0 * math.log(u[2]))
            normals = (radius_n * math.cos(2.0 * math.pi * u[1]), radius_n * math.sin(2.0 * math.pi * u[1]))
            second = (radius_z * math.cos(2.0 * math.pi * u[3]), radius_z * math.sin(2.0 * math.pi * u[3]))
            row = []
            for c in range(2):
                d = math.sqrt(S_e) * p["sigma"][c] * normals[c]
                if p.get("sampling", "nln") == "nln":
                    d *= math.exp(p["mu_ln"] + p["sigma_ln"] * second[c])
                row.append(d)
            rows.append(row)
        out.append(rows)
    return out


# --- dynamics ------------------------------------------------------------------

def saturate(p, u):
    return [min(max(u[c], p["u_min"][c]), p["u_max"][c]) for c in range(2)]


def derivative(p, x, u):
    """f(x, u) of the continuous model (u already saturated)."""
    m, g = p["mass"], p["gravity"]
    if p["model"] == "quad6":
        thrust = (0.5 * m * g + u[0]) + (0.5 * m * g + u[1])
        torque = ((0.5 * m * g + u[1]) - (0.5 * m * g + u[0])) * p["arm"]
        return [x[3], x[4], x[5], -thrust * math.sin(x[2]) / m, thrust * math.cos(x[2]) / m - g,
                torque / p["inertia"]]
    if p["model"] == "quad5":
        a = (m * g + u[1]) / m
        return [x[3], x[4], u[0], -a * math.sin(x[2]), a * math.cos(x[2]) - g]
    return [x[3] * math.cos(x[2]), x[3] * math.sin(x[2]), x[3] * math.tan(u[0]) / p["wheelbase"], u[1]]


def euler(p, x, v):
    f = derivative(p, x, saturate(p, v))
    return [xi + p["dt"] * fi for xi, fi in zip(x, f)]


# --- geometry and the barrier ----------------------------------------------------

def body_points(p, x):
    c, s = math.cos(x[2]), math.sin(x[2])
    return [(x[0] + c * a - s * b, x[1] + s * a + c * b) for a, b in p["shape"]]


def bilinear(world, px, py):
    """Bilinear reading of a grid of signed distances stored at cell centres,
    clamped to the grid, and its two partial derivatives (zero along a
    clamped axis)."""
    sdf, (ox, oy), res = world["sdf"], world["origin"], world["res"]
    H, W = len(sdf), len(sdf[0])
    fx_raw, fy_raw = (px - ox) / res - 0.5, (py - oy) / res - 0.5
    gx, gy = min(max(fx_raw, 0.0), W - 1.0), min(max(fy_raw, 0.0), H - 1.0)
    i, j = min(int(math.floor(gx)), W - 2), min(int(math.floor(gy)), H - 2)
    ax, ay = gx - i, gy - j
    c00, c10, c01, c11 = sdf[j][i], sdf[j][i + 1], sdf[j + 1][i], sdf[j + 1][i + 1]
    value = c00 * (1 - ax) * (1 - ay) + c10 * ax * (1 - ay) + c01 * (1 - ax) * ay + c11 * ax * ay
    dvx = 0.0 if fx_raw != gx else ((c10 - c00) * (1 - ay) + (c11 - c01) * ay) / res
    dvy = 0.0 if fy_raw != gy else ((c01 - c00) * (1 - ax) + (c11 - c10) * ax) / res
    return value, dvx, dvy


def constraint_values(p, world, x):
    """Every h of state x: one per (shape point, circle), one per shape point
    for the costmap.  Each entry is (h, dh/dpx, dh/dpy)."""
    hs = []
    for (px, py) in body_points(p, x):
        for (cx, cy, r) in world["obstacles"]:
            hs.append(((px - cx) ** 2 + (py - cy) ** 2 - r * r, 2.0 * (px - cx), 2.0 * (py - cy)))
        if world.get("sdf") is not None:
            hs.append(bilinear(world, px, py))
    return hs


def fused_barrier(p, world, x):
    return sum(1.0 / max(h, p["h_eps"]) for h, _, _ in constraint_values(p, world, x))


def clearance(p, world, x):
    return min((h for h, _, _ in constraint_values(p, world, x)), default=math.inf)


def sensitivity(p, world, x):
    """Bound on the change of the fused barrier per metre of shape-point move
    (at most `sens_reach` per coordinate): each term's |grad h|_1 times the
    largest |dB/dh| of B(h) = 1/max(h, h_eps) for h within |grad h|_1 reach
    of its value (first order, over the unclamped terms, at reach 0)."""
    reach, eps = p.get("sens_reach", 0.0), p["h_eps"]
    total = 0.0
    for h, dx, dy in constraint_values(p, world, x):
        g = abs(dx) + abs(dy)
        lowest = h - reach * g
        if h + reach * g > eps:
            total += g / max(lowest, eps) ** 2
    return total


# --- one iteration ---------------------------------------------------------------

def rollout(p, world, x0, U, du_k, x_ref, S_e, beta_d):
    """Cost, smallest clearance over steps 1..T and the cost's barrier
    sensitivity of one sample."""
    indicator = p.get("cost_mode", "dbas") == "indicator"
    n = STATE_DIM[p["model"]]
    x = list(x0)
    beta = 0.0 if indicator else fused_barrier(p, world, x)
    total, lowest, sens = 0.0, math.inf, 0.0
    for t in range(p["T"]):
        v = [U[t][c] + du_k[t][c] for c in range(2)]
        x = euler(p, x, v)
        tracking = sum(p["Q"][a] * (x[a] - x_ref[t + 1][a]) ** 2 for a in range(n))
        control = sum(p["gamma_u"] * U[t][c] * v[c] / (S_e * p["sigma"][c] ** 2)
                      for c in range(2) if p["sigma"][c] > 0.0)
        if indicator:
            collision = p.get("collision_weight", 1000.0) * (1.0 if clearance(p, world, x) < 0.0 else 0.0)
        else:
            beta = fused_barrier(p, world, x) - p["gamma_b"] * (beta_d - beta)
            collision = p["r_b"] * beta
            sens += p["r_b"] / (1.0 - p["gamma_b"]) * sensitivity(p, world, x)
        total += tracking + control + collision
        lowest = min(lowest, clearance(p, world, x))
    total += sum(p["Qf"][a] * (x[a] - x_ref[p["T"]][a]) ** 2 for a in range(n))
    return total, lowest, sens


def iterate(p, world, x0, U, x_ref, S_e, counter):
    """One iteration; returns the same quantities as the oracle's step."""
    K, T = p["K"], p["T"]
    U = [list(map(float, row)) for row in U]
    x_ref = [list(map(float, row)) for row in x_ref]
    x0 = [float(v) for v in x0]
    du = noise(p, counter, S_e)
    beta_d = fused_barrier(p, world, x_ref[T])
    S, clear, sens = [], [], []
    for k in range(K):
        s, c, e = rollout(p, world, x0, U, du[k], x_ref, S_e, beta_d)
        S.append(s)
        clear.append(c)
        sens.append(e)
    rho = min(S)
    e = [math.exp(-(s - rho) / p["lambda"]) for s in S]
    eta = sum(e)
    w = [v / eta for v in e]
    Ustar = [[U[t][c] + sum(w[k] * du[k][t][c] for k in range(K)) for c in range(2)] for t in range(T)]
    last = [0.0, 0.0] if p.get("init_mode", "repeat") == "zero" else list(Ustar[T - 1])
    Unext = [list(row) for row in Ustar[1:]] + [last]
    return {"du": du, "S": S, "w": w, "rho": rho, "eta": eta, "Ustar": Ustar, "Unext": Unext,
            "u0": list(Ustar[0]), "beta0": fused_barrier(p, world, x0), "beta_d": beta_d,
            "clear": clear, "sens": sens}

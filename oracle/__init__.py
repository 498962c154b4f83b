"""FP64 CPU oracle for the DBaS-Log-MPPI iteration -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding in ``paper_2504_06437_amd``) never does, and this package imports
nothing from it: both sides receive the same plain parameter dictionaries and
arrays from the seeded generators in ``paper_2504_06437_amd.workloads`` (which
hold no arithmetic of the method).

The numerics live in ``oracle.c`` (plain C, FP64, libm); this module only
marshals numpy arrays through ctypes -- except the Savitzky-Golay smoothing of
the update (``sgf``), written here in numpy from its definition.  See
``oracle.h`` for which passage of the paper each C function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

MODELS = {"quad6": 0, "quad5": 1, "car": 2}
STATE_DIM = {"quad6": 6, "quad5": 5, "car": 4}
OK, INVALID, NUMERIC = 0, 1, 4
PMAX = 16


GCC_FLAGS = ["-O2", "-fno-fast-math", "-std=c99", "-Wall", "-Wextra", "-fopenmp", "-fPIC", "-shared"]
SAMPLING = {"nln": 0, "normal": 1}
COST_MODE = {"dbas": 0, "indicator": 1}


def compile_library(src: str, out: str, include: str | None = None) -> str:
    """Compile an oracle source file into a shared library (gcc -O2, no
    fast-math, OpenMP over samples)."""
    tmp = out + ".tmp"
    inc = ["-I", include] if include else []
    subprocess.check_call(["gcc", *GCC_FLAGS, *inc, src, "-o", tmp, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile liboracle.so."""
    if force or not os.path.exists(LIB_PATH):
        compile_library(os.path.join(_HERE, "oracle.c"), LIB_PATH)
    return LIB_PATH


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("model", ctypes.c_int), ("K", ctypes.c_int), ("T", ctypes.c_int),
        ("dt", ctypes.c_double),
        ("mass", ctypes.c_double), ("gravity", ctypes.c_double), ("arm", ctypes.c_double),
        ("inertia", ctypes.c_double), ("wheelbase", ctypes.c_double),
        ("u_min", ctypes.c_double * 2), ("u_max", ctypes.c_double * 2),
        ("sigma", ctypes.c_double * 2),
        ("mu_ln", ctypes.c_double), ("sigma_ln", ctypes.c_double),
        ("lam", ctypes.c_double), ("gamma_u", ctypes.c_double), ("gamma_b", ctypes.c_double),
        ("r_b", ctypes.c_double), ("h_eps", ctypes.c_double),
        ("Q", ctypes.c_double * 6), ("Qf", ctypes.c_double * 6),
        ("P", ctypes.c_int), ("shape", (ctypes.c_double * 2) * PMAX),
        ("seed", ctypes.c_uint64), ("init_zero", ctypes.c_int),
        ("sampling", ctypes.c_int), ("cost_mode", ctypes.c_int), ("collision_weight", ctypes.c_double),
        ("sens_reach", ctypes.c_double),
    ]


class _World(ctypes.Structure):
    _fields_ = [
        ("J", ctypes.c_int), ("obs", ctypes.POINTER(ctypes.c_double)),
        ("map_w", ctypes.c_int), ("map_h", ctypes.c_int),
        ("map_x0", ctypes.c_double), ("map_y0", ctypes.c_double), ("map_res", ctypes.c_double),
        ("sdf", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def _load(path: str):
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    cp = ctypes.POINTER(_Cfg)
    wp = ctypes.POINTER(_World)
    L.orc_set_threads.argtypes = [ctypes.c_int]
    L.orc_set_threads.restype = ctypes.c_int
    L.orc_threads.restype = ctypes.c_int
    L.orc_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
    L.orc_uniform.argtypes = [ctypes.c_uint32]
    L.orc_uniform.restype = ctypes.c_double
    L.orc_noise_words.argtypes = [cp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32)]
    L.orc_noise.argtypes = [cp, ctypes.c_double, ctypes.c_uint64, dp]
    L.orc_dynamics.argtypes = [cp, dp, dp, dp]
    L.orc_shape_points.argtypes = [cp, dp, dp]
    L.orc_sdf_lookup.argtypes = [wp, ctypes.c_double, ctypes.c_double]
    L.orc_sdf_lookup.restype = ctypes.c_double
    L.orc_fused_barrier.argtypes = [cp, wp, dp]
    L.orc_fused_barrier.restype = ctypes.c_double
    L.orc_barrier_sensitivity.argtypes = [cp, wp, dp]
    L.orc_barrier_sensitivity.restype = ctypes.c_double
    L.orc_collision.argtypes = [cp, wp, dp]
    L.orc_collision.restype = ctypes.c_int
    L.orc_rollout_one.argtypes = [cp, wp, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double, dp, dp, dp, dp]
    L.orc_rollout_one.restype = ctypes.c_double
    L.orc_exploration.argtypes = [cp, wp, dp, dp, ctypes.c_double, ctypes.c_double, dp]
    L.orc_exploration.restype = ctypes.c_double
    L.orc_clearance.argtypes = [cp, wp, dp]
    L.orc_clearance.restype = ctypes.c_double
    L.orc_margins.argtypes = [cp, wp, dp, dp, dp, dp]
    L.orc_weights.argtypes = [dp, ctypes.c_int, ctypes.c_double, dp, dp, dp]
    L.orc_weights.restype = ctypes.c_int
    L.orc_update.argtypes = [dp, dp, dp, ctypes.c_int, ctypes.c_int, dp]
    L.orc_shift.argtypes = [cp, dp, dp]
    L.orc_step.argtypes = [cp, wp, dp, dp, dp, ctypes.c_double, ctypes.c_uint64,
                           dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp, dp]
    L.orc_step.restype = ctypes.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = _load(LIB_PATH)
        _lib.orc_set_threads(int(os.environ.get("ORACLE_THREADS", "1")))
    return _lib


class use_library:
    """Context manager: run the wrappers below on another build of the oracle
    (a library compiled by ``compile_library``), then restore the usual one.
    The tests use it to check that planted mistakes are caught."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = _load(self.path)
        _lib.orc_set_threads(self.saved.orc_threads())
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def set_threads(n: int) -> int:
    """Threads of the oracle's per-sample loops (results do not depend on it)."""
    return lib().orc_set_threads(int(n))


def threads() -> int:
    return lib().orc_threads()


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def make_cfg(params: dict) -> _Cfg:
    """Fill the oracle's own config struct from a plain parameter dict."""
    c = _Cfg()
    c.model = MODELS[params["model"]]
    c.K = int(params["K"])
    c.T = int(params["T"])
    c.dt = float(params["dt"])
    c.mass = float(params.get("mass", 0.5))
    c.gravity = float(params.get("gravity", 9.81))
    c.arm = float(params.get("arm", 0.2))
    c.inertia = float(params.get("inertia", 0.005))
    c.wheelbase = float(params.get("wheelbase", 4.0))
    for i in range(2):
        c.u_min[i] = float(params["u_min"][i])
        c.u_max[i] = float(params["u_max"][i])
        c.sigma[i] = float(params["sigma"][i])
    c.mu_ln = float(params["mu_ln"])
    c.sigma_ln = float(params["sigma_ln"])
    c.lam = float(params["lambda"])
    c.gamma_u = float(params["gamma_u"])
    c.gamma_b = float(params["gamma_b"])
    c.r_b = float(params["r_b"])
    c.h_eps = float(params["h_eps"])
    n = STATE_DIM[params["model"]]
    for a in range(n):
        c.Q[a] = float(params["Q"][a])
        c.Qf[a] = float(params["Qf"][a])
    shape = np.asarray(params["shape"], dtype=np.float64).reshape(-1, 2)
    c.P = shape.shape[0]
    for i in range(c.P):
        c.shape[i][0] = shape[i, 0]
        c.shape[i][1] = shape[i, 1]
    c.seed = int(params["seed"]) & 0xFFFFFFFFFFFFFFFF
    c.init_zero = 1 if params.get("init_mode", "repeat") == "zero" else 0
    c.sampling = SAMPLING[params.get("sampling", "nln")]
    c.cost_mode = COST_MODE[params.get("cost_mode", "dbas")]
    c.collision_weight = float(params.get("collision_weight", 1000.0))
    c.sens_reach = float(params.get("sens_reach", 0.0))
    return c


class World:
    """Obstacles (J x 3: cx, cy, r) and an optional costmap, held as FP64."""

    def __init__(self, obstacles=None, sdf=None, map_origin=(0.0, 0.0), map_res=1.0):
        obs = np.zeros((0, 3)) if obstacles is None else _f64(obstacles).reshape(-1, 3)
        self._obs = obs if obs.size else np.zeros((1, 3))
        self.s = _World()
        self.s.J = obs.shape[0]
        self.s.obs = _dp(self._obs)
        if sdf is not None:
            self._sdf = _f64(sdf)
            self.s.map_h, self.s.map_w = self._sdf.shape
            self.s.map_x0, self.s.map_y0 = float(map_origin[0]), float(map_origin[1])
            self.s.map_res = float(map_res)
            self.s.sdf = _dp(self._sdf)
        else:
            self._sdf = None
            self.s.map_w = self.s.map_h = 0
            self.s.sdf = ctypes.POINTER(ctypes.c_double)()

    @classmethod
    def from_workload(cls, wl: dict) -> "World":
        m = wl.get("map")
        if m is None:
            return cls(wl["obstacles"])
        return cls(wl["obstacles"], m["sdf"], m["origin"], m["res"])


# ----------------------------------------------------------------------------
# thin wrappers
# ----------------------------------------------------------------------------

def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniform(r: int) -> float:
    return lib().orc_uniform(int(r) & 0xFFFFFFFF)


def noise_words(params: dict, counter: int) -> np.ndarray:
    cfg = make_cfg(params)
    out = np.zeros((cfg.K, cfg.T, 4), dtype=np.uint32)
    lib().orc_noise_words(ctypes.byref(cfg), int(counter),
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
    return out


def noise(params: dict, counter: int, S_e: float = 1.0) -> np.ndarray:
    """du[k, t, c]."""
    cfg = make_cfg(params)
    out = np.zeros((cfg.K, cfg.T, 2))
    lib().orc_noise(ctypes.byref(cfg), float(S_e), int(counter), _dp(out))
    return out


def dynamics(params: dict, x, v) -> np.ndarray:
    cfg = make_cfg(params)
    x = _f64(x)
    v = _f64(v)
    xn = np.zeros_like(x)
    lib().orc_dynamics(ctypes.byref(cfg), _dp(x), _dp(v), _dp(xn))
    return xn


def shape_points(params: dict, x) -> np.ndarray:
    cfg = make_cfg(params)
    x = _f64(x)
    out = np.zeros((cfg.P, 2))
    lib().orc_shape_points(ctypes.byref(cfg), _dp(x), _dp(out))
    return out


def sdf_lookup(world: World, px: float, py: float) -> float:
    return lib().orc_sdf_lookup(ctypes.byref(world.s), float(px), float(py))


def fused_barrier(params: dict, world: World, x) -> float:
    cfg = make_cfg(params)
    x = _f64(x)
    return lib().orc_fused_barrier(ctypes.byref(cfg), ctypes.byref(world.s), _dp(x))


def rollout_one(params: dict, world: World, x0, U, du_k, x_ref, S_e=1.0, beta_d=0.0, with_clearance=False):
    """Returns (S, X[(T+1), n], beta[T+1]) (+ the smallest clearance over
    steps 1..T and the barrier sensitivity when with_clearance)."""
    cfg = make_cfg(params)
    n = STATE_DIM[params["model"]]
    x0, U, du_k, x_ref = _f64(x0), _f64(U), _f64(du_k), _f64(x_ref)
    X = np.zeros((cfg.T + 1, n))
    beta = np.zeros(cfg.T + 1)
    mh, sens = ctypes.c_double(), ctypes.c_double()
    S = lib().orc_rollout_one(ctypes.byref(cfg), ctypes.byref(world.s), _dp(x0), _dp(U), _dp(du_k),
                              _dp(x_ref), float(S_e), float(beta_d), _dp(X), _dp(beta), ctypes.byref(mh),
                              ctypes.byref(sens))
    if with_clearance:
        return S, X, beta, mh.value, sens.value
    return S, X, beta


def exploration(params: dict, world: World, x0, Ustar, beta_d: float, mu: float):
    """(S_e, C_B): the next exploration rate mu ln(e + C_B) and the barrier
    cost of the noise-free rollout of U* from x0 (Sec. IV-B)."""
    cfg = make_cfg(params)
    cb = ctypes.c_double()
    se = lib().orc_exploration(ctypes.byref(cfg), ctypes.byref(world.s), _dp(_f64(x0)), _dp(_f64(Ustar)),
                               float(beta_d), float(mu), ctypes.byref(cb))
    return se, cb.value


def barrier_sensitivity(params: dict, world: World, x) -> float:
    cfg = make_cfg(params)
    return lib().orc_barrier_sensitivity(ctypes.byref(cfg), ctypes.byref(world.s), _dp(_f64(x)))


def collision(params: dict, world: World, x) -> int:
    cfg = make_cfg(params)
    return lib().orc_collision(ctypes.byref(cfg), ctypes.byref(world.s), _dp(_f64(x)))


def margins(params: dict, world: World, x0, U, du) -> np.ndarray:
    """min over t = 1..T of |clearance(x_t)| for every sample's rollout."""
    cfg = make_cfg(params)
    du = _f64(du)
    out = np.zeros(cfg.K)
    lib().orc_margins(ctypes.byref(cfg), ctypes.byref(world.s), _dp(_f64(x0)), _dp(_f64(U)), _dp(du), _dp(out))
    return out


def clearance(params: dict, world: World, x) -> float:
    cfg = make_cfg(params)
    x = _f64(x)
    return lib().orc_clearance(ctypes.byref(cfg), ctypes.byref(world.s), _dp(x))


def weights(S, lam: float):
    """Returns (status, w, rho, eta)."""
    S = _f64(S)
    w = np.zeros_like(S)
    rho = ctypes.c_double()
    eta = ctypes.c_double()
    st = lib().orc_weights(_dp(S), S.size, float(lam), _dp(w), ctypes.byref(rho), ctypes.byref(eta))
    return st, w, rho.value, eta.value


def update(U, du, w) -> np.ndarray:
    U, du, w = _f64(U), _f64(du), _f64(w)
    K, T = du.shape[0], du.shape[1]
    out = np.zeros((T, 2))
    lib().orc_update(_dp(U), _dp(du), _dp(w), K, T, _dp(out))
    return out


def shift(params: dict, Ustar) -> np.ndarray:
    cfg = make_cfg(params)
    Ustar = _f64(Ustar)
    out = np.zeros_like(Ustar)
    lib().orc_shift(ctypes.byref(cfg), _dp(Ustar), _dp(out))
    return out


def sgf(y, half_window: int, order: int) -> np.ndarray:
    """Savitzky-Golay smoothing (Algorithm 1's SGF) of y along its first axis,
    from the definition: every output point is the value, at that point, of
    the least-squares polynomial of degree `order` through the 2m+1 samples
    of its window, m = half_window; near the ends the window is the first
    (or last) 2m+1 samples, so the fitted polynomial is evaluated off-centre.
    Each column is smoothed on its own.  m = 0 returns y unchanged."""
    y = np.asarray(y, dtype=np.float64)
    m = int(half_window)
    if m == 0:
        return y.copy()
    n = y.shape[0]
    W = 2 * m + 1
    assert n >= W and 0 <= order < W
    out = np.empty_like(y)
    for t in range(n):
        start = min(max(t - m, 0), n - W)
        xs = np.arange(start, start + W, dtype=np.float64) - t
        V = np.vander(xs, order + 1, increasing=True)
        coef, *_ = np.linalg.lstsq(V, y[start:start + W], rcond=None)
        out[t] = coef[0]            # the polynomial's value at x = 0, i.e. at t
    return out


def step(params: dict, world: World, x0, U, x_ref, S_e: float, counter: int, diagnostics: bool = True) -> dict:
    """One full iteration; returns every intermediate as FP64 arrays.  With
    params["sgf_half_window"] = m > 0 the weighted increment is smoothed by
    sgf(., m, params["sgf_order"]) before it is added to U (Algorithm 1).
    diagnostics=False skips the per-sample clearance and sensitivity (the
    tolerance diagnostics; "clear" and "sens" are then None): the iteration
    alone, as the CPU baseline times it."""
    cfg = make_cfg(params)
    K, T = cfg.K, cfg.T
    x0, U, x_ref = _f64(x0), _f64(U), _f64(x_ref)
    du = np.zeros((K, T, 2))
    S = np.zeros(K)
    w = np.zeros(K)
    Ustar = np.zeros((T, 2))
    Unext = np.zeros((T, 2))
    u0 = np.zeros(2)
    clear = np.zeros(K) if diagnostics else None
    sens = np.zeros(K) if diagnostics else None
    null = ctypes.POINTER(ctypes.c_double)()
    sc = [ctypes.c_double() for _ in range(4)]
    st = lib().orc_step(ctypes.byref(cfg), ctypes.byref(world.s), _dp(x0), _dp(U), _dp(x_ref),
                        float(S_e), int(counter), _dp(du), _dp(S), _dp(w), _dp(Ustar), _dp(Unext),
                        _dp(u0), *[ctypes.byref(s) for s in sc], _dp(clear) if diagnostics else null,
                        _dp(sens) if diagnostics else null)
    m = int(params.get("sgf_half_window", 0))
    if m > 0 and st == OK:
        inc = np.einsum("k,ktc->tc", w, du)
        Ustar = U + sgf(inc, m, int(params.get("sgf_order", 2)))
        Unext = shift(params, Ustar)
        u0 = Ustar[0].copy()
    return {"status": st, "du": du, "S": S, "w": w, "Ustar": Ustar, "Unext": Unext, "u0": u0,
            "rho": sc[0].value, "eta": sc[1].value, "beta0": sc[2].value, "beta_d": sc[3].value,
            "clear": clear, "sens": sens}

"""Python handles over the C ABI: Controller (one MPPI controller), Batch
(many controllers in one persistent graph launch) and Server (continuous
batching).  Marshalling only; device buffers for the device-pointer calls come
from `hip.DeviceArray`."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib as A


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _fp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def make_config(params: dict) -> A.Config:
    """Fill the C config from a plain parameter dict (see workloads.base_params)."""
    c = A.Config()
    c.abi_version = A.ABI_VERSION
    c.model = A.MODELS[params["model"]]
    c.K = int(params["K"])
    c.T = int(params["T"])
    c.dt = float(params["dt"])
    for f in ("mass", "gravity", "arm", "inertia", "wheelbase"):
        setattr(c, f, float(params.get(f, {"mass": 0.5, "gravity": 9.81, "arm": 0.2, "inertia": 0.005,
                                         "wheelbase": 4.0}[f])))
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
    n = A.STATE_DIM[params["model"]]
    for a in range(n):
        c.Q[a] = float(params["Q"][a])
        c.Qf[a] = float(params["Qf"][a])
    shape = np.asarray(params["shape"], dtype=np.float32).reshape(-1, 2)
    c.P = shape.shape[0]
    for i in range(c.P):
        c.shape[i][0] = float(shape[i, 0])
        c.shape[i][1] = float(shape[i, 1])
    c.seed = int(params["seed"]) & 0xFFFFFFFFFFFFFFFF
    c.normaliser = A.NORMALISER[params.get("normaliser", "auto")]
    c.init_mode = A.INIT_MODE[params.get("init_mode", "repeat")]
    c.tile_samples = int(params.get("tile_samples", 0))
    c.export_noise = int(bool(params.get("export_noise", False)))
    c.adaptive_explore = int(bool(params.get("adaptive_explore", False)))
    c.explore_mu = float(params.get("explore_mu", 0.4))
    c.sgf_half_window = int(params.get("sgf_half_window", 0))
    c.sgf_order = int(params.get("sgf_order", 2))
    c.sampling = A.SAMPLING[params.get("sampling", "nln")]
    c.cost_mode = A.COST_MODE[params.get("cost_mode", "dbas")]
    c.collision_weight = float(params.get("collision_weight", 1000.0))
    return c


class Controller:
    """One DBaS-Log-MPPI controller living on a GPU."""

    def __init__(self, params: dict, device: int = 0, stream=None):
        self.L = A.load()
        self.params = dict(params)
        self.K, self.T = int(params["K"]), int(params["T"])
        self.n = A.STATE_DIM[params["model"]]
        cfg = make_config(params)
        dev = A.Device(device, ctypes.c_void_p(stream) if stream else None)
        h = ctypes.c_void_p()
        st = self.L.mppi_create(ctypes.byref(cfg), ctypes.byref(dev), ctypes.byref(h))
        if st != A.OK:
            raise A.MppiError(st, "mppi_create: " + (self.L.mppi_last_error(None) or b"").decode())
        self.h = h

    # -- lifecycle --
    def close(self):
        if getattr(self, "h", None):
            self.L.mppi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st: int, what: str):
        if st != A.OK:
            raise A.MppiError(st, f"{what}: {self.L.mppi_last_error(self.h).decode()}")

    # -- inputs --
    def set_obstacles(self, obs):
        o = _f32(obs).reshape(-1, 3)
        self._check(self.L.mppi_set_obstacles(self.h, o.shape[0], o.ctypes.data if o.size else None, A.MEM_HOST),
                    "mppi_set_obstacles")

    def set_costmap(self, sdf, origin, res):
        if sdf is None:
            self._check(self.L.mppi_set_costmap(self.h, 0, 0, 0.0, 0.0, 0.0, None, A.MEM_HOST), "mppi_set_costmap")
            return
        s = _f32(sdf)
        H, W = s.shape
        self._check(self.L.mppi_set_costmap(self.h, W, H, float(origin[0]), float(origin[1]), float(res),
                                            s.ctypes.data, A.MEM_HOST), "mppi_set_costmap")

    def set_reference(self, x_ref):
        r = _f32(x_ref).reshape(self.T + 1, self.n)
        self._check(self.L.mppi_set_reference(self.h, r.ctypes.data, A.MEM_HOST), "mppi_set_reference")

    def set_exploration(self, S_e: float):
        self._check(self.L.mppi_set_exploration(self.h, float(S_e)), "mppi_set_exploration")

    def set_controls(self, U):
        u = _f32(U).reshape(self.T, 2)
        self._check(self.L.mppi_set_controls(self.h, u.ctypes.data, A.MEM_HOST), "mppi_set_controls")

    def load_workload(self, wl: dict):
        self.set_obstacles(wl["obstacles"])
        if wl.get("map") is not None:
            m = wl["map"]
            self.set_costmap(m["sdf"], m["origin"], m["res"])
        self.set_reference(wl["x_ref"])
        self.set_controls(wl["U0"])

    # -- iteration --
    def step(self, x0) -> np.ndarray:
        x = _f32(x0)
        u0 = np.zeros(2, dtype=np.float32)
        self._check(self.L.mppi_step(self.h, _fp(x), _fp(u0)), "mppi_step")
        return u0

    def step_status(self, x0):
        """Like step, but returns (status, u0) instead of raising on NUMERIC."""
        x = _f32(x0)
        u0 = np.zeros(2, dtype=np.float32)
        st = self.L.mppi_step(self.h, _fp(x), _fp(u0))
        return st, u0

    def step_async(self, x0_dev_ptr: int, u0_dev_ptr: int = 0):
        """Stream-ordered step with device pointers (e.g. tensor.data_ptr())."""
        self._check(self.L.mppi_step_async(self.h, ctypes.c_void_p(x0_dev_ptr),
                                           ctypes.c_void_p(u0_dev_ptr) if u0_dev_ptr else None),
                    "mppi_step_async")

    def synchronize(self) -> int:
        return self.L.mppi_synchronize(self.h)

    @property
    def stream(self) -> int:
        return self.L.mppi_stream(self.h) or 0

    # -- kernel timing --
    def profile(self, every=1):
        """Time the kernels of every `every`-th iteration (True = 1); 0 or
        False turns kernel timing off."""
        self._check(self.L.mppi_profile_enable(self.h, int(every)), "mppi_profile_enable")

    def profile_read(self) -> dict:
        pr = A.Profile()
        self._check(self.L.mppi_profile_read(self.h, ctypes.byref(pr)), "mppi_profile_read")
        return {"iterations": pr.iterations, "dropped": pr.dropped, "rollout_ms": pr.rollout_ms,
                "update_ms": pr.update_ms}

    # -- inspection --
    def controls(self) -> np.ndarray:
        U = np.zeros((self.T, 2), dtype=np.float32)
        self._check(self.L.mppi_get_controls(self.h, _fp(U)), "mppi_get_controls")
        return U

    def last_optimal(self) -> np.ndarray:
        U = np.zeros((self.T, 2), dtype=np.float32)
        self._check(self.L.mppi_get_last_optimal(self.h, _fp(U)), "mppi_get_last_optimal")
        return U

    def costs(self) -> np.ndarray:
        S = np.zeros(self.K)
        self._check(self.L.mppi_get_costs(self.h, S.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "mppi_get_costs")
        return S

    def weights(self) -> np.ndarray:
        w = np.zeros(self.K)
        self._check(self.L.mppi_get_weights(self.h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                    "mppi_get_weights")
        return w

    def noise(self) -> np.ndarray:
        du = np.zeros((self.K, self.T, 2), dtype=np.float32)
        self._check(self.L.mppi_get_noise(self.h, _fp(du)), "mppi_get_noise")
        return du

    def info(self) -> dict:
        i = A.StepInfo()
        self._check(self.L.mppi_get_step_info(self.h, ctypes.byref(i)), "mppi_get_step_info")
        return {f: getattr(i, f) for f, _ in A.StepInfo._fields_}

    def philox_words(self, counter: int) -> np.ndarray:
        w = np.zeros((self.K, self.T, 4), dtype=np.uint32)
        self._check(self.L.mppi_get_philox_words(self.h, int(counter),
                                                 w.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))),
                    "mppi_get_philox_words")
        return w

    def get_state(self) -> dict:
        U = np.zeros((self.T, 2), dtype=np.float32)
        s = A.State(0, 0.0, self.T, _fp(U))
        self._check(self.L.mppi_get_state(self.h, ctypes.byref(s)), "mppi_get_state")
        return {"counter": int(s.counter), "S_e": float(s.S_e), "U": U}

    def set_state(self, state: dict):
        U = _f32(state["U"]).reshape(self.T, 2)
        s = A.State(int(state["counter"]), float(state["S_e"]), self.T, _fp(U))
        self._check(self.L.mppi_set_state(self.h, ctypes.byref(s)), "mppi_set_state")


class Batch:
    """Many controllers stepped by one persistent, graph-captured launch."""

    def __init__(self, controllers, device: int = 0, stream=None):
        self.L = A.load()
        self.ctrls = list(controllers)
        arr = (ctypes.c_void_p * len(self.ctrls))(*[c.h.value for c in self.ctrls])
        dev = A.Device(device, ctypes.c_void_p(stream) if stream else None)
        b = ctypes.c_void_p()
        st = self.L.mppi_batch_create(arr, len(self.ctrls), ctypes.byref(dev), ctypes.byref(b))
        if st != A.OK:
            raise A.MppiError(st, "mppi_batch_create: " + (self.L.mppi_batch_last_error(None) or b"").decode())
        self.b = b

    def close(self):
        if getattr(self, "b", None):
            self.L.mppi_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, x0s):
        n = len(self.ctrls)
        X = np.zeros((n, A.NMAX), dtype=np.float32)
        for i, x in enumerate(x0s):
            x = np.asarray(x, dtype=np.float32)
            X[i, :x.size] = x
        u0s = np.zeros((n, 2), dtype=np.float32)
        sts = (ctypes.c_int32 * n)()
        st = self.L.mppi_batch_step(self.b, _fp(X), _fp(u0s), sts)
        if st not in (A.OK, A.E_NUMERIC):
            raise A.MppiError(st, "mppi_batch_step: " + self.L.mppi_batch_last_error(self.b).decode())
        return u0s, np.array(list(sts), dtype=np.int32)


class Server:
    """Continuous-batching server: robots with resident state, requests
    admitted by launch slots and a device-memory budget for sample scratch."""

    def __init__(self, budget_bytes: int = 256 << 20, max_slots: int = 256, streams: int = 3,
                 max_batch: int = 64, device: int = 0):
        self.L = A.load()
        cfg = A.ServerConfig()
        cfg.abi_version = A.ABI_VERSION
        cfg.device = device
        cfg.budget_bytes = int(budget_bytes)
        cfg.max_slots = int(max_slots)
        cfg.streams = int(streams)
        cfg.max_batch = int(max_batch)
        s = ctypes.c_void_p()
        st = self.L.mppi_server_create(ctypes.byref(cfg), ctypes.byref(s))
        if st != A.OK:
            raise A.MppiError(st, "mppi_server_create: " + (self.L.mppi_server_last_error(None) or b"").decode())
        self.s = s
        self.dims = []

    def close(self):
        if getattr(self, "s", None):
            self.L.mppi_server_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, st, what):
        raise A.MppiError(st, f"{what}: " + self.L.mppi_server_last_error(self.s).decode())

    def add_robot(self, params: dict, obstacles) -> int:
        cfg = make_config(params)
        obs = _f32(obstacles).reshape(-1, 3)
        rid = ctypes.c_int32()
        st = self.L.mppi_server_add_robot(self.s, ctypes.byref(cfg), obs.shape[0],
                                          obs.ctypes.data if obs.shape[0] else None, ctypes.byref(rid))
        if st != A.OK:
            self._err(st, "mppi_server_add_robot")
        self.dims.append((A.STATE_DIM[params["model"]], int(params["T"])))
        return rid.value

    def now(self) -> float:
        return self.L.mppi_server_now(self.s)

    def submit(self, rid: int, x0, x_ref=None, t_arrival: float | None = None) -> int:
        # an unknown id goes through to the library, which rejects it
        n, T = self.dims[rid] if 0 <= rid < len(self.dims) else (A.NMAX, 0)
        x = _f32(x0).reshape(-1)
        assert x.size >= n
        ref = None
        if x_ref is not None:
            ref = _f32(x_ref).reshape(T + 1, n)
        tk = ctypes.c_int64()
        st = self.L.mppi_server_submit(self.s, rid, _fp(x), _fp(ref) if ref is not None else None,
                                       self.now() if t_arrival is None else float(t_arrival), ctypes.byref(tk))
        if st != A.OK:
            self._err(st, "mppi_server_submit")
        return tk.value

    def poll(self, ticket: int):
        """(u0, latency_s, status) once done, else None."""
        u0 = np.zeros(2, dtype=np.float32)
        lat = ctypes.c_double()
        sts = ctypes.c_int32()
        st = self.L.mppi_server_poll(self.s, ticket, _fp(u0), ctypes.byref(lat), ctypes.byref(sts))
        if st == A.E_BUSY:
            return None
        if st != A.OK:
            self._err(st, "mppi_server_poll")
        return u0, lat.value, sts.value

    def wait(self, ticket: int):
        u0 = np.zeros(2, dtype=np.float32)
        lat = ctypes.c_double()
        sts = ctypes.c_int32()
        st = self.L.mppi_server_wait(self.s, ticket, _fp(u0), ctypes.byref(lat), ctypes.byref(sts))
        if st != A.OK:
            self._err(st, "mppi_server_wait")
        return u0, lat.value, sts.value

    def stats(self) -> dict:
        s = A.ServerStats()
        st = self.L.mppi_server_get_stats(self.s, ctypes.byref(s))
        if st != A.OK:
            self._err(st, "mppi_server_get_stats")
        return {f: getattr(s, f) for f, _ in A.ServerStats._fields_}

    def robot_state(self, rid: int):
        n, T = self.dims[rid]
        U = np.zeros((T, 2), dtype=np.float32)
        c = ctypes.c_uint64()
        st = self.L.mppi_server_get_robot(self.s, rid, _fp(U), ctypes.byref(c))
        if st != A.OK:
            self._err(st, "mppi_server_get_robot")
        return U, int(c.value)

#!/usr/bin/env python3
"""Benchmark of one DBaS-Log-MPPI iteration on one MI355X.

A "step" is one iteration of the hot path -- Philox normal x log-normal
sampling, the barrier-state rollout with its cost, the min-shifted
exponential weights, the weighted update and the warm-start shift -- on the
largest single-GPU workload: the planar quadrotor at scale (K = 16384 samples,
T = 100 steps, 400 circular obstacles, 7 shape points, a 512 x 512
signed-distance costmap, FP64 normaliser).

Prints ONE JSON line.  `value` = rollout-steps/s (K*T per iteration) over
the timed region: W untimed iterations, then `--steps` iterations, each timed
from its launch to u0 available on the host (the world, warm start and
counter resident on the device; the state x0 passed with the launch),
bracketed by device synchronisation.  Also reported:
  * the roofline of the rollout kernel: algorithmic FLOPs per launch (7 per
    (shape point, obstacle) pair, reciprocals counted apart) over its mean
    duration from HIP events recorded on its stream around every launch of
    the timed region, against the FP32 vector peak;
  * the same iterations issued back to back from device-resident states
    (pipelined);
  * the ground vehicle (K=4096, T=50, 100 obstacles) with its own roofline,
    and the small quadrotor (K=256, T=20, 10 obstacles) as a latency case;
  * the batched path: 64 mixed controllers in one graph-captured persistent
    launch vs the same 64 stepped one after another through the plain path;
  * the served path: 256 robots sending Poisson 50 Hz request streams to the
    continuous-batching server for 60 s (p50/p99 arrival-to-response), and
    the server's sustained rate with every robot keeping one request in
    flight for 10 s;
  * the paper's controller and its two baselines (Vanilla MPPI, Log-MPPI) at
    the paper's mission sizes (M = 1024, N = 20), and the closed-loop
    missions with each;
  * the FP64 CPU oracle timed on a bounded sample of the headline workload,
    on one core and on all the host cores it may use.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2504_06437_amd import workloads as W  # noqa: E402

PEAK_FP32_VECTOR_TFLOPS = 157.3       # MI355X published FP32 vector peak
HBM_PEAK_GBS = 8000.0
CUS, XCDS = 256, 8                    # MI355X: compute units, and the dies (XCDs) they sit on
METRIC = "rollout-steps/sec (K·T) and p50/p99 control-step latency, batched vs plain"
# kernel durations of the shorter legs come from HIP events around every
# PROFILE_EVERY-th iteration (the events of one iteration add a few
# microseconds to it, a fifth of a vehicle step if taken around every one)
PROFILE_EVERY = 32

# Algorithmic work of one rollout step of one sample, by term: a
# (shape point, obstacle) pair is dx, dy, two FMAs for h and the sum (7 FLOPs;
# its reciprocal is counted apart); a shape point costs 2 FMAs on the
# quadrotors' body axis and 4 on the vehicle's rectangle; a costmap point 15
# FLOPs and one reciprocal; the dynamics and the stage, control and barrier
# costs a fixed amount per model.
PAIR_FLOPS = 7
SHAPE_FLOPS = {"quad6": 4, "quad5": 4, "car": 8}
DYNAMICS_FLOPS = {"quad6": 14, "quad5": 12, "car": 10}
COST_FLOPS = {"quad6": 27, "quad5": 24, "car": 21}
MAP_FLOPS = 15


def rollout_flops_per_step(params: dict, J: int, with_map: bool) -> int:
    P = len(params["shape"])
    m = params["model"]
    return (PAIR_FLOPS * P * J + SHAPE_FLOPS[m] * P + DYNAMICS_FLOPS[m] + COST_FLOPS[m]
            + (MAP_FLOPS * P if with_map else 0))


def rollout_rcp_per_step(params: dict, J: int, with_map: bool) -> int:
    P = len(params["shape"])
    return P * J + (P if with_map else 0)


def percentile(a, q):
    return float(np.percentile(np.asarray(a), q))


def workload_name(wl) -> str:
    p = wl["params"]
    body = {"quad6": "quadrotor", "quad5": "quadrotor (5-state)", "car": "ground vehicle"}[p["model"]]
    s = f"{body} K={p['K']} T={p['T']} J={len(wl['obstacles'])} P={len(p['shape'])}"
    if wl.get("map") is not None:
        n = wl["map"]["sdf"].shape[0]
        s += f" + {n}x{n} costmap"
    if p.get("normaliser") == "on":
        s += ", fp64 normaliser"
    return s


def make_controller(wl, params=None):
    from paper_2504_06437_amd.controller import Controller
    c = Controller(params or wl["params"])
    c.load_workload(wl)
    return c


def closed_loop_states(c, wl, steps):
    """Run the plain path in closed loop with the simulated plant; return the
    visited states and the per-step latencies (host state in -> u0 out)."""
    from paper_2504_06437_amd.plant import advance
    x = wl["x0"].copy()
    xs, lat = [], []
    for _ in range(steps):
        c.set_reference(W.reference(wl, x))
        t0 = time.perf_counter()
        u = c.step(x)
        lat.append(time.perf_counter() - t0)
        xs.append(x.copy())
        x = advance(wl["params"], x, u)
    return np.asarray(xs, dtype=np.float32), lat


def roofline(p, J, with_map, kernel_ms, launches, extra=None):
    flops = p["K"] * p["T"] * rollout_flops_per_step(p, J, with_map)
    rcp = p["K"] * p["T"] * rollout_rcp_per_step(p, J, with_map)
    achieved = flops / (kernel_ms * 1e-3) / 1e12
    out = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
           "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": None, "kernel": "rollout",
           "kernel_ms_mean": kernel_ms, "flops_per_launch": flops, "rcp_per_launch": rcp,
           "rcp_per_s": rcp / (kernel_ms * 1e-3), "launches_timed": launches}
    if extra:
        out.update(extra)
    return out


def bench_leg(wl, steps, warmup, profile_every, pipelined_steps):
    """One workload: `steps` synchronous iterations (launch to u0 on the host,
    each timed) with HIP events on the controller's stream around the kernels
    of every `profile_every`-th one, then `pipelined_steps` iterations issued
    back to back from device-resident states."""
    from paper_2504_06437_amd import hip
    c = make_controller(wl)
    p = wl["params"]
    K, T = p["K"], p["T"]
    n_states = 200
    states, _ = closed_loop_states(c, wl, n_states)
    for i in range(warmup):
        c.step(states[i % n_states])
    c.profile(profile_every)
    lat = []
    hip.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        t1 = time.perf_counter()
        c.step(states[i % n_states])
        lat.append(time.perf_counter() - t1)
    status = c.synchronize()
    hip.synchronize()
    wall = time.perf_counter() - t0
    prof = c.profile_read()
    c.profile(False)
    assert status == 0, status
    # pipelined: device-resident states, no host round trip per iteration
    x_dev = hip.DeviceArray.from_numpy(states)
    u_dev = hip.DeviceArray((n_states, 2))
    for i in range(warmup):
        c.step_async(x_dev.at(i % n_states), u_dev.at(i % n_states))
    assert c.synchronize() == 0
    hip.synchronize()
    tp = time.perf_counter()
    for i in range(pipelined_steps):
        c.step_async(x_dev.at(i % n_states), u_dev.at(i % n_states))
    assert c.synchronize() == 0
    hip.synchronize()
    wall_p = time.perf_counter() - tp
    info = c.info()
    c.close()
    n_prof = max(prof["iterations"], 1)
    return {
        "workload": workload_name(wl), "wall_s": wall, "steps": steps,
        "rollout_steps_per_s": K * T * steps / wall, "ms_per_step": 1e3 * wall / steps,
        "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
        "rollout_steps_per_s_at_p50": K * T / percentile(lat, 50),
        "rollout_ms_mean": prof["rollout_ms"] / n_prof, "update_ms_mean": prof["update_ms"] / n_prof,
        "profiled": prof["iterations"],
        "pipelined": {"steps": pipelined_steps, "ms_per_step": 1e3 * wall_p / pipelined_steps,
                      "rollout_steps_per_s": K * T * pipelined_steps / wall_p},
        "tile_samples": info["tile_samples"], "tiles": info["tiles"], "fp64_tiles": info["fp64_tiles"],
        "noise_kept": info["noise_kept"], "barrier_form": info["barrier_form"],
    }


def bench_latency(wl, steps=50, rounds=4):
    """The small case: `rounds` receding-horizon runs of `steps` control steps
    each, closed loop through the host plant; every step is a synchronous
    iteration (host state in, u0 out)."""
    c = make_controller(wl)
    lat = []
    for _ in range(rounds):
        c.set_controls(np.zeros((wl["params"]["T"], 2), dtype=np.float32))
        _, l = closed_loop_states(c, wl, steps)
        lat.extend(l[1:])
    c.profile(1)
    closed_loop_states(c, wl, steps)
    prof = c.profile_read()
    c.close()
    p = wl["params"]
    n = max(prof["iterations"], 1)
    return {"workload": workload_name(wl), "steps": len(lat), "p50_ms": 1e3 * percentile(lat, 50),
            "p99_ms": 1e3 * percentile(lat, 99), "rollout_steps_per_s_at_p50": p["K"] * p["T"] / percentile(lat, 50),
            "rollout_kernel_ms_mean": prof["rollout_ms"] / n, "update_kernel_ms_mean": prof["update_ms"] / n}


def bench_controllers(runs_per=200):
    """The paper's controller and its baselines at the mission sizes (M =
    1024 samples, N = 20 steps): the same kernels in the three modes, on the
    first quadrotor and vehicle mission layouts.  Synchronous step latency
    and kernel times, to compare with the paper's finding of no significant
    difference in processing time among the three."""
    from paper_2504_06437_amd import mission
    out = []
    for m in (1, 2):
        wl = mission.layout(m, 0)
        for name in ("vanilla", "log", "dbas"):
            c = make_controller(wl, W.as_controller(wl["params"], name))
            x = wl["x0"]
            for _ in range(20):
                c.step(x)
            lat = []
            c.profile(1)
            for _ in range(runs_per):
                t0 = time.perf_counter()
                c.step(x)
                lat.append(time.perf_counter() - t0)
            prof = c.profile_read()
            c.close()
            n = max(prof["iterations"], 1)
            out.append({"mission": m, "controller": name, "workload": workload_name(wl),
                        "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99),
                        "rollout_kernel_us": 1e3 * prof["rollout_ms"] / n, "update_kernel_us": 1e3 * prof["update_ms"] / n})
    return out


def bench_batched(n_ctrl=64, steps=30, seed=3):
    """64 mixed controllers: one graph launch per step vs the plain path one by one."""
    from paper_2504_06437_amd.controller import Batch
    wls = W.batch(n_ctrl, seed)
    ctrls = [make_controller(wl) for wl in wls]
    total = sum(wl["params"]["K"] * wl["params"]["T"] for wl in wls)
    flops = sum(wl["params"]["K"] * wl["params"]["T"] * rollout_flops_per_step(wl["params"], len(wl["obstacles"]), False)
                for wl in wls)
    x0s = [wl["x0"] for wl in wls]
    # plain path, sequential: every controller synchronously, one after another
    for c, wl in zip(ctrls, wls):
        c.step(wl["x0"])
    seq = []
    for _ in range(max(3, steps // 3)):
        t0 = time.perf_counter()
        for c, wl in zip(ctrls, wls):
            c.step(wl["x0"])
        seq.append(time.perf_counter() - t0)
    batch = Batch(ctrls)
    for _ in range(3):
        batch.step(x0s)
    lat = []
    for _ in range(steps):
        t0 = time.perf_counter()
        _, sts = batch.step(x0s)
        lat.append(time.perf_counter() - t0)
    assert np.all(sts == 0)
    batch.close()
    for c in ctrls:
        c.close()
    return {
        "controllers": n_ctrl, "rollout_steps_per_iteration": int(total), "flops_per_iteration": flops,
        "batched": {"rollout_steps_per_s": total / percentile(lat, 50), "p50_ms": 1e3 * percentile(lat, 50),
                    "p99_ms": 1e3 * percentile(lat, 99), "n": len(lat),
                    "tflops_at_p50": flops / percentile(lat, 50) / 1e12},
        "plain_sequential": {"rollout_steps_per_s": total / percentile(seq, 50), "p50_ms": 1e3 * percentile(seq, 50),
                             "p99_ms": 1e3 * percentile(seq, 99), "n": len(seq)},
    }


def bench_served(seconds=60.0, n_robots=256, rate_hz=50.0, seed=4, budget=256 << 20, streams=3):
    """Poisson request streams from `n_robots` robots (sizes as the mixed
    batch) at `rate_hz` each, closed loop through the host plant, served by the
    continuous-batching server.  Latency = completion - scheduled arrival, so
    any lag of this client counts against the server, never for it."""
    from collections import deque

    from paper_2504_06437_amd.controller import Server
    from paper_2504_06437_amd.plant import advance
    wls = W.batch(n_robots, seed)
    srv = Server(budget_bytes=budget, max_slots=256, streams=streams, max_batch=64)
    t_setup = time.perf_counter()
    ids = [srv.add_robot(wl["params"], wl["obstacles"]) for wl in wls]
    t_setup = time.perf_counter() - t_setup
    states = [wl["x0"].copy() for wl in wls]
    # warm-up: one request per robot
    for i, wl in enumerate(wls):
        srv.wait(srv.submit(ids[i], states[i], W.reference(wl, states[i])))
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    arrivals = []
    for r in range(n_robots):
        t = rng.exponential(1.0 / rate_hz)
        while t < seconds:
            arrivals.append((t, r))
            t += rng.exponential(1.0 / rate_hz)
    arrivals.sort()
    work = [wl["params"]["K"] * wl["params"]["T"] for wl in wls]
    pending = [deque() for _ in wls]
    waiting = set()
    last_ref = [0.0] * n_robots
    lat, statuses, served_steps, lag_max = [], [], 0, 0.0
    t0 = srv.now() + 0.05
    i, t_end = 0, t0
    next_note = 10.0
    while i < len(arrivals) or waiting:
        now = srv.now()
        if now - t0 >= next_note:
            print(f"[bench] served: {next_note:.0f} s, {len(lat)} responses", file=sys.stderr, flush=True)
            next_note += 10.0
        if i < len(arrivals) and now >= t0 + arrivals[i][0]:
            t, r = arrivals[i]
            i += 1
            lag_max = max(lag_max, now - (t0 + t))
            ref = None
            if t - last_ref[r] >= 1.0:
                ref = W.reference(wls[r], states[r])
                last_ref[r] = t
            pending[r].append(srv.submit(ids[r], states[r], ref, t0 + t))
            waiting.add(r)
            continue
        for r in list(waiting):
            while pending[r]:
                res = srv.poll(pending[r][0])
                if res is None:
                    break
                pending[r].popleft()
                u0, l, st = res
                lat.append(l)
                statuses.append(st)
                served_steps += work[r]
                states[r] = advance(wls[r]["params"], states[r], u0)
                t_end = max(t_end, srv.now())
            if not pending[r]:
                waiting.discard(r)
    stats = srv.stats()
    srv.close()
    span = t_end - t0
    return {
        "robots": n_robots, "rate_hz_per_robot": rate_hz, "seconds": seconds, "requests": len(lat),
        "ok": int(sum(1 for s in statuses if s == 0)),
        "rollout_steps_per_s": served_steps / span, "requests_per_s": len(lat) / span,
        "p50_ms": 1e3 * percentile(lat, 50), "p99_ms": 1e3 * percentile(lat, 99), "max_ms": 1e3 * max(lat),
        "client_lag_max_ms": 1e3 * lag_max, "launches": stats["launches"], "mean_batch": stats["mean_batch"],
        "deferred_budget": stats["deferred_budget"], "deferred_slots": stats["deferred_slots"],
        "peak_scratch_bytes": stats["peak_bytes_in_flight"], "budget_bytes": budget, "streams": streams,
        "setup_s": t_setup,
    }



def bench_served_saturation(seconds=10.0, n_robots=256, seed=4, budget=256 << 20, streams=3):
    """The server's sustained rate: every robot (sizes as the mixed batch)
    keeps one request in flight, submitting its next state as soon as the
    previous response arrives, for `seconds`.  Requests/s and rollout-steps/s
    here are what the server completes when the offered load always exceeds
    it; latency is submit -> response."""
    from paper_2504_06437_amd.controller import Server
    from paper_2504_06437_amd.plant import advance
    wls = W.batch(n_robots, seed)
    srv = Server(budget_bytes=budget, max_slots=256, streams=streams, max_batch=64)
    ids = [srv.add_robot(wl["params"], wl["obstacles"]) for wl in wls]
    states = [wl["x0"].copy() for wl in wls]
    for i, wl in enumerate(wls):
        srv.wait(srv.submit(ids[i], states[i], W.reference(wl, states[i])))
    work = [wl["params"]["K"] * wl["params"]["T"] for wl in wls]
    t0 = srv.now()
    tickets = [srv.submit(ids[r], states[r], None, t0) for r in range(n_robots)]
    lat, served_steps, n_done = [], 0, 0
    t_end = t0
    while True:
        now = srv.now()
        if now - t0 >= seconds:
            break
        for r in range(n_robots):
            res = srv.poll(tickets[r])
            if res is None:
                continue
            u0, l, st = res
            lat.append(l)
            served_steps += work[r]
            n_done += 1
            states[r] = advance(wls[r]["params"], states[r], u0)
            t_end = srv.now()
            tickets[r] = srv.submit(ids[r], states[r], None, t_end)
    for r in range(n_robots):
        srv.wait(tickets[r])
    stats = srv.stats()
    srv.close()
    span = t_end - t0
    return {"robots": n_robots, "seconds": seconds, "requests": n_done, "requests_per_s": n_done / span,
            "rollout_steps_per_s": served_steps / span, "p50_ms": 1e3 * percentile(lat, 50),
            "p99_ms": 1e3 * percentile(lat, 99), "launches": stats["launches"], "mean_batch": stats["mean_batch"],
            "streams": streams}

def host_cpu():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model


def host_threads() -> int:
    try:
        n = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        n = 0
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(n, avail) if n > 0 else avail)


def cpu_baseline(wl, single_s=12.0, multi_s=8.0):
    """The FP64 oracle (plain C, gcc -O2, threaded over samples when asked) on
    whole iterations of the same workload: first on one core, then on every
    core this process may use.  The all-core figure is `value`."""
    import oracle
    p = wl["params"]
    world = oracle.World.from_workload(wl)

    def run(threads, budget):
        oracle.set_threads(threads)
        U = wl["U0"].astype(np.float64)
        iters, t0 = 0, time.perf_counter()
        while True:
            r = oracle.step(p, world, wl["x0"], U, wl["x_ref"], 1.0, iters, diagnostics=False)
            U = r["Unext"]
            iters += 1
            el = time.perf_counter() - t0
            if el >= budget or iters >= 50:
                break
        return iters, el

    it1, el1 = run(1, single_s)
    nt = host_threads()
    itn, eln = run(nt, multi_s)
    oracle.set_threads(1)
    kt = p["K"] * p["T"]
    return {"value": kt * itn / eln, "unit": "rollout-steps/s", "cores": nt, "kind": "oracle",
            "sample": f"{itn} full iterations of the headline workload ({workload_name(wl)}), FP64, "
                      f"{nt} threads over samples, {eln:.1f} s",
            "single_core": {"value": kt * it1 / el1, "cores": 1, "iterations": it1, "seconds": el1},
            "cpu_model": host_cpu(), "host_cpus_available": host_threads()}


def _kernel_sources():
    csrc = os.path.join(ROOT, "paper_2504_06437_amd", "csrc")
    names = ["mppi_device.hpp", "mppi_kernels.hip"] + sorted(
        f for f in os.listdir(csrc) if f.startswith("mppi_rollout_") and f.endswith(".hip"))
    return "\n".join(open(os.path.join(csrc, n)).read() for n in names)


def _kernel_digest(text: str | None = None) -> str:
    """SHA-256 (16 hex digits) of the kernels' source code: comments removed
    and whitespace collapsed, so that a comment edit keeps the records."""
    import hashlib
    import re
    if text is None:
        text = _kernel_sources()
    code = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    code = re.sub(r"//[^\n]*", " ", code)
    code = " ".join(code.split())
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def _load_record(name: str, kernel: str, workload: str):
    """A counter record from profiles/<name>, if it was taken on the current
    kernel source."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", name)))
    except (OSError, ValueError):
        return None
    r = rec.get(kernel, {}).get(workload)
    if not r or r.get("kernel_source_sha256_16") != _kernel_digest():
        return None
    return r


def load_traffic(kernel: str, workload: str):
    """HBM bytes per launch measured by rocprofv3 counters, if recorded for
    the current kernel source (profiles/traffic.json)."""
    r = _load_record("traffic.json", kernel, workload)
    return r.get("bytes_per_launch") if r else None


def load_counters(kernel: str, workload: str):
    """VALU figures from rocprofv3 SQ counters, if recorded for the current
    kernel source (profiles/counters.json)."""
    r = _load_record("counters.json", kernel, workload)
    keys = ("active_valu_ratio", "valu_insts_per_wave", "wait_frac", "executed_flops_per_launch")
    return {k: r[k] for k in keys if k in r} if r else None


def copy_calibration(mib: int, copies: int = 5):
    """Plain device-to-device copies of known size, run under rocprofv3 --pmc
    to calibrate FETCH_SIZE / WRITE_SIZE against true bytes."""
    from paper_2504_06437_amd import hip
    n = mib * (1 << 20) // 4
    a, b = hip.DeviceArray((n,)), hip.DeviceArray((n,))
    for _ in range(copies):
        hip.copy_device(b, a)
    hip.synchronize()
    return {"copy_bytes": a.nbytes, "copies": copies}


def _pmc_mean(csv_dir: str, counter: str, kernel_substr: str):
    """Mean over dispatches of `counter` (summed over its instances) for the
    kernels whose name contains `kernel_substr`; (mean, dispatches, names)."""
    import csv
    import glob
    per = {}
    for f in glob.glob(os.path.join(csv_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                name = row.get("Kernel_Name", "")
                if row.get("Counter_Name") != counter or kernel_substr not in name:
                    continue
                key = (name, f, row["Dispatch_Id"])
                per[key] = per.get(key, 0.0) + float(row["Counter_Value"])
    if not per:
        raise SystemExit(f"no {counter} rows for kernels matching {kernel_substr!r} under {csv_dir}")
    # the most dispatched instantiation (autotune candidates run only a few times)
    counts = {}
    for name, _, _ in per:
        counts[name] = counts.get(name, 0) + 1
    top = max(counts, key=counts.get)
    vals = [v for (name, _, _), v in per.items() if name == top]
    return sum(vals) / len(vals), len(vals), [top]


def _pmc_duration_s(csv_dir: str, kernel_substr: str, name: str) -> float:
    """Mean start-to-end time of the dispatches of kernel `name` in a
    rocprofv3 --pmc run (each counter row carries its dispatch's timestamps,
    in ns)."""
    import csv
    import glob
    per = {}
    for f in glob.glob(os.path.join(csv_dir, "**", "*counter_collection.csv"), recursive=True):
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                if row.get("Kernel_Name") != name or kernel_substr not in name:
                    continue
                per[(f, row["Dispatch_Id"])] = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) * 1e-9
    if not per:
        raise SystemExit(f"no timestamps for {name!r} under {csv_dir}")
    return sum(per.values()) / len(per)


def summarize_traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, copy_bytes, workload, out_path):
    """HBM bytes per rollout launch from FETCH_SIZE / WRITE_SIZE (KiB per
    dispatch), each scaled by true bytes / counter reading of a plain copy."""
    cf, _, cnames = _pmc_mean(copy_fetch_dir, "FETCH_SIZE", "copy")
    cw, _, _ = _pmc_mean(copy_write_dir, "WRITE_SIZE", "copy")
    f_scale = copy_bytes / (cf * 1024.0)
    w_scale = copy_bytes / (cw * 1024.0)
    fk, nf, names = _pmc_mean(fetch_dir, "FETCH_SIZE", "k_rollout")
    wk, nw, _ = _pmc_mean(write_dir, "WRITE_SIZE", "k_rollout")
    digest = _kernel_digest()
    fetch_b, write_b = fk * 1024.0 * f_scale, wk * 1024.0 * w_scale
    rec = {}
    if os.path.exists(out_path):
        rec = json.load(open(out_path))
    rec.setdefault("rollout", {})[workload] = {
        "bytes_per_launch": fetch_b + write_b, "fetch_bytes": fetch_b, "write_bytes": write_b,
        "fetch_kib_raw": fk, "write_kib_raw": wk, "dispatches": [nf, nw], "kernels": names,
        "copy_kernel": cnames, "copy_bytes": copy_bytes, "fetch_scale": f_scale, "write_scale": w_scale,
        "kernel_source_sha256_16": digest,
    }
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec["rollout"][workload]


def summarize_counters(sq1_dir, sq2_dir, workload, out_path, sq3_dir=None):
    """VALU use of the rollout from SQ counters (two rocprofv3 passes):
    instructions per wave, the waiting share, the transcendental share, and
    the executed FP32 FLOPs per launch, 64 lanes x (2 FMA + ADD + MUL) over
    the FP32 instruction counts (every lane of a wave counted; the counters
    count wave instructions).  Also SQ_ACTIVE_INST_VALU / (SQ_WAVE_CYCLES /
    4), reported as a ratio: with four waves per SIMD living the whole
    launch it would be the SIMD's VALU busy fraction, but on gfx950 it
    exceeds 1, so the two counters are not in the units that reading needs.

    An optional third pass gives the clock: GRBM_GUI_ACTIVE (summed over the
    XCDs, so divided by their number) over the dispatch's own duration is
    the clock the launch ran at, and SQ_INSTS_VALU over the SIMDs and those
    cycles is the VALU instructions each SIMD issued per cycle.  It also
    records SQ_VALU_MFMA_BUSY_CYCLES, which is 0 for a kernel that issues no
    matrix instruction."""
    act, n, names = _pmc_mean(sq1_dir, "SQ_ACTIVE_INST_VALU", "k_rollout")
    wcyc, _, _ = _pmc_mean(sq1_dir, "SQ_WAVE_CYCLES", "k_rollout")
    waves, _, _ = _pmc_mean(sq1_dir, "SQ_WAVES", "k_rollout")
    insts, _, _ = _pmc_mean(sq1_dir, "SQ_INSTS_VALU", "k_rollout")
    wait, _, _ = _pmc_mean(sq1_dir, "SQ_WAIT_ANY", "k_rollout")
    trans, _, _ = _pmc_mean(sq2_dir, "SQ_INSTS_VALU_TRANS_F32", "k_rollout")
    rec = {}
    if os.path.exists(out_path):
        rec = json.load(open(out_path))
    r = {"active_valu_ratio": act / (wcyc / 4.0), "valu_insts_per_wave": insts / waves, "wait_frac": wait / wcyc,
         "trans_share": trans / insts, "dispatches": n, "kernels": names, "kernel_source_sha256_16": _kernel_digest()}
    try:
        fma, _, _ = _pmc_mean(sq2_dir, "SQ_INSTS_VALU_FMA_F32", "k_rollout")
        add, _, _ = _pmc_mean(sq2_dir, "SQ_INSTS_VALU_ADD_F32", "k_rollout")
        mul, _, _ = _pmc_mean(sq2_dir, "SQ_INSTS_VALU_MUL_F32", "k_rollout")
        r.update({"fma_f32": fma, "add_f32": add, "mul_f32": mul,
                  "executed_flops_per_launch": 64.0 * (2.0 * fma + add + mul)})
    except SystemExit:
        pass
    if sq3_dir:
        gui, _, names3 = _pmc_mean(sq3_dir, "GRBM_GUI_ACTIVE", "k_rollout")
        mfma, _, _ = _pmc_mean(sq3_dir, "SQ_VALU_MFMA_BUSY_CYCLES", "k_rollout")
        dur = _pmc_duration_s(sq3_dir, "k_rollout", names3[0])
        cycles = gui / XCDS
        r.update({"grbm_gui_active_per_xcd": cycles, "pmc_dispatch_s": dur, "clock_ghz": cycles / dur / 1e9,
                  "valu_insts_per_simd_cycle": insts / (CUS * 4) / cycles, "mfma_busy_cycles": mfma})
    rec.setdefault("rollout", {})[workload] = r
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return r


def update_bytes(p: dict, tiles: int) -> int:
    """Algorithmic bytes of one update launch: the tile partials N_b (2T rows
    of `tiles` doubles), the tile scalars (min, normaliser, FP64 flag) read
    by every workgroup, f_b written once, and U read, U* and the shifted U
    written."""
    T, groups = p["T"], (2 * p["T"] + 3) // 4
    return 16 * T * tiles + groups * 20 * tiles + 8 * tiles + 3 * 8 * T


def update_roofline(p: dict, r: dict) -> dict:
    """The update kernel against HBM: algorithmic bytes per launch over its
    mean duration (HIP events around the same sampled launches)."""
    b = update_bytes(p, r["tiles"])
    gbs = b / (r["update_ms_mean"] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "bytes_per_launch": b, "kernel_ms_mean": r["update_ms_mean"],
            "note": f"latency-bound: {b / 1e6:.2f} MB over {(2 * p['T'] + 3) // 4} workgroups"}


WORKLOADS = {"c2": W.quad_large, "c1": W.car, "c0": W.quad_small}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c2",
                    help="headline workload (c2: the quadrotor at scale; c1, c0 for profiling runs)")
    ap.add_argument("--only-headline", action="store_true", help="skip every extra leg")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-missions", action="store_true")
    ap.add_argument("--no-legs", action="store_true", help="skip the vehicle, small-quadrotor and controller legs")
    ap.add_argument("--mission-runs", type=int, default=10)
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--copy-calibration", type=int, metavar="MIB",
                    help="only run plain device copies of MIB MiB (counter calibration)")
    ap.add_argument("--summarize-counters", nargs="+", metavar="SQ",
                    help="two or three rocprofv3 SQ counter folders (the third: GRBM_GUI_ACTIVE and "
                         "SQ_VALU_MFMA_BUSY_CYCLES) -> profiles/counters.json (no GPU use)")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="rocprofv3 --pmc output folders -> profiles/traffic.json (no GPU use)")
    ap.add_argument("--copy-bytes", type=int, default=256 << 20)
    args = ap.parse_args()
    if args.summarize_counters:
        d = args.summarize_counters
        if len(d) not in (2, 3):
            ap.error("--summarize-counters takes two or three folders")
        print(json.dumps(summarize_counters(d[0], d[1], workload_name(WORKLOADS[args.workload]()),
                                            os.path.join(ROOT, "profiles", "counters.json"),
                                            d[2] if len(d) == 3 else None), indent=1))
        return
    if args.summarize_traffic:
        r = summarize_traffic(*args.summarize_traffic, args.copy_bytes, workload_name(WORKLOADS[args.workload]()),
                              os.path.join(ROOT, "profiles", "traffic.json"))
        print(json.dumps(r, indent=1))
        return
    if args.copy_calibration:
        print(json.dumps(copy_calibration(args.copy_calibration)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): every run here uses one GPU; "
              "the multi-GPU design is described but not built.", file=sys.stderr)
        sys.exit(2)
    if args.only_headline:
        args.no_batched = args.no_cpu = args.no_served = args.no_missions = args.no_legs = True

    wl = WORKLOADS[args.workload]()
    p = wl["params"]
    J = len(wl["obstacles"])
    with_map = wl.get("map") is not None
    name = workload_name(wl)
    print(f"[bench] headline: {name}, {args.steps} timed steps", file=sys.stderr, flush=True)
    # events around every launch of the headline's timed region (at this size
    # they cost about one per cent of a step)
    r = bench_leg(wl, args.steps, args.warmup, 1 if args.workload == "c2" else PROFILE_EVERY,
                  pipelined_steps=max(args.steps, 100))
    rl = roofline(p, J, with_map, r["rollout_ms_mean"], r["profiled"],
                  {"update_kernel_ms_mean": r["update_ms_mean"], "timed_every": 1 if args.workload == "c2" else PROFILE_EVERY})
    rl["traffic"] = load_traffic("rollout", name)
    rl["valu"] = load_counters("rollout", name)
    if rl["valu"] and "executed_flops_per_launch" in rl["valu"]:
        ex = rl["valu"]["executed_flops_per_launch"] / (r["rollout_ms_mean"] * 1e-3) / 1e12
        rl["valu"]["executed_tflops"] = ex
        rl["valu"]["executed_frac"] = ex / PEAK_FP32_VECTOR_TFLOPS
    out = {
        "metric": METRIC, "value": r["rollout_steps_per_s"], "unit": "rollout-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": name, "K": p["K"], "T": p["T"], "obstacles": J, "shape_points": len(p["shape"]),
                   "costmap": list(wl["map"]["sdf"].shape) if with_map else None,
                   "normaliser": p.get("normaliser", "auto"), "tile_samples": r["tile_samples"], "tiles": r["tiles"],
                   "timed": "each step from its launch to u0 on the host; world, warm start and counter in HBM"},
        "roofline": rl,
        "update_roofline": update_roofline(p, r),
        "latency_ms": {"p50": r["p50_ms"], "p99": r["p99_ms"], "n": args.steps,
                       "rollout_steps_per_s_at_p50": r["rollout_steps_per_s_at_p50"]},
        "pipelined": r["pipelined"],
        "timing": {"wall_s": r["wall_s"], "fp64_tiles": r["fp64_tiles"], "noise_kept": r["noise_kept"],
                   "barrier_form": r["barrier_form"]},
    }
    if not args.no_legs:
        print("[bench] vehicle leg", file=sys.stderr, flush=True)
        wc = W.car()
        rc = bench_leg(wc, 1024, 20, PROFILE_EVERY, pipelined_steps=1024)
        rc["roofline"] = roofline(wc["params"], len(wc["obstacles"]), False, rc["rollout_ms_mean"], rc["profiled"],
                                  {"timed_every": PROFILE_EVERY})
        rc["update_roofline"] = update_roofline(wc["params"], rc)
        out["vehicle"] = rc
        print("[bench] small quadrotor latency leg", file=sys.stderr, flush=True)
        out["small"] = bench_latency(W.quad_small())
        print("[bench] controllers at the mission sizes", file=sys.stderr, flush=True)
        out["controllers"] = bench_controllers()
    if not args.no_batched:
        print("[bench] batched path: 64 mixed controllers", file=sys.stderr, flush=True)
        out["batched"] = bench_batched()
    if not args.no_served:
        print(f"[bench] served path: 256 robots x 50 Hz for {args.serve_seconds:g} s", file=sys.stderr, flush=True)
        out["served"] = bench_served(args.serve_seconds)
        print("[bench] served path at saturation: 256 robots, one request in flight each, 10 s", file=sys.stderr,
              flush=True)
        out["served_saturation"] = bench_served_saturation()
    if not args.no_missions:
        from paper_2504_06437_amd import mission
        print(f"[bench] missions: {args.mission_runs} closed-loop runs each, three controllers", file=sys.stderr,
              flush=True)
        out["missions"] = {"note": "synthetic layouts with the paper's mission settings; not its layouts",
                           "results": [mission.run_mission(m, args.mission_runs, controller=c)
                                       for c in ("dbas", "log", "vanilla") for m in (1, 2, 3)]}
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

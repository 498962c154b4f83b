#!/usr/bin/env python3
"""Benchmark of one DBaS-Log-MPPI iteration on one MI355X.

A "step" is one iteration of the hot path: Philox normal x log-normal sampling,
the barrier-state rollout with its cost, the min-shifted exponential weights
and the weighted update with the warm-start shift, for the ground-vehicle
workload (K=4096 samples, T=50, 100 circular obstacles, 8 shape points).

Prints ONE JSON line.  `value` = rollout-steps/s (K*T per iteration) over the
timed region: W untimed iterations, then `--steps` iterations issued back to
back on the controller's stream with the states already in device memory,
bracketed by device synchronisation.  Also reported:
  * roofline of the rollout kernel (algorithmic FLOPs per launch / its mean
    duration from HIP events recorded on its stream around every 32nd launch
    of the timed region),
  * p50/p99 control-step latency of the plain path (host state in, u0 out),
  * the quadrotor at scale (K=16384, T=100, 400 obstacles + costmap),
  * the batched path: 64 mixed controllers in one graph-captured persistent
    launch vs the same 64 stepped one after another through the plain path,
  * the served path: 256 robots sending Poisson 50 Hz request streams to the
    continuous-batching server (p50/p99 arrival-to-response latency),
  * the closed-loop missions (success, path error, average speed) on
    synthetic layouts with the paper's mission settings,
  * the FP64 CPU oracle timed on a bounded sample of the same workload.
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
METRIC = "rollout-steps/sec (K·T) and p50/p99 control-step latency, batched vs plain"
# kernel durations come from HIP events around every PROFILE_EVERY-th
# iteration of the timed loop (the events of one iteration add about 9 us to
# it, so around every iteration they would cost a fifth of the step)
PROFILE_EVERY = 32


def rollout_flops_per_step(params: dict, J: int, with_map: bool) -> float:
    """Algorithmic FP32 work of one (sample, step) of the rollout.

    per obstacle pair: dx, dy (2), h = dx^2 + dy^2 - r^2 (2 FMA = 4),
        B = 1/max(h, eps) (1), accumulate (1)                      -> 8
    per shape point: rotate + translate (2 x (mul, FMA, add) = 8)    -> 8
    per shape point with a costmap: 2 FMA coords (4), 3 lerps (9),
        B (1), accumulate (1)                                      -> 15
    per step, fixed: noise (2 x (2 FMA uniforms, log, sqrt, sincos pair,
        mul, FMA + exp, 2 mul) = 34), saturation (4), dynamics (quad 20,
        car 14), heading sincos (2), barrier state (2), stage cost
        (4 n), control cost (6), compensated add (6)
    """
    P = len(params["shape"])
    n = W.MODEL_DIMS[params["model"]]
    fixed = 34 + 4 + (14 if params["model"] == "car" else 20) + 2 + 2 + 4 * n + 6 + 6
    return 8.0 * P * J + 8.0 * P + (15.0 * P if with_map else 0.0) + fixed


def percentile(a, q):
    return float(np.percentile(np.asarray(a), q))


def make_controller(wl):
    from paper_2504_06437_amd.controller import Controller
    c = Controller(wl["params"])
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


def bench_plain(wl, steps, warmup):
    from paper_2504_06437_amd import hip
    c = make_controller(wl)
    p = wl["params"]
    K, T = p["K"], p["T"]
    n_states = 200                      # closed-loop states, cycled through by the timed loop
    states, lat = closed_loop_states(c, wl, n_states)
    lat = lat[min(20, len(lat) // 4):]
    x_dev = hip.DeviceArray.from_numpy(states)
    u_dev = hip.DeviceArray((n_states, 2))
    hip.synchronize()
    for i in range(warmup):
        c.step_async(x_dev.at(i % n_states), u_dev.at(i % n_states))
    assert c.synchronize() == 0
    c.profile(PROFILE_EVERY)
    ev0, ev1 = hip.Event(), hip.Event()
    hip.synchronize()
    t0 = time.perf_counter()
    ev0.record(c.stream)
    for i in range(steps):
        c.step_async(x_dev.at(i % n_states), u_dev.at(i % n_states))
    ev1.record(c.stream)
    status = c.synchronize()
    hip.synchronize()
    wall = time.perf_counter() - t0
    prof = c.profile_read()
    c.profile(False)
    info = c.info()
    ev_ms = ev0.elapsed_ms(ev1)
    c.close()
    assert status == 0, status
    return {
        "wall_s": wall, "event_ms": ev_ms, "rollout_steps_per_s": K * T * steps / wall,
        "ms_per_step": 1e3 * wall / steps, "rollout_ms_mean": prof["rollout_ms"] / max(prof["iterations"], 1),
        "update_ms_mean": prof["update_ms"] / max(prof["iterations"], 1), "profiled": prof["iterations"],
        "latency_ms": {"p50": 1e3 * percentile(lat, 50), "p99": 1e3 * percentile(lat, 99), "n": len(lat)},
        "tile_samples": info["tile_samples"], "tiles": info["tiles"],
    }


def bench_at_scale(steps=20, warmup=3):
    """The quadrotor at scale: K=16384, T=100, 400 obstacles + 512x512
    costmap, FP64 normaliser.  Steps issued back to back from device-resident
    states; rollout-kernel time from HIP events around every launch of this
    short loop (events cost ~1% of an 0.8 ms kernel)."""
    from paper_2504_06437_amd import hip
    wl = W.quad_large()
    p = wl["params"]
    c = make_controller(wl)
    x_dev = hip.DeviceArray.from_numpy(np.stack([wl["x0"]] * 4))
    u_dev = hip.DeviceArray((4, 2))
    for i in range(warmup):
        c.step_async(x_dev.at(i % 4), u_dev.at(i % 4))
    assert c.synchronize() == 0
    c.profile(1)
    hip.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        c.step_async(x_dev.at(i % 4), u_dev.at(i % 4))
    status = c.synchronize()
    wall = time.perf_counter() - t0
    prof = c.profile_read()
    info = c.info()
    c.close()
    assert status == 0, status
    J = len(wl["obstacles"])
    kernel_ms = prof["rollout_ms"] / max(prof["iterations"], 1)
    flops = p["K"] * p["T"] * rollout_flops_per_step(p, J, True)
    achieved = flops / (kernel_ms * 1e-3) / 1e12
    return {"workload": f"quadrotor K={p['K']} T={p['T']} J={J} P={len(p['shape'])} + 512x512 costmap",
            "rollout_steps_per_s": p["K"] * p["T"] * steps / wall, "ms_per_step": 1e3 * wall / steps,
            "rollout_kernel_ms_mean": kernel_ms, "update_kernel_ms_mean": prof["update_ms"] / max(prof["iterations"], 1),
            "achieved_tflops": achieved, "frac_of_fp32_peak": achieved / PEAK_FP32_VECTOR_TFLOPS,
            "tile_samples": info["tile_samples"], "fp64_tiles": info["fp64_tiles"], "steps": steps}


def bench_batched(n_ctrl=64, steps=30, seed=3):
    """64 mixed controllers: one graph launch per step vs the plain path one by one."""
    from paper_2504_06437_amd.controller import Batch
    wls = W.batch(n_ctrl, seed)
    ctrls = [make_controller(wl) for wl in wls]
    total = sum(wl["params"]["K"] * wl["params"]["T"] for wl in wls)
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
        "controllers": n_ctrl, "rollout_steps_per_iteration": int(total),
        "batched": {"rollout_steps_per_s": total / percentile(lat, 50), "p50_ms": 1e3 * percentile(lat, 50),
                    "p99_ms": 1e3 * percentile(lat, 99), "n": len(lat)},
        "plain_sequential": {"rollout_steps_per_s": total / percentile(seq, 50), "p50_ms": 1e3 * percentile(seq, 50),
                             "p99_ms": 1e3 * percentile(seq, 99), "n": len(seq)},
    }


def bench_served(seconds=10.0, n_robots=256, rate_hz=50.0, seed=4, budget=256 << 20, streams=3):
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
    while i < len(arrivals) or waiting:
        now = srv.now()
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


def cpu_baseline(wl, budget_s=12.0):
    """The FP64 oracle, single-threaded, on whole iterations of the same workload."""
    import oracle
    p = wl["params"]
    world = oracle.World.from_workload(wl)
    U = wl["U0"].astype(np.float64)
    iters, t0 = 0, time.perf_counter()
    while True:
        r = oracle.step(p, world, wl["x0"], U, wl["x_ref"], 1.0, iters)
        U = r["Unext"]
        iters += 1
        el = time.perf_counter() - t0
        if (el >= budget_s and iters >= 2) or el >= 3 * budget_s:
            break
    return {"value": p["K"] * p["T"] * iters / el, "unit": "rollout-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} full iterations of the same workload (K={p['K']}, T={p['T']}, J={len(wl['obstacles'])}), "
                      f"FP64, single thread, {el:.1f} s"}


def _kernel_digest(text: str | None = None) -> str:
    """SHA-256 (16 hex digits) of the kernel source's code: comments removed
    and whitespace collapsed, so that a comment edit keeps the records."""
    import hashlib
    import re
    if text is None:
        text = open(os.path.join(ROOT, "paper_2504_06437_amd", "csrc", "mppi_kernels.hip")).read()
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
    return {k: r[k] for k in ("valu_busy", "valu_insts_per_wave", "wait_frac")} if r else None


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


def summarize_counters(sq1_dir, sq2_dir, workload, out_path):
    """VALU use of the rollout from SQ counters (two rocprofv3 passes).  Every
    wave lives for the whole launch (one tile per CU, four waves per SIMD), so
    a SIMD's VALU busy fraction is the VALU-active time of its waves over one
    wave's lifetime: SQ_ACTIVE_INST_VALU / (SQ_WAVE_CYCLES / 4)."""
    act, n, names = _pmc_mean(sq1_dir, "SQ_ACTIVE_INST_VALU", "k_rollout")
    wcyc, _, _ = _pmc_mean(sq1_dir, "SQ_WAVE_CYCLES", "k_rollout")
    waves, _, _ = _pmc_mean(sq1_dir, "SQ_WAVES", "k_rollout")
    insts, _, _ = _pmc_mean(sq1_dir, "SQ_INSTS_VALU", "k_rollout")
    wait, _, _ = _pmc_mean(sq1_dir, "SQ_WAIT_ANY", "k_rollout")
    trans, _, _ = _pmc_mean(sq2_dir, "SQ_INSTS_VALU_TRANS_F32", "k_rollout")
    rec = {}
    if os.path.exists(out_path):
        rec = json.load(open(out_path))
    rec.setdefault("rollout", {})[workload] = {
        "valu_busy": act / (wcyc / 4.0), "valu_insts_per_wave": insts / waves, "wait_frac": wait / wcyc,
        "trans_share": trans / insts, "dispatches": n, "kernels": names, "kernel_source_sha256_16": _kernel_digest(),
    }
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec["rollout"][workload]


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1024)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-scale", action="store_true")
    ap.add_argument("--no-missions", action="store_true")
    ap.add_argument("--mission-runs", type=int, default=10)
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--copy-calibration", type=int, metavar="MIB",
                    help="only run plain device copies of MIB MiB (counter calibration)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("SQ1", "SQ2"),
                    help="rocprofv3 SQ counter folders -> profiles/counters.json (no GPU use)")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="rocprofv3 --pmc output folders -> profiles/traffic.json (no GPU use)")
    ap.add_argument("--copy-bytes", type=int, default=256 << 20)
    args = ap.parse_args()
    if args.summarize_counters:
        wl = W.car()
        p = wl["params"]
        workload = f"ground vehicle K={p['K']} T={p['T']} J={len(wl['obstacles'])} P={len(p['shape'])}"
        print(json.dumps(summarize_counters(*args.summarize_counters, workload,
                                            os.path.join(ROOT, "profiles", "counters.json")), indent=1))
        return
    if args.summarize_traffic:
        wl = W.car()
        p = wl["params"]
        workload = f"ground vehicle K={p['K']} T={p['T']} J={len(wl['obstacles'])} P={len(p['shape'])}"
        r = summarize_traffic(*args.summarize_traffic, args.copy_bytes, workload,
                              os.path.join(ROOT, "profiles", "traffic.json"))
        print(json.dumps(r, indent=1))
        return
    if args.copy_calibration:
        print(json.dumps(copy_calibration(args.copy_calibration)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU design "
              "is described but not built.", file=sys.stderr)
        sys.exit(2)

    wl = W.car()
    p = wl["params"]
    J = len(wl["obstacles"])
    print(f"[bench] plain path: car K={p['K']} T={p['T']} J={J}", file=sys.stderr, flush=True)
    r = bench_plain(wl, args.steps, args.warmup)
    flops = p["K"] * p["T"] * rollout_flops_per_step(p, J, False)
    achieved = flops / (r["rollout_ms_mean"] * 1e-3) / 1e12
    workload = f"ground vehicle K={p['K']} T={p['T']} J={J} P={len(p['shape'])}"
    out = {
        "metric": METRIC, "value": r["rollout_steps_per_s"], "unit": "rollout-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload, "K": p["K"], "T": p["T"], "obstacles": J, "shape_points": len(p["shape"]),
                   "tile_samples": r["tile_samples"], "tiles": r["tiles"], "normaliser": "fp32 (fp64 when |rho|/lambda>=1024)"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
                     "traffic": load_traffic("rollout", workload),
                     "kernel": "rollout", "kernel_ms_mean": r["rollout_ms_mean"],
                     "update_kernel_ms_mean": r["update_ms_mean"], "flops_per_launch": flops,
                     "launches_timed": r["profiled"], "timed_every": PROFILE_EVERY,
                     "valu": load_counters("rollout", workload)},
        "update_roofline": update_roofline(p, r),
        "latency_ms": {"plain_p50": r["latency_ms"]["p50"], "plain_p99": r["latency_ms"]["p99"],
                       "n": r["latency_ms"]["n"], "note": "host state in, u0 out (PCIe-inclusive)"},
        "timing": {"wall_s": r["wall_s"], "event_ms": r["event_ms"]},
    }
    if not args.no_scale:
        print("[bench] quadrotor at scale", file=sys.stderr, flush=True)
        out["at_scale"] = bench_at_scale()
    if not args.no_batched:
        print("[bench] batched path: 64 mixed controllers", file=sys.stderr, flush=True)
        out["batched"] = bench_batched()
    if not args.no_served:
        print(f"[bench] served path: 256 robots x 50 Hz for {args.serve_seconds:g} s", file=sys.stderr, flush=True)
        out["served"] = bench_served(args.serve_seconds)
    if not args.no_missions:
        from paper_2504_06437_amd import mission
        print(f"[bench] missions: {args.mission_runs} closed-loop runs each", file=sys.stderr, flush=True)
        out["missions"] = {"note": "synthetic layouts with the paper's mission settings; not its layouts",
                           "results": [mission.run_mission(m, args.mission_runs) for m in (1, 2, 3)]}
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

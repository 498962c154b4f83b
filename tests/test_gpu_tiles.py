"""Tile-shape choice on the GPU: a shape gets the same tile size in every
process (so its results repeat bit for bit across processes), and a change of
obstacles that would overrun the tile's LDS is refused before any launch."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2504_06437_amd import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import numpy as np
from paper_2504_06437_amd import workloads as W
from paper_2504_06437_amd.controller import Controller
wl = W.car(K=3000, T=37, J=77, seed=12)
c = Controller(wl["params"])
c.load_workload(wl)
c.step(wl["x0"])
np.save(sys.argv[2], np.concatenate([c.costs(), c.last_optimal().ravel().astype(np.float64)]))
print(json.dumps({"tile_samples": c.info()["tile_samples"]}))
c.close()
"""


def test_tile_choice_repeats_across_processes(tmp_path):
    """Two processes step the same controller.  The first times the tile
    candidates (no table entry for this shape) and appends its choice to the
    tuning cache; the second reads it, so both use one tile size and produce
    the same bits."""
    cache = tmp_path / "tiles.txt"
    env = dict(os.environ, MPPI_TUNE_CACHE=str(cache), MPPI_TILE_TABLE="")
    env.pop("MPPI_AUTOTUNE", None)
    outs = []
    for i in range(2):
        print(f"[test] child process {i}", flush=True)
        r = subprocess.run([sys.executable, "-c", CHILD, ROOT, str(tmp_path / f"out{i}.npy")], env=env,
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stdout + r.stderr
        outs.append((json.loads(r.stdout.strip().split("\n")[-1]), np.load(tmp_path / f"out{i}.npy")))
    lines = [ln.split() for ln in open(cache) if ln.strip()]
    assert len(lines) == 1 and lines[0][:4] == ["2", "3000", "37", "77"]
    assert int(lines[0][8]) == outs[0][0]["tile_samples"] == outs[1][0]["tile_samples"]
    np.testing.assert_array_equal(outs[0][1], outs[1][1])


def test_shipped_table_sets_the_benchmark_tiles():
    """The shapes of the benchmark workloads come from the shipped table
    without timing, whatever the process."""
    path = os.path.join(ROOT, "paper_2504_06437_amd", "tile_table.txt")
    if not os.path.exists(path):
        pytest.skip("no tile table shipped yet")
    table = {}
    for line in open(path):
        if not line.startswith("#") and line.strip():
            v = [int(x) for x in line.split()]
            table[tuple(v[:8])] = v[8]
    from paper_2504_06437_amd.controller import Controller
    for wl in (W.car(), W.quad_large(), W.quad_small()):
        p = wl["params"]
        key = ({"quad6": 0, "quad5": 1, "car": 2}[p["model"]], p["K"], p["T"], len(wl["obstacles"]),
               len(p["shape"]), 1 if wl.get("map") is not None else 0, 0, 0)
        assert key in table
        c = Controller(p)
        c.load_workload(wl)
        assert c.info()["tile_samples"] == table[key]
        c.close()


def test_obstacles_that_overrun_the_smoothing_sums_are_refused():
    """A vehicle with T = 1024 and smoothing (half window 2), created without
    obstacles: 2048 obstacles leave a tile's chunk too short for the 2T FP64
    sums it smooths, with the tile size fixed or chosen, so the call fails
    with MPPI_E_INVALID (and the controller keeps working without them)."""
    from paper_2504_06437_amd import _lib as A
    from paper_2504_06437_amd.controller import Controller
    wl = W.car(K=4096, T=1024, J=1)
    obs = W.car(K=16, T=4, J=2048)["obstacles"]
    for S in (16, 0):
        p = dict(wl["params"], sgf_half_window=2, sgf_order=2, tile_samples=S)
        c = Controller(p)
        with pytest.raises(A.MppiError) as e:
            c.set_obstacles(obs)
        assert e.value.status == A.E_INVALID
        c.set_obstacles(wl["obstacles"])
        c.set_reference(wl["x_ref"])
        c.step(wl["x0"])
        assert c.info()["status"] == 0
        c.close()

"""Measure the rollout tile shape of the benchmark and test workloads on an
MI355X and write the table the library reads beside itself (tile_table.txt).

The tile size S fixes the order of the tile's reductions, so a shape must get
the same S in every process for its results to repeat bit for bit.  The
library looks a shape up in this table before it times candidates; this
script runs the library's own autotuner (timing every candidate on the
shape's data) with the shipped table switched off, and writes what it chose.

    python -m paper_2504_06437_amd.tune --out tile_table.txt
"""
from __future__ import annotations

import argparse
import os
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))


def workloads():
    """Every shape the benchmark and the GPU tests build at full size."""
    from . import mission
    from . import workloads as W
    out = [W.quad_small(), W.car(), W.quad_large()]
    out += W.batch(64, 3)
    out += W.batch(256, 4)
    for m in (1, 2, 3):
        out += [mission.layout(m, s) for s in range(10)]
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=os.path.join(HERE, "tile_table.txt"))
    args = ap.parse_args(argv)
    fd, cache = tempfile.mkstemp(prefix="mppi_tiles_", suffix=".txt")
    os.close(fd)
    # the library reads these when it first chooses a tile
    os.environ["MPPI_TILE_TABLE"] = ""
    os.environ["MPPI_TUNE_CACHE"] = cache
    os.environ.pop("MPPI_AUTOTUNE", None)
    from .controller import Controller
    wls = workloads()
    for i, wl in enumerate(wls):
        c = Controller(wl["params"])
        c.load_workload(wl)
        c.close()
        if (i + 1) % 10 == 0:
            print(f"[tune] {i + 1}/{len(wls)} shapes", flush=True)
    rows = {}
    with open(cache) as fh:
        for line in fh:
            f = line.split()
            if len(f) == 9:
                rows.setdefault(tuple(int(v) for v in f[:8]), int(f[8]))
    os.unlink(cache)
    with open(args.out, "w") as fh:
        fh.write("# Rollout tile sizes measured on an MI355X by paper_2504_06437_amd/tune.py.\n")
        fh.write("# model K T J P costmap sgf_half_window cost_mode tile_samples\n")
        for k in sorted(rows):
            fh.write(" ".join(str(v) for v in k) + f" {rows[k]}\n")
    print(f"[tune] {len(rows)} shapes -> {args.out}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

"""Host-only checks of the rollout tile's LDS fitting rule, the one question
every tile choice asks (tile_fits in mppi_internal.hpp): a tile fits when a
chunk holds at least one horizon step and, with Savitzky-Golay smoothing, the
2T FP64 update sums fit in the spent chunk inputs.  Also the tune table the
library ships parses and holds only shapes that fit."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2504_06437_amd", "csrc")


@pytest.fixture(scope="module")
def fit_exe(tmp_path_factory):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("tiles") / "tile_fit_check")
    subprocess.check_call([hipcc, "-O1", "-std=c++17", "-I", CSRC, "-I", os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "native", "tile_fit_check.cpp"), "-o", exe])
    return exe


def _query(exe, rows):
    inp = "\n".join(" ".join(str(v) for v in r) for r in rows) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    return [tuple(int(v) for v in line.split()) for line in out if line.strip()]


def _budget():
    src = open(os.path.join(CSRC, "mppi_internal.hpp")).read()
    import re
    return int(re.search(r"constexpr size_t kLdsLimit = (\d+);", src).group(1))


def test_smoothing_sums_that_do_not_fit_are_rejected(fit_exe):
    """The case of a vehicle with T = 1024 and smoothing: fine with no
    obstacle, but with 2048 obstacles a 16-sample tile's chunk is too short
    to hold the 2T FP64 sums, and the rule says so."""
    (f0, tc0, _, _), (f1, tc1, _, _), (f2, tc2, _, _) = _query(
        fit_exe, [(0, 1024, 4, 16, 2), (2048, 1024, 4, 16, 2), (2048, 1024, 4, 16, 0)])
    assert f0 == 1 and tc0 > 0
    assert f1 == 0 and tc1 > 0 and 2 * 1024 * 8 > 2 * tc1 * 16 * 16
    assert f2 == 1


def test_fitting_rule_invariants(fit_exe):
    budget = _budget()
    rng = np.random.Generator(np.random.PCG64(3))
    rows = []
    for _ in range(3000):
        rows.append((int(rng.integers(0, 2049)), int(rng.integers(1, 1025)), int(rng.choice([4, 5, 6])),
                     int(rng.choice([16, 32, 64, 128, 256])), int(rng.choice([0, 0, 1, 4, 16]))))
    for (J, T, n, S, m), (fits, tc, lds, keep) in zip(rows, _query(fit_exe, rows)):
        if tc > 0:
            assert lds <= budget
        if fits:
            assert tc >= 1
            if m > 0:
                assert 2 * T * 8 <= 2 * tc * S * 16
        else:
            assert tc == 0 or (m > 0 and 2 * T * 8 > 2 * tc * S * 16)
        if keep:
            assert tc > 0


def test_shipped_tile_table_parses_and_fits(fit_exe):
    path = os.path.join(ROOT, "paper_2504_06437_amd", "tile_table.txt")
    if not os.path.exists(path):
        pytest.skip("no tile table shipped yet")
    rows, keys = [], set()
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        model, K, T, J, P, cmap, m, mode, S = (int(v) for v in line.split())
        assert model in (0, 1, 2) and S in (16, 32, 64, 128, 256) and cmap in (0, 1) and mode in (0, 1)
        assert (model, K, T, J, P, cmap, m, mode) not in keys
        keys.add((model, K, T, J, P, cmap, m, mode))
        rows.append((J, T, {0: 6, 1: 5, 2: 4}[model], S, m))
    assert rows
    assert all(f == 1 for f, _, _, _ in _query(fit_exe, rows))

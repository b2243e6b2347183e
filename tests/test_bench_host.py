"""Host-side logic of bench.py (no GPU): the algorithmic byte counts
against the sizes of a generated system's own arrays, the CGS2 step bytes
against a step-by-step count of a restarted run, the traffic lookup's
source-hash rule, and the one-GPU rule of the command line."""
import hashlib
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import bench
import reservoir_inputs as ri

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _system(nx=5, ny=4, nz=3):
    s = ri.blackoil_system(nx, ny, nz, seed=3)
    rowptr = np.asarray(s["rowptr"], dtype=np.int32)
    col = np.asarray(s["col"], dtype=np.int32)
    val = np.asarray(s["val"], dtype=np.float64)
    return rowptr, col, val


def test_spmv_bytes_are_the_arrays_read_and_written():
    rowptr, col, val = _system()
    nb = len(rowptr) - 1
    x = np.zeros(3 * nb)
    # matrix values, int32 column indices and row pointers read once,
    # x read once, y written once
    expect = val.nbytes + col.nbytes + rowptr.nbytes + 2 * x.nbytes
    assert bench.algorithmic_bytes(nb, len(col))["spmv_bsr3"] == expect


def test_sweep_bytes_count_the_triangle_blocks():
    rowptr, col, val = _system()
    nb = len(rowptr) - 1
    rows = np.repeat(np.arange(nb), np.diff(rowptr))
    nl = int(np.sum(col < rows))            # strictly lower blocks
    nu = int(np.sum(col > rows))
    assert nl == nu
    blk = val[0].nbytes + 4                 # one 3x3 FP64 block and its index
    vec = 3 * nb * 8
    ab = bench.algorithmic_bytes(nb, len(col))
    # forward: L blocks, row pointers, b read, y written
    assert ab["ilu_fwd_bsr3_f64"] == nl * blk + rowptr.nbytes + 2 * vec
    # backward: U blocks, the diagonal inverses, row pointers, y read, x written
    assert ab["ilu_bwd_bsr3_f64"] == nu * blk + nb * val[0].nbytes + rowptr.nbytes + 2 * vec


def test_cgs2_average_matches_a_step_by_step_count():
    n, restart = 1000, 30
    for iters, launches in [(1, 1), (29, 30), (30, 30), (61, 62), (2044, 2045)]:
        tot = 0
        for j in range(launches):
            nc = min(j % restart + 1, restart) if j < iters else min(iters % restart + 1, restart)
            # pass 1 reads V (nc columns) and w; passes 2 and 3 read V and w
            # and write one vector each
            tot += ((nc + 1) + (nc + 2) + (nc + 2)) * n * 8
        assert bench.cgs2_avg_bytes(n, iters, launches, restart) == pytest.approx(tot / launches,
                                                                                 rel=1e-15)


def test_lagged_cgs2_average_matches_a_step_by_step_count():
    n, restart = 1000, 30
    for iters, launches in [(1, 1), (29, 30), (30, 30), (61, 62), (2044, 2045)]:
        tot = 0
        for j in range(launches):
            nc = min(j % restart + 1, restart) if j < iters else min(iters % restart + 1, restart)
            # pass A reads the nc columns (u the last) and w; pass B reads
            # them and w again and writes v_j and the next vector
            tot += ((nc + 1) + (nc + 1 + 2)) * n * 8
        avg = bench.cgs2_avg_bytes(n, iters, launches, restart, step_bytes=bench.dcgs2_step_bytes)
        assert avg == pytest.approx(tot / launches, rel=1e-15)


def test_traffic_lookup_requires_the_profiled_source(tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("// kernel v1\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    entry = {"bytes_per_launch": 1234, "source": "kernel.hip",
             "source_sha256": hashlib.sha256(src.read_bytes()).hexdigest()}
    (prof / "traffic.json").write_text(json.dumps({"wl": {"k": entry}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profiles("k", "wl") == 1234.0
    assert bench.traffic_from_profiles("k", "other_workload") is None
    assert bench.traffic_from_profiles("missing", "wl") is None
    src.write_text("// kernel v2\n")          # the kernel changed since the counters
    assert bench.traffic_from_profiles("k", "wl") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""

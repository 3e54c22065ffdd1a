"""Host-side checks of the benchmark's command line (no GPU needed)."""
from __future__ import annotations

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_rate_is_null_without_a_record():
    sys.path.insert(0, ROOT)
    import bench
    r = bench.with_traffic_rate({"traffic": None, "avg_launch_us": 10.0, "peak": 8000.0})
    assert r["traffic_GBps"] is None and r["traffic_frac"] is None
    r = bench.with_traffic_rate({"traffic": 8e7, "avg_launch_us": 10.0, "peak": 8000.0})
    assert abs(r["traffic_GBps"] - 8000.0) < 1e-6 and abs(r["traffic_frac"] - 1.0) < 1e-9


def test_committed_traffic_records_name_known_kernels():
    """Every committed counter record names a kernel whose sources the
    benchmark can hash (a record whose hash no longer matches is reported
    as null by the benchmark, never used)."""
    sys.path.insert(0, ROOT)
    import bench
    prof = os.path.join(ROOT, "profiles")
    for f in sorted(os.listdir(prof)):
        if f.startswith("traffic_") and f.endswith(".json"):
            with open(os.path.join(prof, f)) as fh:
                rec = json.load(fh)
            names = [k for k in bench.KERNEL_SOURCES if k in rec["kernel"]]
            assert names, f
            assert len(bench.kernel_hash(names[0])) == len(rec["kernel_hash"]) == 16
            assert rec["hbm_bytes_per_launch"] > 0 and rec["algorithmic_bytes_per_launch"] > 0


def test_one_gpu_slab_is_the_middle_y_slab_of_the_256_case():
    """The --config 7 workload is rows [111, 145) of the 256^3 umbrella case,
    with voxel centres (grid-centre frame) identical to the full grid's."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    from paper_1907_05709_amd import workloads as W
    slab, _ = bench.workload(7)
    full = W.case_umbrella()
    assert slab.shape == (256, 34, 256)
    assert np.array_equal(slab.labels, full.labels[:, 111:145])
    ys = W.voxel_axes(slab.shape, slab.spacing)[1]
    yf = W.voxel_axes(full.shape, full.spacing)[1][111:145]
    assert np.array_equal(ys, yf)
    assert np.array_equal(slab.needle.pts, full.needle.pts) and slab.n_steps == full.n_steps

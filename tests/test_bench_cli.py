"""bench.py's command-line contract, checked without a GPU: more than one GPU
is refused with a message (this benchmark runs on one GPU), and the kernel
source hash that ties the committed traffic summary to the code is stable."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_summary_names_a_kernel_hash():
    path = os.path.join(ROOT, "profiles", "traffic_layer12_m24n12.json")
    d = json.load(open(path))
    h = bench.kernel_source_hash()
    assert len(h) == 16 and all(c in "0123456789abcdef" for c in h)
    assert len(d["kernel_source_hash"]) == 16
    for v in ("c64comp", "c64", "c128"):
        e = d["variants"][v]
        # the bytes per launch are the scaled counters: FETCH_SIZE x fetch_scale + WRITE_SIZE x write_scale
        want = (e["fetch_kib"] * e["fetch_scale"] + e["write_kib"] * e["write_scale"]) * 1024
        assert abs(e["hbm_bytes_per_launch"] - want) <= 1e-6 * want
        assert e["hbm_bytes_per_launch"] > e["algorithmic_bytes_per_launch"]

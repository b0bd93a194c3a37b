"""Host-side checks of bench.py that need no GPU: the one-GPU guard and the rule that ties the
committed HBM counters to the dominant kernel's code."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

KERNELS = os.path.join(ROOT, "paper_2505_23963_amd", "csrc", "fdtdb_kernels.hip")
HEAD = "void k_update_e_bath(const EArgs a"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_kernel_hash_ignores_comments_but_not_code():
    src = open(KERNELS).read()
    base = bench.source_hash("E_lorentz_bath_nb8", src)
    s = src.index(HEAD)
    body = src.index("{", s) + 1
    commented = src[:body] + "\n    // a comment that changes nothing\n" + src[body:]
    assert bench.source_hash("E_lorentz_bath_nb8", commented) == base
    e = src.index("cf.head[1] * Pc[ci]", s)
    changed = src[:e] + "cf.head[2] * Pc[ci]" + src[e + len("cf.head[1] * Pc[ci]"):]
    assert bench.source_hash("E_lorentz_bath_nb8", changed) != base
    # the component-split kernel of the 512^3 workload has its own hash over its own code
    s2 = src.index("void bath_component(const EArgs &a")
    e2 = src.index("co[1] * Pc", s2)
    changed2 = src[:e2] + "co[2] * Pc" + src[e2 + len("co[1] * Pc"):]
    assert bench.source_hash("E_lorentz_bath_nb16", changed2) != bench.source_hash("E_lorentz_bath_nb16", src)
    assert bench.source_hash("E_lorentz_bath_nb8", changed2) == base


def test_counter_file_is_calibrated():
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic_counters.json")))
    cal = t["calibration"]
    # a device copy reads FETCH_SIZE at half the bytes moved and WRITE_SIZE at all of them
    assert abs(cal["FETCH_SIZE"]["scale"] - 2.0) < 0.01
    assert abs(cal["WRITE_SIZE"]["scale"] - 1.0) < 0.01
    k = t["kernels"]["E_lorentz_bath_nb8"]
    assert abs(k["hbm_bytes_per_launch"] - (k["read_bytes"] + k["write_bytes"])) < 1.0
    # the counted bytes can only exceed the algorithmic 364 B per cell of the 26.2 M-cell layer
    assert k["hbm_bytes_per_launch"] >= 364 * 26214400

"""The parts of bench.py's contract that need no GPU: a request for more
than one GPU ends with a message, the slot model's per-pair counts, and the
rule that committed counter traffic is reported only for the kernel source it
was measured on."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "single MI355X" in r.stderr and not r.stdout.strip()


def test_slot_model():
    assert bench.slots_per_pair("interp", 8) == 30.875
    assert bench.slots_per_pair("interp", 8, nfd=4) == 31.75
    assert bench.slots_per_pair("interp", 8, coef16=True) == 24.875
    assert bench.slots_per_pair("direct", 8) == 135
    assert abs(bench.PEAK_SLOTS - 3.93216e13) < 1e6


def test_comments_do_not_change_the_kernel_hash():
    code = "int f(int x) {\n  return x + 1;  // one more\n}\n"
    assert bench.strip_comments(code) == bench.strip_comments("/* a\n b */\n" + code.replace("// one more", ""))


def test_traffic_only_for_the_measured_kernel_source():
    import json
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        d = json.load(f)
    e = d["demod_interp:config1"]
    b, n = bench.measured_traffic("demod_interp", "config1")
    if e["kernel_source_hash"] == bench.kernel_source_hash():
        assert b == e["bytes_per_pass"] > 0 and n == e["launches_per_pass"] >= 1
    else:
        assert (b, n) == (None, None)
    assert bench.measured_traffic("demod_interp", "no-such-workload") == (None, None)


def test_error_statistics_and_form_names():
    import numpy as np
    e = bench.err_stats([4.0004, 10.0, 2.0], [4.0, 10.0, 2.0002])
    assert abs(e["max_e"] - 1e-4) < 1e-12 and e["n_templates"] == 3 and e["at_metric_tolerance"]
    assert not bench.err_stats([4.01], [4.0])["at_metric_tolerance"]
    assert bench.err_stats([np.nan], [4.0])["finite"] is False
    assert bench.parse_form("bf16+coef16") == ("bf16", False, True)
    assert bench.parse_form("c64+split") == ("c64", True, False)
    assert bench.method_slots(8) == 108 and bench.method_slots(16) == 188
    assert 1 <= bench.host_threads() <= 16

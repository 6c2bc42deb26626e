"""Host helpers of bench.py, no GPU: percentiles, the comment-insensitive
hash of the iteration kernel's source, and the rule that measured traffic
is reported only for the source and workload the counters were taken on."""
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_percentiles_match_linear_interpolation():
    rng = np.random.default_rng(5)
    for size in (1, 2, 7, 100):
        x = rng.random(size).tolist()
        for q in (0, 50, 99, 100):
            assert abs(bench.pct(x, q) - float(np.percentile(x, q))) < 1e-15
    assert bench.pct([], 50) is None


def test_code_text_ignores_comments_and_layout_only():
    a = "int f(int x) { // twice\n  return 2 * x; /* doubled */ }\n"
    b = "int f(int x)\n{\n    return 2 * x;\n}\n"
    c = "int f(int x) { return 3 * x; }"
    assert bench.code_text(a) == bench.code_text(b)
    assert bench.code_text(a) != bench.code_text(c)


def test_traffic_only_for_the_source_and_workload_measured(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("w") is None                 # no file
    f.write_text(json.dumps({"workload": "w", "kernel_sha": bench.kernel_hash(),
                             "bytes_per_iteration": 123.0}))
    assert bench.measured_traffic("w") == 123.0
    assert bench.measured_traffic("other") is None
    f.write_text(json.dumps({"workload": "w", "kernel_sha": "0" * 16, "bytes_per_iteration": 1.0}))
    assert bench.measured_traffic("w") is None                 # kernel changed since

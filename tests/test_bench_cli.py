"""bench.py on the CPU: it refuses more than one GPU, and the roofline record
it builds from the committed rocprofv3 summaries (profiles/traffic.json,
profiles/counters.json) is taken only for the kernel source and variant the
counters were collected on."""
import json
import os
import subprocess
import sys
import types

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_profile_records_match_the_kernel_source():
    traffic = json.load(open(bench.TRAFFIC_FILE))
    counters = json.load(open(bench.COUNTERS_FILE))
    assert traffic and set(traffic) == set(counters)
    sha = bench.kernel_sha()
    for key, rec in traffic.items():
        name, v = key.split("/v")
        v = int(v)
        assert rec["kernel_sha256"] == sha, key
        assert os.path.exists(os.path.join(ROOT, rec["source"])), rec["source"]
        tr = bench.measured_traffic(name, v)
        assert tr is not None and tr["bytes"] == rec["fetch_bytes"] + rec["write_bytes"]
        assert bench.measured_counters(name, v) is not None
        # another variant has no record
        assert bench.measured_traffic(name, v + 100) is None


def test_roofline_fractions():
    key = next(iter(json.load(open(bench.TRAFFIC_FILE))))
    name, v = key.split("/v")
    w = types.SimpleNamespace(name=name, dtype=name.split("-")[1])
    adds, ms = 6.66e10, 4.0
    r = bench.roofline(w, adds, 1.09e9, ms, int(v))
    achieved = adds / (ms * 1e-3) / 1e12
    assert r["bound"] == "alu" and r["unit"] == "Tadd/s"
    assert abs(r["achieved"] - achieved) < 1e-9 * achieved
    assert abs(r["peak"] - 78.6432) < 1e-9 and abs(r["frac"] - achieved / 78.6432) < 1e-12
    assert abs(r["frac_unpacked"] - 2 * r["frac"]) < 1e-12
    assert r["traffic"] is not None and r["traffic"] > 0
    # a kernel the counters were not taken on reports no traffic
    assert bench.roofline(w, adds, 1.09e9, ms, int(v) + 100)["traffic"] is None

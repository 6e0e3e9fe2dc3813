"""The autotuner's cache file (DEDISP_TUNE_CACHE): a tuning result is written
as one line and read back by a later process without timing again; an entry
for another variant that fits is taken as it stands, and a line whose key
names another kernel registry is ignored.  Each step runs in a child process
(the file is read once per process), one after the other."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, %r)
from paper_1111_6399_amd import dedisp as dd
from paper_1111_6399_amd import workloads as wl
w = wl.small_f32()
p = dd.Plan.for_workload(w)
fits = []
for v in range(1, dd.dedisp_variant_count()):
    try:
        p.variant = v
        fits.append(v)
    except dd.DedispError:
        pass
v, ms = dd.dedisp_autotune(p.handle, w.nsamp)  # sets the plan's variant
assert p.variant == v
print(v, repr(ms), ",".join(map(str, fits)), flush=True)
""" % ROOT


def child(cache):
    print("autotune child with cache file %s" % cache, flush=True)
    env = dict(os.environ, DEDISP_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", CHILD], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    v, ms, fits = r.stdout.split()
    return int(v), float(ms), [int(f) for f in fits.split(",")]


def test_tune_cache_file(tmp_path, device):
    cache = tmp_path / "tune.txt"
    v1, ms1, fits = child(cache)
    assert v1 in fits and ms1 > 0
    lines = cache.read_text().split("\n")
    assert lines[-1] == "" and len(lines) == 2, lines
    key, v_file, ms_file = lines[0].split()
    assert int(v_file) == v1 and abs(float(ms_file) - ms1) <= 1e-5 * ms1

    # read back: the same result, no new line
    v2, ms2, _ = child(cache)
    assert (v2, ms2) == (v1, float(ms_file))
    assert len(cache.read_text().split("\n")) == 2

    # another fitting variant under the same key is taken as written
    other = next(v for v in fits if v != v1)
    cache.write_text("%s %d 0.125\n" % (key, other))
    v3, ms3, _ = child(cache)
    assert (v3, ms3) == (other, 0.125)

    # a key from another registry does not match: the plan is tuned again
    parts = key.split(":")  # the device name may hold colons itself
    assert parts[-2].startswith("r")
    stale = ":".join(parts[:-2] + ["r0", parts[-1]])
    cache.write_text("%s %d 0.125\n" % (stale, other))
    v4, ms4, _ = child(cache)
    assert v4 in fits and ms4 != 0.125
    assert len(cache.read_text().split("\n")) == 3

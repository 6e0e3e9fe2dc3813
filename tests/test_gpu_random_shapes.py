"""Seeded random shapes through every kernel variant that fits: bands of the
LOFAR and MeerKAT kinds with random channel counts, trial grids (sorted,
unevenly spaced, some repeated trials), output lengths and input types;
uint8 exact, float within the per-output bound, and every variant's result
identical to the others bit for bit."""
import numpy as np
import pytest

import oracle
from paper_1111_6399_amd import workloads as wl

from gpu_util import abs_sum, check_float, run

pytestmark = pytest.mark.gpu

CASES = 36


@pytest.fixture(scope="module")
def dd(device):
    from paper_1111_6399_amd import dedisp
    return dedisp


def draw(k):
    rng = np.random.default_rng([7, k])
    if rng.random() < 0.5:  # LOFAR kind: wide fractional band, long delays
        nchans = int(rng.integers(8, 200))
        band = wl.Band(nchans, 150.0, float(rng.uniform(0.05, 0.4)), 327.68e-6)
        dm_max = float(rng.uniform(0.5, 12.0))
    else:  # MeerKAT kind: narrow fractional band, short delays
        nchans = int(rng.integers(16, 300))
        band = wl.Band(nchans, 1712.0, 428.0 / nchans, 64e-6)
        dm_max = float(rng.uniform(20.0, 600.0))
    ndm = int(rng.integers(1, 120))
    dms = np.sort(rng.uniform(0.0, dm_max, ndm))
    if ndm > 3:
        dms[1] = dms[2]  # a repeated trial
    nsamp = int(rng.integers(1, 4000))
    dtype = ("f32", "f16", "u8")[k % 3]
    return band, dms, nsamp, dtype, rng


@pytest.mark.parametrize("k", range(CASES))
def test_random_shape_every_variant(dd, k):
    band, dms, nsamp, dtype, rng = draw(k)
    sh, m = oracle.shift_table(band.nchans, band.f_top, band.df, band.tsamp, dms)
    print("case %d: %s, %d ch, %d trials, %d samples, max delay %d" % (k, dtype, band.nchans, len(dms), nsamp, m),
          flush=True)
    plan = dd.Plan(band.nchans, band.f_top, band.df, band.tsamp, dms, dtype)
    assert plan.max_shift == m and np.array_equal(plan.shift_table(), sh)
    shape = (band.nchans, nsamp + m)
    if dtype == "u8":
        x = rng.integers(0, 256, shape).astype(np.uint8)
    else:
        x = rng.standard_normal(shape).astype(np.float32 if dtype == "f32" else np.float16)
    want = oracle.dedisperse(x, sh, nsamp)
    scale = None if dtype == "u8" else abs_sum(x, sh, nsamp)
    first = None
    ran = 0
    for v in range(dd.dedisp_variant_count()):
        try:
            plan.variant = v
        except dd.DedispError:
            continue
        got = run(plan, x, nsamp)
        if dtype == "u8":
            assert np.array_equal(got.astype(np.int64), want), "variant %d" % v
        else:
            check_float(got, want, scale)
        if first is None:
            first = got
        else:
            assert np.array_equal(first.view(np.uint32), got.view(np.uint32)), "variant %d differs" % v
        ran += 1
    assert ran >= 2  # the direct kernel and at least one tile variant

"""GPU parity: the HIP kernels against the oracle, element by element.

Integer (uint8 -> int32) results must be bit-exact; float results within
|y - y64| <= 1e-5 * sum_c |x_c| per output.  Every kernel variant is checked,
and all variants must agree with each other bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_1111_6399_amd import workloads as wl

from gpu_util import REL_TOL, abs_sum, check_float, per_dm_error, run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd(device):
    from paper_1111_6399_amd import dedisp
    return dedisp


def make_case(w: wl.Workload):
    b = w.band
    sh, m = oracle.shift_table(b.nchans, b.f_top, b.df, b.tsamp, w.dms)
    x = wl.generate(w, sh, m)
    return sh, m, x


def all_variants(dd, plan):
    out = [0]
    for v in range(1, dd.dedisp_variant_count()):
        try:
            plan.variant = v
            out.append(v)
        except dd.DedispError:
            pass
    return out


def test_small_f32_every_variant(dd):
    w = wl.small_f32()
    sh, m, x = make_case(w)
    plan = dd.Plan.for_workload(w)
    assert plan.max_shift == m
    assert np.array_equal(plan.shift_table(), sh)
    want = oracle.dedisperse(x, sh, w.nsamp)
    scale = abs_sum(x, sh, w.nsamp)
    first = None
    variants = all_variants(dd, plan)
    assert len(variants) >= 3
    for v in variants:
        got = run(plan, x, w.nsamp, variant=v)
        check_float(got, want, scale)
        if first is None:
            first = got
        else:
            assert np.array_equal(got.view(np.uint32), first.view(np.uint32)), "variant %d differs" % v
    # the planted pulse is found at its trial
    assert np.unravel_index(np.argmax(first), first.shape) == (50, 2000)


@pytest.mark.parametrize("dtype", ["f32", "f16", "u8"])
def test_lofar_shape_reduced_time(dd, dtype):
    """Full channel and trial grid of the LOFAR-shaped beam, 3000 output samples
    (several time tiles and a ragged tail)."""
    w = wl.lofar(dtype, nsamp=3000)
    sh, m, x = make_case(w)
    plan = dd.Plan.for_workload(w)
    rows = np.unique(np.concatenate([np.arange(0, 2048, 37), [0, 1, 2047], [p[0] for p in w.pulses]]))
    want = oracle.dedisperse(x, sh, w.nsamp, rows=rows)
    for v in sorted({0, plan.variant}):
        got = run(plan, x, w.nsamp, variant=v)[rows]
        if dtype == "u8":
            assert got.dtype == np.int32
            assert np.array_equal(got.astype(np.int64), want)
        else:
            check_float(got, want, abs_sum(x, sh, w.nsamp, rows=rows))
            e = per_dm_error(got, want)
            assert e.max() < REL_TOL


def test_meerkat_block_tile_variants(dd):
    """The MeerKAT-shaped block's full channel and trial grid (4096 x 4096,
    uint8), 2100 output samples (two 1008-sample time tiles and a ragged
    tail): the small-spread tile (16 trials x 1008, 8 channels a stage) and
    the 8 x 2016 tile with 4 channels a stage equal the oracle on sampled
    trials."""
    w = wl.meerkat_block(nsamp=2100)
    sh, m, x = make_case(w)
    plan = dd.Plan.for_workload(w)
    rows = np.unique(np.concatenate([np.arange(0, 4096, 97), [0, 1, 15, 16, 17, 4094, 4095]]))
    want = oracle.dedisperse(x, sh, w.nsamp, rows=rows)
    for v in (11, 5):
        got = run(plan, x, w.nsamp, variant=v)[rows]
        assert np.array_equal(got.astype(np.int64), want), "variant %d" % v


def test_f16_error_against_float_data(dd):
    """Per-trial error of the half-precision path against the binary64 oracle on the
    original float32 data (quantisation included), reported, and the exact-input gate."""
    w = wl.lofar("f32", nsamp=2048, ndm=256)
    sh, m, x32 = make_case(w)
    x16 = x32.astype(np.float16)
    plan = dd.Plan(w.band.nchans, w.band.f_top, w.band.df, w.band.tsamp, w.dms, "f16")
    got = run(plan, x16, w.nsamp)
    check_float(got, oracle.dedisperse(x16, sh, w.nsamp), abs_sum(x16, sh, w.nsamp))
    e = per_dm_error(got, oracle.dedisperse(x32, sh, w.nsamp))
    # half has an 11-bit significand: per-sample error <= 2^-11 relative, sums of
    # N(0,1) noise stay well inside 1e-3 of the peak
    assert e.max() < 1e-3


@pytest.mark.parametrize("dtype", ["f32", "u8", "f16"])
def test_closed_forms(dd, dtype):
    b = wl.SMALL
    dms = wl.dm_grid(70, 0.13)
    sh, m = oracle.shift_table(b.nchans, b.f_top, b.df, b.tsamp, dms)
    plan = dd.Plan(b.nchans, b.f_top, b.df, b.tsamp, dms, dtype)
    nsamp = 1500
    npdt = {"f32": np.float32, "f16": np.float16, "u8": np.uint8}[dtype]
    # constant input
    v = 255 if dtype == "u8" else 0.75
    x = np.full((b.nchans, nsamp + m), v, dtype=npdt)
    for var in all_variants(dd, plan):
        assert np.all(run(plan, x, nsamp, variant=var) == b.nchans * v)
    # DM 0 is the channel sum
    rng = np.random.default_rng(9)
    x = rng.integers(0, 200, (b.nchans, nsamp + m)).astype(npdt)
    got = run(plan, x, nsamp)
    assert np.array_equal(got[0].astype(np.float64), x[:, :nsamp].astype(np.float64).sum(axis=0))
    # planted pulse, no noise: exact peak at its trial, unique
    x = np.zeros((b.nchans, nsamp + m), dtype=npdt)
    wl.plant_pulses(x, sh, [(40, 700, 9 if dtype == "u8" else 3.5, 1)])
    got = run(plan, x, nsamp)
    peak = b.nchans * (9 if dtype == "u8" else 3.5)
    assert got[40, 700] == peak
    assert np.count_nonzero(got == got.max()) == 1
    # single-channel impulse recovers the delays
    x = np.zeros((b.nchans, nsamp + m), dtype=npdt)
    c0, t1 = 50, 1200
    x[c0, t1] = 1
    got = run(plan, x, nsamp)
    for d in range(len(dms)):
        assert list(np.flatnonzero(got[d])) == [t1 - sh[c0, d]]


@pytest.mark.parametrize("nchans,ndm,nsamp", [(1, 1, 1), (3, 1, 7), (1, 5, 300), (33, 17, 129), (70, 65, 2049),
                                              (5, 200, 5000)])
def test_edge_shapes(dd, nchans, ndm, nsamp):
    band = wl.Band(nchans, 150.0, 0.5, 327.68e-6)
    rng = np.random.default_rng(nchans * 1000 + ndm)
    dms = np.sort(rng.uniform(0, 20, ndm))
    sh, m = oracle.shift_table(band.nchans, band.f_top, band.df, band.tsamp, dms)
    x = rng.standard_normal((nchans, nsamp + m)).astype(np.float32)
    xu = rng.integers(0, 256, (nchans, nsamp + m)).astype(np.uint8)
    want = oracle.dedisperse(x, sh, nsamp)
    wantu = oracle.dedisperse(xu, sh, nsamp)
    xh = x.astype(np.float16)  # half input: the tail of 1-7 samples past the last 16 bytes
    wanth = oracle.dedisperse(xh, sh, nsamp)
    p = dd.Plan(nchans, band.f_top, band.df, band.tsamp, dms, "f32")
    pu = dd.Plan(nchans, band.f_top, band.df, band.tsamp, dms, "u8")
    ph = dd.Plan(nchans, band.f_top, band.df, band.tsamp, dms, "f16")
    for v in all_variants(dd, p):
        check_float(run(p, x, nsamp, variant=v), want, abs_sum(x, sh, nsamp))
    for v in all_variants(dd, pu):
        assert np.array_equal(run(pu, xu, nsamp, variant=v).astype(np.int64), wantu)
    for v in all_variants(dd, ph):
        check_float(run(ph, xh, nsamp, variant=v), wanth, abs_sum(xh, sh, nsamp))


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_staged_input_beyond_4gib(dd, dtype):
    """A plan whose staged input is larger than 2^32 bytes (the tile kernels
    address each row from its own base) on 1024 channels of a low band, with
    trials dense enough for the tiles: a tiled variant and the direct kernel
    against the oracle on sampled trials, every output sample."""
    import torch
    nchans, nsamp = 1024, 5000
    band = wl.Band(nchans, 150.0, 0.09, 327.68e-6)
    dms = (700.0 if dtype == "u8" else 360.0) + 0.1 * np.arange(64)
    sh, m = oracle.shift_table(nchans, band.f_top, band.df, band.tsamp, dms)
    staged = 2 if dtype == "u8" else 4
    assert nchans * (nsamp + m) * staged > 2 ** 32
    plan = dd.Plan(nchans, band.f_top, band.df, band.tsamp, dms, dtype)
    assert plan.max_shift == m
    print("staged input %.2f GB, max_shift %d" % (nchans * (nsamp + m) * staged / 1e9, m), flush=True)
    g = torch.Generator(device="cuda")
    g.manual_seed(11)
    if dtype == "u8":
        xin = torch.randint(0, 256, (nchans, nsamp + m), generator=g, device="cuda", dtype=torch.uint8)
    else:
        xin = torch.randn((nchans, nsamp + m), generator=g, device="cuda")
    x = xin.cpu().numpy()
    rows = np.array([0, 1, 7, 8, 31, 32, 63])
    want = oracle.dedisperse(x, sh, nsamp, rows=rows)
    scale = None if dtype == "u8" else abs_sum(x, sh, nsamp, rows=rows)
    odt = torch.int32 if dtype == "u8" else torch.float32
    for v in (1, 0):
        plan.variant = v
        out = torch.full((64, nsamp), -7, dtype=odt, device="cuda")
        plan.execute(xin, out, nsamp, torch.cuda.current_stream())
        torch.cuda.synchronize()
        got = out.cpu().numpy()[rows]
        if dtype == "u8":
            assert np.array_equal(got.astype(np.int64), want), "variant %d" % v
        else:
            check_float(got, want, scale)
        del out
    del xin
    torch.cuda.empty_cache()


@pytest.mark.parametrize("nchans,dm_max,dtype,nsamp,rows", [
    (256, 200.0, "f32", 2500, None),
    (2000, 100.0, "f32", 1200, [0, 1, 7, 8, 999, 1000, 1998, 1999]),
    (2000, 400.0, "u8", 1200, [0, 1, 7, 8, 999, 1000, 1998, 1999]),
])
def test_fig4_sweep_shapes(dd, nchans, dm_max, dtype, nsamp, rows):
    """Points of the Figure 4 sweeps (as many trials as channels, equally spaced
    up to a maximum DM, on the stand-in band) with the trials from the
    library's grid planner, against the oracle's own grid and delay table."""
    import torch
    band = wl.fig4_band(nchans)
    dms = dd.dedisp_dm_grid(dm_max, nchans)
    assert np.array_equal(dms, oracle.dm_grid(dm_max, nchans))
    sh, m = oracle.shift_table(nchans, band.f_top, band.df, band.tsamp, oracle.dm_grid(dm_max, nchans))
    plan = dd.Plan(nchans, band.f_top, band.df, band.tsamp, dms, dtype)
    assert plan.max_shift == m
    # 2000 channels and trials fit an 8-trial tile; at 256 the trials are too
    # far apart (an 8-trial tile would span ~24k samples) and the default is a
    # tile of one or two trials
    assert plan.variant >= 1
    if nchans == 256:
        assert dd.dedisp_variant_describe(plan.variant)[0] <= 2  # trials per tile
    g = torch.Generator(device="cuda")
    g.manual_seed(nchans + int(dm_max))
    if dtype == "u8":
        xin = torch.randint(0, 256, (nchans, nsamp + m), generator=g, device="cuda", dtype=torch.uint8)
    else:
        xin = torch.randn((nchans, nsamp + m), generator=g, device="cuda")
    x = xin.cpu().numpy()
    rows = np.arange(nchans) if rows is None else np.array(rows)
    want = oracle.dedisperse(x, sh, nsamp, rows=rows)
    scale = None if dtype == "u8" else abs_sum(x, sh, nsamp, rows=rows)
    odt = torch.int32 if dtype == "u8" else torch.float32
    # at 256 channels: the default, every other tiled variant that fits, and
    # the direct kernel
    for v in all_variants(dd, plan) if nchans <= 256 else [plan.variant]:
        plan.variant = v
        out = torch.full((nchans, nsamp), -7, dtype=odt, device="cuda")
        plan.execute(xin, out, nsamp, torch.cuda.current_stream())
        torch.cuda.synchronize()
        got = out.cpu().numpy()[rows]
        if dtype == "u8":
            assert np.array_equal(got.astype(np.int64), want), "variant %d" % v
        else:
            check_float(got, want, scale)
        del out
    del xin
    torch.cuda.empty_cache()


def test_unsorted_dm_list(dd):
    b = wl.SMALL
    dms = np.random.default_rng(3).permutation(wl.dm_grid(50, 0.2))
    sh, m = oracle.shift_table(b.nchans, b.f_top, b.df, b.tsamp, dms)
    x = np.random.default_rng(4).integers(0, 256, (b.nchans, 1000 + m)).astype(np.uint8)
    p = dd.Plan(b.nchans, b.f_top, b.df, b.tsamp, dms, "u8")
    want = oracle.dedisperse(x, sh, 1000)
    for v in all_variants(dd, p):
        assert np.array_equal(run(p, x, 1000, variant=v).astype(np.int64), want)


def test_zero_samples_is_noop(dd):
    import torch
    p = dd.Plan(8, 150.0, 0.5, 327.68e-6, [0.0, 1.0], "f32")
    out = torch.full((2, 4), 3.0, device="cuda")
    x = torch.zeros((8, 4 + p.max_shift), device="cuda")
    p.execute(x, out, 0)
    torch.cuda.synchronize()
    assert torch.all(out == 3.0)


def test_execute_rejects_bad_pointers(dd):
    import torch
    p = dd.Plan(8, 150.0, 0.5, 327.68e-6, [0.0, 1.0], "f32")
    x = torch.zeros((8, 100 + p.max_shift), device="cuda")
    out = torch.zeros((2, 100), device="cuda")
    with pytest.raises(dd.DedispError):
        dd.dedisp_execute(p.handle, x.data_ptr() + 4, out.data_ptr(), 100)  # misaligned input
    with pytest.raises(dd.DedispError):
        dd.dedisp_execute(p.handle, 0, out.data_ptr(), 100)
    with pytest.raises(dd.DedispError):
        dd.dedisp_execute(p.handle, x.data_ptr(), out.data_ptr(), -1)


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_host_search_bit_identical_to_device(dd, dtype):
    """The vectorised host search sums in the GPU kernels' order: its float
    results equal dedisp_execute's bit for bit (tiled and direct variants)."""
    w = wl.lofar(dtype, nsamp=2600, ndm=300)
    sh, m, x = make_case(w)
    plan = dd.Plan.for_workload(w)
    host = np.empty((w.ndm, w.nsamp), np.float32)
    dd.dedisp_execute_cpu(plan.handle, x, host, w.nsamp, 0)
    for v in sorted({0, plan.variant}):
        got = run(plan, x, w.nsamp, variant=v)
        assert np.array_equal(got.view(np.uint32), host.view(np.uint32)), "variant %d" % v

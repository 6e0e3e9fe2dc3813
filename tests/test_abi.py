"""C-ABI checks that need no GPU: exported symbols, argument checks, and the
binary64 delay table against the oracle (the table is built on the host)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_1111_6399_amd import workloads as wl

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "dedisp.h")


@pytest.fixture(scope="module")
def dd():
    from paper_1111_6399_amd import dedisp
    return dedisp


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dedisp_\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported(dd):
    names = declared_functions()
    assert len(names) >= 25
    for n in names:
        assert hasattr(dd.lib, n), n
    assert dd.MISSING == []
    assert set(dd.EXPORTS) == set(names)


def test_status_strings(dd):
    for code in range(7):
        s = dd.status_string(code)
        assert s and s != "unknown status"
    assert dd.status_string(99) == "unknown status"


@pytest.mark.parametrize("band,ndm,step", [(wl.SMALL, 100, 0.1), (wl.LOFAR, 2048, 0.1), (wl.MEERKAT, 4096, 0.5),
                                           (wl.Band(1024, 1712.0, 428.0 / 1024, 64e-6), 4096, 0.05),
                                           (wl.Band(256, 1712.0, 428.0 / 256, 64e-6), 512, 0.25)])
def test_shift_table_bit_exact(dd, band, ndm, step):
    dms = wl.dm_grid(ndm, step)
    p = dd.Plan(band.nchans, band.f_top, band.df, band.tsamp, dms, "u8")
    want, m = oracle.shift_table(band.nchans, band.f_top, band.df, band.tsamp, dms)
    got = p.shift_table()
    assert got.dtype == np.int32 and got.shape == want.shape
    assert np.array_equal(got, want)
    assert p.max_shift == m


def test_shift_table_batch_beams_bit_exact(dd):
    for w in wl.batch_beams():
        b = w.band
        want, m = oracle.shift_table(b.nchans, b.f_top, b.df, b.tsamp, w.dms)
        p = dd.Plan.for_workload(w)
        assert np.array_equal(p.shift_table(), want) and p.max_shift == m


def test_unsorted_dm_list_table(dd):
    b = wl.SMALL
    dms = np.random.default_rng(1).permutation(wl.dm_grid(80, 0.123))
    p = dd.Plan(b.nchans, b.f_top, b.df, b.tsamp, dms, "f32")
    want, m = oracle.shift_table(b.nchans, b.f_top, b.df, b.tsamp, dms)
    assert np.array_equal(p.shift_table(), want) and p.max_shift == m


BAD_PLANS = [
    dict(nchans=0), dict(nchans=-3), dict(df=0.0), dict(df=-1.0), dict(tsamp=0.0), dict(tsamp=-1e-3),
    dict(f_top=0.0), dict(f_top=float("nan")), dict(df=float("inf")), dict(nchans=800),
    dict(dms=[1.0, -0.5]), dict(dms=[float("nan")]), dict(dms=[float("inf")]), dict(dtype=3), dict(dtype=-1),
    dict(dms=[1e12]),  # a delay beyond int32
]


@pytest.mark.parametrize("bad", BAD_PLANS)
def test_plan_create_rejects(dd, bad):
    args = dict(nchans=64, f_top=150.0, df=0.1953125, tsamp=327.68e-6, dms=[0.0, 1.0], dtype=2)
    args.update(bad)
    dm = np.asarray(args["dms"], dtype=np.float64)
    h = ctypes.c_void_p(12345)
    st = dd.lib.dedisp_plan_create(args["nchans"], args["f_top"], args["df"], args["tsamp"],
                                   dm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(dm.size), args["dtype"],
                                   ctypes.byref(h))
    assert st == dd.DEDISP_ERR_INVALID_ARG
    assert h.value == 12345  # out-parameter untouched


def test_plan_create_null_and_empty(dd):
    h = ctypes.c_void_p()
    dm = np.zeros(1)
    assert dd.lib.dedisp_plan_create(8, 150.0, 0.5, 1e-3, None, 1, 2, ctypes.byref(h)) == dd.DEDISP_ERR_INVALID_ARG
    assert dd.lib.dedisp_plan_create(8, 150.0, 0.5, 1e-3, dm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0, 2,
                                     ctypes.byref(h)) == dd.DEDISP_ERR_INVALID_ARG
    assert dd.lib.dedisp_plan_create(8, 150.0, 0.5, 1e-3, dm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1, 2,
                                     None) == dd.DEDISP_ERR_INVALID_ARG


def test_null_handles(dd):
    out = ctypes.c_int32(7)
    assert dd.lib.dedisp_plan_max_shift(None, ctypes.byref(out)) == dd.DEDISP_ERR_INVALID_ARG
    assert out.value == 7
    assert dd.lib.dedisp_plan_destroy(None) == dd.DEDISP_OK
    assert dd.lib.dedisp_batch_destroy(None) == dd.DEDISP_OK
    assert dd.lib.dedisp_server_destroy(None) == dd.DEDISP_OK
    assert dd.lib.dedisp_execute(None, None, None, 1, None) == dd.DEDISP_ERR_INVALID_ARG
    assert dd.lib.dedisp_server_create(1 << 30, 4, None) == dd.DEDISP_ERR_INVALID_ARG
    assert dd.lib.dedisp_server_create(0, 4, ctypes.byref(ctypes.c_void_p())) == dd.DEDISP_ERR_INVALID_ARG
    assert dd.lib.dedisp_submit(None, 0, None, None, None) == dd.DEDISP_ERR_INVALID_ARG


def test_execute_argument_checks_before_device(dd):
    p = dd.Plan(8, 150.0, 0.5, 327.68e-6, [0.0, 1.0], "f32")
    # zero samples is a no-op that never touches the device, even with NULL buffers
    assert dd.lib.dedisp_execute(p.handle, None, None, 0, None) == dd.DEDISP_OK
    assert dd.lib.dedisp_execute(p.handle, None, None, -1, None) == dd.DEDISP_ERR_INVALID_ARG
    assert dd.lib.dedisp_execute(p.handle, None, ctypes.c_void_p(4096), 10, None) == dd.DEDISP_ERR_INVALID_ARG
    # misaligned input (needs 16 bytes), misaligned output (needs 4)
    assert dd.lib.dedisp_execute(p.handle, ctypes.c_void_p(4100), ctypes.c_void_p(4096), 10, None) == \
        dd.DEDISP_ERR_INVALID_ARG
    assert dd.lib.dedisp_execute(p.handle, ctypes.c_void_p(4096), ctypes.c_void_p(4098), 10, None) == \
        dd.DEDISP_ERR_INVALID_ARG
    assert dd.lib.dedisp_execute(p.handle, ctypes.c_void_p(4096), ctypes.c_void_p(4096), 1 << 31, None) == \
        dd.DEDISP_ERR_INVALID_ARG


def test_variants(dd):
    n = dd.dedisp_variant_count()
    assert n >= 3
    for v in range(n):
        dms, samples, threads = dd.dedisp_variant_describe(v)
        assert dms >= 1 and samples >= 1 and threads in (256, 512, 1024)
    with pytest.raises(dd.DedispError):
        dd.dedisp_variant_describe(n)
    p = dd.Plan(64, 150.0, 0.1953125, 327.68e-6, wl.dm_grid(100, 0.1), "f32")
    assert 0 <= p.variant < n
    p.variant = 0
    assert p.variant == 0
    with pytest.raises(dd.DedispError):
        p.variant = n
    # a delay spread no multi-trial tile can stage leaves the one-trial tile
    # (whose window is its own samples only) and the direct kernel
    wide = dd.Plan(16, 150.0, 4.0, 327.68e-6, wl.dm_grid(4, 200.0), "f32")
    assert wide.variant >= 1 and dd.dedisp_variant_describe(wide.variant)[0] == 1
    for v in range(1, n):
        if dd.dedisp_variant_describe(v)[0] == 1:
            wide.variant = v
        else:
            with pytest.raises(dd.DedispError):
                wide.variant = v
    wide.variant = 0
    assert wide.variant == 0


def test_batch_create_checks(dd):
    p = dd.Plan(8, 150.0, 0.5, 327.68e-6, [0.0, 1.0], "f32")
    for plans, ns in [([p.handle], [0]), ([p.handle], [-4]), ([None], [10])]:
        with pytest.raises(dd.DedispError):
            dd.dedisp_batch_create(plans, ns)
    b = dd.dedisp_batch_create([p.handle, p.handle], [100, 200])
    assert dd.dedisp_batch_info(b) == (0, 0)
    assert dd.dedisp_batch_get_variant(b) >= 1
    for bad in (-2, dd.dedisp_variant_count()):
        with pytest.raises(dd.DedispError):
            dd.dedisp_batch_set_variant(b, bad)
    # 0: split by the plans' own variants (host bookkeeping only, no device work)
    dd.dedisp_batch_set_variant(b, 0)
    assert dd.dedisp_batch_get_variant(b) >= 1
    # -1: every beam on its own
    dd.dedisp_batch_set_variant(b, -1)
    assert dd.dedisp_batch_get_variant(b) == -1
    # graph layouts: 0-2 (host bookkeeping only before the first execute)
    assert dd.dedisp_batch_get_layout(b) == 0
    for layout in (1, 2, 0):
        dd.dedisp_batch_set_layout(b, layout)
        assert dd.dedisp_batch_get_layout(b) == layout
    for bad in (-1, 3):
        with pytest.raises(dd.DedispError):
            dd.dedisp_batch_set_layout(b, bad)
    dd.dedisp_batch_set_layout(b, 2)
    dd.dedisp_batch_set_variant(b, -1)  # resets the layout
    assert dd.dedisp_batch_get_layout(b) == 0
    dd.dedisp_batch_destroy(b)


@pytest.mark.parametrize("dm_max,ndm", [(200.0, 2000), (0.1, 4), (1000.0, 3), (0.0, 7), (25.0, 1)])
def test_dm_grid_matches_oracle(dd, dm_max, ndm):
    assert np.array_equal(dd.dedisp_dm_grid(dm_max, ndm).view(np.uint64), oracle.dm_grid(dm_max, ndm).view(np.uint64))


def test_dm_grid_rejects(dd):
    out = np.full(4, -1.0)
    for bad in [(-1.0, 4), (float("nan"), 4), (float("inf"), 4), (1.0, 0), (1.0, -3)]:
        assert dd.lib.dedisp_dm_grid(bad[0], bad[1], out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == \
            dd.DEDISP_ERR_INVALID_ARG
    assert np.all(out == -1.0)
    assert dd.lib.dedisp_dm_grid(1.0, 4, None) == dd.DEDISP_ERR_INVALID_ARG


@pytest.mark.parametrize("dtype,es,staged", [("u8", 1, 2), ("f16", 2, 0), ("f32", 4, 0)])
def test_plan_footprint(dd, dtype, es, staged):
    band = wl.LOFAR
    dms = oracle.dm_grid(200.0, 64)
    sh, m = oracle.shift_table(band.nchans, band.f_top, band.df, band.tsamp, dms)
    plan = dd.Plan(band.nchans, band.f_top, band.df, band.tsamp, dms, dtype)
    for nsamp in (0, 1, 4097):
        total = band.nchans * (nsamp + m)
        i, o, s = dd.dedisp_plan_footprint(plan.handle, nsamp)
        assert i == total * es
        assert o == 64 * nsamp * 4
        assert s == (0 if staged == 0 else (total + 7) // 8 * 8 * staged)
    with pytest.raises(dd.DedispError):
        dd.dedisp_plan_footprint(plan.handle, -1)
    assert dd.lib.dedisp_plan_footprint(None, 10, None, None, None) == dd.DEDISP_ERR_INVALID_ARG


def _sigproc(fields):
    from sigproc_util import SIGPROC_FIELDS, write_sigproc
    return write_sigproc(fields), SIGPROC_FIELDS


def test_sigproc_parse_matches_oracle(dd):
    buf, fields = _sigproc({"nchans": 3})
    buf, _ = _sigproc(fields)
    for extra in (b"", bytes(100)):
        got = dd.dedisp_sigproc_parse(buf + extra)
        want = oracle.sigproc_header(buf + extra)
        for k in ("nchans", "nbits", "nifs", "data_type", "telescope_id", "machine_id", "tsamp", "fch1", "foff",
                  "tstart", "refdm", "source_name", "header_bytes"):
            assert got[k] == want[k], k
        assert got["dtype"] == dd.DEDISP_U8


def test_sigproc_parse_rejects(dd):
    good, _ = _sigproc({"nchans": 4, "nbits": 8, "tsamp": 1e-3, "foff": -1.0, "fch1": 100.0})
    assert dd.dedisp_sigproc_parse(good)["dtype"] == dd.DEDISP_U8
    f32, _ = _sigproc({"nchans": 4, "nbits": 32, "tsamp": 1e-3, "foff": 1.0, "fch1": 100.0})
    assert dd.dedisp_sigproc_parse(f32)["dtype"] == dd.DEDISP_F32
    bads = [good[:-3], good[4:], _sigproc({"nchans": 4, "nbits": 8, "tsamp": 1e-3, "foff": 0.0})[0],
            _sigproc({"nchans": 0, "nbits": 8, "tsamp": 1e-3, "foff": 1.0})[0],
            _sigproc({"nchans": 4, "nbits": 12, "tsamp": 1e-3, "foff": 1.0})[0],
            good.replace(b"nchans", b"nchanz")]
    for b in bads:
        with pytest.raises(dd.DedispError):
            dd.dedisp_sigproc_parse(b)
    assert dd.lib.dedisp_sigproc_parse(None, 10, None) == dd.DEDISP_ERR_INVALID_ARG


def test_corner_turn_argument_checks(dd):
    f = dd.lib.dedisp_corner_turn
    assert f(None, 16, 10, 4, 10, dd.DEDISP_U8, 0, None) == dd.DEDISP_ERR_INVALID_ARG
    assert f(16, 16, 10, 4, 9, dd.DEDISP_U8, 0, None) == dd.DEDISP_ERR_INVALID_ARG  # pitch < nsamp
    assert f(16, 16, 10, 0, 10, dd.DEDISP_U8, 0, None) == dd.DEDISP_ERR_INVALID_ARG
    assert f(16, 16, 10, 4, 10, 7, 0, None) == dd.DEDISP_ERR_INVALID_ARG
    assert f(16, 16, 0, 4, 10, dd.DEDISP_U8, 0, None) == dd.DEDISP_OK  # nothing to do, no device call


# ------------------------------------------------- vectorised host search --

@pytest.mark.parametrize("dtype", ["f32", "f16", "u8"])
@pytest.mark.parametrize("nchans,ndm,nsamp", [(1, 1, 1), (33, 17, 257), (70, 40, 1000), (496, 64, 3000)])
def test_execute_cpu_matches_oracle(dd, dtype, nchans, ndm, nsamp):
    """The host search (host code, no device): exact for 8-bit input, within
    the float tolerance otherwise; full and ragged tiles of 16 trials x 256
    samples, channel counts that are not multiples of 32."""
    band = wl.Band(nchans, 150.0, 0.1953125, 327.68e-6)
    dms = np.arange(ndm) * 0.37
    sh, m = oracle.shift_table(nchans, band.f_top, band.df, band.tsamp, dms)
    rng = np.random.default_rng([41, nchans, ndm])
    if dtype == "u8":
        x = rng.integers(0, 256, size=(nchans, nsamp + m)).astype(np.uint8)
    else:
        x = rng.standard_normal((nchans, nsamp + m)).astype(np.float32 if dtype == "f32" else np.float16)
    plan = dd.Plan(nchans, band.f_top, band.df, band.tsamp, dms, dtype)
    out = np.empty((ndm, nsamp), dtype=np.int32 if dtype == "u8" else np.float32)
    for nt in (1, 3, 0):
        out[:] = -7
        isa = dd.dedisp_execute_cpu(plan.handle, x, out, nsamp, nt)
        assert isa in (0, 1, 2)
        want = oracle.dedisperse(x, sh, nsamp)
        if dtype == "u8":
            assert np.array_equal(out.astype(np.int64), want)
        else:
            scale = oracle.dedisperse(np.abs(x.astype(np.float32)), sh, nsamp)
            assert np.all(np.abs(out - want) <= 1e-5 * scale)


def test_execute_cpu_same_result_any_threads(dd):
    """Float results do not depend on the thread count (fixed summation order)."""
    w = wl.lofar("f32", nsamp=1500, ndm=100)
    b = w.band
    sh, m = oracle.shift_table(b.nchans, b.f_top, b.df, b.tsamp, w.dms)
    x = wl.generate(w, sh, m)
    plan = dd.Plan.for_workload(w)
    outs = []
    for nt in (1, 2, 7):
        o = np.empty((w.ndm, w.nsamp), np.float32)
        dd.dedisp_execute_cpu(plan.handle, x, o, w.nsamp, nt)
        outs.append(o)
    assert all(np.array_equal(o.view(np.uint32), outs[0].view(np.uint32)) for o in outs)


def test_execute_cpu_argument_checks(dd):
    plan = dd.Plan(4, 150.0, 0.5, 1e-3, [0.0, 1.0], "f32")
    f = dd.lib.dedisp_execute_cpu
    assert f(None, 16, 16, 10, 0, None) == dd.DEDISP_ERR_INVALID_ARG
    assert f(plan.handle, None, 16, 10, 0, None) == dd.DEDISP_ERR_INVALID_ARG
    assert f(plan.handle, 16, 16, -1, 0, None) == dd.DEDISP_ERR_INVALID_ARG
    assert f(plan.handle, 16, 16, 10, -2, None) == dd.DEDISP_ERR_INVALID_ARG
    assert f(plan.handle, None, None, 0, 0, None) == dd.DEDISP_OK  # nothing to do


class _FakeDeviceTensor:
    """Stands in for a device tensor: only what the binding's checks read."""

    class _Dev:
        type = "cuda"

    def __init__(self, dtype, numel, contiguous=True):
        self.dtype, self._n, self._c, self.device = dtype, numel, contiguous, self._Dev()

    def numel(self):
        return self._n

    def is_contiguous(self):
        return self._c

    def data_ptr(self):
        return 0x1000


@pytest.mark.parametrize("dtype", ["u8", "f16", "f32"])
def test_execute_checks_tensors_before_the_library(dd, dtype, monkeypatch):
    """Plan.execute rejects a buffer of the wrong element type, too few
    elements, non-contiguous or on the host, before any call into the library
    (whose kernels cannot see the size of an allocation)."""
    import torch
    p = dd.Plan(8, 150.0, 0.5, 327.68e-6, [0.0, 1.0, 2.0], dtype)
    n = 100
    nin = 8 * (n + p.max_shift)
    tin = {"u8": torch.uint8, "f16": torch.float16, "f32": torch.float32}[dtype]
    tout = torch.int32 if dtype == "u8" else torch.float32
    wrong_in = torch.float32 if dtype != "f32" else torch.uint8
    wrong_out = torch.float32 if dtype == "u8" else torch.int32
    good_out = _FakeDeviceTensor(tout, 3 * n)
    cases = [
        (_FakeDeviceTensor(wrong_in, nin), good_out),                 # element type of the input
        (_FakeDeviceTensor(tin, nin - 1), good_out),                  # one input element short
        (_FakeDeviceTensor(tin, nin, contiguous=False), good_out),    # strided view
        (torch.zeros(nin, dtype=tin), good_out),                      # host tensor
        (_FakeDeviceTensor(tin, nin), _FakeDeviceTensor(wrong_out, 3 * n)),
        (_FakeDeviceTensor(tin, nin), _FakeDeviceTensor(tout, 3 * n - 1)),
    ]
    def no_call(*a, **k):
        raise AssertionError("the library was called with a rejected buffer")

    monkeypatch.setattr(dd, "dedisp_execute", no_call)
    for xin, out in cases:
        with pytest.raises(dd.DedispError) as e:
            p.execute(xin, out, n)
        assert e.value.status == dd.DEDISP_ERR_INVALID_ARG


def test_library_rounds_exact_ties_half_up(dd):
    """The library's delay table at binary64 products that are exactly n + 1/2
    (gives n + 1) or the double just below (gives n): tests/golden/tie_pins.json."""
    import json
    doc = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "tie_pins.json")))
    for case in doc["cases"]:
        b = doc["bands"][case["band"]]
        c = case["channel"]
        p = dd.Plan(c + 1, b["f_top"], b["df"], b["tsamp"], [float.fromhex(case["dm"])], "u8")
        assert p.shift_table()[c, 0] == case["value"], case

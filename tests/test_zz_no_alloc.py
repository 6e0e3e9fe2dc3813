"""The allocation-free entry point (dedisp_execute_static) against
dedisp_execute: two calls in a row on the same device (the second smaller),
8-bit input (whose widened copy lives in the library's static scratch) and
float32 input, every output compared; the entry captured into a HIP graph
and replayed; and its refusals (too large for the scratch, device tables not
yet created)."""
import numpy as np
import pytest

import oracle
from paper_1111_6399_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd(device):
    from paper_1111_6399_amd import dedisp
    return dedisp


def case(dd, dtype, nchans, ndm, nsamp, seed):
    import torch
    band = wl.Band(nchans, 1712.0, 428.0 / nchans, 64e-6)
    dms = wl.dm_grid(ndm, 0.5)
    plan = dd.Plan(nchans, band.f_top, band.df, band.tsamp, dms, dtype)
    sh, m = oracle.shift_table(nchans, band.f_top, band.df, band.tsamp, dms)
    assert plan.max_shift == m
    rng = np.random.default_rng(seed)
    if dtype == "u8":
        x = rng.integers(0, 256, (nchans, nsamp + m)).astype(np.uint8)
    else:
        x = rng.standard_normal((nchans, nsamp + m)).astype(np.float32)
    xin = torch.from_numpy(x).to("cuda")
    odt = torch.int32 if dtype == "u8" else torch.float32
    ref = torch.full((ndm, nsamp), -9, dtype=odt, device="cuda")
    got = torch.full((ndm, nsamp), -9, dtype=odt, device="cuda")
    return plan, sh, x, xin, ref, got


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_static_entry_matches_execute(dd, dtype):
    import torch
    stream = torch.cuda.current_stream()
    # two calls in a row on one device, the second smaller: the scratch keeps
    # the first call's contents, which must not leak into the second
    for (nchans, ndm, nsamp, seed) in ((1024, 300, 20000, 1), (256, 70, 3001, 2)):
        plan, sh, x, xin, ref, got = case(dd, dtype, nchans, ndm, nsamp, seed)
        plan.execute(xin, ref, nsamp, stream)  # also creates the device tables
        dd.dedisp_execute_static(plan.handle, xin.data_ptr(), got.data_ptr(), nsamp, stream)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), got.cpu().numpy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (nchans, ndm, nsamp)
        rows = np.array([0, ndm // 2, ndm - 1])
        want = oracle.dedisperse(x, sh, nsamp, rows=rows)
        if dtype == "u8":
            assert np.array_equal(b[rows].astype(np.int64), want)
        else:
            scale = oracle.dedisperse(np.abs(x), sh, nsamp, rows=rows)
            assert np.all(np.abs(b[rows] - want) <= 1e-5 * scale)


@pytest.mark.parametrize("dtype", ["u8", "f32"])
def test_static_entry_in_a_captured_graph(dd, dtype):
    """Captured into a HIP graph (nothing is allocated, so capture records
    only its kernels) and replayed three times, new input written eagerly
    between the replays: every replay equals dedisp_execute on that input."""
    import torch
    nsamp = 3001
    plan, sh, x, xin, ref, got = case(dd, dtype, 256, 70, nsamp, 4)
    stream = torch.cuda.current_stream()
    plan.execute(xin, ref, nsamp, stream)  # device tables
    dd.dedisp_execute_static(plan.handle, xin.data_ptr(), got.data_ptr(), nsamp, stream)  # warm-up
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        dd.dedisp_execute_static(plan.handle, xin.data_ptr(), got.data_ptr(), nsamp, torch.cuda.current_stream())
    torch.cuda.synchronize()
    rng = np.random.default_rng(6)
    for k in range(3):
        if dtype == "u8":
            x2 = rng.integers(0, 256, x.shape).astype(np.uint8)
        else:
            x2 = rng.standard_normal(x.shape).astype(np.float32)
        xin.copy_(torch.from_numpy(x2))
        got.fill_(-9)
        graph.replay()
        plan.execute(xin, ref, nsamp, stream)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), "replay %d" % k
    rows = np.array([0, 35, 69])
    want = oracle.dedisperse(x2, sh, nsamp, rows=rows)
    b = got.cpu().numpy()
    if dtype == "u8":
        assert np.array_equal(b[rows].astype(np.int64), want)
    else:
        scale = oracle.dedisperse(np.abs(x2), sh, nsamp, rows=rows)
        assert np.all(np.abs(b[rows] - want) <= 1e-5 * scale)
    del graph


def test_static_entry_refusals(dd):
    import torch
    # device tables not created yet on this device: refused, nothing allocated
    plan, sh, x, xin, ref, got = case(dd, "u8", 64, 16, 1000, 3)
    with pytest.raises(dd.DedispError) as e:
        dd.dedisp_execute_static(plan.handle, xin.data_ptr(), got.data_ptr(), 1000)
    assert e.value.status == dd.DEDISP_ERR_INVALID_ARG
    # an 8-bit problem whose widened copy exceeds the 1 GiB scratch
    band = wl.Band(4096, 1712.0, 0.104492, 64e-6)
    big = dd.Plan(4096, band.f_top, band.df, band.tsamp, wl.dm_grid(64, 0.5), "u8")
    nsamp = (1 << 30) // (2 * 4096) + 16
    with pytest.raises(dd.DedispError) as e:
        dd.dedisp_execute_static(big.handle, xin.data_ptr(), got.data_ptr(), nsamp)
    assert e.value.status == dd.DEDISP_ERR_INVALID_ARG
    torch.cuda.synchronize()

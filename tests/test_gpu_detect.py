"""GPU parity of the detection step against the oracle.

The detection input is a seeded synthetic block uploaded to the device (the
oracle never sees a GPU result).  Int32 blocks (the output type of 8-bit
plans): statistics and S/N within 1e-9, best times exact (equal boxcar sums
give equal S/N on both sides, and different integer sums differ by far more
than rounding).  Float32 blocks: S/N within 1e-9, and the reported time must
reach the oracle's best S/N within that tolerance (another time may tie).
Candidates are compared as sets, leaving out pairs within the tolerance of the
threshold.
"""
import numpy as np
import pytest

import oracle
from paper_1111_6399_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module")
def dd(device):
    from paper_1111_6399_amd import dedisp
    return dedisp


def plan_for(dd, ndm, dtype):
    # any plan with ndm trials: detection uses only its trial count and output type
    return dd.Plan(8, 150.0, 0.1953125, 327.68e-6, np.arange(ndm) * 0.1, dtype)


def run_detect(dd, plan, block, nwidths, threshold, cap=4096):
    import torch
    ndm, n = block.shape
    x = torch.from_numpy(np.ascontiguousarray(block)).to("cuda")
    stats = torch.empty((ndm, 2), dtype=torch.float64, device="cuda")
    snr = torch.empty((ndm, nwidths), dtype=torch.float64, device="cuda")
    t = torch.empty((ndm, nwidths), dtype=torch.int32, device="cuda")
    cand = torch.zeros(cap * 4, dtype=torch.int32, device="cuda")
    count = torch.full((1,), 12345, dtype=torch.int32, device="cuda")
    dd.dedisp_detect(plan.handle, x.data_ptr(), n, nwidths, threshold, stats.data_ptr(), snr.data_ptr(),
                     t.data_ptr(), cand.data_ptr(), cap, count.data_ptr(), torch.cuda.current_stream())
    torch.cuda.synchronize()
    k = int(count.item())
    c = cand.cpu().numpy().view(dd.CANDIDATE_DTYPE)[:min(k, cap)]
    return stats.cpu().numpy(), snr.cpu().numpy(), t.cpu().numpy().astype(np.int64), c, k


def planted(rng, ndm, n, kind):
    if kind == "int":
        x = rng.integers(60000, 70000, size=(ndm, n)).astype(np.int32)
    else:
        x = rng.standard_normal((ndm, n)).astype(np.float32)
    for d in range(0, ndm, 5):
        w = int(rng.choice([1, 3, 8, 20, 64]))
        t0 = int(rng.integers(0, n - w))
        x[d, t0:t0 + w] += (3000 if kind == "int" else 2.0)
    return x


def compare(got, want, block, threshold, exact_t):
    gs, gb, gt, gc, k = got
    ws, wb, wt, wc = want
    assert np.allclose(gs, ws, rtol=1e-12, atol=1e-9)
    finite = np.isfinite(wb)
    assert np.array_equal(finite, np.isfinite(gb)) and np.all(gb[~finite] == -np.inf)
    assert np.all(gt[~finite] == -1)
    assert np.all(np.abs(gb[finite] - wb[finite]) <= TOL * np.maximum(1.0, np.abs(wb[finite])))
    if exact_t:
        assert np.array_equal(gt, wt)
    else:
        # the reported time reaches the best S/N (recomputed by the oracle's formula)
        x = block.astype(np.float64)
        mean, std = ws[:, 0], ws[:, 1]
        for d, kk in zip(*np.nonzero(finite)):
            w = 1 << kk
            s = gt[d, kk]
            v = (x[d, s:s + w].sum() - w * mean[d]) / (std[d] * np.sqrt(w)) if std[d] > 0 else 0.0
            assert v >= wb[d, kk] - TOL * max(1.0, abs(wb[d, kk]))
    assert k == len(gc) or k > len(gc)
    got_set = {(int(c["dm_index"]), int(c["width"])) for c in gc}
    sure = {(d, 1 << kk) for d, kk in zip(*np.nonzero(np.abs(wb - threshold) > 1e-6))}
    assert got_set & sure == wc & sure
    for c in gc:
        kk = int(c["width"]).bit_length() - 1
        assert c["time"] == gt[c["dm_index"], kk]
        assert abs(c["snr"] - gb[c["dm_index"], kk]) <= 1e-6 * max(1.0, abs(gb[c["dm_index"], kk]))


@pytest.mark.parametrize("kind,ndm,n,nw", [("int", 37, 10000, 8), ("float", 37, 9000, 8), ("int", 5, 5000, 12),
                                            ("float", 3, 4097, 12)])
def test_detect_matches_oracle(dd, kind, ndm, n, nw):
    rng = np.random.default_rng([21, ndm, n])
    block = planted(rng, ndm, n, kind)
    plan = plan_for(dd, ndm, "u8" if kind == "int" else "f32")
    thr = 6.0
    got = run_detect(dd, plan, block, nw, thr)
    compare(got, oracle.detect(block, nw, thr), block, thr, exact_t=(kind == "int"))


@pytest.mark.parametrize("n,nw", [(1, 1), (1, 3), (7, 4), (4096, 1), (4097, 2), (8193, 5)])
def test_detect_edge_shapes(dd, n, nw):
    rng = np.random.default_rng([22, n])
    block = rng.integers(0, 9, size=(4, n)).astype(np.int32)
    block[1] = 5  # a constant trial: S/N 0 everywhere
    plan = plan_for(dd, 4, "u8")
    got = run_detect(dd, plan, block, nw, 1.0)
    compare(got, oracle.detect(block, nw, 1.0), block, 1.0, exact_t=True)


@pytest.mark.parametrize("nw", [10, 12])
def test_detect_int_ties(dd, nw):
    """Integer rows of a few levels (negative ones too): every width has many
    starts with equal sums, so the earliest one must be reported; chunks end
    inside the widest boxcars and the last chunk is partial."""
    rng = np.random.default_rng([24, nw])
    block = rng.integers(-3, 4, size=(9, 20000)).astype(np.int32)
    block[4] = -7  # constant
    plan = plan_for(dd, 9, "u8")
    got = run_detect(dd, plan, block, nw, 2.0)
    compare(got, oracle.detect(block, nw, 2.0), block, 2.0, exact_t=True)


def test_detect_capacity_and_count(dd):
    """More candidates than room: the count is the true number, only the
    capacity is written."""
    rng = np.random.default_rng(23)
    block = planted(rng, 40, 3000, "int")
    plan = plan_for(dd, 40, "u8")
    want = oracle.detect(block, 6, -1e9)[3]  # every (trial, width) is a candidate
    got = run_detect(dd, plan, block, 6, -1e9, cap=17)
    assert got[4] == len(want) == 240 and len(got[3]) == 17
    assert {(int(c["dm_index"]), int(c["width"])) for c in got[3]} <= want


def test_detect_rejects(dd):
    import torch
    plan = plan_for(dd, 4, "f32")
    x = torch.zeros((4, 100), device="cuda")
    s = torch.empty((4, 4), dtype=torch.float64, device="cuda")
    t = torch.empty((4, 4), dtype=torch.int32, device="cuda")
    for args in [(0, 4), (100, 0), (100, 13)]:
        with pytest.raises(dd.DedispError):
            dd.dedisp_detect(plan.handle, x.data_ptr(), args[0], args[1], 5.0, None, s.data_ptr(), t.data_ptr(),
                             None, 0, None)
    with pytest.raises(dd.DedispError):
        dd.dedisp_detect(plan.handle, x.data_ptr(), 100, 4, float("nan"), None, s.data_ptr(), t.data_ptr(), None,
                         0, None)
    with pytest.raises(dd.DedispError):  # candidates without a counter
        dd.dedisp_detect(plan.handle, x.data_ptr(), 100, 4, 5.0, None, s.data_ptr(), t.data_ptr(), x.data_ptr(),
                         4, None)


def test_search_then_detect_finds_the_planted_pulse(dd):
    """End to end on the 64-channel workload: de-dispersion on the GPU, then
    detection on the GPU; the planted pulse (amplitude 5 in every channel at
    trial 50, t = 2000) is the strongest width-1 candidate, at its trial and
    time."""
    import torch
    w = wl.small_f32()
    b = w.band
    sh, m = oracle.shift_table(b.nchans, b.f_top, b.df, b.tsamp, w.dms)
    x = wl.generate(w, sh, m)
    plan = dd.Plan.for_workload(w)
    xin = torch.from_numpy(x).to("cuda")
    out = torch.empty((w.ndm, w.nsamp), dtype=torch.float32, device="cuda")
    plan.execute(xin, out, w.nsamp, torch.cuda.current_stream())
    torch.cuda.synchronize()
    got = run_detect(dd, plan, out.cpu().numpy(), 4, 8.0)
    cands = got[3]
    assert len(cands) >= 1
    top = cands[np.argmax(cands["snr"])]
    assert (int(top["dm_index"]), int(top["width"]), int(top["time"])) == (50, 1, 2000)
    # the oracle on its own de-dispersion of the same input agrees
    want = oracle.detect(oracle.dedisperse(x, sh, w.nsamp), 4, 8.0)
    assert want[2][50, 0] == 2000 and abs(want[1][50, 0] - got[1][50, 0]) < 1e-3 * want[1][50, 0]

"""Batched persistent launch (HIP graph) against solo launches and the oracle.

Each beam's output from the batch must be bit-identical to dedisp_execute of
that beam alone (same accumulation order), and match the oracle (uint8 exact,
float within the per-output bound).  The graph is replayed several times with
eager work and synchronisations in between, and with changed buffers.
"""
import numpy as np
import pytest

import oracle
from paper_1111_6399_amd import workloads as wl

from gpu_util import abs_sum, check_float, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd(device):
    from paper_1111_6399_amd import dedisp
    return dedisp


def small_beams(seed=11, nbeams=7):
    """Uneven beams shaped like the batched workload, scaled down in time and trials."""
    rng = np.random.default_rng(seed)
    beams = []
    for b in range(nbeams):
        nchans = int(rng.choice([64, 96, 128]))
        nsamp = int(rng.integers(700, 5000))
        ndm = int(rng.integers(20, 90))
        step = float(rng.choice([0.5, 1.0, 2.0]))
        dtype = ["f32", "u8", "f16"][b % 3]
        band = wl.Band(nchans, 1712.0, 428.0 / nchans, 64e-6)
        beams.append(wl.Workload("b%d" % b, band, wl.dm_grid(ndm, step), nsamp, dtype, 300 + b, []))
    # one beam whose delay spread is too wide for any tile: it runs on its own
    wide = wl.Workload("wide", wl.Band(16, 150.0, 4.0, 327.68e-6), wl.dm_grid(4, 200.0), 300, "f32", 399, [])
    beams.append(wide)
    return beams


def make_inputs(beams):
    out = []
    for w in beams:
        b = w.band
        sh, m = oracle.shift_table(b.nchans, b.f_top, b.df, b.tsamp, w.dms)
        rng = np.random.default_rng(w.seed)
        n_in = w.nsamp + m
        if w.dtype == "u8":
            x = rng.integers(0, 256, (b.nchans, n_in)).astype(np.uint8)
        else:
            x = rng.standard_normal((b.nchans, n_in)).astype(np.float32)
            if w.dtype == "f16":
                x = x.astype(np.float16)
        out.append((sh, m, x))
    return out


def alloc_out(w):
    import torch
    return torch.full((w.ndm, w.nsamp), -5, dtype=torch.int32 if w.dtype == "u8" else torch.float32,
                      device="cuda")


def test_batch_matches_solo_and_oracle(dd):
    import torch
    beams = small_beams()
    data = make_inputs(beams)
    plans = [dd.Plan.for_workload(w) for w in beams]
    ins = [to_device(x) for (_, _, x) in data]
    outs = [alloc_out(w) for w in beams]
    batch = dd.dedisp_batch_create([p.handle for p in plans], [w.nsamp for w in beams])
    try:
        stream = torch.cuda.current_stream()
        # solo references
        solo = []
        for p, w, xi in zip(plans, beams, ins):
            o = alloc_out(w)
            p.execute(xi, o, w.nsamp, stream)
            solo.append(o)
        torch.cuda.synchronize()
        solo = [o.cpu().numpy() for o in solo]
        for rep in range(4):
            for o in outs:
                o.fill_(-5)
            dd.dedisp_batch_execute(batch, [t.data_ptr() for t in ins], [t.data_ptr() for t in outs], stream)
            torch.cuda.synchronize()
            for w, o, s, (sh, m, x) in zip(beams, outs, solo, data):
                got = o.cpu().numpy()
                assert np.array_equal(got.view(np.uint32), s.view(np.uint32)), "beam %s replay %d" % (w.name, rep)
            # eager work between replays
            torch.cuda.synchronize()
            _ = (ins[0].float().sum() if ins[0].dtype != torch.uint8 else ins[0].sum()).item()
        items, groups = dd.dedisp_batch_info(batch)
        assert items > 0 and groups > 0
        for w, s, (sh, m, x) in zip(beams, solo, data):
            want = oracle.dedisperse(x, sh, w.nsamp)
            if w.dtype == "u8":
                assert np.array_equal(s.astype(np.int64), want)
            else:
                check_float(s, want, abs_sum(x, sh, w.nsamp))
        # new output buffers: the argument table is refreshed, no rebuild needed
        outs2 = [alloc_out(w) for w in beams]
        dd.dedisp_batch_execute(batch, [t.data_ptr() for t in ins], [t.data_ptr() for t in outs2], stream)
        torch.cuda.synchronize()
        for o, s in zip(outs2, solo):
            assert np.array_equal(o.cpu().numpy().view(np.uint32), s.view(np.uint32))
    finally:
        dd.dedisp_batch_destroy(batch)


def test_batch_every_variant(dd):
    import torch
    beams = small_beams(seed=5, nbeams=4)
    data = make_inputs(beams)
    plans = [dd.Plan.for_workload(w) for w in beams]
    ins = [to_device(x) for (_, _, x) in data]
    batch = dd.dedisp_batch_create([p.handle for p in plans], [w.nsamp for w in beams])
    try:
        ref = None
        for v in range(1, dd.dedisp_variant_count()):
            dd.dedisp_batch_set_variant(batch, v)
            outs = [alloc_out(w) for w in beams]
            dd.dedisp_batch_execute(batch, [t.data_ptr() for t in ins], [t.data_ptr() for t in outs])
            torch.cuda.synchronize()
            res = [o.cpu().numpy().view(np.uint32) for o in outs]
            if ref is None:
                ref = res
            else:
                for a, b in zip(ref, res):
                    assert np.array_equal(a, b), "variant %d" % v
        tune_outs = [alloc_out(w) for w in beams]
        v, ms = dd.dedisp_batch_autotune(batch, [t.data_ptr() for t in ins], [t.data_ptr() for t in tune_outs])
        assert (v >= 1 or v == -1) and ms > 0
        torch.cuda.synchronize()
        for a, o in zip(ref, tune_outs):
            assert np.array_equal(a, o.cpu().numpy().view(np.uint32)), "autotuned split"
    finally:
        dd.dedisp_batch_destroy(batch)


def test_batch_split_by_plan_variants(dd):
    """Beams whose plans carry different variants (one tiled variant for most
    of the work, others tiled differently or direct): split by the plans' own
    variants, every beam equals its solo launch bit for bit, over replays."""
    import torch
    beams = small_beams(seed=9, nbeams=6)
    data = make_inputs(beams)
    plans = [dd.Plan.for_workload(w) for w in beams]
    plans[0].variant = 1
    plans[1].variant = 5
    plans[2].variant = 1
    plans[3].variant = 0
    plans[4].variant = 11
    ins = [to_device(x) for (_, _, x) in data]
    stream = torch.cuda.current_stream()
    solo = []
    for p, w, xi in zip(plans, beams, ins):
        o = alloc_out(w)
        p.execute(xi, o, w.nsamp, stream)
        solo.append(o)
    torch.cuda.synchronize()
    solo = [o.cpu().numpy().view(np.uint32) for o in solo]
    batch = dd.dedisp_batch_create([p.handle for p in plans], [w.nsamp for w in beams])
    try:
        dd.dedisp_batch_set_variant(batch, 0)
        for rep in range(3):
            outs = [alloc_out(w) for w in beams]
            dd.dedisp_batch_execute(batch, [t.data_ptr() for t in ins], [t.data_ptr() for t in outs], stream)
            torch.cuda.synchronize()
            for w, o, s in zip(beams, outs, solo):
                assert np.array_equal(o.cpu().numpy().view(np.uint32), s), "beam %s replay %d" % (w.name, rep)
        assert dd.dedisp_batch_get_variant(batch) >= 1
        # every beam launched on its own inside the graph, in each layout of
        # the graph's branches (balanced, one branch, one per staging kind)
        dd.dedisp_batch_set_variant(batch, -1)
        assert dd.dedisp_batch_get_variant(batch) == -1
        for layout in (0, 1, 2):
            dd.dedisp_batch_set_layout(batch, layout)
            for rep in range(2):
                outs = [alloc_out(w) for w in beams]
                dd.dedisp_batch_execute(batch, [t.data_ptr() for t in ins], [t.data_ptr() for t in outs], stream)
                torch.cuda.synchronize()
                for w, o, s in zip(beams, outs, solo):
                    assert np.array_equal(o.cpu().numpy().view(np.uint32), s), \
                        "beam %s per-beam layout %d replay %d" % (w.name, layout, rep)
        # persistent groups in the per-kind layout
        dd.dedisp_batch_set_variant(batch, 0)
        dd.dedisp_batch_set_layout(batch, 2)
        outs = [alloc_out(w) for w in beams]
        dd.dedisp_batch_execute(batch, [t.data_ptr() for t in ins], [t.data_ptr() for t in outs], stream)
        torch.cuda.synchronize()
        for w, o, s in zip(beams, outs, solo):
            assert np.array_equal(o.cpu().numpy().view(np.uint32), s), "beam %s groups by kind" % w.name
        v, ms = dd.dedisp_batch_autotune(batch, [t.data_ptr() for t in ins], [t.data_ptr() for t in outs])
        assert (v >= 1 or v == -1) and ms > 0
        outs = [alloc_out(w) for w in beams]
        dd.dedisp_batch_execute(batch, [t.data_ptr() for t in ins], [t.data_ptr() for t in outs], stream)
        torch.cuda.synchronize()
        for w, o, s in zip(beams, outs, solo):
            assert np.array_equal(o.cpu().numpy().view(np.uint32), s), "beam %s after autotune" % w.name
    finally:
        dd.dedisp_batch_destroy(batch)


def test_batch_rejects_bad_args(dd):
    p = dd.Plan(8, 150.0, 0.5, 327.68e-6, [0.0, 1.0], "f32")
    with pytest.raises(dd.DedispError):
        dd.dedisp_batch_create([p.handle], [0])
    with pytest.raises(dd.DedispError):
        dd.dedisp_batch_create([], [])

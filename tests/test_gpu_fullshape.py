"""GPU parity at the workloads' real shapes, in the launch configuration the
bench times (each plan autotuned).

* LOFAR-shaped beam (496 channels x 2048 trials x 65536 output samples) in
  float32, uint8 and float16: every output sample of about 300 trials that
  cover every position inside a trial tile, both ends of the grid and every
  planted pulse's trial.  uint8 is bit-exact; float within the per-output
  bound; for float16 the per-trial error against the binary64 oracle on the
  original float32 data (quantisation included) is printed and bounded.
* MeerKAT-shaped block (4096 x 4096 x 32768, uint8): sampled trials, exact.
* The 32 uneven beams of the batched workload through one batch, under the
  per-group persistent kernels and under per-beam launches: every beam equal
  to its solo launch bit for bit (compared on the device), and sampled trials
  of every beam against the oracle.
* The streaming server at the MeerKAT shape (4096 channels, 4096 trials,
  blocks of 32768): two beams x three blocks, mixed and alone, against the
  oracle's streaming reference on sampled trials.
"""
import numpy as np
import pytest

import oracle
from paper_1111_6399_amd import workloads as wl

from gpu_util import REL_TOL, abs_sum, check_float, per_dm_error

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd(device):
    from paper_1111_6399_amd import dedisp
    return dedisp


def sampled_rows(ndm, extra=()):
    """Every 7th trial (7 is prime to every tile height, so every position in a
    trial tile appears), the first and last two, tile edges of 8 and 16."""
    r = set(range(0, ndm, 7)) | {0, 1, ndm - 2, ndm - 1} | set(int(e) for e in extra)
    r |= {x for x in (7, 8, 15, 16, 17, ndm // 2 - 1, ndm // 2) if 0 <= x < ndm}
    return np.array(sorted(r), dtype=np.int64)


def device_rows(out, rows):
    import torch
    return out[torch.from_numpy(rows).to(out.device)].cpu().numpy()


@pytest.mark.parametrize("dtype", ["f32", "u8", "f16"])
def test_lofar_full_shape(dd, dtype):
    import torch
    w = wl.lofar(dtype)
    b = w.band
    sh, m = oracle.shift_table(b.nchans, b.f_top, b.df, b.tsamp, w.dms)
    x = wl.generate(w, sh, m)
    plan = dd.Plan.for_workload(w)
    assert plan.max_shift == m and np.array_equal(plan.shift_table(), sh)
    v, ms = dd.dedisp_autotune(plan.handle, w.nsamp)
    print("lofar %s: autotuned variant %d, %.3f ms" % (dtype, v, ms), flush=True)
    xin = torch.from_numpy(x).to("cuda")
    out = torch.full((w.ndm, w.nsamp), -7, dtype=torch.int32 if dtype == "u8" else torch.float32, device="cuda")
    plan.execute(xin, out, w.nsamp)
    torch.cuda.synchronize()
    rows = sampled_rows(w.ndm, [p[0] for p in w.pulses])
    got = device_rows(out, rows)
    want = oracle.dedisperse(x, sh, w.nsamp, rows=rows)
    if dtype == "u8":
        assert np.array_equal(got.astype(np.int64), want)
    else:
        worst = check_float(got, want, abs_sum(x, sh, w.nsamp, rows=rows))
        print("lofar %s: %d trials x %d samples, max |err| / sum|x| = %.3g" % (dtype, rows.size, w.nsamp, worst))
    if dtype == "f16":
        # error against the binary64 sum of the original float32 data, per trial
        x32 = wl.generate(wl.lofar("f32"), sh, m)
        e = per_dm_error(got, oracle.dedisperse(x32, sh, w.nsamp, rows=rows))
        print("lofar f16 per-trial error vs float32 data: min %.3g median %.3g max %.3g"
              % (e.min(), np.median(e), e.max()), flush=True)
        assert e.max() < 1e-3
    # every pulse comes back at its trial and time (amplitude 3-10 over N(0,1) noise)
    for (d, t, a, _) in w.pulses:
        i = int(np.searchsorted(rows, d))
        assert rows[i] == d and int(np.argmax(got[i])) == t
    del xin, out
    torch.cuda.empty_cache()


def test_meerkat_block_full_shape(dd):
    import torch
    w = wl.meerkat_block()
    b = w.band
    sh, m = oracle.shift_table(b.nchans, b.f_top, b.df, b.tsamp, w.dms)
    x = wl.generate(w, sh, m)
    plan = dd.Plan.for_workload(w)
    v, ms = dd.dedisp_autotune(plan.handle, w.nsamp)
    print("meerkat block: autotuned variant %d, %.3f ms" % (v, ms), flush=True)
    xin = torch.from_numpy(x).to("cuda")
    out = torch.full((w.ndm, w.nsamp), -7, dtype=torch.int32, device="cuda")
    plan.execute(xin, out, w.nsamp)
    torch.cuda.synchronize()
    rows = sampled_rows(w.ndm)[::2]
    assert np.array_equal(device_rows(out, rows).astype(np.int64), oracle.dedisperse(x, sh, w.nsamp, rows=rows))
    del xin, out
    torch.cuda.empty_cache()


def beam_input(w, max_shift):
    """Input of one beam of the batched mix drawn on the device (torch Philox
    seeded per beam): float32 N(0,1), or round(clip(64 + 16 z, 0, 255))."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(int(w.seed))
    z = torch.randn((w.band.nchans, w.nsamp + int(max_shift)), generator=g, device="cuda", dtype=torch.float32)
    if w.dtype == "f32":
        return z
    return torch.clamp(torch.round(64.0 + 16.0 * z), 0.0, 255.0).to(torch.uint8)


def test_batch_32_beams_full_shape(dd):
    import torch
    beams = wl.batch_beams()
    plans = [dd.Plan.for_workload(w) for w in beams]
    for p, w in zip(plans, beams):
        dd.dedisp_autotune(p.handle, w.nsamp)
    ins = [beam_input(w, p.max_shift) for w, p in zip(beams, plans)]

    def alloc():
        return [torch.full((w.ndm, w.nsamp), -5, dtype=torch.int32 if w.dtype == "u8" else torch.float32,
                           device="cuda") for w in beams]

    solo = alloc()
    for p, w, xi, o in zip(plans, beams, ins, solo):
        p.execute(xi, o, w.nsamp)
    torch.cuda.synchronize()
    batch = dd.dedisp_batch_create([p.handle for p in plans], [w.nsamp for w in beams])
    try:
        # 0: persistent kernels per group of the plans' own variants; 1: one
        # variant for every beam; -1: per-beam launches in the graph
        for mode in (0, 1, -1):
            dd.dedisp_batch_set_variant(batch, mode)
            outs = alloc()
            for rep in range(2):
                dd.dedisp_batch_execute(batch, [t.data_ptr() for t in ins], [t.data_ptr() for t in outs])
                torch.cuda.synchronize()
                if rep == 0:
                    # the persistent groups are laid out by the first execute
                    items, wgs = dd.dedisp_batch_info(batch)
                    print("batch mode %d: %d items on %d workgroups" % (mode, items, wgs), flush=True)
                    assert (items > 0 and wgs > 0) if mode >= 0 else items == 0
                for w, o, s in zip(beams, outs, solo):
                    assert torch.equal(o.view(torch.int32), s.view(torch.int32)), \
                        "beam %s mode %d replay %d" % (w.name, mode, rep)
                outs[0].fill_(-5)
            del outs
        v, ms = dd.dedisp_batch_autotune(batch, [t.data_ptr() for t in ins], [t.data_ptr() for t in solo])
        print("batch autotune: split %d, %.2f ms" % (v, ms), flush=True)
    finally:
        dd.dedisp_batch_destroy(batch)
    # the oracle on sampled trials of every beam, every output sample
    for w, p, xi, s in zip(beams, plans, ins, solo):
        b = w.band
        sh, m = oracle.shift_table(b.nchans, b.f_top, b.df, b.tsamp, w.dms)
        assert m == p.max_shift
        x = xi.cpu().numpy()
        rows = np.array(sorted({0, 1, 15, 16, w.ndm // 2, w.ndm - 2, w.ndm - 1}), dtype=np.int64)
        got = device_rows(s, rows)
        want = oracle.dedisperse(x, sh, w.nsamp, rows=rows)
        if w.dtype == "u8":
            assert np.array_equal(got.astype(np.int64), want), w.name
        else:
            check_float(got, want, abs_sum(x, sh, w.nsamp, rows=rows))
        del x
    del ins, solo
    torch.cuda.empty_cache()


def test_server_meerkat_shape(dd):
    """Two MeerKAT-shaped beams (4096 channels, 4096 trials, blocks of 32768
    uint8 samples, history of max_shift samples on the device), three blocks
    each, submitted interleaved; then beam 0 alone.  Sampled trials of every
    block equal the oracle's streaming reference; alone equals mixed."""
    import time
    import torch
    band = wl.MEERKAT
    dms = wl.dm_grid(4096, 0.5)
    B, nblocks = 32768, 3
    sh, m = oracle.shift_table(band.nchans, band.f_top, band.df, band.tsamp, dms)
    streams = [np.concatenate([wl.stream_block(77, beam, k, band.nchans, B) for k in range(nblocks)], axis=1)
               for beam in range(2)]
    rows = sampled_rows(4096)[::6]

    def wait(server, ticket):
        t0 = time.time()
        while True:
            done, _ = dd.dedisp_poll(server, ticket)
            if done:
                return
            assert time.time() - t0 < 60.0, "ticket %d did not finish" % ticket
            time.sleep(0.002)

    def serve(beam_ids):
        plan = dd.Plan(band.nchans, band.f_top, band.df, band.tsamp, dms, "u8")
        server = dd.dedisp_server_create(24 << 30, 4)
        outs = {i: [] for i in beam_ids}
        try:
            bids = {i: dd.dedisp_server_add_beam(server, plan.handle, B) for i in beam_ids}
            blocks = {i: [torch.from_numpy(np.ascontiguousarray(streams[i][:, k * B:(k + 1) * B])).pin_memory()
                          for k in range(nblocks)] for i in beam_ids}
            pending = []
            for k in range(nblocks):
                for i in beam_ids:
                    out = torch.full((4096, B), -3, dtype=torch.int32, device="cuda")
                    # the server's streams do not wait for torch's: the fill must be done
                    torch.cuda.current_stream().synchronize()
                    while True:
                        t = dd.dedisp_submit(server, bids[i], blocks[i][k].data_ptr(), out.data_ptr())
                        if t is not None:
                            break
                        assert pending, "not admitted with nothing in flight"
                        wait(server, pending.pop(0))
                    pending.append(t)
                    outs[i].append(out)
            for t in pending:
                wait(server, t)
            return {i: [device_rows(o, rows) for o in outs[i]] for i in beam_ids}
        finally:
            dd.dedisp_server_destroy(server)

    mixed = serve([0, 1])
    alone = serve([0])
    for i in (0, 1):
        for k in range(nblocks):
            want = oracle.stream_reference(streams[i], sh, m, B, k, rows=rows)
            assert np.array_equal(mixed[i][k].astype(np.int64), want), "beam %d block %d" % (i, k)
    for k in range(nblocks):
        assert np.array_equal(alone[0][k], mixed[0][k])
    torch.cuda.empty_cache()

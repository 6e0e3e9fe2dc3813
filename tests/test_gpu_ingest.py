"""GPU parity of filterbank ingestion: the corner turn against the oracle's
definition (bit-exact: it only moves samples), and a synthetic sigproc file
read, corner-turned into a plan's input behind a zero history and searched,
against the oracle reading the same bytes itself."""
import numpy as np
import pytest

import oracle
from sigproc_util import write_sigproc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dd(device):
    from paper_1111_6399_amd import dedisp
    return dedisp


NP = {"u8": np.uint8, "f16": np.float16, "f32": np.float32}


@pytest.mark.parametrize("dtype", ["u8", "f16", "f32"])
@pytest.mark.parametrize("nsamp,nchans", [(1, 1), (64, 64), (65, 63), (1000, 100), (4097, 513), (5, 4), (300, 260),
                                          (129, 1024)])
@pytest.mark.parametrize("reverse", [False, True])
def test_corner_turn_matches_oracle(dd, dtype, nsamp, nchans, reverse):
    import torch
    rng = np.random.default_rng([31, nsamp, nchans])
    x = (rng.integers(0, 256, size=(nsamp, nchans)) if dtype == "u8" else rng.standard_normal((nsamp, nchans)))
    x = x.astype(NP[dtype])
    pitch = nsamp + 37
    tin = torch.from_numpy(x).to("cuda")
    sentinel = np.full((nchans + 1, pitch), 77, dtype=NP[dtype])  # one spare row after the last
    tout = torch.from_numpy(sentinel.copy()).to("cuda")
    dd.dedisp_corner_turn(tin.data_ptr(), tout.data_ptr(), nsamp, nchans, pitch, dtype, reverse,
                          torch.cuda.current_stream())
    torch.cuda.synchronize()
    got = tout.cpu().numpy()
    want = oracle.corner_turn(x, reverse)
    assert np.array_equal(got[:nchans, :nsamp].view(np.uint8), want.view(np.uint8))
    assert np.array_equal(got[:, nsamp:], sentinel[:, nsamp:]) and np.array_equal(got[nchans], sentinel[nchans])


@pytest.mark.parametrize("offset", [0, 1, 3, 8, 15])
@pytest.mark.parametrize("nsamp,nchans,extra", [(300, 260, 37), (1, 4, 0), (17, 512, 3), (1000, 8, 16)])
def test_corner_turn_u8_any_output_alignment(dd, offset, nsamp, nchans, extra):
    """8-bit rows written at any byte alignment (the plan's input places a
    block behind the history, max_shift samples into each row): every sample
    lands once, nothing outside the rows is touched."""
    import torch
    rng = np.random.default_rng([33, offset, nsamp, nchans])
    x = rng.integers(0, 256, size=(nsamp, nchans)).astype(np.uint8)
    pitch = nsamp + extra
    tin = torch.from_numpy(x).to("cuda")
    size = offset + nchans * pitch + 64
    sentinel = rng.integers(0, 256, size=size).astype(np.uint8)
    tout = torch.from_numpy(sentinel.copy()).to("cuda")
    for reverse in (False, True):
        dd.dedisp_corner_turn(tin.data_ptr(), tout.data_ptr() + offset, nsamp, nchans, pitch, "u8", reverse,
                              torch.cuda.current_stream())
        torch.cuda.synchronize()
        got = tout.cpu().numpy()
        rows = got[offset:offset + nchans * pitch].reshape(nchans, pitch)
        assert np.array_equal(rows[:, :nsamp], oracle.corner_turn(x, reverse))
        keep = np.ones(size, dtype=bool)
        keep[offset:offset + nchans * pitch] = np.tile(np.arange(pitch) >= nsamp, nchans)
        assert np.array_equal(got[keep], sentinel[keep])


def test_corner_turn_meerkat_block(dd):
    """The MeerKAT-shaped block of the pipeline (32768 samples x 4096 uint8
    channels) into rows behind a history of max_shift samples, exactly."""
    import torch
    from paper_1111_6399_amd import workloads as wl
    w = wl.meerkat_block()
    nch, n = w.band.nchans, w.nsamp
    m = dd.Plan.for_workload(w).max_shift
    rng = np.random.default_rng(34)
    x = rng.integers(0, 256, size=(n, nch)).astype(np.uint8)
    tin = torch.from_numpy(x).to("cuda")
    rows = torch.zeros((nch, n + m), dtype=torch.uint8, device="cuda")
    dd.dedisp_corner_turn(tin.data_ptr(), rows.data_ptr() + m, n, nch, n + m, "u8", False,
                          torch.cuda.current_stream())
    torch.cuda.synchronize()
    got = rows.cpu().numpy()
    assert not got[:, :m].any()
    assert np.array_equal(got[:, m:], x.T)


@pytest.mark.parametrize("foff", [-0.390625, 0.390625])
def test_filterbank_file_search(dd, foff):
    """8-bit sigproc data (channel 0 highest for a negative foff, lowest for a
    positive one) with a dispersed pulse: library parse + corner turn + search
    equals the oracle's parse, rows and sum exactly."""
    import torch
    nchans, nsamp, tsamp = 96, 6000, 1.31072e-4
    fch1 = 400.0 if foff < 0 else 400.0 - (nchans - 1) * 0.390625
    hdr = write_sigproc({"source_name": "SYNTH", "fch1": fch1, "foff": foff, "nchans": nchans, "nbits": 8,
                         "tsamp": tsamp, "nifs": 1, "tstart": 60000.0})
    rng = np.random.default_rng(32)
    data = rng.integers(0, 200, size=(nsamp, nchans)).astype(np.uint8)
    blob = hdr + data.tobytes()

    # library: header, then the samples it says follow
    h = dd.dedisp_sigproc_parse(blob)
    assert h["header_bytes"] == len(hdr) and h["dtype"] == dd.DEDISP_U8
    top = h["fch1"] if h["foff"] < 0 else h["fch1"] + (h["nchans"] - 1) * h["foff"]
    dms = np.arange(40) * 2.5
    plan = dd.Plan(h["nchans"], top, abs(h["foff"]), h["tsamp"], dms, "u8")
    m = plan.max_shift
    n_out = nsamp - m
    assert n_out > 1000
    samples = np.frombuffer(blob, dtype=np.uint8, offset=h["header_bytes"]).reshape(-1, h["nchans"])
    tin = torch.from_numpy(samples.copy()).to("cuda")
    rows = torch.zeros((nchans, nsamp), dtype=torch.uint8, device="cuda")  # the plan's input: pitch n_out + m
    dd.dedisp_corner_turn(tin.data_ptr(), rows.data_ptr(), nsamp, nchans, nsamp, "u8", h["foff"] > 0,
                          torch.cuda.current_stream())
    out = torch.empty((40, n_out), dtype=torch.int32, device="cuda")
    plan.execute(rows, out, n_out, torch.cuda.current_stream())
    torch.cuda.synchronize()

    # oracle: its own reading of the same bytes
    oh = oracle.sigproc_header(blob)
    otop = oh["fch1"] if oh["foff"] < 0 else oh["fch1"] + (oh["nchans"] - 1) * oh["foff"]
    sh, om = oracle.shift_table(oh["nchans"], otop, abs(oh["foff"]), oh["tsamp"], dms)
    assert om == m
    orows = oracle.corner_turn(np.frombuffer(blob, dtype=np.uint8, offset=oh["header_bytes"])
                               .reshape(-1, oh["nchans"]), oh["foff"] > 0)
    want = oracle.dedisperse(orows, sh, n_out)
    assert np.array_equal(out.cpu().numpy().astype(np.int64), want)

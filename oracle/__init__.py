"""Oracle for brute-force incoherent de-dispersion -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct CPU reference written from the paper
("A GPU-based survey for millisecond radio transients using ARTEMIS").  Only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may import
it.  It shares no code with the GPU library (``paper_1111_6399_amd``) and
neither imports the other; inputs come from the seeded generators in
``paper_1111_6399_amd.workloads``, which hold none of the method's arithmetic.

Functions and the passages they follow:

* :func:`shift_table` -- per-channel dispersion delays in samples, section
  "Searching for radio transients" (quadratic cold-plasma law, DM as the single
  free parameter).  Constant 4148.808 s MHz^2 pc^-1 cm^3, delays relative to the
  top of the band, round half up.  Binary64, fixed operation order, no fused
  multiply-add (plain C, ``-ffp-contract=off``).
* :func:`dedisperse` -- ``out[d][t] = sum_c in[c][t + shift[c][d]]``: shift each
  channel, then integrate over frequency, for every trial DM (sections
  "Searching for radio transients" and "Acceleration via GPU computing").
  Binary64 accumulation for float input, int64 for uint8 input.
* :func:`stream_reference` -- the same sum over a stream cut into blocks, with a
  zero history before the first block (the paper does not describe block
  buffering; this is the reading the streaming tests use).
* :func:`dm_grid` -- trial DMs equally spaced from 0 up to a maximum DM, the
  grid of the timing comparisons (section "Comparisons of GPU and CPU
  algorithms", Figure 4: as many trials as channels).
* :func:`sigproc_header`, :func:`corner_turn` -- ingestion of sigproc
  filterbank data (the paper's test data were sigproc simulations, section
  "Searching for radio transients"): the header's keywords and values, and the
  time-major samples rearranged into one row per channel.
* :func:`detect` -- the detection step after the search (section
  "Introduction": the pipeline ends in detection; Figure 3: the recovered pulse
  at its trial DM): per trial mean and standard deviation, boxcar S/N for
  widths 1, 2, 4, ..., the best (S/N, time) per width, the candidates above a
  threshold.  The paper gives no formula; the function's docstring states the
  reading used.

Every function here is pinned by ``tests/test_oracle_pins.py`` against results
the mathematics fixes (exact rational arithmetic, closed forms, invariants, an
independent dense-matrix formulation on tiny grids).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dedisp_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` (gcc, OpenMP, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
           "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build(force=False)
    lib = ctypes.CDLL(_LIB)
    i32p = ctypes.POINTER(ctypes.c_int32)
    f64p = ctypes.POINTER(ctypes.c_double)
    lib.oracle_shift_table.restype = ctypes.c_int64
    lib.oracle_shift_table.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       f64p, ctypes.c_int, i32p]
    common = [ctypes.c_int64, ctypes.c_int, i32p, ctypes.c_int, i32p, ctypes.c_int, ctypes.c_int64,
              ctypes.c_int64]
    lib.oracle_dedisperse_f32.restype = None
    lib.oracle_dedisperse_f32.argtypes = [ctypes.c_void_p] + common + [ctypes.c_void_p]
    lib.oracle_dedisperse_u8.restype = None
    lib.oracle_dedisperse_u8.argtypes = [ctypes.c_void_p] + common + [ctypes.c_void_p]
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_num_threads.argtypes = []
    _lib = lib
    return lib


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use on this host."""
    return int(_load().oracle_num_threads())


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def shift_table(nchans: int, f_top: float, df: float, tsamp: float, dm_list) -> tuple[np.ndarray, int]:
    """Integer delay of every (channel, trial DM) in samples.

    Returns ``(shift, max_shift)`` with ``shift`` an int32 array of shape
    ``(nchans, ndm)``: ``shift[c][d] = round_half_up(DM_d * k_c)`` with
    ``f_c = f_top - c*df`` and ``k_c = 4148.808*(1/f_c^2 - 1/f_top^2)/tsamp``
    (frequencies in MHz, tsamp in seconds).  Section "Searching for radio
    transients": the delay follows the quadratic cold-plasma law and depends on
    DM alone.
    """
    dm = np.ascontiguousarray(np.asarray(dm_list, dtype=np.float64))
    ndm = int(dm.shape[0])
    if nchans <= 0 or ndm <= 0:
        raise ValueError("nchans and ndm must be positive")
    if not (df > 0 and tsamp > 0 and f_top > 0 and f_top - (nchans - 1) * df > 0):
        raise ValueError("band must be positive and descending")
    if not np.all(np.isfinite(dm)) or np.any(dm < 0):
        raise ValueError("trial DMs must be finite and non-negative")
    out = np.empty((nchans, ndm), dtype=np.int32)
    m = _load().oracle_shift_table(int(nchans), float(f_top), float(df), float(tsamp),
                                   _ptr(dm, ctypes.c_double), ndm, _ptr(out, ctypes.c_int32))
    if m < 0:
        raise ValueError("a delay does not fit in int32")
    return out, int(m)


_SIGPROC_INT = {"telescope_id", "machine_id", "data_type", "nchans", "nbits", "nifs", "nbeams", "ibeam",
                 "barycentric", "pulsarcentric", "nsamples"}
_SIGPROC_DOUBLE = {"tsamp", "fch1", "foff", "tstart", "src_raj", "src_dej", "az_start", "za_start", "refdm",
                   "period"}
_SIGPROC_STRING = {"source_name", "rawdatafile"}


def sigproc_header(buf: bytes) -> dict:
    """Keywords and values of a sigproc filterbank header: length-prefixed
    (32-bit little-endian) keyword strings between HEADER_START and
    HEADER_END, each followed by a 32-bit integer, a binary64 value or a
    length-prefixed string.  Adds ``header_bytes``, the offset of the first
    sample.  Raises ValueError on a malformed header or unknown keyword."""
    import struct

    pos = 0

    def string():
        nonlocal pos
        (n,) = struct.unpack_from("<i", buf, pos)
        if not 0 < n <= 256 or pos + 4 + n > len(buf):
            raise ValueError("bad string at %d" % pos)
        v = bytes(buf[pos + 4:pos + 4 + n]).decode("latin-1")
        pos += 4 + n
        return v

    try:
        if string() != "HEADER_START":
            raise ValueError("no HEADER_START")
        out = {}
        while True:
            key = string()
            if key == "HEADER_END":
                break
            if key in _SIGPROC_INT:
                (out[key],) = struct.unpack_from("<i", buf, pos)
                pos += 4
            elif key in _SIGPROC_DOUBLE:
                (out[key],) = struct.unpack_from("<d", buf, pos)
                pos += 8
            elif key in _SIGPROC_STRING:
                out[key] = string()
            else:
                raise ValueError("unknown keyword %r" % key)
    except struct.error as e:
        raise ValueError("truncated header") from e
    out["header_bytes"] = pos
    return out


def corner_turn(samples: np.ndarray, reverse_channels: bool = False) -> np.ndarray:
    """Time-major ``samples[t][c]`` as channel rows ``out[c][t]``; with
    ``reverse_channels`` input channel c becomes row ``nchans-1-c``."""
    out = np.ascontiguousarray(np.asarray(samples).T)
    return np.ascontiguousarray(out[::-1]) if reverse_channels else out


def dm_grid(dm_max: float, ndm: int) -> np.ndarray:
    """Trial DMs equally spaced over [0, dm_max]: ``dm_max * (d / (ndm - 1))``
    in binary64 for ``d = 0 .. ndm-1`` (the quotient first, so the last trial is
    ``dm_max`` itself); one trial is ``[0]``.  Section "Comparisons of GPU and
    CPU algorithms" (Figure 4 holds the maximum DM and spaces the trials
    equally)."""
    if ndm < 1 or not np.isfinite(dm_max) or dm_max < 0:
        raise ValueError("ndm >= 1 and a finite dm_max >= 0 are required")
    if ndm == 1:
        return np.zeros(1)
    return float(dm_max) * (np.arange(ndm, dtype=np.float64) / float(ndm - 1))


def detect(block: np.ndarray, nwidths: int, threshold: float):
    """Detection on a de-dispersed block ``(ndm, n)`` (int or float), binary64.

    Per trial ``d``: ``mean`` and population ``std`` of its ``n`` values; for
    ``w = 2**k`` (``k < nwidths``) and every ``t`` with ``t + w <= n``:
    ``snr = (sum(x[t:t+w]) - w*mean) / (std*sqrt(w))`` (0 where ``std == 0``);
    ``best_snr[d][k]``, ``best_t[d][k]``: the largest ``snr`` and the earliest
    ``t`` reaching it (``-inf``, ``-1`` when ``w > n``).  Candidates: the set of
    ``(d, w)`` whose best S/N is ``>= threshold``.
    Returns ``(stats (ndm, 2), best_snr, best_t, candidates)``.
    """
    x = np.asarray(block).astype(np.float64)
    ndm, n = x.shape
    mean = x.mean(axis=1)
    std = np.sqrt(((x - mean[:, None]) ** 2).mean(axis=1))
    best_snr = np.full((ndm, nwidths), -np.inf)
    best_t = np.full((ndm, nwidths), -1, dtype=np.int64)
    rows = np.arange(ndm)
    for k in range(nwidths):
        w = 1 << k
        if w > n:
            continue
        box = np.lib.stride_tricks.sliding_window_view(x, w, axis=1).sum(axis=2)
        with np.errstate(divide="ignore", invalid="ignore"):
            snr = (box - w * mean[:, None]) / (std[:, None] * np.sqrt(float(w)))
        snr[std == 0.0] = 0.0
        t = np.argmax(snr, axis=1)
        best_t[:, k] = t
        best_snr[:, k] = snr[rows, t]
    cands = {(int(d), 1 << int(k)) for d, k in zip(*np.nonzero(best_snr >= threshold))}
    return np.stack([mean, std], axis=1), best_snr, best_t, cands


def dedisperse(data: np.ndarray, shift: np.ndarray, nsamp: int, rows=None,
               t_begin: int = 0, t_count: int | None = None) -> np.ndarray:
    """``out[i][t] = sum_c data[c][t_begin + t + shift[c][rows[i]]]``.

    ``data`` is ``(nchans, >= nsamp + max(shift))`` float32, float16 or uint8.
    float16 input is widened exactly to float32 first.  Returns float64 for
    float input and int64 for uint8 input, shape ``(len(rows), t_count)``.
    """
    nchans, ndm = shift.shape
    if data.ndim != 2 or data.shape[0] != nchans:
        raise ValueError("data must be (nchans, samples)")
    rows = np.arange(ndm, dtype=np.int32) if rows is None else np.ascontiguousarray(rows, dtype=np.int32)
    if t_count is None:
        t_count = nsamp - t_begin
    if t_begin < 0 or t_count < 0 or t_begin + t_count > nsamp:
        raise ValueError("time range outside [0, nsamp)")
    if rows.size and (rows.min() < 0 or rows.max() >= ndm):
        raise ValueError("row index out of range")
    if nsamp + int(shift.max(initial=0)) > data.shape[1]:
        raise ValueError("data rows shorter than nsamp + max_shift")
    sh = np.ascontiguousarray(shift, dtype=np.int32)
    if data.dtype == np.float16:
        data = data.astype(np.float32)
    lib = _load()
    if data.dtype == np.float32:
        out = np.empty((rows.size, t_count), dtype=np.float64)
        fn = lib.oracle_dedisperse_f32
    elif data.dtype == np.uint8:
        out = np.empty((rows.size, t_count), dtype=np.int64)
        fn = lib.oracle_dedisperse_u8
    else:
        raise TypeError("unsupported input dtype %s" % data.dtype)
    if data.strides[1] != data.itemsize:
        data = np.ascontiguousarray(data)
    stride = data.strides[0] // data.itemsize
    fn(data.ctypes.data, int(stride), int(nchans), _ptr(sh, ctypes.c_int32), int(ndm),
       _ptr(rows, ctypes.c_int32), int(rows.size), int(t_begin), int(t_count), out.ctypes.data)
    return out


def stream_reference(stream: np.ndarray, shift: np.ndarray, max_shift: int, block: int,
                     b: int, rows=None) -> np.ndarray:
    """Output block ``b`` of a beam streamed in blocks of ``block`` samples.

    ``stream`` is ``(nchans, n)`` holding the blocks back to back.  The history
    before sample 0 is zero.  Output block ``b`` holds the de-dispersed series
    at stream times ``[b*block - max_shift, (b+1)*block - max_shift)``, i.e. the
    sum over the ``max_shift`` samples of history plus the new block.
    """
    nchans = stream.shape[0]
    lo = b * block - max_shift
    hi = (b + 1) * block
    padded = np.zeros((nchans, block + max_shift), dtype=stream.dtype)
    src_lo = max(lo, 0)
    padded[:, src_lo - lo:] = stream[:, src_lo:hi]
    return dedisperse(padded, shift, block, rows=rows)

"""Seeded synthetic workloads for de-dispersion.

This module only draws random numbers and lays out arrays.  It holds none of
the de-dispersion arithmetic: where a dispersed pulse is planted, the caller
passes in the integer delay table (``shift[c][d]``) to plant it along.  Both the
GPU library's tests and the oracle's tests take their inputs from here.

The shapes follow the workloads the paper describes (filterbank data of the
LOFAR kind: 496 channels below 150 MHz, and a MeerKAT L-band-shaped stream),
which were sigproc simulations.  None of those files exist here; every array is
drawn from a seeded generator, row by row, so any single channel can be redrawn
on its own.

Recipes (``seed`` is per workload):

* noise row ``c``: ``numpy.random.default_rng([seed, c]).standard_normal(n, float32)``
* uint8 samples: ``round(clip(64 + 16*z, 0, 255))`` of the same ``z``
* float16 samples: the float32 samples cast to float16
* pulses: drawn from ``default_rng([seed, 1_000_000])``; amplitudes are
  multiples of 1/16 so that sums of them are exact in float32.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PULSE_STREAM = 1_000_000


@dataclass(frozen=True)
class Band:
    """Channel 0 sits at ``f_top`` MHz; channel c at ``f_top - c*df``."""

    nchans: int
    f_top: float
    df: float
    tsamp: float


LOFAR = Band(496, 150.0, 0.1953125, 327.68e-6)
SMALL = Band(64, 150.0, 0.1953125, 327.68e-6)
MEERKAT = Band(4096, 1712.0, 0.104492, 64e-6)


def dm_grid(ndm: int, step: float) -> np.ndarray:
    """Equally spaced trial DMs ``d*step`` for ``d < ndm`` (pc cm^-3)."""
    return np.arange(ndm, dtype=np.float64) * float(step)


@dataclass
class Workload:
    """One de-dispersion problem: band, trial DMs, output length, input dtype."""

    name: str
    band: Band
    dms: np.ndarray
    nsamp: int
    dtype: str = "f32"
    seed: int = 0
    pulses: list = field(default_factory=list)  # (d, t, amplitude, width)

    @property
    def ndm(self) -> int:
        return int(self.dms.shape[0])


def small_f32() -> Workload:
    """64 channels, 100 trials 0-9.9 in steps of 0.1, 8192 output samples,
    one pulse of amplitude 5 at DM 5.0 (trial 50), t = 2000."""
    return Workload("small-f32", SMALL, dm_grid(100, 0.1), 8192, "f32", 1, [(50, 2000, 5.0, 1)])


def lofar(dtype: str = "f32", nsamp: int = 65536, ndm: int = 2048, seed: int = 2) -> Workload:
    """LOFAR-shaped beam: 496 channels from 150 MHz, 2048 trials 0-204.7,
    65536 output samples, 8 pulses at random trials, times and amplitudes 3-10."""
    rng = np.random.default_rng([seed, PULSE_STREAM])
    pulses = []
    used_t = []
    while len(pulses) < 8:
        d = int(rng.integers(0, ndm))
        t = int(rng.integers(0, nsamp))
        a = float(np.round(rng.uniform(3.0, 10.0) * 16.0) / 16.0)
        if all(abs(t - u) > 64 for u in used_t):
            used_t.append(t)
            pulses.append((d, t, a, 1))
    return Workload("lofar-%s" % dtype, LOFAR, dm_grid(ndm, 0.1), nsamp, dtype, seed, pulses)


# Timing sweeps in the manner of the paper's Figure 4 (its band, sampling
# interval and data length are not stated): the LOFAR-shaped band (150 MHz
# top, 496 x 0.1953125 = 96.875 MHz wide, 327.68 us) cut into nchans
# channels, as many trials as channels spaced equally up to a maximum DM,
# 65536 output samples (21.5 s of data), float32 N(0,1) noise drawn on the
# device.
FIG4_BANDWIDTH = 496 * 0.1953125
FIG4_CHANNELS = (256, 512, 1024, 2048, 4096)  # at a maximum DM of 200
FIG4_DM_MAX = (25.0, 50.0, 100.0, 200.0, 400.0, 800.0)  # at 2000 channels and trials


def fig4_band(nchans: int) -> Band:
    """The LOFAR-shaped band cut into ``nchans`` channels."""
    return Band(nchans, 150.0, FIG4_BANDWIDTH / nchans, 327.68e-6)


def fig4_points():
    """(sweep, nchans, maximum DM) of every point of both sweeps."""
    pts = [("channels", n, 200.0) for n in FIG4_CHANNELS]
    pts += [("max_dm", 2000, m) for m in FIG4_DM_MAX]
    return pts


def meerkat_block(nsamp: int = 32768, ndm: int = 4096, step: float = 0.5) -> Workload:
    """MeerKAT L-band-shaped block: 4096 channels from 1712 MHz, df 0.104492,
    tsamp 64 us, trials 0-2047.5 in steps of 0.5, uint8 samples."""
    return Workload("meerkat-u8", MEERKAT, dm_grid(ndm, step), nsamp, "u8", 5, [])


def noise_rows(seed: int, nchans: int, nsamp_in: int, rows=None) -> np.ndarray:
    """float32 N(0,1) samples, one independent seeded stream per channel."""
    rows = range(nchans) if rows is None else rows
    out = np.empty((len(rows), nsamp_in), dtype=np.float32)
    for i, c in enumerate(rows):
        out[i] = np.random.default_rng([seed, int(c)]).standard_normal(nsamp_in, dtype=np.float32)
    return out


def to_u8(z: np.ndarray) -> np.ndarray:
    """8-bit quantisation of unit-variance samples: round(clip(64 + 16 z, 0, 255))."""
    return np.rint(np.clip(64.0 + 16.0 * z.astype(np.float64), 0.0, 255.0)).astype(np.uint8)


def plant_pulses(data: np.ndarray, shift: np.ndarray, pulses) -> None:
    """Add each pulse ``(d, t, a, w)`` along the delay curve of trial ``d``:
    ``data[c][t + shift[c][d] + j] += a`` for ``j < w`` (in place)."""
    nchans = data.shape[0]
    for (d, t, a, w) in pulses:
        for c in range(nchans):
            j0 = t + int(shift[c][d])
            data[c, j0:j0 + w] += data.dtype.type(a)


def generate(w: Workload, shift: np.ndarray, max_shift: int) -> np.ndarray:
    """Input array of shape ``(nchans, nsamp + max_shift)`` in the workload's dtype.

    ``shift``/``max_shift`` are only used to place the pulses and size the rows.
    """
    n_in = w.nsamp + int(max_shift)
    z = noise_rows(w.seed, w.band.nchans, n_in)
    if w.dtype in ("f32", "f16"):
        plant_pulses(z, shift, w.pulses)
        return z if w.dtype == "f32" else z.astype(np.float16)
    if w.dtype == "u8":
        # pulses in units of 1/16 of the noise rms land as integers after x16
        zz = z.astype(np.float64)
        plant_pulses(zz, shift, w.pulses)
        return to_u8(zz)
    raise ValueError(w.dtype)


def batch_beams(nbeams: int = 32, seed: int = 4):
    """Uneven beams for the batched launch, drawn in this order per beam:
    nchans in {256, 496, 1024}; nsamp in [2^14, 2^17]; ndm in [512, 4096];
    DM step in {0.05, 0.1, 0.2, 0.25, 0.5}; dtype in {f32, u8}.  Every beam
    uses the MeerKAT half-L band (f_top 1712 MHz, df = 428/nchans MHz, 64 us)."""
    rng = np.random.default_rng(seed)
    beams = []
    for b in range(nbeams):
        nchans = int(rng.choice([256, 496, 1024]))
        nsamp = int(rng.integers(1 << 14, (1 << 17) + 1))
        ndm = int(rng.integers(512, 4097))
        step = float(rng.choice([0.05, 0.1, 0.2, 0.25, 0.5]))
        dtype = str(rng.choice(["f32", "u8"]))
        band = Band(nchans, 1712.0, 428.0 / nchans, 64e-6)
        beams.append(Workload("beam%02d" % b, band, dm_grid(ndm, step), nsamp, dtype, 100 + b, []))
    return beams


def stream_block(seed: int, beam: int, block: int, nchans: int, nsamp: int, pool: int = 0) -> np.ndarray:
    """uint8 block ``block`` of beam ``beam`` in a served stream, from its own
    seeded stream (``pool > 0`` folds (beam, block) onto ``pool`` distinct blocks,
    which lets a long served run cycle through pre-drawn data)."""
    key = [seed, beam, block] if pool <= 0 else [seed, (beam * 7919 + block) % pool]
    rng = np.random.default_rng(key)
    z = rng.standard_normal((nchans, nsamp), dtype=np.float32)
    return to_u8(z)

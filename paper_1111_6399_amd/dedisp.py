"""ctypes binding of libdedisp.so: the C-ABI calls under the same names.

Argument marshalling only: every step of de-dispersion runs in the library's
HIP kernels.  Device buffers are passed as integer addresses (for example
``tensor.data_ptr()`` of a ROCm torch tensor) and streams as ``hipStream_t``
handles (``torch.cuda.current_stream().cuda_stream``).  Importing this module
fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdedisp.so")

DEDISP_U8, DEDISP_F16, DEDISP_F32 = 0, 1, 2
DTYPES = {"u8": DEDISP_U8, "f16": DEDISP_F16, "f32": DEDISP_F32}
(DEDISP_OK, DEDISP_ERR_INVALID_ARG, DEDISP_ERR_OUT_OF_MEMORY, DEDISP_ERR_DEVICE, DEDISP_ERR_AGAIN,
 DEDISP_ERR_NOT_FOUND, DEDISP_ERR_INTERNAL) = range(7)


class DedispError(RuntimeError):
    def __init__(self, status: int, call: str):
        self.status = status
        super().__init__("%s: %s (status %d)" % (call, status_string(status), status))


if not os.path.exists(LIB_PATH):
    raise ImportError("libdedisp.so is not built (python -m paper_1111_6399_amd.build): %s" % LIB_PATH)

lib = ctypes.CDLL(LIB_PATH)

_p = ctypes.c_void_p
_i = ctypes.c_int
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_d = ctypes.c_double
_pp = ctypes.POINTER(ctypes.c_void_p)

_SIGS = {
    "dedisp_status_string": (ctypes.c_char_p, [_i]),
    "dedisp_plan_create": (_i, [_i, _d, _d, _d, ctypes.POINTER(_d), _i, _i, _pp]),
    "dedisp_plan_destroy": (_i, [_p]),
    "dedisp_plan_max_shift": (_i, [_p, ctypes.POINTER(ctypes.c_int32)]),
    "dedisp_plan_shift_table": (_i, [_p, ctypes.POINTER(ctypes.c_int32)]),
    "dedisp_plan_dims": (_i, [_p, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "dedisp_dm_grid": (_i, [_d, _i, ctypes.POINTER(_d)]),
    "dedisp_plan_footprint": (_i, [_p, _i64, ctypes.POINTER(_u64), ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    "dedisp_variant_count": (_i, []),
    "dedisp_variant_describe": (_i, [_i, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "dedisp_plan_set_variant": (_i, [_p, _i]),
    "dedisp_plan_get_variant": (_i, [_p, ctypes.POINTER(_i)]),
    "dedisp_autotune": (_i, [_p, _i64, ctypes.POINTER(_i), ctypes.POINTER(_d)]),
    "dedisp_execute": (_i, [_p, _p, _p, _i64, _p]),
    "dedisp_execute_static": (_i, [_p, _p, _p, _i64, _p]),
    "dedisp_detect": (_i, [_p, _p, _i64, _i, _d, _p, _p, _p, _p, _i, _p, _p]),
    "dedisp_sigproc_parse": (_i, [_p, ctypes.c_size_t, _p]),
    "dedisp_execute_cpu": (_i, [_p, _p, _p, _i64, _i, ctypes.POINTER(_i)]),
    "dedisp_corner_turn": (_i, [_p, _p, _i64, _i, _i64, _i, _i, _p]),
    "dedisp_batch_create": (_i, [_pp, ctypes.POINTER(_i64), _i, _pp]),
    "dedisp_batch_execute": (_i, [_p, _pp, _pp, _p]),
    "dedisp_batch_info": (_i, [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i)]),
    "dedisp_batch_destroy": (_i, [_p]),
    "dedisp_batch_get_variant": (_i, [_p, ctypes.POINTER(_i)]),
    "dedisp_batch_set_variant": (_i, [_p, _i]),
    "dedisp_batch_get_layout": (_i, [_p, ctypes.POINTER(_i)]),
    "dedisp_batch_set_layout": (_i, [_p, _i]),
    "dedisp_batch_autotune": (_i, [_p, _pp, _pp, _p, ctypes.POINTER(_i), ctypes.POINTER(_d)]),
    "dedisp_server_create": (_i, [ctypes.c_size_t, _i, _pp]),
    "dedisp_server_add_beam": (_i, [_p, _p, _i64, ctypes.POINTER(_i)]),
    "dedisp_submit": (_i, [_p, _i, _p, _p, ctypes.POINTER(_u64)]),
    "dedisp_poll": (_i, [_p, _u64, ctypes.POINTER(_i), ctypes.POINTER(_d)]),
    "dedisp_server_drain": (_i, [_p]),
    "dedisp_server_stats": (_i, [_p, ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "dedisp_server_destroy": (_i, [_p]),
}

EXPORTS = sorted(_SIGS)
MISSING = []
for _name, (_res, _args) in _SIGS.items():
    try:
        _f = getattr(lib, _name)
    except AttributeError:
        MISSING.append(_name)
        continue
    _f.restype = _res
    _f.argtypes = _args


def status_string(status: int) -> str:
    return lib.dedisp_status_string(int(status)).decode()


def _check(status: int, call: str) -> None:
    if status != DEDISP_OK:
        raise DedispError(status, call)


def _stream(stream) -> int | None:
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return int(stream.cuda_stream)
    return int(stream)


# ------------------------------------------------------------------ plans

def dedisp_plan_create(nchans: int, f_top: float, df: float, tsamp: float, dm_list, in_dtype) -> int:
    dm = np.ascontiguousarray(np.asarray(dm_list, dtype=np.float64))
    dt = DTYPES[in_dtype] if isinstance(in_dtype, str) else int(in_dtype)
    h = ctypes.c_void_p()
    _check(lib.dedisp_plan_create(int(nchans), float(f_top), float(df), float(tsamp),
                                  dm.ctypes.data_as(ctypes.POINTER(_d)), int(dm.size), dt, ctypes.byref(h)),
           "dedisp_plan_create")
    return h.value


def dedisp_plan_destroy(plan: int) -> None:
    _check(lib.dedisp_plan_destroy(plan), "dedisp_plan_destroy")


def dedisp_plan_max_shift(plan: int) -> int:
    v = ctypes.c_int32()
    _check(lib.dedisp_plan_max_shift(plan, ctypes.byref(v)), "dedisp_plan_max_shift")
    return v.value


def dedisp_plan_dims(plan: int):
    n, d, t = _i(), _i(), _i()
    _check(lib.dedisp_plan_dims(plan, ctypes.byref(n), ctypes.byref(d), ctypes.byref(t)), "dedisp_plan_dims")
    return n.value, d.value, t.value


def dedisp_dm_grid(dm_max: float, ndm: int) -> np.ndarray:
    out = np.empty(max(int(ndm), 1), dtype=np.float64)
    _check(lib.dedisp_dm_grid(float(dm_max), int(ndm), out.ctypes.data_as(ctypes.POINTER(_d))), "dedisp_dm_grid")
    return out


def dedisp_plan_footprint(plan: int, nsamp: int):
    a, b, c = _u64(), _u64(), _u64()
    _check(lib.dedisp_plan_footprint(plan, int(nsamp), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "dedisp_plan_footprint")
    return a.value, b.value, c.value


def dedisp_plan_shift_table(plan: int) -> np.ndarray:
    nchans, ndm, _ = dedisp_plan_dims(plan)
    out = np.empty((nchans, ndm), dtype=np.int32)
    _check(lib.dedisp_plan_shift_table(plan, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
           "dedisp_plan_shift_table")
    return out


def dedisp_variant_count() -> int:
    return int(lib.dedisp_variant_count())


def dedisp_variant_describe(variant: int):
    a, b, c = _i(), _i(), _i()
    _check(lib.dedisp_variant_describe(int(variant), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "dedisp_variant_describe")
    return a.value, b.value, c.value


def dedisp_plan_set_variant(plan: int, variant: int) -> None:
    _check(lib.dedisp_plan_set_variant(plan, int(variant)), "dedisp_plan_set_variant")


def dedisp_plan_get_variant(plan: int) -> int:
    v = _i()
    _check(lib.dedisp_plan_get_variant(plan, ctypes.byref(v)), "dedisp_plan_get_variant")
    return v.value


def dedisp_autotune(plan: int, nsamp: int):
    v, ms = _i(), _d()
    _check(lib.dedisp_autotune(plan, int(nsamp), ctypes.byref(v), ctypes.byref(ms)), "dedisp_autotune")
    return v.value, ms.value


def dedisp_execute(plan: int, in_ptr: int, out_ptr: int, nsamp: int, stream=None) -> None:
    _check(lib.dedisp_execute(plan, in_ptr, out_ptr, int(nsamp), _stream(stream)), "dedisp_execute")


def dedisp_execute_static(plan: int, in_ptr: int, out_ptr: int, nsamp: int, stream=None) -> None:
    _check(lib.dedisp_execute_static(plan, in_ptr, out_ptr, int(nsamp), _stream(stream)), "dedisp_execute_static")


# ------------------------------------------------------------------- host

def dedisp_execute_cpu(plan: int, in_array, out_array, nsamp: int, nthreads: int = 0) -> int:
    """Host arrays (numpy, C-contiguous); returns the vector ISA level used."""
    isa = _i()
    _check(lib.dedisp_execute_cpu(plan, in_array.ctypes.data, out_array.ctypes.data, int(nsamp), int(nthreads),
                                  ctypes.byref(isa)), "dedisp_execute_cpu")
    return isa.value


# -------------------------------------------------------------- ingestion

# Layout of dedisp_sigproc_header (C struct with natural alignment).
SIGPROC_HEADER_DTYPE = np.dtype([("nchans", np.int32), ("nbits", np.int32), ("nifs", np.int32),
                                 ("data_type", np.int32), ("telescope_id", np.int32), ("machine_id", np.int32),
                                 ("nbeams", np.int32), ("ibeam", np.int32), ("nsamples", np.int32),
                                 ("dtype", np.int32), ("tsamp", np.float64), ("fch1", np.float64),
                                 ("foff", np.float64), ("tstart", np.float64), ("refdm", np.float64),
                                 ("header_bytes", np.int64), ("source_name", "S80")], align=True)


def dedisp_sigproc_parse(buf: bytes) -> dict:
    """Parse a sigproc header from the start of ``buf`` (bytes)."""
    raw = np.frombuffer(bytes(buf), dtype=np.uint8)
    h = np.zeros(1, dtype=SIGPROC_HEADER_DTYPE)
    _check(lib.dedisp_sigproc_parse(raw.ctypes.data, raw.size, h.ctypes.data), "dedisp_sigproc_parse")
    out = {k: h[0][k].item() for k in SIGPROC_HEADER_DTYPE.names}
    out["source_name"] = h[0]["source_name"].decode("latin-1")
    return out


def dedisp_corner_turn(in_ptr: int, out_ptr: int, nsamp: int, nchans: int, out_pitch: int, in_dtype,
                       reverse_channels: bool = False, stream=None) -> None:
    dt = DTYPES[in_dtype] if isinstance(in_dtype, str) else int(in_dtype)
    _check(lib.dedisp_corner_turn(in_ptr, out_ptr, int(nsamp), int(nchans), int(out_pitch), dt,
                                  1 if reverse_channels else 0, _stream(stream)), "dedisp_corner_turn")


# -------------------------------------------------------------- detection

# Layout of dedisp_candidate (four 4-byte fields).
CANDIDATE_DTYPE = np.dtype([("dm_index", np.int32), ("width", np.int32), ("time", np.int32), ("snr", np.float32)])


def dedisp_detect(plan: int, out_ptr: int, nsamp: int, nwidths: int, threshold: float, stats_ptr, snr_ptr: int,
                  t_ptr: int, cand_ptr, cand_capacity: int, count_ptr, stream=None) -> None:
    """Device pointers as integers (``stats_ptr``, ``cand_ptr``, ``count_ptr`` may be None)."""
    _check(lib.dedisp_detect(plan, out_ptr, int(nsamp), int(nwidths), float(threshold), stats_ptr, snr_ptr, t_ptr,
                             cand_ptr, int(cand_capacity), count_ptr, _stream(stream)), "dedisp_detect")


# ---------------------------------------------------------------- batches

def dedisp_batch_create(plans, nsamps) -> int:
    n = len(plans)
    arr = (ctypes.c_void_p * n)(*plans)
    ns = (_i64 * n)(*[int(x) for x in nsamps])
    h = ctypes.c_void_p()
    _check(lib.dedisp_batch_create(arr, ns, n, ctypes.byref(h)), "dedisp_batch_create")
    return h.value


def dedisp_batch_execute(batch: int, ins, outs, stream=None) -> None:
    n = len(ins)
    a = (ctypes.c_void_p * n)(*ins)
    b = (ctypes.c_void_p * n)(*outs)
    _check(lib.dedisp_batch_execute(batch, a, b, _stream(stream)), "dedisp_batch_execute")


def dedisp_batch_info(batch: int):
    w, g = _i64(), _i()
    _check(lib.dedisp_batch_info(batch, ctypes.byref(w), ctypes.byref(g)), "dedisp_batch_info")
    return w.value, g.value


def dedisp_batch_get_variant(batch: int) -> int:
    v = _i()
    _check(lib.dedisp_batch_get_variant(batch, ctypes.byref(v)), "dedisp_batch_get_variant")
    return v.value


def dedisp_batch_set_variant(batch: int, variant: int) -> None:
    _check(lib.dedisp_batch_set_variant(batch, int(variant)), "dedisp_batch_set_variant")


def dedisp_batch_get_layout(batch: int) -> int:
    v = _i()
    _check(lib.dedisp_batch_get_layout(batch, ctypes.byref(v)), "dedisp_batch_get_layout")
    return v.value


def dedisp_batch_set_layout(batch: int, layout: int) -> None:
    _check(lib.dedisp_batch_set_layout(batch, int(layout)), "dedisp_batch_set_layout")


def dedisp_batch_autotune(batch: int, ins, outs, stream=None):
    n = len(ins)
    a = (ctypes.c_void_p * n)(*ins)
    b = (ctypes.c_void_p * n)(*outs)
    v, ms = _i(), _d()
    _check(lib.dedisp_batch_autotune(batch, a, b, _stream(stream), ctypes.byref(v), ctypes.byref(ms)),
           "dedisp_batch_autotune")
    return v.value, ms.value


def dedisp_batch_destroy(batch: int) -> None:
    _check(lib.dedisp_batch_destroy(batch), "dedisp_batch_destroy")


# ---------------------------------------------------------------- serving

def dedisp_server_create(hbm_budget_bytes: int, max_inflight: int) -> int:
    h = ctypes.c_void_p()
    _check(lib.dedisp_server_create(int(hbm_budget_bytes), int(max_inflight), ctypes.byref(h)),
           "dedisp_server_create")
    return h.value


def dedisp_server_add_beam(server: int, plan: int, block_nsamp: int) -> int:
    b = _i()
    _check(lib.dedisp_server_add_beam(server, plan, int(block_nsamp), ctypes.byref(b)), "dedisp_server_add_beam")
    return b.value


def dedisp_submit(server: int, beam: int, block_ptr: int, out_ptr: int):
    """Returns the ticket, or None when the request was not admitted (retry later)."""
    t = _u64()
    st = lib.dedisp_submit(server, int(beam), block_ptr, out_ptr, ctypes.byref(t))
    if st == DEDISP_ERR_AGAIN:
        return None
    _check(st, "dedisp_submit")
    return t.value


def dedisp_poll(server: int, ticket: int):
    """Returns (done, latency_s)."""
    d, lat = _i(), _d()
    _check(lib.dedisp_poll(server, _u64(ticket), ctypes.byref(d), ctypes.byref(lat)), "dedisp_poll")
    return bool(d.value), lat.value


def dedisp_server_drain(server: int) -> None:
    _check(lib.dedisp_server_drain(server), "dedisp_server_drain")


def dedisp_server_stats(server: int):
    a, b, c = _d(), _d(), _d()
    _check(lib.dedisp_server_stats(server, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
           "dedisp_server_stats")
    return a.value, b.value, c.value


def dedisp_server_destroy(server: int) -> None:
    _check(lib.dedisp_server_destroy(server), "dedisp_server_destroy")


# ------------------------------------------------------- convenience layer

# Element type names (torch dtype names) of a plan's input and output, by dtype code.
_IN_DTYPES = {DEDISP_U8: "uint8", DEDISP_F16: "float16", DEDISP_F32: "float32"}
_OUT_DTYPES = {DEDISP_U8: "int32", DEDISP_F16: "float32", DEDISP_F32: "float32"}


def device_address(buf, dtype_name: str, min_numel: int, what: str) -> int:
    """Address of a device buffer.  A tensor (anything with ``data_ptr()``) must
    be on the GPU, contiguous, of element type ``dtype_name`` and hold at least
    ``min_numel`` elements, else DedispError(INVALID_ARG) is raised before any
    library call; a plain integer is taken as an address as it is."""
    if not hasattr(buf, "data_ptr"):
        return int(buf)
    problems = []
    dev = getattr(buf, "device", None)
    if dev is not None and getattr(dev, "type", "cuda") != "cuda":
        problems.append("not on the GPU (%s)" % dev)
    if hasattr(buf, "is_contiguous") and not buf.is_contiguous():
        problems.append("not contiguous")
    dt = str(getattr(buf, "dtype", dtype_name)).replace("torch.", "")
    if dt != dtype_name:
        problems.append("element type %s, expected %s" % (dt, dtype_name))
    n = int(buf.numel()) if hasattr(buf, "numel") else min_numel
    if n < min_numel:
        problems.append("%d elements, expected at least %d" % (n, min_numel))
    if problems:
        raise DedispError(DEDISP_ERR_INVALID_ARG, "%s buffer: %s" % (what, "; ".join(problems)))
    return int(buf.data_ptr())


class Plan:
    """Owning wrapper of a plan handle."""

    def __init__(self, nchans, f_top, df, tsamp, dm_list, in_dtype="f32"):
        self.handle = dedisp_plan_create(nchans, f_top, df, tsamp, dm_list, in_dtype)
        self.nchans, self.ndm, self.dtype_code = dedisp_plan_dims(self.handle)
        self.max_shift = dedisp_plan_max_shift(self.handle)

    @classmethod
    def for_workload(cls, w):
        return cls(w.band.nchans, w.band.f_top, w.band.df, w.band.tsamp, w.dms, w.dtype)

    def shift_table(self) -> np.ndarray:
        return dedisp_plan_shift_table(self.handle)

    @property
    def variant(self) -> int:
        return dedisp_plan_get_variant(self.handle)

    @variant.setter
    def variant(self, v: int) -> None:
        dedisp_plan_set_variant(self.handle, v)

    def execute(self, inp, out, nsamp: int, stream=None) -> None:
        """``inp``/``out`` are device tensors or raw addresses.  Tensors are
        checked first (on the GPU, contiguous, element type of the plan, at
        least ``nchans*(nsamp+max_shift)`` input and ``ndm*nsamp`` output
        elements), since the library cannot see the size of an allocation."""
        nsamp = int(nsamp)
        n = max(nsamp, 0)  # the library itself rejects a negative count and does nothing for 0
        ip = device_address(inp, _IN_DTYPES[self.dtype_code], self.nchans * (n + self.max_shift) if n else 0, "input")
        op = device_address(out, _OUT_DTYPES[self.dtype_code], self.ndm * n, "output")
        dedisp_execute(self.handle, ip, op, nsamp, stream)

    def close(self) -> None:
        if self.handle:
            dedisp_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

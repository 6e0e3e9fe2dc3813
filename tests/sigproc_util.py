"""Test helper: sigproc filterbank headers written from the format's definition."""
import struct


def write_sigproc(fields, order=None):
    """A sigproc header written from the format's definition: each keyword
    as a little-endian 32-bit length and its characters, then its value."""
    ints = {"telescope_id", "machine_id", "data_type", "nchans", "nbits", "nifs", "nbeams", "ibeam",
            "barycentric", "pulsarcentric", "nsamples"}
    strs = {"source_name", "rawdatafile"}

    def s(x):
        b = x.encode("latin-1")
        return struct.pack("<i", len(b)) + b

    out = s("HEADER_START")
    for k in (order or list(fields)):
        v = fields[k]
        out += s(k)
        if k in ints:
            out += struct.pack("<i", v)
        elif k in strs:
            out += s(v)
        else:
            out += struct.pack("<d", v)
    return out + s("HEADER_END")


SIGPROC_FIELDS = {"telescope_id": 64, "machine_id": 10, "data_type": 1, "source_name": "FAKE_DM50",
                  "fch1": 1711.9478, "foff": -0.208984375, "nchans": 2048, "nbits": 8, "tstart": 59000.25,
                  "tsamp": 6.4e-05, "nifs": 1, "src_raj": 123456.7, "src_dej": -301234.5, "refdm": 50.0}

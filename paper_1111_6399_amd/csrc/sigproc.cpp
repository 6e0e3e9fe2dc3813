// Reader of sigproc filterbank headers (the file format the paper's test data
// came in: section "Searching for radio transients", data simulated with the
// sigproc package).  A header is a sequence of keywords, each written as a
// 32-bit little-endian length followed by that many characters, opened by
// HEADER_START and closed by HEADER_END; each keyword is followed by its
// value: a 32-bit integer, a binary64 number, or (for the two name keywords)
// another length-prefixed string.  Host code only.
#include <cstdint>
#include <cstring>
#include <string>

#include "../../include/dedisp.h"

namespace {

enum Kind { kInt, kDouble, kString, kNone };

struct Key {
  const char* name;
  Kind kind;
};

const Key kKeys[] = {
    {"HEADER_START", kNone}, {"HEADER_END", kNone},      {"telescope_id", kInt},  {"machine_id", kInt},
    {"data_type", kInt},     {"nchans", kInt},           {"nbits", kInt},         {"nifs", kInt},
    {"nbeams", kInt},        {"ibeam", kInt},            {"barycentric", kInt},   {"pulsarcentric", kInt},
    {"nsamples", kInt},      {"tsamp", kDouble},         {"fch1", kDouble},       {"foff", kDouble},
    {"tstart", kDouble},     {"src_raj", kDouble},       {"src_dej", kDouble},    {"az_start", kDouble},
    {"za_start", kDouble},   {"refdm", kDouble},         {"period", kDouble},     {"source_name", kString},
    {"rawdatafile", kString},
};

struct Reader {
  const unsigned char* p;
  size_t n, at;
  bool get_u32(uint32_t* v) {
    if (n - at < 4) return false;
    *v = static_cast<uint32_t>(p[at]) | (static_cast<uint32_t>(p[at + 1]) << 8) |
         (static_cast<uint32_t>(p[at + 2]) << 16) | (static_cast<uint32_t>(p[at + 3]) << 24);
    at += 4;
    return true;
  }
  bool get_f64(double* v) {
    if (n - at < 8) return false;
    uint64_t u = 0;
    for (int i = 7; i >= 0; --i) u = (u << 8) | p[at + i];
    std::memcpy(v, &u, 8);
    at += 8;
    return true;
  }
  bool get_str(std::string* s) {
    uint32_t len = 0;
    if (!get_u32(&len) || len == 0 || len > 256 || n - at < len) return false;
    s->assign(reinterpret_cast<const char*>(p + at), len);
    at += len;
    return true;
  }
};

}  // namespace

extern "C" int dedisp_sigproc_parse(const void* buf, size_t len, dedisp_sigproc_header* out) {
  if (buf == nullptr || out == nullptr) return DEDISP_ERR_INVALID_ARG;
  Reader r{static_cast<const unsigned char*>(buf), len, 0};
  dedisp_sigproc_header h;
  std::memset(&h, 0, sizeof(h));
  h.nifs = 1;
  std::string key;
  if (!r.get_str(&key) || key != "HEADER_START") return DEDISP_ERR_INVALID_ARG;
  for (;;) {
    if (!r.get_str(&key)) return DEDISP_ERR_INVALID_ARG;
    if (key == "HEADER_END") break;
    const Key* k = nullptr;
    for (const Key& x : kKeys)
      if (key == x.name) k = &x;
    if (k == nullptr || k->kind == kNone) return DEDISP_ERR_INVALID_ARG;  // unknown keyword: length of its value unknown
    if (k->kind == kInt) {
      uint32_t u = 0;
      if (!r.get_u32(&u)) return DEDISP_ERR_INVALID_ARG;
      const int32_t v = static_cast<int32_t>(u);
      if (key == "nchans") h.nchans = v;
      else if (key == "nbits") h.nbits = v;
      else if (key == "nifs") h.nifs = v;
      else if (key == "data_type") h.data_type = v;
      else if (key == "telescope_id") h.telescope_id = v;
      else if (key == "machine_id") h.machine_id = v;
      else if (key == "nbeams") h.nbeams = v;
      else if (key == "ibeam") h.ibeam = v;
      else if (key == "nsamples") h.nsamples = v;
    } else if (k->kind == kDouble) {
      double v = 0.0;
      if (!r.get_f64(&v)) return DEDISP_ERR_INVALID_ARG;
      if (key == "tsamp") h.tsamp = v;
      else if (key == "fch1") h.fch1 = v;
      else if (key == "foff") h.foff = v;
      else if (key == "tstart") h.tstart = v;
      else if (key == "refdm") h.refdm = v;
    } else {
      std::string v;
      if (!r.get_str(&v)) return DEDISP_ERR_INVALID_ARG;
      if (key == "source_name") {
        const size_t m = v.size() < sizeof(h.source_name) - 1 ? v.size() : sizeof(h.source_name) - 1;
        std::memcpy(h.source_name, v.data(), m);
      }
    }
  }
  if (h.nchans < 1 || h.tsamp <= 0.0 || h.foff == 0.0 || h.nifs < 1) return DEDISP_ERR_INVALID_ARG;
  if (h.nbits != 8 && h.nbits != 16 && h.nbits != 32) return DEDISP_ERR_INVALID_ARG;
  h.dtype = h.nbits == 8 ? DEDISP_U8 : h.nbits == 32 ? DEDISP_F32 : -1;  // 16-bit integers have no plan type
  h.header_bytes = static_cast<int64_t>(r.at);
  *out = h;
  return DEDISP_OK;
}

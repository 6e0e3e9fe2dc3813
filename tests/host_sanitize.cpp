// Host parts of the library run under AddressSanitizer + UndefinedBehavior-
// Sanitizer or ThreadSanitizer (test infrastructure, built and run by
// tests/test_host_sanitizers.py): the binary64 delay table builder on the
// workloads' bands, the sigproc header parser on a valid header, every
// truncation of it and corrupted copies, and the threaded host search on
// small plans of every input type against a plain loop written here.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "dedisp_internal.h"
#include "shift_table.h"

namespace {

int failures = 0;

#define CHECK(cond)                                                      \
  do {                                                                   \
    if (!(cond)) {                                                       \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                        \
    }                                                                    \
  } while (0)

// --------------------------------------------------------------- delays --

int32_t max_shift_of(int nchans, double f_top, double df, double tsamp, int ndm, double step) {
  std::vector<double> dms(ndm);
  for (int d = 0; d < ndm; ++d) dms[d] = d * step;
  std::vector<int32_t> table;
  int32_t m = -1;
  CHECK(dedisp::build_shift_table(nchans, f_top, df, tsamp, dms.data(), ndm, &table, &m));
  CHECK(table.size() == static_cast<size_t>(nchans) * ndm);
  for (int d = 0; d < ndm; ++d) CHECK(table[d] == 0);  // channel 0 is the reference
  return m;
}

void delays() {
  // the small band, the LOFAR-shaped band and the MeerKAT-shaped band
  CHECK(max_shift_of(64, 150.0, 0.1953125, 327.68e-6, 100, 0.1) == 1040);
  CHECK(max_shift_of(496, 150.0, 0.1953125, 327.68e-6, 2048, 0.1) == 796415);
  CHECK(max_shift_of(4096, 1712.0, 428.0 / 4096, 64e-6, 4096, 0.5) == 35209);
}

// -------------------------------------------------------------- sigproc --

void put_i32(std::vector<uint8_t>& b, int32_t v) {
  uint8_t x[4];
  std::memcpy(x, &v, 4);
  b.insert(b.end(), x, x + 4);
}
void put_f64(std::vector<uint8_t>& b, double v) {
  uint8_t x[8];
  std::memcpy(x, &v, 8);
  b.insert(b.end(), x, x + 8);
}
void put_str(std::vector<uint8_t>& b, const char* s) {
  put_i32(b, static_cast<int32_t>(std::strlen(s)));
  b.insert(b.end(), s, s + std::strlen(s));
}

std::vector<uint8_t> header() {
  std::vector<uint8_t> b;
  put_str(b, "HEADER_START");
  put_str(b, "telescope_id");
  put_i32(b, 64);
  put_str(b, "source_name");
  put_str(b, "FAKE");
  put_str(b, "fch1");
  put_f64(b, 1711.9478);
  put_str(b, "foff");
  put_f64(b, -0.208984375);
  put_str(b, "nchans");
  put_i32(b, 2048);
  put_str(b, "nbits");
  put_i32(b, 8);
  put_str(b, "tstart");
  put_f64(b, 59000.25);
  put_str(b, "tsamp");
  put_f64(b, 6.4e-05);
  put_str(b, "nifs");
  put_i32(b, 1);
  put_str(b, "HEADER_END");
  return b;
}

void sigproc() {
  const std::vector<uint8_t> h = header();
  dedisp_sigproc_header out;
  CHECK(dedisp_sigproc_parse(h.data(), h.size(), &out) == DEDISP_OK);
  CHECK(out.nchans == 2048 && out.nbits == 8 && out.nifs == 1 && out.header_bytes == static_cast<int64_t>(h.size()));
  // every truncation is refused, reading nothing past the given length (each
  // prefix is copied into a buffer of exactly that size)
  for (size_t n = 0; n < h.size(); ++n) {
    std::vector<uint8_t> cut(h.begin(), h.begin() + n);
    CHECK(dedisp_sigproc_parse(cut.empty() ? nullptr : cut.data(), n, &out) != DEDISP_OK);
  }
  // corrupted copies: accepted or refused, never read out of bounds
  std::mt19937 rng(12345);
  for (int k = 0; k < 3000; ++k) {
    std::vector<uint8_t> c = h;
    const int flips = 1 + static_cast<int>(rng() % 4);
    for (int f = 0; f < flips; ++f) c[rng() % c.size()] = static_cast<uint8_t>(rng());
    const int st = dedisp_sigproc_parse(c.data(), c.size(), &out);
    CHECK(st == DEDISP_OK || st == DEDISP_ERR_INVALID_ARG);
  }
}

// ---------------------------------------------------------- host search --

float half_to_float(uint16_t h) {  // IEEE 754 binary16
  const int e = (h >> 10) & 0x1f, m = h & 0x3ff;
  const double s = (h & 0x8000) ? -1.0 : 1.0;
  if (e == 0) return static_cast<float>(s * std::ldexp(m, -24));
  if (e == 31) return m ? NAN : static_cast<float>(s * INFINITY);
  return static_cast<float>(s * std::ldexp(1024 + m, e - 25));
}

uint16_t float_to_half_small(float v) {  // |v| < 2^15, normal or zero; round to nearest even
  if (v == 0.0f) return 0;
  const uint16_t sign = v < 0 ? 0x8000 : 0;
  double a = std::fabs(static_cast<double>(v));
  int e = 0;
  const double f = std::frexp(a, &e);  // a = f * 2^e, 0.5 <= f < 1
  double m = std::nearbyint(f * 2048.0);  // 11 significant bits
  if (m == 2048.0) {
    m = 1024.0;
    ++e;
  }
  const int be = e - 1 + 15;
  if (be <= 0) return sign;  // flushed (never for these inputs)
  return static_cast<uint16_t>(sign | (be << 10) | (static_cast<int>(m) - 1024));
}

void search(int dtype, int nchans, int ndm, double step, int64_t nsamp, int nthreads) {
  dedisp_plan_s p;
  p.nchans = nchans;
  p.ndm = ndm;
  p.dtype = dtype;
  p.f_top = 150.0;
  p.df = 0.1953125 * 8;
  p.tsamp = 327.68e-6;
  for (int d = 0; d < ndm; ++d) p.dms.push_back(d * step);
  CHECK(dedisp::build_shift_table(nchans, p.f_top, p.df, p.tsamp, p.dms.data(), ndm, &p.shift, &p.max_shift));
  const int64_t pitch = nsamp + p.max_shift;
  std::mt19937 rng(static_cast<uint32_t>(dtype * 1000 + nsamp + nthreads));
  std::normal_distribution<float> z(0.0f, 1.0f);
  std::vector<uint8_t> in8;
  std::vector<uint16_t> in16;
  std::vector<float> in32, x(static_cast<size_t>(nchans) * pitch);
  for (size_t i = 0; i < x.size(); ++i) {
    if (dtype == DEDISP_U8) {
      in8.push_back(static_cast<uint8_t>(rng() & 0xff));
      x[i] = in8.back();
    } else if (dtype == DEDISP_F16) {
      in16.push_back(float_to_half_small(z(rng)));
      x[i] = half_to_float(in16.back());
    } else {
      in32.push_back(z(rng));
      x[i] = in32.back();
    }
  }
  const void* in = dtype == DEDISP_U8 ? static_cast<const void*>(in8.data())
                   : dtype == DEDISP_F16 ? static_cast<const void*>(in16.data())
                                         : static_cast<const void*>(in32.data());
  std::vector<int32_t> out_i(static_cast<size_t>(ndm) * nsamp, -1);
  std::vector<float> out_f(static_cast<size_t>(ndm) * nsamp, -1.0f);
  void* out = dtype == DEDISP_U8 ? static_cast<void*>(out_i.data()) : static_cast<void*>(out_f.data());
  int isa = -1;
  CHECK(dedisp_execute_cpu(&p, in, out, nsamp, nthreads, &isa) == DEDISP_OK);
  CHECK(isa >= 0 && isa <= 2);
  for (int d = 0; d < ndm; ++d)
    for (int64_t t = 0; t < nsamp; ++t) {
      double sum = 0.0, mag = 0.0;
      for (int c = 0; c < nchans; ++c) {
        const double v = x[static_cast<size_t>(c) * pitch + t + p.shift[static_cast<size_t>(c) * ndm + d]];
        sum += v;
        mag += std::fabs(v);
      }
      const size_t o = static_cast<size_t>(d) * nsamp + t;
      if (dtype == DEDISP_U8)
        CHECK(out_i[o] == static_cast<int32_t>(sum));
      else
        CHECK(std::fabs(out_f[o] - sum) <= 1e-5 * mag + 1e-30);
    }
}

}  // namespace

int main() {
  delays();
  sigproc();
  for (int dtype : {DEDISP_U8, DEDISP_F16, DEDISP_F32})
    for (int64_t nsamp : {1, 7, 129, 300})
      for (int nthreads : {1, 3}) search(dtype, 37, 21, 2.5, nsamp, nthreads);
  // an empty request, and refused arguments
  dedisp_plan_s p;
  p.nchans = 4;
  p.ndm = 2;
  p.dms = {0.0, 1.0};
  CHECK(dedisp::build_shift_table(4, 150.0, 1.0, 1e-3, p.dms.data(), 2, &p.shift, &p.max_shift));
  CHECK(dedisp_execute_cpu(&p, nullptr, nullptr, 0, 1, nullptr) == DEDISP_OK);
  CHECK(dedisp_execute_cpu(&p, nullptr, nullptr, 5, 1, nullptr) == DEDISP_ERR_INVALID_ARG);
  CHECK(dedisp_execute_cpu(nullptr, nullptr, nullptr, 5, 1, nullptr) == DEDISP_ERR_INVALID_ARG);
  int isa = -1;
  dedisp_execute_cpu(&p, nullptr, nullptr, 0, 1, &isa);
  std::printf("host checks %s (%d failures; host search vector level %d)\n", failures ? "FAILED" : "passed",
              failures, isa);
  return failures ? 1 : 0;
}

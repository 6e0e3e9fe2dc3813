// Binary64 dispersion-delay table (host).  Built with -ffp-contract=off: the
// operation order below is part of the definition, so that every table entry
// is reproducible bit for bit.
//
// Section "Searching for radio transients": the cold-plasma law delays a
// channel by an amount proportional to DM * f^-2; incoherent de-dispersion
// removes that delay, measured from the top of the band, channel by channel.
#include <cmath>
#include <cstdint>

#include "shift_table.h"

namespace dedisp {

// Delay, in samples per unit DM, of channel c relative to channel 0.
static double delay_per_dm(double f_top, double df, double tsamp, int c) {
  const double f = f_top - static_cast<double>(c) * df;
  const double lo = 1.0 / (f * f);
  const double hi = 1.0 / (f_top * f_top);
  return kDispersionConstant * (lo - hi) / tsamp;
}

// Round half up for x >= 0.  x - floor(x) is exact for non-negative x.
static bool round_half_up(double x, int64_t* r) {
  const double fl = std::floor(x);
  const double v = fl + ((x - fl) >= 0.5 ? 1.0 : 0.0);
  if (!(v >= 0.0) || v > 2147483647.0) return false;
  *r = static_cast<int64_t>(v);
  return true;
}

bool build_shift_table(int nchans, double f_top, double df, double tsamp, const double* dm, int ndm,
                       std::vector<int32_t>* table, int32_t* max_shift) {
  table->assign(static_cast<size_t>(nchans) * ndm, 0);
  int64_t m = 0;
  for (int c = 0; c < nchans; ++c) {
    const double k = delay_per_dm(f_top, df, tsamp, c);
    int32_t* row = table->data() + static_cast<size_t>(c) * ndm;
    for (int d = 0; d < ndm; ++d) {
      int64_t s;
      if (!round_half_up(dm[d] * k, &s)) return false;
      row[d] = static_cast<int32_t>(s);
      if (s > m) m = s;
    }
  }
  *max_shift = static_cast<int32_t>(m);
  return true;
}

}  // namespace dedisp

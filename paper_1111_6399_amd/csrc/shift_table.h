// Binary64 delay table builder (host only, no HIP dependency).
#pragma once

#include <cstdint>
#include <vector>

namespace dedisp {

// Dispersion constant, s MHz^2 pc^-1 cm^3.
constexpr double kDispersionConstant = 4148.808;

// table[c*ndm + d] = round_half_up(dm[d] * 4148.808*(1/(f_c*f_c) - 1/(f_top*f_top))/tsamp),
// f_c = f_top - c*df.  Returns false if an entry does not fit in int32.
bool build_shift_table(int nchans, double f_top, double df, double tsamp, const double* dm, int ndm,
                       std::vector<int32_t>* table, int32_t* max_shift);

}  // namespace dedisp

// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/dedisp.h"
#include "shift_table.h"

namespace dedisp {

// Float sums are accumulated in blocks of this many channels (see dedisp.h).
constexpr int kChanBlock = 32;


inline size_t dtype_size(int dtype) { return dtype == DEDISP_U8 ? 1 : dtype == DEDISP_F16 ? 2 : 4; }
inline size_t out_size(int) { return 4; }

// Shape of a tiled kernel variant.
struct TileShape {
  int dw;   // trials per wave
  int ks;   // 64-bit LDS reads per lane per trial (2 samples each)
  int wd;   // waves along the trial axis
  int wt;   // waves along the time axis
  int dms() const { return dw * wd; }
  int samples() const { return 128 * ks * wt; }
  int threads() const { return 64 * wd * wt; }
};

// Per-device state of a plan: the delay table padded to a multiple of 64
// trials per channel, and per tile shape the (min, max) delay of every
// (trial tile, channel).
struct DeviceTables {
  int32_t* shift = nullptr;  // [nchans][ndm_pad]
  std::map<int, int2*> windows;  // dms-per-tile -> [ntiles][nchans]
};

struct Launch;

}  // namespace dedisp

struct dedisp_plan_s {
  int nchans = 0;
  int ndm = 0;
  int ndm_pad = 0;
  int dtype = DEDISP_F32;
  double f_top = 0, df = 0, tsamp = 0;
  std::vector<double> dms;
  std::vector<int32_t> shift;  // [nchans][ndm]
  int32_t max_shift = 0;
  std::atomic<int> variant{-1};  // -1: library default
  std::mutex mu;
  std::map<int, dedisp::DeviceTables> dev;  // per device id
  std::map<int, std::vector<int2>> host_windows;  // dms-per-tile -> [ntiles][nchans]
};

namespace dedisp {

// Device table of a plan on the current device (uploaded on first use).
int device_tables(dedisp_plan p, int device, DeviceTables** out);
// Window table for a trial-tile size on the current device.
int device_windows(dedisp_plan p, int device, int dms_per_tile, const int2** out);
const std::vector<int2>& host_windows(dedisp_plan p, int dms_per_tile);

// Kernel registry (kernels.hip).
int variant_count();
TileShape variant_shape(int v);   // v >= 1
// Largest window (in samples) a tiled variant can stage for this plan, and
// whether the plan fits it.
bool variant_fits(dedisp_plan p, int v);
int default_variant(dedisp_plan p);

// Launch one plan's kernel over the whole problem.
int launch(dedisp_plan p, int variant, const void* in, void* out, int64_t nsamp, hipStream_t s);

inline int hip_status(hipError_t e) {
  if (e == hipSuccess) return DEDISP_OK;
  if (e == hipErrorOutOfMemory) return DEDISP_ERR_OUT_OF_MEMORY;
  return DEDISP_ERR_DEVICE;
}

}  // namespace dedisp

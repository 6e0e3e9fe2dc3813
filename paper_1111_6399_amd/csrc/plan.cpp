// Plans: argument checks, the binary64 delay table, per-device copies, and the
// plain execute entry point.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "dedisp_internal.h"

using dedisp::DeviceTables;

extern "C" const char* dedisp_status_string(int status) {
  switch (status) {
    case DEDISP_OK: return "ok";
    case DEDISP_ERR_INVALID_ARG: return "invalid argument";
    case DEDISP_ERR_OUT_OF_MEMORY: return "out of memory";
    case DEDISP_ERR_DEVICE: return "device error";
    case DEDISP_ERR_AGAIN: return "not admitted, try again";
    case DEDISP_ERR_NOT_FOUND: return "not found";
    case DEDISP_ERR_INTERNAL: return "internal error";
    default: return "unknown status";
  }
}

extern "C" int dedisp_plan_create(int nchans, double f_top, double df, double tsamp, const double* dm_list,
                                  int ndm, int in_dtype, dedisp_plan* out_plan) {
  if (out_plan == nullptr || dm_list == nullptr) return DEDISP_ERR_INVALID_ARG;
  if (nchans < 1 || ndm < 1) return DEDISP_ERR_INVALID_ARG;
  if (!(std::isfinite(f_top) && std::isfinite(df) && std::isfinite(tsamp))) return DEDISP_ERR_INVALID_ARG;
  if (!(f_top > 0.0 && df > 0.0 && tsamp > 0.0)) return DEDISP_ERR_INVALID_ARG;
  if (!(f_top - static_cast<double>(nchans - 1) * df > 0.0)) return DEDISP_ERR_INVALID_ARG;
  if (in_dtype != DEDISP_U8 && in_dtype != DEDISP_F16 && in_dtype != DEDISP_F32) return DEDISP_ERR_INVALID_ARG;
  for (int d = 0; d < ndm; ++d)
    if (!std::isfinite(dm_list[d]) || dm_list[d] < 0.0) return DEDISP_ERR_INVALID_ARG;
  // padded rows and the int32 index arithmetic of the kernels
  if (static_cast<int64_t>(ndm) > (1 << 30)) return DEDISP_ERR_INVALID_ARG;

  dedisp_plan p = new (std::nothrow) dedisp_plan_s();
  if (p == nullptr) return DEDISP_ERR_OUT_OF_MEMORY;
  p->nchans = nchans;
  p->ndm = ndm;
  p->ndm_pad = (ndm + 63) / 64 * 64;
  p->dtype = in_dtype;
  p->f_top = f_top;
  p->df = df;
  p->tsamp = tsamp;
  try {
    p->dms.assign(dm_list, dm_list + ndm);
    if (!dedisp::build_shift_table(nchans, f_top, df, tsamp, dm_list, ndm, &p->shift, &p->max_shift)) {
      delete p;
      return DEDISP_ERR_INVALID_ARG;
    }
  } catch (const std::bad_alloc&) {
    delete p;
    return DEDISP_ERR_OUT_OF_MEMORY;
  }
  *out_plan = p;
  return DEDISP_OK;
}

extern "C" int dedisp_plan_destroy(dedisp_plan p) {
  if (p == nullptr) return DEDISP_OK;
  int dev0 = -1;
  if (!p->dev.empty()) (void)hipGetDevice(&dev0);
  for (auto& kv : p->dev) {
    if (hipSetDevice(kv.first) != hipSuccess) continue;
    if (kv.second.shift) (void)hipFree(kv.second.shift);
    for (auto& w : kv.second.window_base) (void)hipFree(w.second);
    for (auto& w : kv.second.slot_pos) (void)hipFree(w.second);
  }
  if (dev0 >= 0) (void)hipSetDevice(dev0);
  delete p;
  return DEDISP_OK;
}

extern "C" int dedisp_plan_max_shift(dedisp_plan p, int32_t* out) {
  if (p == nullptr || out == nullptr) return DEDISP_ERR_INVALID_ARG;
  *out = p->max_shift;
  return DEDISP_OK;
}

extern "C" int dedisp_plan_shift_table(dedisp_plan p, int32_t* host_out) {
  if (p == nullptr || host_out == nullptr) return DEDISP_ERR_INVALID_ARG;
  std::memcpy(host_out, p->shift.data(), p->shift.size() * sizeof(int32_t));
  return DEDISP_OK;
}

extern "C" int dedisp_plan_dims(dedisp_plan p, int* nchans, int* ndm, int* in_dtype) {
  if (p == nullptr) return DEDISP_ERR_INVALID_ARG;
  if (nchans) *nchans = p->nchans;
  if (ndm) *ndm = p->ndm;
  if (in_dtype) *in_dtype = p->dtype;
  return DEDISP_OK;
}

extern "C" int dedisp_dm_grid(double dm_max, int ndm, double* dm_out) {
  if (dm_out == nullptr || ndm < 1 || !std::isfinite(dm_max) || dm_max < 0.0) return DEDISP_ERR_INVALID_ARG;
  if (ndm == 1) {
    dm_out[0] = 0.0;
    return DEDISP_OK;
  }
  const double den = static_cast<double>(ndm - 1);
  for (int d = 0; d < ndm; ++d) dm_out[d] = dm_max * (static_cast<double>(d) / den);
  return DEDISP_OK;
}

extern "C" int dedisp_plan_footprint(dedisp_plan p, int64_t nsamp, uint64_t* in_bytes, uint64_t* out_bytes,
                                     uint64_t* staged_bytes) {
  if (p == nullptr || nsamp < 0 || nsamp > static_cast<int64_t>(INT32_MAX) - p->max_shift)
    return DEDISP_ERR_INVALID_ARG;
  const uint64_t total = static_cast<uint64_t>(p->nchans) * static_cast<uint64_t>(nsamp + p->max_shift);
  if (in_bytes) *in_bytes = total * dedisp::dtype_size(p->dtype);
  if (out_bytes) *out_bytes = static_cast<uint64_t>(p->ndm) * static_cast<uint64_t>(nsamp) * 4u;
  if (staged_bytes)
    *staged_bytes = p->dtype != DEDISP_U8 ? 0u
                                          : static_cast<uint64_t>(dedisp::widened_samples(static_cast<int64_t>(total))) *
                                                static_cast<uint64_t>(dedisp::staged_size(p->dtype));
  return DEDISP_OK;
}

extern "C" int dedisp_plan_set_variant(dedisp_plan p, int variant) {
  if (p == nullptr || variant < 0 || variant >= dedisp::variant_count()) return DEDISP_ERR_INVALID_ARG;
  if (variant > 0 && !dedisp::variant_fits(p, variant)) return DEDISP_ERR_INVALID_ARG;
  p->variant.store(variant);
  return DEDISP_OK;
}

extern "C" int dedisp_plan_get_variant(dedisp_plan p, int* variant) {
  if (p == nullptr || variant == nullptr) return DEDISP_ERR_INVALID_ARG;
  const int v = p->variant.load();
  *variant = v >= 0 ? v : dedisp::default_variant(p);
  return DEDISP_OK;
}

namespace dedisp {

bool trace_enabled() {
  static const bool on = std::getenv("DEDISP_TRACE") != nullptr;
  return on;
}

void trace_hip_error(hipError_t e, const char* file, int line) {
  std::fprintf(stderr, "[dedisp] %s:%d: %s\n", file, line, hipGetErrorString(e));
}

const std::vector<int2>& host_windows(dedisp_plan p, int dms_per_tile) {
  std::lock_guard<std::mutex> g(p->mu);
  auto it = p->host_windows.find(dms_per_tile);
  if (it != p->host_windows.end()) return it->second;
  const int ntiles = (p->ndm + dms_per_tile - 1) / dms_per_tile;
  std::vector<int2> w(static_cast<size_t>(ntiles) * p->nchans);
  for (int t = 0; t < ntiles; ++t) {
    const int d0 = t * dms_per_tile;
    const int d1 = std::min(p->ndm, d0 + dms_per_tile);
    for (int c = 0; c < p->nchans; ++c) {
      const int32_t* row = p->shift.data() + static_cast<size_t>(c) * p->ndm;
      int lo = row[d0], hi = row[d0];
      for (int d = d0 + 1; d < d1; ++d) {
        lo = std::min(lo, row[d]);
        hi = std::max(hi, row[d]);
      }
      w[static_cast<size_t>(t) * p->nchans + c] = make_int2(lo, hi);
    }
  }
  return p->host_windows.emplace(dms_per_tile, std::move(w)).first->second;
}

int device_tables(dedisp_plan p, int device, DeviceTables** out, bool create) {
  std::lock_guard<std::mutex> g(p->mu);
  auto found = p->dev.find(device);
  if (!create && (found == p->dev.end() || found->second.shift == nullptr)) return DEDISP_ERR_INVALID_ARG;
  DeviceTables& t = p->dev[device];
  if (t.shift == nullptr) {
    // Rows padded to a multiple of 64 trials, pad entries repeat the last trial
    // so that every padded read stays inside the window of its tile.  Rows
    // of zeros follow the last channel: kernels read the delays of channels
    // ahead without a bounds check.
    std::vector<int32_t> padded(static_cast<size_t>(p->nchans + kShiftPadRows) * p->ndm_pad, 0);
    for (int c = 0; c < p->nchans; ++c) {
      const int32_t* src = p->shift.data() + static_cast<size_t>(c) * p->ndm;
      int32_t* dst = padded.data() + static_cast<size_t>(c) * p->ndm_pad;
      std::memcpy(dst, src, sizeof(int32_t) * p->ndm);
      for (int d = p->ndm; d < p->ndm_pad; ++d) dst[d] = src[p->ndm - 1];
    }
    int32_t* dptr = nullptr;
    hipError_t e = hipMalloc(&dptr, padded.size() * sizeof(int32_t));
    if (e != hipSuccess) return hip_status(e);
    e = hipMemcpy(dptr, padded.data(), padded.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      (void)hipFree(dptr);
      return hip_status(e);
    }
    t.shift = dptr;
  }
  *out = &t;
  return DEDISP_OK;
}

namespace {

template <typename T>
int upload(const std::vector<T>& h, T** out) {
  T* dptr = nullptr;
  hipError_t e = hipMalloc(&dptr, h.size() * sizeof(T));
  if (e != hipSuccess) return hip_status(e);
  e = hipMemcpy(dptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(dptr);
    return hip_status(e);
  }
  *out = dptr;
  return DEDISP_OK;
}

// Alignment of row c's start in samples: (c*pitch + start) mod align.
inline int row_phase(int c, int pitch_mod, int start_mod, int align) {
  return static_cast<int>((static_cast<int64_t>(c) * pitch_mod + start_mod) % align);
}

// Alignment of the window start c*pitch + start + t0 + lo (t0 is a multiple
// of align).
inline int window_mis(int c, int pitch_mod, int start_mod, int lo, int align) {
  return (row_phase(c, pitch_mod, start_mod, align) + lo % align) % align;
}

}  // namespace

int device_window_base(dedisp_plan p, int device, int dms_per_tile, int samples, int align, int es, int pitch_mod,
                       int start_mod, int halo, const uint32_t** out, bool create) {
  const std::vector<int2>& hw = host_windows(p, dms_per_tile);
  std::lock_guard<std::mutex> g(p->mu);
  DeviceTables& t = p->dev[device];
  const auto key = std::make_tuple(dms_per_tile, samples, align, es, pitch_mod, start_mod, halo);
  auto it = t.window_base.find(key);
  if (it == t.window_base.end() && !create) return DEDISP_ERR_INVALID_ARG;
  if (it == t.window_base.end()) {
    const int ntiles = static_cast<int>(hw.size() / p->nchans);
    const int stride = p->nchans + kGeoPad;
    // rows of each tile end with kGeoPad zero entries: kernels read the
    // entries of channels ahead without a bounds check
    std::vector<uint32_t> base(2 * static_cast<size_t>(ntiles) * stride, 0u);
    for (int tile = 0; tile < ntiles; ++tile)
      for (int c = 0; c < p->nchans; ++c) {
        const int2 w = hw[static_cast<size_t>(tile) * p->nchans + c];
        const int mis = window_mis(c, pitch_mod, start_mod, w.x, align);
        // from the row's start rounded down to align: its phase, then lo - mis
        const int64_t start = row_phase(c, pitch_mod, start_mod, align) + w.x - mis;
        // bytes the tile's reads reach: its samples, the delay spread, the
        // start alignment and the halo lane's neighbour read
        const int64_t bytes = es * (static_cast<int64_t>(w.y) - w.x + mis + samples) + halo;
        uint32_t* e = base.data() + 2 * (static_cast<size_t>(tile) * stride + c);
        e[0] = static_cast<uint32_t>(es * start);
        e[1] = static_cast<uint32_t>((bytes + 1023) / 1024);
      }
    uint32_t* d = nullptr;
    const int st = upload(base, &d);
    if (st != DEDISP_OK) return st;
    it = t.window_base.emplace(key, d).first;
  }
  *out = it->second;
  return DEDISP_OK;
}

int device_slot_pos(dedisp_plan p, int device, int dms_per_tile, int align, int es, int pitch_mod, int start_mod,
                    const int32_t** out, bool create) {
  const std::vector<int2>& hw = host_windows(p, dms_per_tile);
  std::lock_guard<std::mutex> g(p->mu);
  DeviceTables& t = p->dev[device];
  const auto key = std::make_tuple(dms_per_tile, align, es, pitch_mod, start_mod);
  auto it = t.slot_pos.find(key);
  if (it == t.slot_pos.end() && !create) return DEDISP_ERR_INVALID_ARG;
  if (it == t.slot_pos.end()) {
    const int ntiles = static_cast<int>(hw.size() / p->nchans);
    const size_t stride = static_cast<size_t>(p->nchans + kGeoPad) * dms_per_tile;
    std::vector<int32_t> pos(static_cast<size_t>(ntiles) * stride, 0);
    for (int tile = 0; tile < ntiles; ++tile)
      for (int c = 0; c < p->nchans; ++c) {
        const int lo = hw[static_cast<size_t>(tile) * p->nchans + c].x;
        const int mis = window_mis(c, pitch_mod, start_mod, lo, align);
        const int32_t* row = p->shift.data() + static_cast<size_t>(c) * p->ndm;
        int32_t* dst = pos.data() + tile * stride + static_cast<size_t>(c) * dms_per_tile;
        for (int j = 0; j < dms_per_tile; ++j) {
          // trials past the last repeat it, so that they stay inside the window
          const int d = std::min(p->ndm - 1, tile * dms_per_tile + j);
          dst[j] = es * (row[d] - lo + mis);
        }
      }
    int32_t* d = nullptr;
    const int st = upload(pos, &d);
    if (st != DEDISP_OK) return st;
    it = t.slot_pos.emplace(key, d).first;
  }
  *out = it->second;
  return DEDISP_OK;
}

}  // namespace dedisp

extern "C" int dedisp_execute_static(dedisp_plan p, const void* in, void* out, int64_t nsamp, void* stream) {
  if (p == nullptr || nsamp < 0) return DEDISP_ERR_INVALID_ARG;
  if (nsamp == 0) return DEDISP_OK;
  if (in == nullptr || out == nullptr) return DEDISP_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(in) & 15) != 0 || (reinterpret_cast<uintptr_t>(out) & 3) != 0)
    return DEDISP_ERR_INVALID_ARG;
  if (nsamp > static_cast<int64_t>(INT32_MAX) - p->max_shift) return DEDISP_ERR_INVALID_ARG;
  int v = p->variant.load();
  if (v < 0) v = dedisp::default_variant(p);
  void* ws = nullptr;
  if (p->dtype == DEDISP_U8 && v > 0) {
    // the widened copy goes to the library's static scratch
    if (dedisp::staged_bytes(p, nsamp) > dedisp::static_scratch_bytes()) return DEDISP_ERR_INVALID_ARG;
    const int st = dedisp::static_scratch(&ws);
    if (st != DEDISP_OK) return st;
  }
  return dedisp::launch(p, v, in, out, nsamp, static_cast<hipStream_t>(stream), ws, true);
}

extern "C" int dedisp_execute(dedisp_plan p, const void* in, void* out, int64_t nsamp, void* stream) {
  if (p == nullptr || nsamp < 0) return DEDISP_ERR_INVALID_ARG;
  if (nsamp == 0) return DEDISP_OK;
  if (in == nullptr || out == nullptr) return DEDISP_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(in) & 15) != 0 || (reinterpret_cast<uintptr_t>(out) & 3) != 0)
    return DEDISP_ERR_INVALID_ARG;
  if (nsamp > static_cast<int64_t>(INT32_MAX) - p->max_shift) return DEDISP_ERR_INVALID_ARG;
  int v = p->variant.load();
  if (v < 0) v = dedisp::default_variant(p);
  return dedisp::launch(p, v, in, out, nsamp, static_cast<hipStream_t>(stream));
}

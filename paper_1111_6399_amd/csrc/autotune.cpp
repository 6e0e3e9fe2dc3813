// Autotuner: time every kernel variant that fits a plan on scratch buffers of
// the plan's shape and keep the fastest.  Results are cached in memory per
// (shape, device) and optionally in a text file named by DEDISP_TUNE_CACHE,
// one line per entry: "<key> <variant> <ms>".
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>

#include "dedisp_internal.h"

namespace {

std::mutex g_mu;
std::map<std::string, std::pair<int, double>> g_cache;
bool g_file_loaded = false;

// The delay table fixes everything the kernels' speed depends on apart from
// the output length, the device and the kernels themselves, so the key
// hashes the table and the variant registry (shapes and kernel generation).
std::string tune_key(dedisp_plan p, int64_t nsamp, int device) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the table
  const unsigned char* b = reinterpret_cast<const unsigned char*>(p->shift.data());
  for (size_t i = 0; i < p->shift.size() * sizeof(int32_t); ++i) h = (h ^ b[i]) * 1099511628211ull;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) arch = prop.gcnArchName;
  std::ostringstream os;
  os << arch << ':' << p->nchans << 'x' << p->ndm << 'x' << nsamp << ":t" << p->dtype << ":r" << std::hex
     << dedisp::registry_signature() << ':' << h;
  return os.str();
}

void load_file_locked() {
  if (g_file_loaded) return;
  g_file_loaded = true;
  const char* path = std::getenv("DEDISP_TUNE_CACHE");
  if (path == nullptr) return;
  std::ifstream f(path);
  std::string key;
  int v;
  double ms;
  while (f >> key >> v >> ms) g_cache[key] = {v, ms};
}

void append_file(const std::string& key, int v, double ms) {
  const char* path = std::getenv("DEDISP_TUNE_CACHE");
  if (path == nullptr) return;
  std::ofstream f(path, std::ios::app);
  f << key << ' ' << v << ' ' << ms << '\n';
}

}  // namespace

extern "C" int dedisp_autotune(dedisp_plan p, int64_t nsamp, int* best_variant, double* best_ms) {
  if (p == nullptr || best_variant == nullptr || nsamp < 1) return DEDISP_ERR_INVALID_ARG;
  if (nsamp > static_cast<int64_t>(INT32_MAX) - p->max_shift) return DEDISP_ERR_INVALID_ARG;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  const std::string key = tune_key(p, nsamp, dev);
  {
    std::lock_guard<std::mutex> g(g_mu);
    load_file_locked();
    auto it = g_cache.find(key);
    if (it != g_cache.end() && it->second.first < dedisp::variant_count() &&
        (it->second.first == 0 || dedisp::variant_fits(p, it->second.first))) {
      p->variant.store(it->second.first);
      *best_variant = it->second.first;
      if (best_ms) *best_ms = it->second.second;
      return DEDISP_OK;
    }
  }
  const bool trace = std::getenv("DEDISP_TRACE") != nullptr;
  const size_t in_bytes = static_cast<size_t>(p->nchans) * (nsamp + p->max_shift) * dedisp::dtype_size(p->dtype);
  const size_t out_bytes = static_cast<size_t>(p->ndm) * nsamp * 4;
  void* din = nullptr;
  void* dout = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int st = DEDISP_OK;
  int best = -1;
  double best_t = 1e30;
  do {
    if ((e = hipMalloc(&din, in_bytes)) != hipSuccess) break;
    if ((e = hipMalloc(&dout, out_bytes)) != hipSuccess) break;
    if ((e = hipMemset(din, 0, in_bytes)) != hipSuccess) break;
    if ((e = hipStreamCreate(&s)) != hipSuccess) break;
    if ((e = hipEventCreate(&e0)) != hipSuccess) break;
    if ((e = hipEventCreate(&e1)) != hipSuccess) break;
    for (int v = 1; v < dedisp::variant_count() && st == DEDISP_OK; ++v) {
      if (!dedisp::variant_fits(p, v)) continue;
      st = dedisp::launch(p, v, din, dout, nsamp, s);  // warm-up
      if (st != DEDISP_OK) break;
      double tmin = 1e30;
      for (int rep = 0; rep < 3 && st == DEDISP_OK; ++rep) {
        if ((e = hipEventRecord(e0, s)) != hipSuccess) break;
        st = dedisp::launch(p, v, din, dout, nsamp, s);
        if ((e = hipEventRecord(e1, s)) != hipSuccess) break;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
        tmin = std::min(tmin, static_cast<double>(ms));
      }
      if (e != hipSuccess) break;
      if (trace) {
        const dedisp::TileShape sh = dedisp::variant_shape(v);
        std::fprintf(stderr, "[dedisp] autotune variant %d (%d trials x %d samples, %d threads): %.4f ms\n", v,
                     sh.dms(), sh.samples(), sh.threads(), tmin);
      }
      if (tmin < best_t) {
        best_t = tmin;
        best = v;
      }
    }
  } while (false);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (din) (void)hipFree(din);
  if (dout) (void)hipFree(dout);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  if (st != DEDISP_OK) return st;
  if (best < 0) {  // nothing tiled fits: the direct kernel
    best = 0;
    best_t = 0.0;
  }
  p->variant.store(best);
  {
    std::lock_guard<std::mutex> g(g_mu);
    g_cache[key] = {best, best_t};
    append_file(key, best, best_t);
  }
  *best_variant = best;
  if (best_ms) *best_ms = best_t;
  return DEDISP_OK;
}

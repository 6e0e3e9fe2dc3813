// Batched launch: many beams of any shape in one persistent kernel, replayed
// from a HIP graph.
//
// Work items are (beam, trial tile, time tile) of one tile variant; beams are
// ordered by the cost of one of their items (channels, then trials), so the
// item list runs longest items first and resident workgroups that pull items
// from one atomic counter finish close together.  The graph holds a counter
// reset kernel and the persistent kernel; the per-beam argument table the
// kernel reads (pointers included) lives in device memory and is refreshed
// with a stream-ordered copy when the caller's pointers change, so the graph
// itself never needs to be rebuilt for new buffers.  Beams that the chosen
// variant cannot stage (delay spread too wide) run as their own launches,
// captured in the same graph.  8-bit and half inputs are widened into
// buffers the batch owns (one per such beam) by one kernel at the head of the
// graph, which reads its jobs from a device table refreshed like the argument
// table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "dedisp_internal.h"

struct dedisp_batch_s {
  std::vector<dedisp_plan> plans;
  std::vector<int64_t> nsamps;
  int nbeams = 0;
  int variant = -1;              // persistent-kernel tile variant
  std::vector<int> order;        // beams in the persistent kernel, longest items first
  std::vector<int> solo;         // beams launched on their own
  std::vector<int> solo_variant;
  int device = -1;
  // device state
  dedisp::TiledArgs* d_args = nullptr;
  int64_t* d_item_end = nullptr;
  int* d_dtype = nullptr;
  unsigned long long* d_counter = nullptr;
  dedisp::WidenJob* d_jobs = nullptr;
  int njobs = 0;
  std::vector<void*> ws;                // widened input per beam (8-bit and half beams)
  dedisp::TiledArgs* h_args = nullptr;  // pinned staging, two halves
  dedisp::WidenJob* h_jobs = nullptr;   // pinned staging, two halves
  int h_half = 0;
  hipEvent_t h_done[2] = {nullptr, nullptr};
  hipStream_t capture = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> ins;
  std::vector<void*> outs;
  int64_t n_items = 0;
  int grid = 0;
  size_t lds = 0;
  int threads = 0;
};

namespace {

int free_graph(dedisp_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  return DEDISP_OK;
}

int free_device(dedisp_batch b) {
  free_graph(b);
  if (b->d_args) (void)hipFree(b->d_args);
  if (b->d_item_end) (void)hipFree(b->d_item_end);
  if (b->d_dtype) (void)hipFree(b->d_dtype);
  if (b->d_counter) (void)hipFree(b->d_counter);
  if (b->h_args) (void)hipHostFree(b->h_args);
  if (b->d_jobs) (void)hipFree(b->d_jobs);
  if (b->h_jobs) (void)hipHostFree(b->h_jobs);
  for (void* w : b->ws)
    if (w) (void)hipFree(w);
  b->ws.clear();
  b->d_jobs = nullptr;
  b->h_jobs = nullptr;
  b->njobs = 0;
  for (auto& e : b->h_done)
    if (e) (void)hipEventDestroy(e);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  b->d_args = nullptr;
  b->d_item_end = nullptr;
  b->d_dtype = nullptr;
  b->d_counter = nullptr;
  b->h_args = nullptr;
  b->h_done[0] = b->h_done[1] = nullptr;
  b->capture = nullptr;
  b->device = -1;
  return DEDISP_OK;
}

// Split the beams between the persistent kernel (variant v) and solo launches.
void assign(dedisp_batch b, int v) {
  b->variant = v;
  b->order.clear();
  b->solo.clear();
  b->solo_variant.clear();
  for (int i = 0; i < b->nbeams; ++i) {
    if (v >= 1 && dedisp::variant_fits(b->plans[i], v)) {
      b->order.push_back(i);
    } else {
      b->solo.push_back(i);
      b->solo_variant.push_back(dedisp::default_variant(b->plans[i]));
    }
  }
  std::stable_sort(b->order.begin(), b->order.end(), [b](int x, int y) {
    const dedisp_plan px = b->plans[x], py = b->plans[y];
    if (px->nchans != py->nchans) return px->nchans > py->nchans;
    return px->ndm > py->ndm;
  });
}

// Variant that fits the most work of the batch (ties: library order).
int pick_variant(dedisp_batch b) {
  int best = -1;
  double best_work = -1.0;
  for (int v = 1; v < dedisp::variant_count(); ++v) {
    double work = 0.0;
    for (int i = 0; i < b->nbeams; ++i)
      if (dedisp::variant_fits(b->plans[i], v))
        work += static_cast<double>(b->plans[i]->nchans) * b->plans[i]->ndm * b->nsamps[i];
    if (work > best_work * (1.0 + 1e-12)) {
      best_work = work;
      best = v;
    }
  }
  return best_work > 0.0 ? best : -1;
}

int64_t total_samples(dedisp_batch b, int i) {
  return (b->nsamps[i] + b->plans[i]->max_shift) * b->plans[i]->nchans;
}

// Fill the argument and widening tables for the current pointers into the
// next pinned half.
int build_args(dedisp_batch b, const void* const* ins, void* const* outs, dedisp::TiledArgs** host,
               std::vector<int64_t>* ends, std::vector<int>* dtypes) {
  dedisp::TiledArgs* h = b->h_args + b->h_half * b->nbeams;
  dedisp::WidenJob* hj = b->h_jobs + b->h_half * b->nbeams;
  int64_t acc = 0;
  size_t lds = 0;
  b->njobs = 0;
  for (size_t k = 0; k < b->order.size(); ++k) {
    const int i = b->order[k];
    size_t l = 0;
    int64_t nblocks = 0;
    int threads = 0;
    const void* src = ins[i];
    if (b->ws[i] != nullptr) {
      const int64_t n = total_samples(b, i);
      hj[b->njobs++] = dedisp::WidenJob{ins[i], b->ws[i], n, dedisp::widened_samples(n), b->plans[i]->dtype};
      src = b->ws[i];
    }
    const int st = dedisp::tiled_args(b->plans[i], b->variant, src, outs[i], b->nsamps[i], &h[k], &l, &nblocks,
                                      &threads);
    if (st != DEDISP_OK) return st;
    lds = std::max(lds, l);
    b->threads = threads;
    const dedisp::TiledArgs& a = h[k];
    const int64_t items = static_cast<int64_t>(a.n_dm_groups) * ((a.n_t_tiles + a.gt - 1) / a.gt) * a.gd * a.gt;
    acc += items;
    if (ends) ends->push_back(acc);
    if (dtypes) dtypes->push_back(b->plans[i]->dtype);
  }
  b->n_items = acc;
  b->lds = lds;
  *host = h;
  return DEDISP_OK;
}

int setup_device(dedisp_batch b, int dev, const void* const* ins, void* const* outs) {
  hipError_t e;
  const size_t n = std::max<size_t>(1, b->order.size());
  if ((e = hipMalloc(&b->d_args, n * sizeof(dedisp::TiledArgs))) != hipSuccess) return DEDISP_HIP_STATUS(e);
  if ((e = hipMalloc(&b->d_item_end, n * sizeof(int64_t))) != hipSuccess) return DEDISP_HIP_STATUS(e);
  if ((e = hipMalloc(&b->d_dtype, n * sizeof(int))) != hipSuccess) return DEDISP_HIP_STATUS(e);
  if ((e = hipMalloc(&b->d_counter, sizeof(unsigned long long))) != hipSuccess) return DEDISP_HIP_STATUS(e);
  if ((e = hipHostMalloc(&b->h_args, 2 * std::max(1, b->nbeams) * sizeof(dedisp::TiledArgs))) != hipSuccess)
    return DEDISP_HIP_STATUS(e);
  if ((e = hipHostMalloc(&b->h_jobs, 2 * std::max(1, b->nbeams) * sizeof(dedisp::WidenJob))) != hipSuccess)
    return DEDISP_HIP_STATUS(e);
  if ((e = hipMalloc(&b->d_jobs, std::max(1, b->nbeams) * sizeof(dedisp::WidenJob))) != hipSuccess)
    return DEDISP_HIP_STATUS(e);
  b->ws.assign(b->nbeams, nullptr);
  for (int i = 0; i < b->nbeams; ++i) {
    const int dt = b->plans[i]->dtype;
    if (dt == DEDISP_F32) continue;
    const size_t bytes = static_cast<size_t>(dedisp::widened_samples(total_samples(b, i))) * dedisp::staged_size(dt);
    if ((e = hipMalloc(&b->ws[i], bytes)) != hipSuccess) return DEDISP_HIP_STATUS(e);
  }
  for (auto& ev : b->h_done)
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return DEDISP_HIP_STATUS(e);
  if ((e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking)) != hipSuccess) return DEDISP_HIP_STATUS(e);
  b->device = dev;
  if (b->order.empty()) return DEDISP_OK;
  dedisp::TiledArgs* h = nullptr;
  std::vector<int64_t> ends;
  std::vector<int> dtypes;
  int st = build_args(b, ins, outs, &h, &ends, &dtypes);
  if (st != DEDISP_OK) return st;
  if ((e = hipMemcpy(b->d_args, h, b->order.size() * sizeof(dedisp::TiledArgs), hipMemcpyHostToDevice)) != hipSuccess)
    return DEDISP_HIP_STATUS(e);
  if ((e = hipMemcpy(b->d_item_end, ends.data(), ends.size() * sizeof(int64_t), hipMemcpyHostToDevice)) != hipSuccess)
    return DEDISP_HIP_STATUS(e);
  if ((e = hipMemcpy(b->d_dtype, dtypes.data(), dtypes.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
    return DEDISP_HIP_STATUS(e);
  if (b->njobs > 0 &&
      (e = hipMemcpy(b->d_jobs, b->h_jobs + b->h_half * b->nbeams, b->njobs * sizeof(dedisp::WidenJob),
                     hipMemcpyHostToDevice)) != hipSuccess)
    return DEDISP_HIP_STATUS(e);
  return DEDISP_OK;
}

int build_graph(dedisp_batch b, const void* const* ins, void* const* outs) {
  hipError_t e;
  const void* fn = nullptr;
  if (!b->order.empty()) {
    fn = dedisp::batch_kernel(b->variant);
    if (fn == nullptr) return DEDISP_ERR_INTERNAL;
    if (b->lds > 64 * 1024) {
      const int st = dedisp::allow_large_lds(fn);
      if (st != DEDISP_OK) return st;
    }
    int per_cu = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, b->threads, b->lds)) != hipSuccess)
      return DEDISP_HIP_STATUS(e);
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, b->device)) != hipSuccess) return DEDISP_HIP_STATUS(e);
    const int64_t resident = static_cast<int64_t>(std::max(1, per_cu)) * prop.multiProcessorCount;
    b->grid = static_cast<int>(std::min<int64_t>(resident, std::max<int64_t>(1, b->n_items)));
  }
  // what solo launches need must exist before capture (allocations, attributes)
  for (size_t k = 0; k < b->solo.size(); ++k) {
    const int st = dedisp::prepare(b->plans[b->solo[k]], b->solo_variant[k], b->nsamps[b->solo[k]]);
    if (st != DEDISP_OK) return st;
  }
  if ((e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed)) != hipSuccess)
    return DEDISP_HIP_STATUS(e);
  int st = DEDISP_OK;
  if (!b->order.empty()) {
    void* rargs[] = {&b->d_counter};
    e = hipLaunchKernel(dedisp::reset_kernel(), dim3(1), dim3(1), rargs, 0, b->capture);
    if (e == hipSuccess && b->njobs > 0) {
      st = dedisp::widen_jobs(b->d_jobs, b->njobs, b->capture);
      if (st != DEDISP_OK) e = hipErrorUnknown;
    }
    if (e == hipSuccess) {
      dedisp::BatchArgs ba;
      ba.beams = b->d_args;
      ba.item_end = b->d_item_end;
      ba.dtype = b->d_dtype;
      ba.nbeams = static_cast<int>(b->order.size());
      ba.n_items = b->n_items;
      ba.counter = b->d_counter;
      void* kargs[] = {&ba};
      e = hipLaunchKernel(fn, dim3(b->grid), dim3(b->threads), kargs, b->lds, b->capture);
    }
    if (e != hipSuccess && st == DEDISP_OK) st = DEDISP_HIP_STATUS(e);
  }
  for (size_t k = 0; k < b->solo.size() && st == DEDISP_OK; ++k) {
    const int i = b->solo[k];
    st = dedisp::launch(b->plans[i], b->solo_variant[k], ins[i], outs[i], b->nsamps[i], b->capture, b->ws[i]);
  }
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->capture, &g);
  if (st != DEDISP_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  b->graph = g;
  if ((e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0)) != hipSuccess) return DEDISP_HIP_STATUS(e);
  return DEDISP_OK;
}

}  // namespace

extern "C" int dedisp_batch_create(const dedisp_plan* plans, const int64_t* nsamps, int nbeams,
                                   dedisp_batch* out) {
  if (plans == nullptr || nsamps == nullptr || out == nullptr || nbeams < 1) return DEDISP_ERR_INVALID_ARG;
  for (int i = 0; i < nbeams; ++i) {
    if (plans[i] == nullptr || nsamps[i] < 1) return DEDISP_ERR_INVALID_ARG;
    if (nsamps[i] > static_cast<int64_t>(INT32_MAX) - plans[i]->max_shift) return DEDISP_ERR_INVALID_ARG;
  }
  dedisp_batch b = new (std::nothrow) dedisp_batch_s();
  if (b == nullptr) return DEDISP_ERR_OUT_OF_MEMORY;
  b->plans.assign(plans, plans + nbeams);
  b->nsamps.assign(nsamps, nsamps + nbeams);
  b->nbeams = nbeams;
  assign(b, pick_variant(b));
  *out = b;
  return DEDISP_OK;
}

extern "C" int dedisp_batch_destroy(dedisp_batch b) {
  if (b == nullptr) return DEDISP_OK;
  int dev0 = -1;
  if (b->device >= 0 && hipGetDevice(&dev0) == hipSuccess) (void)hipSetDevice(b->device);
  free_device(b);
  if (dev0 >= 0) (void)hipSetDevice(dev0);
  delete b;
  return DEDISP_OK;
}

extern "C" int dedisp_batch_info(dedisp_batch b, int64_t* work_items, int* workgroups) {
  if (b == nullptr) return DEDISP_ERR_INVALID_ARG;
  if (work_items) *work_items = b->n_items;
  if (workgroups) *workgroups = b->grid;
  return DEDISP_OK;
}

static int check_ptrs(dedisp_batch b, const void* const* ins, void* const* outs) {
  if (ins == nullptr || outs == nullptr) return DEDISP_ERR_INVALID_ARG;
  for (int i = 0; i < b->nbeams; ++i) {
    if (ins[i] == nullptr || outs[i] == nullptr) return DEDISP_ERR_INVALID_ARG;
    if ((reinterpret_cast<uintptr_t>(ins[i]) & 15) != 0 || (reinterpret_cast<uintptr_t>(outs[i]) & 3) != 0)
      return DEDISP_ERR_INVALID_ARG;
  }
  return DEDISP_OK;
}

extern "C" int dedisp_batch_execute(dedisp_batch b, const void* const* ins, void* const* outs, void* stream_v) {
  if (b == nullptr) return DEDISP_ERR_INVALID_ARG;
  int st = check_ptrs(b, ins, outs);
  if (st != DEDISP_OK) return st;
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  if (b->device != dev) {
    free_device(b);
    st = setup_device(b, dev, ins, outs);
    if (st != DEDISP_OK) {
      free_device(b);
      return st;
    }
    b->ins.assign(ins, ins + b->nbeams);
    b->outs.assign(outs, outs + b->nbeams);
  }
  bool changed = false;
  for (int i = 0; i < b->nbeams; ++i) changed |= (b->ins[i] != ins[i] || b->outs[i] != outs[i]);
  if (changed) {
    bool solo_changed = false;
    for (int i : b->solo) solo_changed |= (b->ins[i] != ins[i] || b->outs[i] != outs[i]);
    if (!b->order.empty()) {
      // the half we are about to fill was last read by the copy two updates ago
      b->h_half ^= 1;
      if ((e = hipEventSynchronize(b->h_done[b->h_half])) != hipSuccess) return DEDISP_HIP_STATUS(e);
      dedisp::TiledArgs* h = nullptr;
      st = build_args(b, ins, outs, &h, nullptr, nullptr);
      if (st != DEDISP_OK) return st;
      e = hipMemcpyAsync(b->d_args, h, b->order.size() * sizeof(dedisp::TiledArgs), hipMemcpyHostToDevice, stream);
      if (e == hipSuccess && b->njobs > 0)
        e = hipMemcpyAsync(b->d_jobs, b->h_jobs + b->h_half * b->nbeams, b->njobs * sizeof(dedisp::WidenJob),
                           hipMemcpyHostToDevice, stream);
      if (e == hipSuccess) e = hipEventRecord(b->h_done[b->h_half], stream);
      if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
    }
    b->ins.assign(ins, ins + b->nbeams);
    b->outs.assign(outs, outs + b->nbeams);
    if (solo_changed) free_graph(b);
  }
  if (b->exec == nullptr) {
    st = build_graph(b, ins, outs);
    if (st != DEDISP_OK) {
      free_graph(b);
      return st;
    }
  }
  return DEDISP_HIP_STATUS(hipGraphLaunch(b->exec, stream));
}

extern "C" int dedisp_batch_autotune(dedisp_batch b, const void* const* ins, void* const* outs, void* stream_v,
                                     int* best_variant, double* best_ms) {
  if (b == nullptr || best_variant == nullptr) return DEDISP_ERR_INVALID_ARG;
  int st = check_ptrs(b, ins, outs);
  if (st != DEDISP_OK) return st;
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return DEDISP_HIP_STATUS(e);
  }
  int best = -1;
  double best_t = 1e30;
  for (int v = 1; v < dedisp::variant_count() && st == DEDISP_OK; ++v) {
    bool any = false;
    for (int i = 0; i < b->nbeams; ++i) any |= dedisp::variant_fits(b->plans[i], v);
    if (!any) continue;
    (void)hipStreamSynchronize(stream);
    free_device(b);
    assign(b, v);
    st = dedisp_batch_execute(b, ins, outs, stream);  // builds the graph, warms up
    if (st != DEDISP_OK) break;
    double tmin = 1e30;
    for (int rep = 0; rep < 2; ++rep) {
      if ((e = hipEventRecord(e0, stream)) != hipSuccess) break;
      if ((st = dedisp_batch_execute(b, ins, outs, stream)) != DEDISP_OK) break;
      if ((e = hipEventRecord(e1, stream)) != hipSuccess) break;
      if ((e = hipEventSynchronize(e1)) != hipSuccess) break;
      float ms = 0.f;
      if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
      tmin = std::min(tmin, static_cast<double>(ms));
    }
    if (e != hipSuccess) st = DEDISP_HIP_STATUS(e);
    if (st == DEDISP_OK && tmin < best_t) {
      best_t = tmin;
      best = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != DEDISP_OK) return st;
  (void)hipStreamSynchronize(stream);
  free_device(b);
  assign(b, best);
  *best_variant = best;
  if (best_ms) *best_ms = best_t;
  return DEDISP_OK;
}

extern "C" int dedisp_batch_get_variant(dedisp_batch b, int* variant) {
  if (b == nullptr || variant == nullptr) return DEDISP_ERR_INVALID_ARG;
  *variant = b->variant;
  return DEDISP_OK;
}

extern "C" int dedisp_batch_set_variant(dedisp_batch b, int variant) {
  if (b == nullptr || variant < 1 || variant >= dedisp::variant_count()) return DEDISP_ERR_INVALID_ARG;
  int dev0 = -1;
  if (b->device >= 0 && hipGetDevice(&dev0) == hipSuccess) (void)hipSetDevice(b->device);
  if (b->device >= 0) (void)hipDeviceSynchronize();
  free_device(b);
  if (dev0 >= 0) (void)hipSetDevice(dev0);
  assign(b, variant);
  return DEDISP_OK;
}

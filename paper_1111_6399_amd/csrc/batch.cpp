// Batched launch: many beams of any shape in persistent kernels, replayed
// from a HIP graph.
//
// The beams that run persistently form groups of one tile variant, one
// staging kind (8-bit beams are staged as 16-bit pairs, half beams as halves,
// float beams as float) and one LDS occupancy (a launch sizes its slots for its widest
// window, so a beam with a wide delay spread would hold every other beam of
// its kernel to fewer workgroups per CU), one persistent kernel per group,
// each compiled for its path only.  Work items are (beam, trial tile, time tile); inside a group beams
// are ordered by the cost of one of their items (channels, then trials), so
// the item list runs longest items first and resident workgroups that pull
// items from the group's atomic counter finish close together.  The graph
// holds, per group, a counter reset kernel and the persistent kernel; the
// per-beam argument tables the kernels read (pointers included) live in
// device memory and are refreshed with stream-ordered copies when the
// caller's pointers change, so the graph itself never needs to be rebuilt for
// new buffers.  Beams that no persistent group takes run as their own
// launches, captured in the same graph: with one variant for the whole batch,
// those it cannot stage (delay spread too wide); in the split that follows
// each plan's own variant, the beams whose plan runs the direct kernel.
// 8-bit inputs are widened into buffers the batch owns (one per such beam) by
// one kernel at the head of the graph, which reads its jobs from a device
// table refreshed like the argument tables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <numeric>
#include <tuple>
#include <utility>
#include <vector>

#include "dedisp_internal.h"

namespace {

constexpr int kBranches = 4;

struct BatchGroup {
  int variant = -1;
  int kind = 0;                         // staging kind of its beams (dedisp::StageKind)
  std::vector<int> order;               // beams, longest items first
  int off = 0;                          // first argument slot of the group in each pinned half
  double work = 0.0;                    // adds of its beams
  dedisp::TiledArgs* d_args = nullptr;  // [order.size()]
  int64_t* d_item_end = nullptr;        // [order.size()]
  unsigned long long* d_counter = nullptr;  // [kBatchCounters]
  int64_t n_items = 0;
  int grid = 0;
  size_t lds = 0;
  int threads = 0;
};

}  // namespace

struct dedisp_batch_s {
  std::vector<dedisp_plan> plans;
  std::vector<int64_t> nsamps;
  int nbeams = 0;
  int variant = -1;  // variant of the group that carries the most work
  // how the graph spreads its launches over the branches: 0 each on the
  // branch with the least work so far, 1 all on one branch in order (the
  // plain sequence, without its launch overheads), 2 one branch per staging
  // kind (float and 16-bit beams side by side)
  int layout = 0;
  std::vector<BatchGroup> groups;
  std::vector<int> solo;  // beams launched on their own
  std::vector<int> solo_variant;
  int device = -1;
  // device state
  dedisp::WidenJob* d_jobs = nullptr;
  int njobs = 0;
  std::vector<void*> ws;                // widened input per beam (8-bit beams)
  dedisp::TiledArgs* h_args = nullptr;  // pinned staging, two halves of nbeams slots
  dedisp::WidenJob* h_jobs = nullptr;   // pinned staging, two halves
  int h_half = 0;
  hipEvent_t h_done[2] = {nullptr, nullptr};
  hipStream_t capture = nullptr;
  // graph branches: the group kernels and solo launches are captured on
  // these, forked from and joined back to the capture stream, so that the
  // graph runs them concurrently and one kernel's tail overlaps the others
  hipStream_t branch[kBranches] = {};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[kBranches] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> ins;
  std::vector<void*> outs;
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
  for (BatchGroup& g : b->groups) {
    if (g.d_args) (void)hipFree(g.d_args);
    if (g.d_item_end) (void)hipFree(g.d_item_end);
    if (g.d_counter) (void)hipFree(g.d_counter);
    g.d_args = nullptr;
    g.d_item_end = nullptr;
    g.d_counter = nullptr;
    g.n_items = 0;
    g.grid = 0;
  }
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
  for (auto& x : b->branch)
    if (x) (void)hipStreamDestroy(x);
  for (auto& x : b->join_ev)
    if (x) (void)hipEventDestroy(x);
  if (b->fork_ev) (void)hipEventDestroy(b->fork_ev);
  for (auto& x : b->branch) x = nullptr;
  for (auto& x : b->join_ev) x = nullptr;
  b->fork_ev = nullptr;
  b->h_args = nullptr;
  b->h_done[0] = b->h_done[1] = nullptr;
  b->capture = nullptr;
  b->device = -1;
  return DEDISP_OK;
}

double beam_work(dedisp_batch b, int i) {
  return static_cast<double>(b->plans[i]->nchans) * b->plans[i]->ndm * b->nsamps[i];
}

// Form the groups: beam i runs persistently with variant tiled[i] >= 1 (in
// the group of that variant and its staging kind), or on its own with
// variant solo_v[i] when tiled[i] < 1.
void form_groups(dedisp_batch b, const std::vector<int>& tiled, const std::vector<int>& solo_v) {
  b->groups.clear();
  b->solo.clear();
  b->solo_variant.clear();
  std::map<std::tuple<int, int, int>, size_t> index;
  for (int i = 0; i < b->nbeams; ++i) {
    if (tiled[i] < 1) {
      b->solo.push_back(i);
      b->solo_variant.push_back(solo_v[i]);
      continue;
    }
    const auto key = std::make_tuple(tiled[i], dedisp::stage_kind(b->plans[i]->dtype),
                                     dedisp::tiled_per_cu(b->plans[i], tiled[i]));
    auto it = index.find(key);
    if (it == index.end()) {
      it = index.emplace(key, b->groups.size()).first;
      BatchGroup g;
      g.variant = std::get<0>(key);
      g.kind = std::get<1>(key);
      b->groups.push_back(g);
    }
    BatchGroup& g = b->groups[it->second];
    g.order.push_back(i);
    g.work += beam_work(b, i);
  }
  int off = 0;
  double most = -1.0;
  b->variant = -1;
  for (BatchGroup& g : b->groups) {
    std::stable_sort(g.order.begin(), g.order.end(), [b](int x, int y) {
      const dedisp_plan px = b->plans[x], py = b->plans[y];
      if (px->nchans != py->nchans) return px->nchans > py->nchans;
      return px->ndm > py->ndm;
    });
    g.off = off;
    off += static_cast<int>(g.order.size());
    if (g.work > most) {
      most = g.work;
      b->variant = g.variant;
    }
  }
}

// One variant for the 8-bit beams (v8) and one for the float and half beams
// (vf): every beam its variant fits runs persistently with it, the others on
// their own with their library default.
void assign_kinds(dedisp_batch b, int v8, int vf) {
  std::vector<int> tiled(b->nbeams, -1), solo_v(b->nbeams, 0);
  for (int i = 0; i < b->nbeams; ++i) {
    const int v = b->plans[i]->dtype == DEDISP_U8 ? v8 : vf;
    if (v >= 1 && dedisp::variant_fits(b->plans[i], v))
      tiled[i] = v;
    else
      solo_v[i] = dedisp::default_variant(b->plans[i]);
  }
  form_groups(b, tiled, solo_v);
}

// One variant for the whole batch.
void assign(dedisp_batch b, int v) { assign_kinds(b, v, v); }

// Variant beam i runs with on its own: its plan's (set or tuned) if that
// still fits, else the library default (0: the direct kernel).
int own_variant(dedisp_batch b, int i) {
  const int v = b->plans[i]->variant.load();
  if (v == 0 || (v >= 1 && dedisp::variant_fits(b->plans[i], v))) return v;
  return dedisp::default_variant(b->plans[i]);
}

// Split by each plan's own variant: tiled beams run persistently in the
// group of their variant and staging kind, direct ones on their own.
// Returns false if that is the same split as assign() with one variant.
bool assign_own(dedisp_batch b) {
  std::vector<int> tiled(b->nbeams, -1), solo_v(b->nbeams, 0);
  bool same = true;
  for (int i = 0; i < b->nbeams; ++i) {
    const int v = own_variant(b, i);
    if (v >= 1)
      tiled[i] = v;
    else
      solo_v[i] = v;
    same = same && v == own_variant(b, 0);
  }
  form_groups(b, tiled, solo_v);
  return !same;
}

// Every beam on its own with its plan's variant, the launches captured in the
// graph (no persistent kernel).
void assign_solo(dedisp_batch b) {
  std::vector<int> tiled(b->nbeams, -1), solo_v(b->nbeams, 0);
  for (int i = 0; i < b->nbeams; ++i) solo_v[i] = own_variant(b, i);
  form_groups(b, tiled, solo_v);
}

// Variant that fits the most work of the batch (ties: library order).
int pick_variant(dedisp_batch b) {
  int best = -1;
  double best_work = -1.0;
  for (int v = 1; v < dedisp::variant_count(); ++v) {
    double work = 0.0;
    for (int i = 0; i < b->nbeams; ++i)
      if (dedisp::variant_fits(b->plans[i], v)) work += beam_work(b, i);
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
// current pinned half (ends: per group, the prefix sums of work items).
int build_args(dedisp_batch b, const void* const* ins, void* const* outs,
               std::vector<std::vector<int64_t>>* ends) {
  dedisp::TiledArgs* h = b->h_args + b->h_half * b->nbeams;
  dedisp::WidenJob* hj = b->h_jobs + b->h_half * b->nbeams;
  b->njobs = 0;
  if (ends) ends->assign(b->groups.size(), {});
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    BatchGroup& g = b->groups[gi];
    int64_t acc = 0;
    size_t lds = 0;
    for (size_t k = 0; k < g.order.size(); ++k) {
      const int i = g.order[k];
      size_t l = 0;
      int64_t nblocks = 0;
      int threads = 0;
      const void* src = ins[i];
      if (b->ws[i] != nullptr) {
        const int64_t n = total_samples(b, i);
        hj[b->njobs++] = dedisp::WidenJob{ins[i], b->ws[i], n, dedisp::widened_samples(n), b->plans[i]->dtype};
        src = b->ws[i];
      }
      dedisp::TiledArgs& a = h[g.off + k];
      const int st = dedisp::tiled_args(b->plans[i], g.variant, src, outs[i], b->nsamps[i], &a, &l, &nblocks,
                                        &threads);
      if (st != DEDISP_OK) return st;
      lds = std::max(lds, l);
      g.threads = threads;
      const int64_t items = static_cast<int64_t>(a.n_dm_groups) * ((a.n_t_tiles + a.gt - 1) / a.gt) * a.gd * a.gt;
      acc += items;
      if (ends) (*ends)[gi].push_back(acc);
    }
    g.n_items = acc;
    g.lds = lds;
  }
  return DEDISP_OK;
}

int setup_device(dedisp_batch b, int dev, const void* const* ins, void* const* outs) {
  hipError_t e;
  const int nb = std::max(1, b->nbeams);
  if ((e = hipHostMalloc(&b->h_args, 2 * nb * sizeof(dedisp::TiledArgs))) != hipSuccess) return DEDISP_HIP_STATUS(e);
  if ((e = hipHostMalloc(&b->h_jobs, 2 * nb * sizeof(dedisp::WidenJob))) != hipSuccess) return DEDISP_HIP_STATUS(e);
  if ((e = hipMalloc(&b->d_jobs, nb * sizeof(dedisp::WidenJob))) != hipSuccess) return DEDISP_HIP_STATUS(e);
  for (BatchGroup& g : b->groups) {
    const size_t n = g.order.size();
    if ((e = hipMalloc(&g.d_args, n * sizeof(dedisp::TiledArgs))) != hipSuccess) return DEDISP_HIP_STATUS(e);
    if ((e = hipMalloc(&g.d_item_end, n * sizeof(int64_t))) != hipSuccess) return DEDISP_HIP_STATUS(e);
    if ((e = hipMalloc(&g.d_counter, dedisp::kBatchCounters * sizeof(unsigned long long))) != hipSuccess)
      return DEDISP_HIP_STATUS(e);
  }
  b->ws.assign(b->nbeams, nullptr);
  for (int i = 0; i < b->nbeams; ++i) {
    const int dt = b->plans[i]->dtype;
    if (dt != DEDISP_U8) continue;
    const size_t bytes = static_cast<size_t>(dedisp::widened_samples(total_samples(b, i))) * dedisp::staged_size(dt);
    if ((e = hipMalloc(&b->ws[i], bytes)) != hipSuccess) return DEDISP_HIP_STATUS(e);
  }
  for (auto& ev : b->h_done)
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return DEDISP_HIP_STATUS(e);
  if ((e = hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking)) != hipSuccess) return DEDISP_HIP_STATUS(e);
  for (auto& x : b->branch)
    if ((e = hipStreamCreateWithFlags(&x, hipStreamNonBlocking)) != hipSuccess) return DEDISP_HIP_STATUS(e);
  for (auto& x : b->join_ev)
    if ((e = hipEventCreateWithFlags(&x, hipEventDisableTiming)) != hipSuccess) return DEDISP_HIP_STATUS(e);
  if ((e = hipEventCreateWithFlags(&b->fork_ev, hipEventDisableTiming)) != hipSuccess) return DEDISP_HIP_STATUS(e);
  b->device = dev;
  if (b->groups.empty()) return DEDISP_OK;
  std::vector<std::vector<int64_t>> ends;
  int st = build_args(b, ins, outs, &ends);
  if (st != DEDISP_OK) return st;
  const dedisp::TiledArgs* h = b->h_args + b->h_half * b->nbeams;
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    const BatchGroup& g = b->groups[gi];
    if ((e = hipMemcpy(g.d_args, h + g.off, g.order.size() * sizeof(dedisp::TiledArgs), hipMemcpyHostToDevice)) !=
        hipSuccess)
      return DEDISP_HIP_STATUS(e);
    if ((e = hipMemcpy(g.d_item_end, ends[gi].data(), ends[gi].size() * sizeof(int64_t), hipMemcpyHostToDevice)) !=
        hipSuccess)
      return DEDISP_HIP_STATUS(e);
  }
  if (b->njobs > 0 &&
      (e = hipMemcpy(b->d_jobs, b->h_jobs + b->h_half * b->nbeams, b->njobs * sizeof(dedisp::WidenJob),
                     hipMemcpyHostToDevice)) != hipSuccess)
    return DEDISP_HIP_STATUS(e);
  return DEDISP_OK;
}

int build_graph(dedisp_batch b, const void* const* ins, void* const* outs) {
  hipError_t e;
  std::vector<const void*> fns;
  if (!b->groups.empty()) {
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, b->device)) != hipSuccess) return DEDISP_HIP_STATUS(e);
    for (BatchGroup& g : b->groups) {
      const void* fn = dedisp::batch_kernel(g.variant, g.kind);
      if (fn == nullptr) return DEDISP_ERR_INTERNAL;
      if (g.lds > 64 * 1024) {
        const int st = dedisp::allow_large_lds(fn);
        if (st != DEDISP_OK) return st;
      }
      int per_cu = 0;
      if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, g.threads, g.lds)) != hipSuccess)
        return DEDISP_HIP_STATUS(e);
      const int64_t resident = static_cast<int64_t>(std::max(1, per_cu)) * prop.multiProcessorCount;
      g.grid = static_cast<int>(std::min<int64_t>(resident, std::max<int64_t>(1, g.n_items)));
      fns.push_back(fn);
    }
  }
  // what solo launches need must exist before capture (allocations, attributes)
  for (size_t k = 0; k < b->solo.size(); ++k) {
    const int st = dedisp::prepare(b->plans[b->solo[k]], b->solo_variant[k], b->nsamps[b->solo[k]]);
    if (st != DEDISP_OK) return st;
  }
  if ((e = hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed)) != hipSuccess)
    return DEDISP_HIP_STATUS(e);
  int st = DEDISP_OK;
  if (b->njobs > 0) st = dedisp::widen_jobs(b->d_jobs, b->njobs, b->capture);
  // fork: branch k waits for the widening, then runs its share
  if (st == DEDISP_OK) st = DEDISP_HIP_STATUS(hipEventRecord(b->fork_ev, b->capture));
  for (int k = 0; k < kBranches && st == DEDISP_OK; ++k)
    st = DEDISP_HIP_STATUS(hipStreamWaitEvent(b->branch[k], b->fork_ev, 0));
  // the groups in order of their work (largest first), each on the branch
  // with the least work so far; then the solo launches the same way
  double load[kBranches] = {};
  auto pick = [&load, b](int kind) {
    if (b->layout == 1) return 0;
    if (b->layout == 2) return kind == dedisp::kStageFloat ? 0 : 1;
    int k = 0;
    for (int j = 1; j < kBranches; ++j)
      if (load[j] < load[k]) k = j;
    return k;
  };
  std::vector<size_t> gorder(b->groups.size());
  std::iota(gorder.begin(), gorder.end(), size_t{0});
  std::stable_sort(gorder.begin(), gorder.end(),
                   [b](size_t x, size_t y) { return b->groups[x].work > b->groups[y].work; });
  for (size_t n = 0; n < gorder.size() && st == DEDISP_OK; ++n) {
    const size_t gi = gorder[n];
    BatchGroup& g = b->groups[gi];
    const int k = pick(g.kind);
    load[k] += g.work;
    hipStream_t bs = b->branch[k];
    void* rargs[] = {&g.d_counter};
    e = hipLaunchKernel(dedisp::reset_kernel(), dim3(1), dim3(dedisp::reset_kernel_threads()), rargs, 0, bs);
    if (e == hipSuccess) {
      dedisp::BatchArgs ba;
      ba.beams = g.d_args;
      ba.item_end = g.d_item_end;
      ba.nbeams = static_cast<int>(g.order.size());
      ba.n_items = g.n_items;
      ba.counter = g.d_counter;
      void* kargs[] = {&ba};
      e = hipLaunchKernel(fns[gi], dim3(g.grid), dim3(g.threads), kargs, g.lds, bs);
    }
    if (e != hipSuccess) st = DEDISP_HIP_STATUS(e);
  }
  for (size_t n = 0; n < b->solo.size() && st == DEDISP_OK; ++n) {
    const int i = b->solo[n];
    const int k = pick(dedisp::stage_kind(b->plans[i]->dtype));
    load[k] += beam_work(b, i);
    st = dedisp::launch(b->plans[i], b->solo_variant[n], ins[i], outs[i], b->nsamps[i], b->branch[k], b->ws[i]);
  }
  // join every branch back into the capture stream
  for (int k = 0; k < kBranches; ++k) {
    hipError_t e1 = hipEventRecord(b->join_ev[k], b->branch[k]);
    if (e1 == hipSuccess) e1 = hipStreamWaitEvent(b->capture, b->join_ev[k], 0);
    if (e1 != hipSuccess && st == DEDISP_OK) st = DEDISP_HIP_STATUS(e1);
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
  int64_t items = 0;
  int grid = 0;
  for (const BatchGroup& g : b->groups) {
    items += g.n_items;
    grid += g.grid;
  }
  if (work_items) *work_items = items;
  if (workgroups) *workgroups = grid;
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
    if (!b->groups.empty()) {
      // the half we are about to fill was last read by the copies two updates ago
      b->h_half ^= 1;
      if ((e = hipEventSynchronize(b->h_done[b->h_half])) != hipSuccess) return DEDISP_HIP_STATUS(e);
      st = build_args(b, ins, outs, nullptr);
      if (st != DEDISP_OK) return st;
      const dedisp::TiledArgs* h = b->h_args + b->h_half * b->nbeams;
      for (size_t gi = 0; gi < b->groups.size() && e == hipSuccess; ++gi) {
        const BatchGroup& g = b->groups[gi];
        e = hipMemcpyAsync(g.d_args, h + g.off, g.order.size() * sizeof(dedisp::TiledArgs), hipMemcpyHostToDevice,
                           stream);
      }
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
  b->layout = 0;  // the groups are timed on balanced branches, whatever was set before
  hipStream_t stream = static_cast<hipStream_t>(stream_v);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return DEDISP_HIP_STATUS(e);
  }
  // time the current split: one warm-up execute (builds the graph), best of two
  auto time_split = [&](double* tmin) -> int {
    (void)hipStreamSynchronize(stream);
    int r = dedisp_batch_execute(b, ins, outs, stream);
    *tmin = 1e30;
    for (int rep = 0; rep < 2 && r == DEDISP_OK; ++rep) {
      hipError_t x = hipEventRecord(e0, stream);
      if (x == hipSuccess) r = dedisp_batch_execute(b, ins, outs, stream);
      if (r != DEDISP_OK) break;
      if (x == hipSuccess) x = hipEventRecord(e1, stream);
      if (x == hipSuccess) x = hipEventSynchronize(e1);
      float ms = 0.f;
      if (x == hipSuccess) x = hipEventElapsedTime(&ms, e0, e1);
      if (x != hipSuccess) return DEDISP_HIP_STATUS(x);
      *tmin = std::min(*tmin, static_cast<double>(ms));
    }
    return r;
  };
  int best = -1;
  bool best_own = false, best_solo = false;
  double best_t = 1e30;
  for (int v = 1; v < dedisp::variant_count() && st == DEDISP_OK; ++v) {
    bool any = false;
    for (int i = 0; i < b->nbeams; ++i) any |= dedisp::variant_fits(b->plans[i], v);
    if (!any) continue;
    (void)hipStreamSynchronize(stream);
    free_device(b);
    assign(b, v);
    double t = 0.0;
    st = time_split(&t);
    if (st == DEDISP_OK && t < best_t) {
      best_t = t;
      best = v;
    }
  }
  // with both kinds of beams: the 8-bit beams' variant, then the float beams',
  // each over every variant with the other held (the kinds run as separate
  // kernels, so their times nearly add up)
  int best8 = best, bestf = best;
  bool kinds = false, has8 = false, hasf = false;
  for (int i = 0; i < b->nbeams; ++i) (b->plans[i]->dtype == DEDISP_U8 ? has8 : hasf) = true;
  for (int pass = 0; pass < 2 && has8 && hasf && best >= 1 && st == DEDISP_OK; ++pass) {
    for (int v = 1; v < dedisp::variant_count() && st == DEDISP_OK; ++v) {
      const int v8 = pass == 0 ? v : best8, vf = pass == 0 ? bestf : v;
      if (v8 == best8 && vf == bestf) continue;  // timed already
      (void)hipStreamSynchronize(stream);
      free_device(b);
      assign_kinds(b, v8, vf);
      double t = 0.0;
      st = time_split(&t);
      if (st == DEDISP_OK && t < best_t) {
        best_t = t;
        best8 = v8;
        bestf = vf;
        kinds = true;
      }
    }
  }
  if (st == DEDISP_OK) {
    (void)hipStreamSynchronize(stream);
    free_device(b);
    if (assign_own(b)) {
      double t = 0.0;
      st = time_split(&t);
      if (st == DEDISP_OK && t < best_t) {
        best_t = t;
        best = b->variant;
        best_own = true;
        kinds = false;
      }
    }
  }
  // the per-beam launches, in each layout of the branches
  int best_layout = 0, solo_layout = -1;
  for (int layout = 0; layout < 3 && st == DEDISP_OK; ++layout) {
    (void)hipStreamSynchronize(stream);
    free_device(b);
    assign_solo(b);
    b->layout = layout;
    double t = 0.0;
    st = time_split(&t);
    if (st == DEDISP_OK && t < best_t) {
      best_t = t;
      best_solo = true;
      best_own = kinds = false;
      solo_layout = layout;
    }
  }
  if (best_solo) best_layout = solo_layout;
  b->layout = 0;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != DEDISP_OK) return st;
  (void)hipStreamSynchronize(stream);
  free_device(b);
  if (best_solo)
    assign_solo(b);
  else if (best_own)
    assign_own(b);
  else if (kinds)
    assign_kinds(b, best8, bestf);
  else
    assign(b, best);
  b->layout = best_layout;
  *best_variant = b->variant;
  if (best_ms) *best_ms = best_t;
  return DEDISP_OK;
}

extern "C" int dedisp_batch_get_layout(dedisp_batch b, int* layout) {
  if (b == nullptr || layout == nullptr) return DEDISP_ERR_INVALID_ARG;
  *layout = b->layout;
  return DEDISP_OK;
}

extern "C" int dedisp_batch_set_layout(dedisp_batch b, int layout) {
  if (b == nullptr || layout < 0 || layout > 2) return DEDISP_ERR_INVALID_ARG;
  int dev0 = -1;
  if (b->device >= 0 && hipGetDevice(&dev0) == hipSuccess) (void)hipSetDevice(b->device);
  if (b->device >= 0) (void)hipDeviceSynchronize();
  free_graph(b);
  if (dev0 >= 0) (void)hipSetDevice(dev0);
  b->layout = layout;
  return DEDISP_OK;
}

extern "C" int dedisp_batch_get_variant(dedisp_batch b, int* variant) {
  if (b == nullptr || variant == nullptr) return DEDISP_ERR_INVALID_ARG;
  *variant = b->variant;
  return DEDISP_OK;
}

extern "C" int dedisp_batch_set_variant(dedisp_batch b, int variant) {
  if (b == nullptr || variant < -1 || variant >= dedisp::variant_count()) return DEDISP_ERR_INVALID_ARG;
  int dev0 = -1;
  if (b->device >= 0 && hipGetDevice(&dev0) == hipSuccess) (void)hipSetDevice(b->device);
  if (b->device >= 0) (void)hipDeviceSynchronize();
  free_device(b);
  if (dev0 >= 0) (void)hipSetDevice(dev0);
  b->layout = 0;
  if (variant == -1)
    assign_solo(b);
  else if (variant == 0)
    (void)assign_own(b);
  else
    assign(b, variant);
  return DEDISP_OK;
}

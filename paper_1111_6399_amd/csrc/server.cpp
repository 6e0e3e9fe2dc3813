// Streaming server: blocks of many beams are submitted as they arrive and run
// concurrently on a pool of streams; each beam keeps its last max_shift input
// samples on the device so that consecutive blocks overlap correctly.
//
// Per beam there is one ring buffer of [nchans][R] samples in staged form
// (8-bit samples widened to 16 bits; half and float as they are) and one
// buffer for a raw block.  Stream sample tau of a beam sits at ring position
// (tau + H) mod R, H = max_shift rounded up to 8, R >= max_shift + B plus a
// tile's overrun, a multiple of 8.  Block b of a beam is copied as one
// contiguous transfer into the raw buffer; one kernel writes it into the ring
// (widened where needed; nothing else is copied: the history stays where it
// is), and the de-dispersion kernel reads the window of stream samples
// [b*B - max_shift, (b+1)*B) straight from the ring, starting at position
// (b*B + H - max_shift) mod R and wrapping at R.  Every operation of a beam
// goes to the same stream, so blocks of one beam run in order and a block is
// not written over history that an earlier kernel still reads; different
// beams use different streams of the pool and overlap on the device (copies
// of one beam under the kernels of others).
//
// Admission: a beam's ring and raw buffer are charged to the memory budget
// when it is added; a request is charged its output (ndm*B values) and is
// admitted while that fits the budget and fewer than max_inflight requests are
// running.  Completion is recorded by a host callback enqueued after the
// kernel, which also returns the request's charge and slot.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "dedisp_internal.h"

namespace {

double now_s() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket = 0;
  int beam = 0;
  size_t footprint = 0;
  double work = 0.0;  // DM x channel x samples
  double t_submit = 0.0;
  std::atomic<double> t_done{0.0};
  std::atomic<int> finished{0};
  int status = DEDISP_OK;
  dedisp_server owner = nullptr;
};

struct Beam {
  dedisp_plan plan = nullptr;
  int64_t block = 0;  // B
  int64_t ring = 0;   // R: samples per ring row
  int64_t head = 0;   // H: ring position of stream sample 0
  size_t es = 1;      // bytes per raw sample
  void* rows = nullptr;  // ring rows [nchans][R], staged
  void* raw = nullptr;   // one raw block
  size_t ring_bytes = 0;
  size_t bytes = 0;
  int64_t next = 0;        // index of the next block since the history last restarted
  bool zero_tail = true;   // next block starts from a zero history
  int stream = 0;
};

// Ring length for a beam: the history and a block, plus the samples a tile
// may read past the block (4032 samples, its halo and the rounding of its
// loads to 1 KB; the one-trial tile of 8064 samples reads further, and those
// reads wrap or return zeros and feed only outputs past the block), a
// multiple of 8 samples.
int64_t ring_samples(int64_t max_shift, int64_t block) { return (max_shift + block + 4608 + 7) / 8 * 8; }

}  // namespace

struct dedisp_server_s {
  size_t budget = 0;
  int max_inflight = 0;
  int device = -1;
  std::atomic<size_t> used{0};
  std::atomic<int> inflight{0};
  std::vector<Beam> beams;
  std::vector<hipStream_t> streams;
  std::map<uint64_t, std::shared_ptr<Request>> reqs;
  uint64_t next_ticket = 1;
  std::mutex mu;
  // statistics over completed requests
  std::vector<double> latencies;
  double first_submit = -1.0;
  double last_done = 0.0;
  double work_done = 0.0;
  int64_t fault_at = -1;  // test hook: the n-th submission fails as a device fault
  int64_t submissions = 0;
};

namespace {

constexpr int kStreams = 4;

void on_done(void* arg) {
  Request* r = static_cast<Request*>(arg);
  r->t_done.store(now_s());
  r->owner->used.fetch_sub(r->footprint);
  r->owner->inflight.fetch_sub(1);
  r->finished.store(1);
}

// Move completed requests' latencies into the statistics (caller holds mu).
void harvest(dedisp_server s) {
  for (auto& kv : s->reqs) {
    Request* r = kv.second.get();
    if (r->finished.load() == 1) {
      r->finished.store(2);  // counted
      if (r->status == DEDISP_OK) {
        const double done = r->t_done.load();
        s->latencies.push_back(done - r->t_submit);
        s->last_done = std::max(s->last_done, done);
        s->work_done += r->work;
      }
    }
  }
}

}  // namespace

extern "C" int dedisp_server_create(size_t hbm_budget_bytes, int max_inflight, dedisp_server* out) {
  if (out == nullptr || hbm_budget_bytes == 0 || max_inflight < 1) return DEDISP_ERR_INVALID_ARG;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  dedisp_server s = new (std::nothrow) dedisp_server_s();
  if (s == nullptr) return DEDISP_ERR_OUT_OF_MEMORY;
  s->budget = hbm_budget_bytes;
  s->max_inflight = max_inflight;
  s->device = dev;
  for (int i = 0; i < kStreams; ++i) {
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) {
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      return DEDISP_HIP_STATUS(e);
    }
    s->streams.push_back(st);
  }
  if (const char* f = std::getenv("DEDISP_FAULT_INJECT")) {
    // "submit:N": the N-th submission (1-based) fails as a device fault
    if (std::strncmp(f, "submit:", 7) == 0) s->fault_at = std::atoll(f + 7);
  }
  *out = s;
  return DEDISP_OK;
}

extern "C" int dedisp_server_add_beam(dedisp_server s, dedisp_plan p, int64_t block_nsamp, int* beam_id) {
  if (s == nullptr || p == nullptr || beam_id == nullptr || block_nsamp < 1) return DEDISP_ERR_INVALID_ARG;
  if (block_nsamp > static_cast<int64_t>(INT32_MAX) - p->max_shift) return DEDISP_ERR_INVALID_ARG;
  Beam b;
  b.plan = p;
  b.block = block_nsamp;
  b.ring = ring_samples(p->max_shift, block_nsamp);
  b.head = (static_cast<int64_t>(p->max_shift) + 7) / 8 * 8;
  b.es = dedisp::dtype_size(p->dtype);
  b.ring_bytes = static_cast<size_t>(p->nchans) * static_cast<size_t>(b.ring) * dedisp::staged_size(p->dtype);
  const size_t raw_bytes = static_cast<size_t>(p->nchans) * b.block * b.es;
  b.bytes = b.ring_bytes + raw_bytes;
  std::lock_guard<std::mutex> g(s->mu);
  if (s->used.load() + b.bytes > s->budget) return DEDISP_ERR_AGAIN;
  hipError_t e = hipSetDevice(s->device);
  if (e == hipSuccess) e = hipMalloc(&b.rows, b.ring_bytes);
  if (e == hipSuccess) e = hipMalloc(&b.raw, raw_bytes);
  if (e != hipSuccess) {
    for (void* x : {b.rows, b.raw})
      if (x) (void)hipFree(x);
    return DEDISP_HIP_STATUS(e);
  }
  b.stream = static_cast<int>(s->beams.size() % s->streams.size());
  s->used.fetch_add(b.bytes);
  s->beams.push_back(b);
  *beam_id = static_cast<int>(s->beams.size() - 1);
  return DEDISP_OK;
}

extern "C" int dedisp_submit(dedisp_server s, int beam_id, const void* block, void* out_dev, uint64_t* ticket) {
  if (s == nullptr || block == nullptr || out_dev == nullptr || ticket == nullptr) return DEDISP_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(out_dev) & 3) != 0) return DEDISP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  if (beam_id < 0 || beam_id >= static_cast<int>(s->beams.size())) return DEDISP_ERR_NOT_FOUND;
  Beam& b = s->beams[beam_id];
  const dedisp_plan p = b.plan;
  const size_t in_bytes = static_cast<size_t>(p->nchans) * b.block * b.es;
  const size_t footprint = static_cast<size_t>(p->ndm) * b.block * 4;
  if (s->inflight.load() >= s->max_inflight || s->used.load() + footprint > s->budget) return DEDISP_ERR_AGAIN;
  hipError_t e = hipSetDevice(s->device);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);

  auto r = std::make_shared<Request>();
  r->ticket = s->next_ticket++;
  r->beam = beam_id;
  r->footprint = footprint;
  r->work = static_cast<double>(p->ndm) * p->nchans * b.block;
  r->t_submit = now_s();
  r->owner = s;
  if (s->first_submit < 0) s->first_submit = r->t_submit;
  s->submissions += 1;

  if (s->submissions == s->fault_at) {
    // injected device fault: nothing runs, the ticket reports the error and
    // the beam restarts from a zero history (a discontinuity of the stream)
    r->status = DEDISP_ERR_DEVICE;
    r->t_done.store(r->t_submit);
    r->finished.store(1);
    b.zero_tail = true;
    b.next += 1;
    s->reqs[r->ticket] = r;
    *ticket = r->ticket;
    return DEDISP_OK;
  }

  hipStream_t st = s->streams[b.stream];
  int status = DEDISP_OK;
  if (b.zero_tail) {  // a new history: zeros before the first block
    b.next = 0;
    status = DEDISP_HIP_STATUS(hipMemsetAsync(b.rows, 0, b.ring_bytes, st));
  }
  const int64_t first = (b.next % b.ring) * (b.block % b.ring) % b.ring;  // b*B mod R
  if (status == DEDISP_OK) status = DEDISP_HIP_STATUS(hipMemcpyAsync(b.raw, block, in_bytes, hipMemcpyDefault, st));
  if (status == DEDISP_OK)
    status = dedisp::ring_append(p->dtype, b.raw, b.rows, b.block, b.ring, (first + b.head) % b.ring, p->nchans, st);
  if (status == DEDISP_OK) {
    int v = p->variant.load();
    if (v < 0) v = dedisp::default_variant(p);
    const int64_t start = (first + b.head - p->max_shift) % b.ring;
    const dedisp::StagedRows rows{b.rows, b.ring, static_cast<int64_t>(p->nchans) * b.ring, start, b.ring};
    status = dedisp::launch_rows(p, v, rows, out_dev, b.block, st);
  }
  if (status == DEDISP_OK) status = DEDISP_HIP_STATUS(hipLaunchHostFunc(st, on_done, r.get()));
  if (status != DEDISP_OK) {
    // nothing usable was queued for this block: restart the beam's history
    b.zero_tail = true;
    b.next += 1;
    return status;
  }
  s->used.fetch_add(footprint);
  s->inflight.fetch_add(1);
  b.zero_tail = false;
  b.next += 1;
  s->reqs[r->ticket] = r;
  *ticket = r->ticket;
  return DEDISP_OK;
}

extern "C" int dedisp_poll(dedisp_server s, uint64_t ticket, int* done, double* latency_s) {
  if (s == nullptr || done == nullptr) return DEDISP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return DEDISP_ERR_NOT_FOUND;
  Request* r = it->second.get();
  if (r->finished.load() == 0) {
    *done = 0;
    return DEDISP_OK;
  }
  harvest(s);
  const int status = r->status;
  const double lat = r->t_done.load() - r->t_submit;
  s->reqs.erase(it);
  if (status != DEDISP_OK) return status;
  *done = 1;
  if (latency_s) *latency_s = lat;
  return DEDISP_OK;
}

extern "C" int dedisp_server_drain(dedisp_server s) {
  if (s == nullptr) return DEDISP_ERR_INVALID_ARG;
  std::vector<hipStream_t> streams;
  {
    std::lock_guard<std::mutex> g(s->mu);
    streams = s->streams;
  }
  int st = DEDISP_OK;
  for (hipStream_t x : streams) {
    const int r = DEDISP_HIP_STATUS(hipStreamSynchronize(x));
    if (r != DEDISP_OK) st = r;
  }
  std::lock_guard<std::mutex> g(s->mu);
  harvest(s);
  return st;
}

extern "C" int dedisp_server_stats(dedisp_server s, double* p50_s, double* p99_s, double* dm_ch_samp_per_s) {
  if (s == nullptr) return DEDISP_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  harvest(s);
  std::vector<double> l = s->latencies;
  std::sort(l.begin(), l.end());
  auto pct = [&l](double q) {
    if (l.empty()) return 0.0;
    const size_t i = std::min(l.size() - 1, static_cast<size_t>(q * (l.size() - 1) + 0.5));
    return l[i];
  };
  if (p50_s) *p50_s = pct(0.50);
  if (p99_s) *p99_s = pct(0.99);
  if (dm_ch_samp_per_s) {
    const double span = s->last_done - s->first_submit;
    *dm_ch_samp_per_s = (span > 0 && !l.empty()) ? s->work_done / span : 0.0;
  }
  return DEDISP_OK;
}

extern "C" int dedisp_server_destroy(dedisp_server s) {
  if (s == nullptr) return DEDISP_OK;
  (void)dedisp_server_drain(s);
  int dev0 = -1;
  if (hipGetDevice(&dev0) == hipSuccess) (void)hipSetDevice(s->device);
  for (Beam& b : s->beams)
    for (void* x : {b.rows, b.raw})
      if (x) (void)hipFree(x);
  for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
  if (dev0 >= 0) (void)hipSetDevice(dev0);
  delete s;
  return DEDISP_OK;
}

// The streaming server's host logic (csrc/server.cpp) on the CPU under
// sanitizers (test infrastructure, built and run by
// tests/test_host_sanitizers.py; nothing here is part of the library).
//
// The HIP runtime calls the server makes are stood in for here: a stream is a
// worker thread that runs its queued operations in order, device memory is
// host memory, and a host function queued on a stream runs on that worker, as
// the runtime's callback thread would run it.  The two device steps the server
// queues, appending a block to a beam's ring rows and de-dispersing the
// window that ends with it, are plain loops here that first check what the GPU
// kernels assume of their arguments.  Each output block is compared with the
// plain definition over the beam's whole stream (zeros before its first
// block), so that the ring positions the server computes are checked too.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <random>
#include <thread>
#include <vector>

#include "dedisp_internal.h"
#include "shift_table.h"

namespace {

std::atomic<int> failures{0};

#define CHECK(cond)                                                      \
  do {                                                                   \
    if (!(cond)) {                                                       \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #cond); \
      failures.fetch_add(1);                                             \
    }                                                                    \
  } while (0)

// Streams hold their queued work while this is set (to keep requests in
// flight for the admission checks).
std::mutex hold_mu;
std::condition_variable hold_cv;
bool hold = false;

}  // namespace

// ------------------------------------------------- runtime stand-ins --

struct ihipStream_t {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::function<void()>> q;
  bool busy = false;
  bool stop = false;
  std::thread worker;

  void run() {
    std::unique_lock<std::mutex> g(mu);
    for (;;) {
      cv.wait(g, [this] { return stop || !q.empty(); });
      if (q.empty()) return;  // stopping with nothing left
      std::function<void()> f = std::move(q.front());
      q.pop_front();
      busy = true;
      g.unlock();
      {
        std::unique_lock<std::mutex> h(hold_mu);
        hold_cv.wait(h, [] { return !hold; });
      }
      f();
      g.lock();
      busy = false;
      cv.notify_all();
    }
  }
  void push(std::function<void()> f) {
    std::lock_guard<std::mutex> g(mu);
    q.push_back(std::move(f));
    cv.notify_all();
  }
  void sync() {
    std::unique_lock<std::mutex> g(mu);
    cv.wait(g, [this] { return q.empty() && !busy; });
  }
};

hipError_t hipGetDevice(int* id) {
  *id = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int id) { return id == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  *s = new ihipStream_t();
  (*s)->worker = std::thread([st = *s] { st->run(); });
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  s->worker.join();
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  s->sync();
  return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t n) {
  *p = std::malloc(n);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
  s->push([=] { std::memcpy(dst, src, n); });
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t s) {
  s->push([=] { std::memset(dst, v, n); });
  return hipSuccess;
}
hipError_t hipLaunchHostFunc(hipStream_t s, hipHostFn_t fn, void* arg) {
  s->push([=] { fn(arg); });
  return hipSuccess;
}

namespace {

float half_to_float(uint16_t h) {  // IEEE 754 binary16 (normal numbers and zero here)
  const int e = (h >> 10) & 0x1f, m = h & 0x3ff;
  const double s = (h & 0x8000) ? -1.0 : 1.0;
  if (e == 0) return static_cast<float>(s * std::ldexp(m, -24));
  return static_cast<float>(s * std::ldexp(1024 + m, e - 25));
}

// An integer in [-64, 64] as binary16.
uint16_t half_of_int(int v) {
  if (v == 0) return 0;
  const uint16_t sign = v < 0 ? 0x8000 : 0;
  int a = std::abs(v), e = 0;
  while ((a >> e) > 1) ++e;  // a = 1.f * 2^e
  const int m = (a << (10 - e)) & 0x3ff;
  return static_cast<uint16_t>(sign | ((e + 15) << 10) | m);
}

double staged_value(int dtype, const void* rows, int64_t i) {
  if (dtype == DEDISP_U8) return static_cast<const uint16_t*>(rows)[i];
  if (dtype == DEDISP_F16) return half_to_float(static_cast<const uint16_t*>(rows)[i]);
  return static_cast<const float*>(rows)[i];
}

}  // namespace

// Device steps the server queues, as plain loops.
namespace dedisp {

bool trace_enabled() { return false; }
void trace_hip_error(hipError_t, const char*, int) {}
int default_variant(dedisp_plan) { return 1; }

int ring_append(int dtype, const void* blk, void* ring_rows, int64_t block, int64_t ring, int64_t pos, int nchans,
                hipStream_t s) {
  CHECK(block >= 1 && block <= ring && pos >= 0 && pos < ring && ring % 8 == 0);
  s->push([=] {
    for (int c = 0; c < nchans; ++c)
      for (int64_t j = 0; j < block; ++j) {
        const int64_t src = static_cast<int64_t>(c) * block + j, dst = static_cast<int64_t>(c) * ring + (pos + j) % ring;
        if (dtype == DEDISP_U8)
          static_cast<uint16_t*>(ring_rows)[dst] = static_cast<const uint8_t*>(blk)[src];
        else if (dtype == DEDISP_F16)
          static_cast<uint16_t*>(ring_rows)[dst] = static_cast<const uint16_t*>(blk)[src];
        else
          static_cast<float*>(ring_rows)[dst] = static_cast<const float*>(blk)[src];
      }
  });
  return DEDISP_OK;
}

int launch_rows(dedisp_plan p, int v, const StagedRows& rows, void* out, int64_t nsamp, hipStream_t s) {
  // what the tile kernels assume of ring rows
  CHECK(v >= 1);
  CHECK(rows.ring > 0 && rows.pitch == rows.ring && rows.ring % 8 == 0);
  CHECK(rows.start >= 0 && rows.start < rows.ring);
  CHECK(rows.total == static_cast<int64_t>(p->nchans) * rows.ring);
  // a window (the history and the block) fits the ring without wrapping
  // onto itself (loads past the ring return zeros and feed only samples past
  // the block)
  CHECK(rows.ring >= p->max_shift + nsamp);
  const dedisp_plan_s* pp = p;
  const StagedRows r = rows;
  s->push([=] {
    for (int d = 0; d < pp->ndm; ++d)
      for (int64_t t = 0; t < nsamp; ++t) {
        double sum = 0.0;
        for (int c = 0; c < pp->nchans; ++c) {
          const int64_t k = (r.start + t + pp->shift[static_cast<size_t>(c) * pp->ndm + d]) % r.ring;
          sum += staged_value(pp->dtype, r.in, static_cast<int64_t>(c) * r.ring + k);
        }
        if (pp->dtype == DEDISP_U8)
          static_cast<int32_t*>(out)[d * nsamp + t] = static_cast<int32_t>(sum);
        else
          static_cast<float*>(out)[d * nsamp + t] = static_cast<float>(sum);
      }
  });
  return DEDISP_OK;
}

}  // namespace dedisp

// ------------------------------------------------------------- checks --

namespace {

struct Stream {
  dedisp_plan_s plan;
  int64_t block = 0;
  int beam = -1;
  std::vector<double> x;  // [nchans][nblocks * block] values of the stream
  std::vector<std::vector<uint8_t>> raw;  // per block, [nchans][block] in the input type
};

void make_plan(dedisp_plan_s& p, int dtype, int nchans, int ndm, double step) {
  p.nchans = nchans;
  p.ndm = ndm;
  p.dtype = dtype;
  p.f_top = 150.0;
  p.df = 0.1953125 * 8;
  p.tsamp = 327.68e-6;
  for (int d = 0; d < ndm; ++d) p.dms.push_back(d * step);
  CHECK(dedisp::build_shift_table(nchans, p.f_top, p.df, p.tsamp, p.dms.data(), ndm, &p.shift, &p.max_shift));
}

void make_stream(Stream& s, int nblocks, uint32_t seed) {
  std::mt19937 rng(seed);
  const int n = s.plan.nchans;
  const int64_t len = nblocks * s.block;
  s.x.assign(static_cast<size_t>(n) * len, 0.0);
  const size_t es = dedisp::dtype_size(s.plan.dtype);
  for (int b = 0; b < nblocks; ++b) {
    std::vector<uint8_t> r(static_cast<size_t>(n) * s.block * es);
    for (int c = 0; c < n; ++c)
      for (int64_t j = 0; j < s.block; ++j) {
        const size_t i = static_cast<size_t>(c) * s.block + j;
        double v;
        if (s.plan.dtype == DEDISP_U8) {
          r[i] = static_cast<uint8_t>(rng() & 0xff);
          v = r[i];
        } else if (s.plan.dtype == DEDISP_F16) {
          const uint16_t h = half_of_int(static_cast<int>(rng() % 129) - 64);
          std::memcpy(&r[2 * i], &h, 2);
          v = half_to_float(h);
        } else {
          const float f = static_cast<float>(static_cast<int>(rng() % 2001) - 1000) / 64.0f;
          std::memcpy(&r[4 * i], &f, 4);
          v = f;
        }
        s.x[static_cast<size_t>(c) * len + b * s.block + j] = v;
      }
    s.raw.push_back(std::move(r));
  }
}

// Block b of a stream whose history restarted at block b0: the plain sum over
// the stream from block b0 on (zeros before it), output times
// [b*B - max_shift, (b+1)*B - max_shift) counted from block b0.
void check_block(const Stream& s, int b0, int b, const std::vector<uint8_t>& out) {
  const dedisp_plan_s& p = s.plan;
  const int64_t B = s.block, len = static_cast<int64_t>(s.x.size()) / p.nchans;
  int bad = 0;
  for (int d = 0; d < p.ndm; ++d)
    for (int64_t t = 0; t < B; ++t) {
      double sum = 0.0;
      for (int c = 0; c < p.nchans; ++c) {
        const int64_t tau = (b - b0) * B - p.max_shift + t + p.shift[static_cast<size_t>(c) * p.ndm + d];
        if (tau >= 0) sum += s.x[static_cast<size_t>(c) * len + b0 * B + tau];
      }
      if (p.dtype == DEDISP_U8) {
        int32_t got;
        std::memcpy(&got, &out[4 * (d * B + t)], 4);
        bad += got != static_cast<int32_t>(sum);
      } else {
        float got;
        std::memcpy(&got, &out[4 * (d * B + t)], 4);
        bad += got != static_cast<float>(sum);
      }
    }
  if (bad) std::fprintf(stderr, "dtype %d block %d (history from %d): %d outputs differ\n", p.dtype, b, b0, bad);
  CHECK(bad == 0);
}

// Submit every block of the given streams in order (from this thread), polling
// until each is done; DEDISP_ERR_AGAIN is retried after a poll.
void feed(dedisp_server srv, std::vector<Stream*> streams, int nblocks) {
  for (int b = 0; b < nblocks; ++b)
    for (Stream* s : streams) {
      std::vector<uint8_t> out(static_cast<size_t>(s->plan.ndm) * s->block * 4);
      uint64_t tk = 0;
      int st;
      while ((st = dedisp_submit(srv, s->beam, s->raw[b].data(), out.data(), &tk)) == DEDISP_ERR_AGAIN)
        std::this_thread::yield();
      CHECK(st == DEDISP_OK);
      int done = 0;
      double lat = -1.0;
      while (st == DEDISP_OK && !done) {
        st = dedisp_poll(srv, tk, &done, &lat);
        if (!done) std::this_thread::yield();
      }
      CHECK(st == DEDISP_OK && lat >= 0.0);
      check_block(*s, 0, b, out);
    }
}

void concurrent_beams() {
  // three beams, one per input type, ragged block lengths; two submitting
  // threads; at most three requests in flight
  Stream s[3];
  make_plan(s[0].plan, DEDISP_U8, 12, 7, 2.5);
  make_plan(s[1].plan, DEDISP_F16, 9, 5, 3.5);
  make_plan(s[2].plan, DEDISP_F32, 10, 6, 1.5);
  const int64_t blocks[3] = {64, 100, 37};
  const int nblocks = 6;
  dedisp_server srv = nullptr;
  CHECK(dedisp_server_create(size_t{1} << 30, 3, &srv) == DEDISP_OK);
  for (int k = 0; k < 3; ++k) {
    s[k].block = blocks[k];
    make_stream(s[k], nblocks, 100 + k);
    CHECK(dedisp_server_add_beam(srv, &s[k].plan, s[k].block, &s[k].beam) == DEDISP_OK);
  }
  std::thread t1(feed, srv, std::vector<Stream*>{&s[0], &s[1]}, nblocks);
  std::thread t2(feed, srv, std::vector<Stream*>{&s[2]}, nblocks);
  t1.join();
  t2.join();
  double p50 = -1, p99 = -1, rate = -1;
  CHECK(dedisp_server_drain(srv) == DEDISP_OK);
  CHECK(dedisp_server_stats(srv, &p50, &p99, &rate) == DEDISP_OK);
  CHECK(p50 >= 0.0 && p99 >= p50 && rate > 0.0);
  CHECK(dedisp_server_destroy(srv) == DEDISP_OK);
}

void admission() {
  Stream s;
  make_plan(s.plan, DEDISP_U8, 8, 4, 2.0);
  s.block = 48;
  make_stream(s, 3, 7);
  // a budget smaller than the beam's buffers refuses the beam
  dedisp_server small = nullptr;
  CHECK(dedisp_server_create(1024, 2, &small) == DEDISP_OK);
  int id = -1;
  CHECK(dedisp_server_add_beam(small, &s.plan, s.block, &id) == DEDISP_ERR_AGAIN);
  CHECK(dedisp_server_destroy(small) == DEDISP_OK);
  // one slot: a second request waits for the first
  dedisp_server srv = nullptr;
  CHECK(dedisp_server_create(size_t{1} << 30, 1, &srv) == DEDISP_OK);
  CHECK(dedisp_server_add_beam(srv, &s.plan, s.block, &s.beam) == DEDISP_OK);
  std::vector<std::vector<uint8_t>> out(3, std::vector<uint8_t>(static_cast<size_t>(s.plan.ndm) * s.block * 4));
  uint64_t tk[3] = {};
  {
    std::lock_guard<std::mutex> g(hold_mu);
    hold = true;
  }
  CHECK(dedisp_submit(srv, s.beam, s.raw[0].data(), out[0].data(), &tk[0]) == DEDISP_OK);
  CHECK(dedisp_submit(srv, s.beam, s.raw[1].data(), out[1].data(), &tk[1]) == DEDISP_ERR_AGAIN);
  int done = -1;
  CHECK(dedisp_poll(srv, tk[0], &done, nullptr) == DEDISP_OK && done == 0);
  {
    std::lock_guard<std::mutex> g(hold_mu);
    hold = false;
  }
  hold_cv.notify_all();
  CHECK(dedisp_server_drain(srv) == DEDISP_OK);
  CHECK(dedisp_poll(srv, tk[0], &done, nullptr) == DEDISP_OK && done == 1);
  CHECK(dedisp_poll(srv, tk[0], &done, nullptr) == DEDISP_ERR_NOT_FOUND);  // reported once
  for (int b = 1; b < 3; ++b) {
    CHECK(dedisp_submit(srv, s.beam, s.raw[b].data(), out[b].data(), &tk[b]) == DEDISP_OK);
    CHECK(dedisp_server_drain(srv) == DEDISP_OK);
    CHECK(dedisp_poll(srv, tk[b], &done, nullptr) == DEDISP_OK && done == 1);
  }
  for (int b = 0; b < 3; ++b) check_block(s, 0, b, out[b]);
  // refused arguments
  CHECK(dedisp_submit(srv, 5, s.raw[0].data(), out[0].data(), &tk[0]) == DEDISP_ERR_NOT_FOUND);
  CHECK(dedisp_submit(srv, s.beam, nullptr, out[0].data(), &tk[0]) == DEDISP_ERR_INVALID_ARG);
  CHECK(dedisp_poll(srv, 12345, &done, nullptr) == DEDISP_ERR_NOT_FOUND);
  CHECK(dedisp_server_destroy(srv) == DEDISP_OK);
}

void injected_fault() {
  // the third submission fails: its ticket reports the fault once and the
  // beam's next block starts from a zero history
  setenv("DEDISP_FAULT_INJECT", "submit:3", 1);
  Stream s;
  make_plan(s.plan, DEDISP_F32, 10, 6, 1.5);
  s.block = 40;
  make_stream(s, 5, 11);
  dedisp_server srv = nullptr;
  CHECK(dedisp_server_create(size_t{1} << 30, 4, &srv) == DEDISP_OK);
  unsetenv("DEDISP_FAULT_INJECT");
  CHECK(dedisp_server_add_beam(srv, &s.plan, s.block, &s.beam) == DEDISP_OK);
  for (int b = 0; b < 5; ++b) {
    std::vector<uint8_t> out(static_cast<size_t>(s.plan.ndm) * s.block * 4);
    uint64_t tk = 0;
    CHECK(dedisp_submit(srv, s.beam, s.raw[b].data(), out.data(), &tk) == DEDISP_OK);
    CHECK(dedisp_server_drain(srv) == DEDISP_OK);
    int done = 0;
    const int st = dedisp_poll(srv, tk, &done, nullptr);
    if (b == 2) {
      CHECK(st == DEDISP_ERR_DEVICE);
    } else {
      CHECK(st == DEDISP_OK && done == 1);
      check_block(s, b < 2 ? 0 : 3, b, out);
    }
  }
  CHECK(dedisp_server_destroy(srv) == DEDISP_OK);
}

}  // namespace

int main() {
  concurrent_beams();
  admission();
  injected_fault();
  std::printf("server checks %s (%d failures)\n", failures.load() ? "FAILED" : "passed", failures.load());
  return failures.load() ? 1 : 0;
}

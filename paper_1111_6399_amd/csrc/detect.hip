// Detection on a de-dispersed block (the search's last step: after every
// trial DM has been integrated, a pulse shows up as a significant excess in
// one trial's time series).  One workgroup per trial:
//   1. the trial's mean and standard deviation over the block (binary64, one
//      pass of sums shifted by the trial's first value);
//   2. the row in chunks: a chunk (and the longest boxcar's overlap into the
//      next) is loaded into LDS and turned in place into its prefix sums P
//      (per-thread runs, then a scan over the workgroup), so every boxcar is
//      one difference, b_w(t) = P[t + w] - P[t]; the S/N of every complete
//      boxcar (b_w(t) - w*mean) / (std*sqrt(w)) and the best (S/N, time) per
//      width, the earliest time on ties (integer rows: the best sum, whose
//      S/N is the best S/N at the same time, see boxcars());
//   3. (trial, width) pairs whose best S/N reaches the threshold appended to
//      a candidate list through one atomic counter.
// Values are converted to binary64 on load, so the prefix sums of the int32
// outputs of 8-bit input are exact (below 2^53) and the S/N of both sides of a
// comparison is taken in the same precision.
#include <hip/hip_runtime.h>

#include <cmath>
#include <map>
#include <mutex>
#include <type_traits>

#include "dedisp_internal.h"

namespace dedisp {
namespace {

constexpr int kDetThreads = 256;
constexpr int kDetChunk = 4096;  // boxcar start times per LDS chunk
constexpr int kUnroll = 8;       // global loads in flight per thread (moments pass)
constexpr int kChunkUnroll = 18; // global loads in flight per thread (chunk loads: one round for 4096 + 511)

// The S/N of a boxcar of width 2^k with sum b is (b - snr_base) * snr_scale.
__device__ __forceinline__ double snr_base(int k, double mean) { return static_cast<double>(1 << k) * mean; }
__device__ __forceinline__ double snr_scale(int k, double sd) {
  return sd > 0.0 ? 1.0 / (sd * sqrt(static_cast<double>(1 << k))) : 0.0;
}

// Sum over the workgroup (every thread gets the result).
__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int s = kDetThreads / 2; s > 0; s >>= 1) {
    if (tid < s) red[tid] += red[tid + s];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

// Every complete boxcar starting at i < ni of a chunk held as prefix sums
// P[0..L] from time t0, folded into the best (value, time) per width.  All
// NW + 1 sums a start needs are read before any is used; kGuard: the chunk
// ends at the row's end, so the widest boxcars of its last starts are
// incomplete (and P is read at L instead).  kSums: the value is the boxcar
// sum itself.  That is for integer rows, whose sums are exact integers below
// 2^53: there (b - base) * inv, with inv > 0, is strictly increasing in b
// (distinct integers stay distinct through both roundings), and all S/N are 0
// when inv is 0 (a constant row, all sums equal), so the largest sum is at the
// same earliest time as the largest S/N.  Otherwise the value is the S/N.
template <int NW, bool kGuard, bool kSums>
__device__ __forceinline__ void boxcars(const double* P, int ni, int L, int t0, const double* base,
                                        const double* inv, double* bs, int* bt) {
  for (int i = threadIdx.x; i < ni; i += kDetThreads) {
    double q[NW + 1];
    q[0] = P[i];
#pragma unroll
    for (int k = 0; k < NW; ++k) q[k + 1] = P[kGuard ? min(i + (1 << k), L) : i + (1 << k)];
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      double v;
      if constexpr (kSums)
        v = q[k + 1] - q[0];
      else
        v = (q[k + 1] - q[0] - base[k]) * inv[k];
      // times increase along a thread, so the first of equals stays
      const bool take = v > bs[k] && (!kGuard || i + (1 << k) <= L);
      bs[k] = take ? v : bs[k];
      bt[k] = take ? t0 + i : bt[k];
    }
  }
}

template <typename T, int NW>
__global__ __launch_bounds__(kDetThreads) void detect_rows(const T* __restrict__ out, int64_t nsamp,
                                                           double threshold, double* __restrict__ stats,
                                                           double* __restrict__ best_snr,
                                                           int32_t* __restrict__ best_t,
                                                           dedisp_candidate* __restrict__ cand, int cap,
                                                           unsigned* __restrict__ count) {
  extern __shared__ double sh[];  // [kDetChunk + 2^(NW-1)] prefix sums, reused for the reductions
  __shared__ double red[kDetThreads];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int d = blockIdx.x;
  const T* row = out + static_cast<int64_t>(d) * nsamp;

  constexpr bool kSums = std::is_same<T, int32_t>::value;  // track sums, S/N at the end

  // moments about the first value (no cancellation for rows far from zero):
  // a pass of their own for float rows, whose S/N every start needs; integer
  // rows add them up while the chunks are loaded
  const double k0 = static_cast<double>(row[0]);
  double s1 = 0.0, s2 = 0.0;
  double mean = 0.0, sd = 0.0;
  auto finish_moments = [&]() {
    const double m1 = block_sum(s1, red) / static_cast<double>(nsamp);
    const double m2 = block_sum(s2, red) / static_cast<double>(nsamp);
    mean = k0 + m1;
    sd = sqrt(fmax(m2 - m1 * m1, 0.0));
    if (stats != nullptr && tid == 0) {
      stats[2 * d] = mean;
      stats[2 * d + 1] = sd;
    }
  };
  for (int64_t t = tid; !kSums && t < nsamp; t += kUnroll * kDetThreads) {
    double v[kUnroll];  // independent loads, all in flight before the first is used
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      const int64_t u = t + j * kDetThreads;  // clamped, so every load is issued unconditionally
      const double x = static_cast<double>(row[u < nsamp ? u : nsamp - 1]);
      v[j] = u < nsamp ? x : k0;
    }
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      const double e = v[j] - k0;
      s1 += e;
      s2 += e * e;
    }
  }
  if constexpr (!kSums) finish_moments();

  constexpr int W = 1 << (NW - 1);
  constexpr int span = kDetChunk + W - 1;
  constexpr int NS = kSums ? 1 : NW;  // integer rows need the S/N terms only at the end
  double base[NS] = {}, inv[NS] = {};
  if constexpr (!kSums) {
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      base[k] = snr_base(k, mean);
      inv[k] = snr_scale(k, sd);
    }
  }
  double bs[NW];  // best value (S/N, or the boxcar sum for integer rows) of this thread's starts
  int bt[NW];     // its time; times are below 2^31 (nsamp is checked)
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    bs[k] = -INFINITY;
    bt[k] = -1;
  }
  double* P = sh;
  for (int64_t t0 = 0; t0 < nsamp; t0 += kDetChunk) {
    const int L = static_cast<int>(min(static_cast<int64_t>(span), nsamp - t0));  // samples held
    for (int i = tid; i < L; i += kChunkUnroll * kDetThreads) {
      T v[kChunkUnroll];  // raw samples, converted as they are stored
#pragma unroll
      for (int j = 0; j < kChunkUnroll; ++j) {
        const int u = i + j * kDetThreads;
        v[j] = row[t0 + (u < L ? u : L - 1)];
      }
#pragma unroll
      for (int j = 0; j < kChunkUnroll; ++j) {
        const int u = i + j * kDetThreads;
        const double x = static_cast<double>(v[j]);
        if (u < L) P[u] = x;
        if constexpr (kSums) {
          // each sample once: the chunk's own samples, not the overlap into the next
          const double e = u < min(L, kDetChunk) ? x - k0 : 0.0;
          s1 += e;
          s2 += e * e;
        }
      }
    }
    __syncthreads();
    // in place: P[i] = sum of the chunk's samples before i, P[L] = all of them.
    // Runs of an odd length start on different LDS banks.
    const int seg = ((L + kDetThreads - 1) / kDetThreads) | 1;
    const int i0 = min(tid * seg, L), i1 = min(i0 + seg, L);
    double own = 0.0;
    for (int i = i0; i < i1; ++i) own += P[i];
    double incl = own;  // inclusive scan over the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    if (lane == 63) red[wave] = incl;
    __syncthreads();
    double run = incl - own;
    for (int j = 0; j < wave; ++j) run += red[j];
    for (int i = i0; i < i1; ++i) {
      const double v = P[i];
      P[i] = run;
      run += v;
    }
    if (i1 == L && i0 < i1) P[L] = run;
    if (L == 0 && tid == 0) P[0] = 0.0;
    __syncthreads();
    // complete boxcars starting in this chunk: i < kDetChunk and t0 + i + w <= nsamp;
    // a chunk that holds its whole span has them all
    const int ni = min(kDetChunk, L);
    if (L == span)
      boxcars<NW, false, kSums>(P, ni, L, static_cast<int>(t0), base, inv, bs, bt);
    else
      boxcars<NW, true, kSums>(P, ni, L, static_cast<int>(t0), base, inv, bs, bt);
    __syncthreads();  // the chunk's sums are read before the next load
  }
  if constexpr (kSums) finish_moments();

  // best over the workgroup, per width: largest S/N, then earliest time
  double* rs = sh;
  int* rt = reinterpret_cast<int*>(sh + kDetThreads * NW);
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    // the S/N of the best sum, the same expression as for every start
    rs[k * kDetThreads + tid] = kSums && bt[k] >= 0 ? (bs[k] - snr_base(k, mean)) * snr_scale(k, sd) : bs[k];
    rt[k * kDetThreads + tid] = bt[k];
  }
  __syncthreads();
  if (tid < NW) {
    const int k = tid;
    double v = -INFINITY;
    int tb = -1;
    for (int j = 0; j < kDetThreads; ++j) {
      const double x = rs[k * kDetThreads + j];
      const int tx = rt[k * kDetThreads + j];
      if (tx < 0) continue;
      if (tb < 0 || x > v || (x == v && tx < tb)) {
        v = x;
        tb = tx;
      }
    }
    best_snr[static_cast<int64_t>(d) * NW + k] = v;
    best_t[static_cast<int64_t>(d) * NW + k] = tb;
    if (tb >= 0 && v >= threshold && cand != nullptr) {
      const unsigned idx = atomicAdd(count, 1u);
      if (static_cast<int>(idx) < cap) {
        dedisp_candidate c;
        c.dm_index = d;
        c.width = 1 << k;
        c.time = tb;
        c.snr = static_cast<float>(v);
        cand[idx] = c;
      }
    }
  }
}

__global__ void zero_counter(unsigned* c) { *c = 0u; }

// Raise a detection kernel's dynamic LDS limit to what the widest boxcar set
// needs (once per kernel and device; its static LDS comes on top).
int allow_detect_lds(const void* fn) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, bool> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  std::lock_guard<std::mutex> g(mu);
  const auto key = std::make_pair(fn, dev);
  if (done.count(key)) return DEDISP_OK;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                          static_cast<int>(detect_lds_bytes(kMaxDetectWidths)));
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  done[key] = true;
  return DEDISP_OK;
}

}  // namespace

size_t detect_lds_bytes(int nwidths) {
  const size_t span = kDetChunk + (static_cast<size_t>(1) << (nwidths - 1)) - 1;
  const size_t boxes = (span + 1) * sizeof(double);
  const size_t reduce = static_cast<size_t>(kDetThreads) * nwidths * (sizeof(double) + sizeof(int64_t));
  return boxes > reduce ? boxes : reduce;
}

namespace {

template <typename T, int NW>
int launch_detect(int nrows, const T* out, int64_t nsamp, double threshold, double* stats, double* best_snr,
                  int32_t* best_t, dedisp_candidate* cand, int cap, unsigned* count, hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&detect_rows<T, NW>);
  const int st = allow_detect_lds(fn);
  if (st != DEDISP_OK) return st;
  hipLaunchKernelGGL((detect_rows<T, NW>), dim3(static_cast<unsigned>(nrows)), dim3(kDetThreads),
                     detect_lds_bytes(NW), s, out, nsamp, threshold, stats, best_snr, best_t, cand, cap, count);
  return DEDISP_HIP_STATUS(hipGetLastError());
}

template <typename T>
int launch_detect_any(int nw, int nrows, const T* out, int64_t nsamp, double threshold, double* stats,
                      double* best_snr, int32_t* best_t, dedisp_candidate* cand, int cap, unsigned* count,
                      hipStream_t s) {
  static_assert(kMaxDetectWidths == 12, "one instantiation per number of widths");
#define DEDISP_DETECT_CASE(N) \
  case N:                     \
    return launch_detect<T, N>(nrows, out, nsamp, threshold, stats, best_snr, best_t, cand, cap, count, s);
  switch (nw) {
    DEDISP_DETECT_CASE(1)
    DEDISP_DETECT_CASE(2)
    DEDISP_DETECT_CASE(3)
    DEDISP_DETECT_CASE(4)
    DEDISP_DETECT_CASE(5)
    DEDISP_DETECT_CASE(6)
    DEDISP_DETECT_CASE(7)
    DEDISP_DETECT_CASE(8)
    DEDISP_DETECT_CASE(9)
    DEDISP_DETECT_CASE(10)
    DEDISP_DETECT_CASE(11)
    DEDISP_DETECT_CASE(12)
    default:
      return DEDISP_ERR_INVALID_ARG;
  }
#undef DEDISP_DETECT_CASE
}

}  // namespace

int detect(dedisp_plan p, const void* out, int64_t nsamp, int nwidths, double threshold, double* stats,
           double* best_snr, int32_t* best_t, dedisp_candidate* cand, int cap, unsigned* count, hipStream_t s) {
  if (cand != nullptr) hipLaunchKernelGGL(zero_counter, dim3(1), dim3(1), 0, s, count);
  if (p->dtype == DEDISP_U8)
    return launch_detect_any(nwidths, p->ndm, static_cast<const int32_t*>(out), nsamp, threshold, stats, best_snr,
                             best_t, cand, cap, count, s);
  return launch_detect_any(nwidths, p->ndm, static_cast<const float*>(out), nsamp, threshold, stats, best_snr,
                           best_t, cand, cap, count, s);
}

}  // namespace dedisp

extern "C" int dedisp_detect(dedisp_plan p, const void* out_dev, int64_t nsamp, int nwidths, double threshold,
                             double* stats_dev, double* best_snr_dev, int32_t* best_t_dev,
                             dedisp_candidate* cand_dev, int cand_capacity, uint32_t* cand_count_dev,
                             void* stream) {
  if (p == nullptr || out_dev == nullptr || best_snr_dev == nullptr || best_t_dev == nullptr)
    return DEDISP_ERR_INVALID_ARG;
  if (nsamp < 1 || nsamp > INT32_MAX || nwidths < 1 || nwidths > dedisp::kMaxDetectWidths || !std::isfinite(threshold))
    return DEDISP_ERR_INVALID_ARG;
  if ((reinterpret_cast<uintptr_t>(out_dev) & 3) != 0) return DEDISP_ERR_INVALID_ARG;
  if (cand_dev != nullptr && (cand_capacity < 0 || cand_count_dev == nullptr)) return DEDISP_ERR_INVALID_ARG;
  return dedisp::detect(p, out_dev, nsamp, nwidths, threshold, stats_dev, best_snr_dev, best_t_dev, cand_dev,
                        cand_capacity, reinterpret_cast<unsigned*>(cand_count_dev),
                        static_cast<hipStream_t>(stream));
}

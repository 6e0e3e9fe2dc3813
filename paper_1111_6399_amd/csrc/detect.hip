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
//      width, the earliest time on ties;
//   3. (trial, width) pairs whose best S/N reaches the threshold appended to
//      a candidate list through one atomic counter.
// Values are converted to binary64 on load, so the prefix sums of the int32
// outputs of 8-bit input are exact (below 2^53) and the S/N of both sides of a
// comparison is taken in the same precision.
#include <hip/hip_runtime.h>

#include <cmath>
#include <map>
#include <mutex>

#include "dedisp_internal.h"

namespace dedisp {
namespace {

constexpr int kDetThreads = 256;
constexpr int kDetChunk = 4096;  // boxcar start times per LDS chunk
constexpr int kUnroll = 8;       // global loads in flight per thread

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

template <typename T>
__global__ __launch_bounds__(kDetThreads) void detect_rows(const T* __restrict__ out, int64_t nsamp, int nw,
                                                           double threshold, double* __restrict__ stats,
                                                           double* __restrict__ best_snr,
                                                           int32_t* __restrict__ best_t,
                                                           dedisp_candidate* __restrict__ cand, int cap,
                                                           unsigned* __restrict__ count) {
  extern __shared__ double sh[];  // [kDetChunk + 2^(nw-1)] prefix sums, reused for the reductions
  __shared__ double red[kDetThreads];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int d = blockIdx.x;
  const T* row = out + static_cast<int64_t>(d) * nsamp;

  // moments about the first value (no cancellation for rows far from zero)
  const double k0 = static_cast<double>(row[0]);
  double s1 = 0.0, s2 = 0.0;
  for (int64_t t = tid; t < nsamp; t += kUnroll * kDetThreads) {
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
  const double m1 = block_sum(s1, red) / static_cast<double>(nsamp);
  const double m2 = block_sum(s2, red) / static_cast<double>(nsamp);
  const double mean = k0 + m1;
  const double sd = sqrt(fmax(m2 - m1 * m1, 0.0));
  if (stats != nullptr && tid == 0) {
    stats[2 * d] = mean;
    stats[2 * d + 1] = sd;
  }

  const int W = 1 << (nw - 1);
  const int span = kDetChunk + W - 1;
  double inv[kMaxDetectWidths], base[kMaxDetectWidths];
  double bs[kMaxDetectWidths];
  int64_t bt[kMaxDetectWidths];
#pragma unroll
  for (int k = 0; k < kMaxDetectWidths; ++k) {
    const double w = static_cast<double>(1 << k);
    inv[k] = sd > 0.0 ? 1.0 / (sd * sqrt(w)) : 0.0;
    base[k] = w * mean;
    bs[k] = -INFINITY;
    bt[k] = -1;
  }
  double* P = sh;
  for (int64_t t0 = 0; t0 < nsamp; t0 += kDetChunk) {
    const int L = static_cast<int>(min(static_cast<int64_t>(span), nsamp - t0));  // samples held
    for (int i = tid; i < L; i += kUnroll * kDetThreads) {
      double v[kUnroll];
#pragma unroll
      for (int j = 0; j < kUnroll; ++j) {
        const int u = i + j * kDetThreads;
        v[j] = static_cast<double>(row[t0 + (u < L ? u : L - 1)]);
      }
#pragma unroll
      for (int j = 0; j < kUnroll; ++j)
        if (i + j * kDetThreads < L) P[i + j * kDetThreads] = v[j];
    }
    __syncthreads();
    // in place: P[i] = sum of the chunk's samples before i, P[L] = all of them
    const int seg = (L + kDetThreads - 1) / kDetThreads;
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
    // complete boxcars starting in this chunk: i < kDetChunk and t0 + i + w <= nsamp
    const int ni = min(kDetChunk, L);
    for (int i = tid; i < ni; i += kDetThreads) {
      const double p0 = P[i];
      // fully unrolled (uniform guards only), so that bs/bt stay in registers
#pragma unroll
      for (int k = 0; k < kMaxDetectWidths; ++k) {
        if (k < nw) {
          const int w = 1 << k;
          const bool fits = i + w <= L;  // a complete boxcar
          const double snr = (P[fits ? i + w : L] - p0 - base[k]) * inv[k];
          if (fits && snr > bs[k]) {  // times increase along a thread, so the first of equals stays
            bs[k] = snr;
            bt[k] = t0 + i;
          }
        }
      }
    }
    __syncthreads();  // the chunk's sums are read before the next load
  }

  // best over the workgroup, per width: largest S/N, then earliest time
  double* rs = sh;
  int64_t* rt = reinterpret_cast<int64_t*>(sh + kDetThreads * nw);
#pragma unroll
  for (int k = 0; k < kMaxDetectWidths; ++k) {
    if (k < nw) {
      rs[k * kDetThreads + tid] = bs[k];
      rt[k * kDetThreads + tid] = bt[k];
    }
  }
  __syncthreads();
  if (tid < nw) {
    const int k = tid;
    double v = -INFINITY;
    int64_t tb = -1;
    for (int j = 0; j < kDetThreads; ++j) {
      const double x = rs[k * kDetThreads + j];
      const int64_t tx = rt[k * kDetThreads + j];
      if (tx < 0) continue;
      if (tb < 0 || x > v || (x == v && tx < tb)) {
        v = x;
        tb = tx;
      }
    }
    best_snr[static_cast<int64_t>(d) * nw + k] = v;
    best_t[static_cast<int64_t>(d) * nw + k] = static_cast<int32_t>(tb);
    if (tb >= 0 && v >= threshold && cand != nullptr) {
      const unsigned idx = atomicAdd(count, 1u);
      if (static_cast<int>(idx) < cap) {
        dedisp_candidate c;
        c.dm_index = d;
        c.width = 1 << k;
        c.time = static_cast<int32_t>(tb);
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

int detect(dedisp_plan p, const void* out, int64_t nsamp, int nwidths, double threshold, double* stats,
           double* best_snr, int32_t* best_t, dedisp_candidate* cand, int cap, unsigned* count, hipStream_t s) {
  const size_t lds = detect_lds_bytes(nwidths);
  if (cand != nullptr) hipLaunchKernelGGL(zero_counter, dim3(1), dim3(1), 0, s, count);
  if (p->dtype == DEDISP_U8) {
    const void* fn = reinterpret_cast<const void*>(&detect_rows<int32_t>);
    int st = allow_detect_lds(fn);
    if (st != DEDISP_OK) return st;
    hipLaunchKernelGGL(detect_rows<int32_t>, dim3(p->ndm), dim3(kDetThreads), lds, s,
                       static_cast<const int32_t*>(out), nsamp, nwidths, threshold, stats, best_snr, best_t, cand,
                       cap, count);
  } else {
    const void* fn = reinterpret_cast<const void*>(&detect_rows<float>);
    int st = allow_detect_lds(fn);
    if (st != DEDISP_OK) return st;
    hipLaunchKernelGGL(detect_rows<float>, dim3(p->ndm), dim3(kDetThreads), lds, s, static_cast<const float*>(out),
                       nsamp, nwidths, threshold, stats, best_snr, best_t, cand, cap, count);
  }
  return DEDISP_HIP_STATUS(hipGetLastError());
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

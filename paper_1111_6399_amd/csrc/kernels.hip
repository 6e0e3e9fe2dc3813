// De-dispersion kernels for gfx950 (CDNA4) and the variant registry.
//
// Every kernel computes out[d][t] = sum_c in[c][t + shift[c][d]] (the paper's
// brute-force search: each channel shifted by its delay for every trial, then
// integrated over frequency).  Float sums follow one fixed order (channels
// ascending, in blocks of kChanBlock, each block summed into a partial that is
// added to the total), so every variant gives bit-identical float results.
//
// Mapping to the paper's three requirements (section "Acceleration via GPU
// computing"):
//  (i)  accumulators in the fastest memory: per-lane registers, several trials
//       x several samples per lane (a rectangle of (DM, t) per workgroup);
//  (ii) the right (f, t) data on chip: each workgroup stages, channel by
//       channel, the window of samples its tile of trials needs into LDS, so a
//       sample fetched once from HBM/L2 serves every trial of the tile;
//  (iii) few operations for the shift: delays are read from a precomputed
//       table with scalar (wave-uniform) loads, no arithmetic per lane.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "dedisp_internal.h"

namespace dedisp {
namespace {

// ---------------------------------------------------------------- loads --

template <typename T>
struct Elem;
template <>
struct Elem<float> {
  static __device__ __forceinline__ float get(const float* p, int64_t i) { return p[i]; }
};
template <>
struct Elem<__half> {
  static __device__ __forceinline__ float get(const __half* p, int64_t i) { return __half2float(p[i]); }
};
template <>
struct Elem<uint8_t> {
  static __device__ __forceinline__ float get(const uint8_t* p, int64_t i) { return static_cast<float>(p[i]); }
};

// Four consecutive samples starting at element i (i a multiple of 4, so the
// vector load is naturally aligned for a 16-byte aligned buffer) plus the
// fifth; elements at or past `total` read as zero.
template <typename T>
__device__ __forceinline__ void load5(const T* __restrict__ p, int64_t i, int64_t total, float4& v, float& e) {
  if (i + 4 < total) {
    if constexpr (sizeof(T) == 4) {
      v = *reinterpret_cast<const float4*>(p + i);
    } else if constexpr (sizeof(T) == 2) {
      const uint2 raw = *reinterpret_cast<const uint2*>(p + i);
      const __half2 lo = *reinterpret_cast<const __half2*>(&raw.x);
      const __half2 hi = *reinterpret_cast<const __half2*>(&raw.y);
      v = make_float4(__low2float(lo), __high2float(lo), __low2float(hi), __high2float(hi));
    } else {
      const uint32_t raw = *reinterpret_cast<const uint32_t*>(p + i);
      v = make_float4(static_cast<float>(raw & 0xffu), static_cast<float>((raw >> 8) & 0xffu),
                      static_cast<float>((raw >> 16) & 0xffu), static_cast<float>(raw >> 24));
    }
    e = Elem<T>::get(p, i + 4);
  } else {
    v.x = i < total ? Elem<T>::get(p, i) : 0.f;
    v.y = i + 1 < total ? Elem<T>::get(p, i + 1) : 0.f;
    v.z = i + 2 < total ? Elem<T>::get(p, i + 2) : 0.f;
    v.w = i + 3 < total ? Elem<T>::get(p, i + 3) : 0.f;
    e = i + 4 < total ? Elem<T>::get(p, i + 4) : 0.f;
  }
}

// ------------------------------------------------------------ direct --

// One lane per output sample.  The reference-simple variant, also the
// fallback for plans whose delay spread does not fit any tiled variant.
template <typename In>
__global__ __launch_bounds__(256) void dedisp_direct(const In* __restrict__ in, int64_t pitch,
                                                     void* __restrict__ out_v, int64_t nsamp,
                                                     const int32_t* __restrict__ shift, int ndm_pad,
                                                     int nchans, int64_t tblocks) {
  const int64_t bid = blockIdx.x;
  const int d = static_cast<int>(bid / tblocks);
  const int64_t t = (bid % tblocks) * 256 + threadIdx.x;
  if (t >= nsamp) return;
  const int32_t* sh = shift + d;
  if constexpr (sizeof(In) == 1) {
    int32_t acc = 0;
    for (int c = 0; c < nchans; ++c)
      acc += static_cast<int32_t>(in[c * pitch + t + sh[static_cast<int64_t>(c) * ndm_pad]]);
    static_cast<int32_t*>(out_v)[d * nsamp + t] = acc;
  } else {
    float tot = 0.f;
    for (int c0 = 0; c0 < nchans; c0 += kChanBlock) {
      const int c1 = min(nchans, c0 + kChanBlock);
      float part = 0.f;
      for (int c = c0; c < c1; ++c)
        part += Elem<In>::get(in, c * pitch + t + sh[static_cast<int64_t>(c) * ndm_pad]);
      tot += part;
    }
    static_cast<float*>(out_v)[d * nsamp + t] = tot;
  }
}

// ------------------------------------------------------------- tiled --

// Workgroup tile: WD*DW trials x WT*128*KS samples.  Wave (wd, wt) owns DW
// trials and 128*KS samples; lane l owns samples 2l, 2l+1 (+128k).
//
// Per channel the workgroup stages the window of input its tile needs into
// LDS twice: copy0[j] = x[a0 + j] and copy1[j] = x[a0 + j + 1], both 8-byte
// aligned, so a trial with either parity of delay reads its samples as
// naturally aligned 64-bit pairs (misaligned 64-bit LDS reads are more than
// an order of magnitude slower on this chip).
//
// Tiles are numbered so that the workgroups an XCD runs (block i runs on XCD
// i mod 8) take consecutive trial tiles of the same time tile: their windows
// overlap, so that XCD's L2 serves most of the staging traffic.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
  const int xcd = bid & 7;
  const int idx = bid >> 3;
  const int q = nblocks >> 3, r = nblocks & 7;
  return xcd * q + min(xcd, r) + idx;
}

template <typename In, int DW, int KS, int WD, int WT>
__global__ __launch_bounds__(64 * WD * WT) void dedisp_tiled(
    const In* __restrict__ in, int64_t pitch, int64_t total, void* __restrict__ out_v, int64_t nsamp, int ndm,
    const int32_t* __restrict__ shift, int ndm_pad, int nchans, const int2* __restrict__ win, int cap,
    int n_dm_tiles) {
  constexpr int NT = 64 * WD * WT;
  constexpr int T = 128 * KS * WT;
  extern __shared__ float4 lds4[];
  float4* copy0_4 = lds4;
  float4* copy1_4 = lds4 + (cap >> 2);
  const float2* copy0_2 = reinterpret_cast<const float2*>(copy0_4);
  const float2* copy1_2 = reinterpret_cast<const float2*>(copy1_4);

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int wd = wave % WD;
  const int wt = wave / WD;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int dm_tile = tile % n_dm_tiles;
  const int t_tile = tile / n_dm_tiles;
  const int64_t t0 = static_cast<int64_t>(t_tile) * T;
  const int dw0 = dm_tile * (DW * WD) + wd * DW;
  const int tw = wt * 128 * KS;

  float part[DW][2 * KS];
  float tot[DW][2 * KS];
#pragma unroll
  for (int j = 0; j < DW; ++j)
#pragma unroll
    for (int k = 0; k < 2 * KS; ++k) {
      part[j][k] = 0.f;
      tot[j][k] = 0.f;
    }

  const int2* wrow = win + static_cast<int64_t>(dm_tile) * nchans;
  for (int c = 0; c < nchans; ++c) {
    const int2 mm = wrow[c];
    const int64_t g0 = static_cast<int64_t>(c) * pitch + t0 + mm.x;
    const int64_t a0 = g0 & ~static_cast<int64_t>(3);
    const int mis = static_cast<int>(g0 - a0);
    const int len = mis + T + (mm.y - mm.x);
    const int n4 = (len + 3) >> 2;
    __syncthreads();
    for (int i = tid; i < n4; i += NT) {
      float4 v;
      float e;
      load5(in, a0 + 4 * static_cast<int64_t>(i), total, v, e);
      copy0_4[i] = v;
      copy1_4[i] = make_float4(v.y, v.z, v.w, e);
    }
    __syncthreads();
    const int32_t* srow = shift + static_cast<int64_t>(c) * ndm_pad + dw0;
#pragma unroll
    for (int j = 0; j < DW; ++j) {
      const int s = srow[j];
      const int r = mis + (s - mm.x) + tw;
      const float2* b = (r & 1) ? (copy1_2 + ((r - 1) >> 1)) : (copy0_2 + (r >> 1));
#pragma unroll
      for (int k = 0; k < KS; ++k) {
        const float2 v = b[lane + 64 * k];
        part[j][2 * k] += v.x;
        part[j][2 * k + 1] += v.y;
      }
    }
    if (((c + 1) % kChanBlock) == 0 || c + 1 == nchans) {
#pragma unroll
      for (int j = 0; j < DW; ++j)
#pragma unroll
        for (int k = 0; k < 2 * KS; ++k) {
          tot[j][k] += part[j][k];
          part[j][k] = 0.f;
        }
    }
  }

#pragma unroll
  for (int j = 0; j < DW; ++j) {
    const int d = dw0 + j;
    if (d >= ndm) break;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int64_t t = t0 + tw + 2 * lane + 128 * k;
      if (t + 1 < nsamp) {
        if constexpr (sizeof(In) == 1) {
          int32_t* o = static_cast<int32_t*>(out_v) + d * nsamp + t;
          const int2 w = make_int2(static_cast<int32_t>(tot[j][2 * k]), static_cast<int32_t>(tot[j][2 * k + 1]));
          __builtin_memcpy(o, &w, 8);
        } else {
          float* o = static_cast<float*>(out_v) + d * nsamp + t;
          const float2 w = make_float2(tot[j][2 * k], tot[j][2 * k + 1]);
          __builtin_memcpy(o, &w, 8);
        }
      } else if (t < nsamp) {
        if constexpr (sizeof(In) == 1)
          static_cast<int32_t*>(out_v)[d * nsamp + t] = static_cast<int32_t>(tot[j][2 * k]);
        else
          static_cast<float*>(out_v)[d * nsamp + t] = tot[j][2 * k];
      }
    }
  }
}

// ----------------------------------------------------------- registry --

using TiledFn = void (*)(const void*, int64_t, int64_t, void*, int64_t, int, const int32_t*, int, int,
                         const int2*, int, int);

struct Variant {
  TileShape shape;
  const void* fn[3];  // by dtype: U8, F16, F32
};

#define DEDISP_VARIANT(DW, KS, WD, WT)                                                              \
  Variant {                                                                                        \
    TileShape{DW, KS, WD, WT}, {                                                                   \
      reinterpret_cast<const void*>(&dedisp_tiled<uint8_t, DW, KS, WD, WT>),                        \
          reinterpret_cast<const void*>(&dedisp_tiled<__half, DW, KS, WD, WT>),                     \
          reinterpret_cast<const void*>(&dedisp_tiled<float, DW, KS, WD, WT>)                       \
    }                                                                                              \
  }

const Variant kVariants[] = {
    DEDISP_VARIANT(4, 4, 4, 2),   // 16 trials x 1024 samples, 512 threads
    DEDISP_VARIANT(4, 4, 8, 1),   // 32 x 512
    DEDISP_VARIANT(4, 8, 4, 2),   // 16 x 2048
    DEDISP_VARIANT(4, 8, 8, 1),   // 32 x 1024
    DEDISP_VARIANT(8, 4, 4, 2),   // 32 x 1024
    DEDISP_VARIANT(2, 8, 4, 4),   // 8 x 4096
    DEDISP_VARIANT(4, 4, 4, 1),   // 16 x 512, 256 threads
};
constexpr int kNumTiled = sizeof(kVariants) / sizeof(kVariants[0]);

constexpr size_t kMaxLds = 160 * 1024;

// Floats per LDS copy a tiled variant needs for this plan, or 0 if too many.
int lds_cap(dedisp_plan p, const TileShape& s) {
  const std::vector<int2>& w = host_windows(p, s.dms());
  int spread = 0;
  for (const int2& x : w) spread = std::max(spread, x.y - x.x);
  const int64_t cap = (static_cast<int64_t>(s.samples()) + spread + 3 + 4 + 3) / 4 * 4;
  if (2 * cap * 4 > static_cast<int64_t>(kMaxLds)) return 0;
  return static_cast<int>(cap);
}

}  // namespace

int variant_count() { return 1 + kNumTiled; }

TileShape variant_shape(int v) { return kVariants[v - 1].shape; }

bool variant_fits(dedisp_plan p, int v) {
  if (v == 0) return true;
  if (v < 0 || v > kNumTiled) return false;
  return lds_cap(p, kVariants[v - 1].shape) > 0;
}

int default_variant(dedisp_plan p) {
  static const int order[] = {3, 1, 2, 4, 5, 6, 7};
  for (int v : order)
    if (v <= kNumTiled && variant_fits(p, v)) return v;
  return 0;
}

int launch(dedisp_plan p, int v, const void* in, void* out, int64_t nsamp, hipStream_t s) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e);
  DeviceTables* dt = nullptr;
  int st = device_tables(p, dev, &dt);
  if (st != DEDISP_OK) return st;
  const int64_t pitch = nsamp + p->max_shift;
  const int64_t total = pitch * p->nchans;
  if (v == 0) {
    const int64_t tblocks = (nsamp + 255) / 256;
    const int64_t nblocks = tblocks * p->ndm;
    if (nblocks > INT32_MAX) return DEDISP_ERR_INVALID_ARG;
    switch (p->dtype) {
      case DEDISP_U8:
        hipLaunchKernelGGL(dedisp_direct<uint8_t>, dim3(static_cast<unsigned>(nblocks)), dim3(256), 0, s,
                           static_cast<const uint8_t*>(in), pitch, out, nsamp, dt->shift, p->ndm_pad, p->nchans,
                           tblocks);
        break;
      case DEDISP_F16:
        hipLaunchKernelGGL(dedisp_direct<__half>, dim3(static_cast<unsigned>(nblocks)), dim3(256), 0, s,
                           static_cast<const __half*>(in), pitch, out, nsamp, dt->shift, p->ndm_pad, p->nchans,
                           tblocks);
        break;
      default:
        hipLaunchKernelGGL(dedisp_direct<float>, dim3(static_cast<unsigned>(nblocks)), dim3(256), 0, s,
                           static_cast<const float*>(in), pitch, out, nsamp, dt->shift, p->ndm_pad, p->nchans,
                           tblocks);
    }
    return hip_status(hipGetLastError());
  }
  if (v < 0 || v > kNumTiled) return DEDISP_ERR_INVALID_ARG;
  const Variant& var = kVariants[v - 1];
  const int cap = lds_cap(p, var.shape);
  if (cap == 0) return DEDISP_ERR_INVALID_ARG;
  const int2* win = nullptr;
  st = device_windows(p, dev, var.shape.dms(), &win);
  if (st != DEDISP_OK) return st;
  const int n_dm_tiles = (p->ndm + var.shape.dms() - 1) / var.shape.dms();
  const int64_t n_t_tiles = (nsamp + var.shape.samples() - 1) / var.shape.samples();
  const int64_t nblocks = n_t_tiles * n_dm_tiles;
  if (nblocks > INT32_MAX) return DEDISP_ERR_INVALID_ARG;
  const size_t lds = 2 * static_cast<size_t>(cap) * 4;
  const void* fn = var.fn[p->dtype];
  if (lds > 64 * 1024) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kMaxLds));
    if (e != hipSuccess) return hip_status(e);
  }
  int ndm = p->ndm, ndm_pad = p->ndm_pad, nchans = p->nchans;
  const int32_t* sh = dt->shift;
  void* args[] = {const_cast<void**>(&in), (void*)&pitch, (void*)&total, &out, (void*)&nsamp, &ndm,
                  (void*)&sh, &ndm_pad, &nchans, (void*)&win, (void*)&cap, (void*)&n_dm_tiles};
  e = hipLaunchKernel(fn, dim3(static_cast<unsigned>(nblocks)), dim3(var.shape.threads()), args, lds, s);
  return hip_status(e);
}

}  // namespace dedisp

extern "C" int dedisp_variant_count(void) { return dedisp::variant_count(); }

extern "C" int dedisp_variant_describe(int v, int* dms, int* samples, int* threads) {
  if (v < 0 || v >= dedisp::variant_count()) return DEDISP_ERR_INVALID_ARG;
  if (v == 0) {
    if (dms) *dms = 1;
    if (samples) *samples = 256;
    if (threads) *threads = 256;
    return DEDISP_OK;
  }
  const dedisp::TileShape s = dedisp::variant_shape(v);
  if (dms) *dms = s.dms();
  if (samples) *samples = s.samples();
  if (threads) *threads = s.threads();
  return DEDISP_OK;
}

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

// Raw (unconverted) staging registers: four consecutive samples plus the fifth.
// Kept raw until they are written to LDS so that the load latency overlaps
// the previous channel's accumulation.
template <typename T>
struct Raw;
template <>
struct Raw<float> {
  float4 v;
  float e;
};
template <>
struct Raw<__half> {
  uint2 v;
  unsigned short e;
};
template <>
struct Raw<uint8_t> {
  uint32_t v;
  uint32_t e;
};

// Staging loads go through a buffer resource that covers exactly the
// channel's window: lanes past the window, and a window that runs past the end
// of the input, read zeros from the range check instead of touching memory.
// Every thread issues the same number of loads per channel whatever the
// window length, so the compiler can count them and wait for exactly the
// channel it is about to consume while the later channels stay in flight.
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ void load_raw(__amdgpu_buffer_rsrc_t rs, int i, Raw<T>& r) {
  if constexpr (sizeof(T) == 4) {
    const v4i v = __builtin_amdgcn_raw_buffer_load_b128(rs, 16 * i, 0, 0);
    r.v = make_float4(__int_as_float(v.x), __int_as_float(v.y), __int_as_float(v.z), __int_as_float(v.w));
    r.e = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, 16 * i + 16, 0, 0));
  } else if constexpr (sizeof(T) == 2) {
    const v2i v = __builtin_amdgcn_raw_buffer_load_b64(rs, 8 * i, 0, 0);
    r.v = make_uint2(static_cast<uint32_t>(v.x), static_cast<uint32_t>(v.y));
    r.e = static_cast<unsigned short>(__builtin_amdgcn_raw_buffer_load_b16(rs, 8 * i + 8, 0, 0));
  } else {
    r.v = static_cast<uint32_t>(__builtin_amdgcn_raw_buffer_load_b32(rs, 4 * i, 0, 0));
    r.e = static_cast<uint32_t>(__builtin_amdgcn_raw_buffer_load_b8(rs, 4 * i + 4, 0, 0));
  }
}

__device__ __forceinline__ float h2f(uint32_t bits) { return __half2float(__ushort_as_half(static_cast<unsigned short>(bits))); }

template <typename T>
__device__ __forceinline__ void to_float(const Raw<T>& r, float4& v, float& e) {
  if constexpr (sizeof(T) == 4) {
    v = r.v;
    e = r.e;
  } else if constexpr (sizeof(T) == 2) {
    v = make_float4(h2f(r.v.x & 0xffffu), h2f(r.v.x >> 16), h2f(r.v.y & 0xffffu), h2f(r.v.y >> 16));
    e = h2f(r.e);
  } else {
    v = make_float4(static_cast<float>(r.v & 0xffu), static_cast<float>((r.v >> 8) & 0xffu),
                    static_cast<float>((r.v >> 16) & 0xffu), static_cast<float>(r.v >> 24));
    e = static_cast<float>(r.e);
  }
}

// Barrier that orders LDS traffic only: global loads issued before it stay in
// flight (a full __syncthreads() would also wait for every outstanding global
// load, i.e. for the prefetch of the next channels).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Block i of a launch runs on XCD i mod 8.  xcd_rank() renumbers blocks so
// that each XCD takes one contiguous run of logical indices.
__device__ __forceinline__ int xcd_rank(int bid, int nblocks) {
  const int xcd = bid & 7;
  const int idx = bid >> 3;
  const int q = nblocks >> 3, r = nblocks & 7;
  return xcd * q + min(xcd, r) + idx;
}

// Read-only tables are read through the constant address space so that the
// wave-uniform reads become scalar loads (s_load): they then neither occupy
// vector registers nor wait behind the outstanding global loads of the
// staging pipeline.
typedef __attribute__((address_space(4))) const int32_t cint32;

struct TiledArgs {
  const void* in;
  int64_t pitch;  // samples per input row (nsamp + max_shift)
  int64_t total;  // samples in the input buffer
  void* out;
  int64_t nsamp;
  const int32_t* shift;  // [nchans][ndm_pad]
  const int2* win;       // [n_dm_tiles][nchans] (min, max) delay
  int ndm, ndm_pad, nchans;
  int cap;  // floats per LDS copy
  int n_dm_tiles, n_t_tiles;
  int gd, gt;        // tiles per group along trials and time
  int n_dm_groups;   // groups along trials
};

// Logical tile of this block.  Consecutive logical indices form groups of
// gd trial tiles x gt time tiles; an XCD runs whole groups at a time, and the
// windows of a group overlap (neighbouring trial tiles share the top of the
// band, neighbouring time tiles share the delay spread at the bottom), so the
// XCD's L2 serves most of the staging traffic.
__device__ __forceinline__ bool tile_of(const TiledArgs& a, int& dm_tile, int& t_tile) {
  const int l = xcd_rank(blockIdx.x, gridDim.x);
  const int bs = a.gd * a.gt;
  const int g = l / bs;
  const int i = l - g * bs;
  const int gdm = g % a.n_dm_groups;
  const int gtm = g / a.n_dm_groups;
  dm_tile = gdm * a.gd + i % a.gd;
  t_tile = gtm * a.gt + i / a.gd;
  return dm_tile < a.n_dm_tiles && t_tile < a.n_t_tiles;
}

struct Geo {
  int64_t a0;  // first staged element (multiple of 4)
  int mis;     // offset of the window start past a0
  int n4;      // float4 groups staged
  int lo;      // smallest delay of the tile at this channel
};

// Workgroup tile: WD*DW trials x WT*128*KS samples.  Wave (wd, wt) owns DW
// trials and 128*KS samples; lane l owns samples 2l, 2l+1 (+128k).
//
// Per channel the workgroup stages the window of input its tile needs into
// LDS twice: copy0[j] = x[a0 + j] and copy1[j] = x[a0 + j + 1], both 8-byte
// aligned, so a trial with either parity of delay reads its samples as
// naturally aligned 64-bit pairs (misaligned 64-bit LDS reads are more than
// an order of magnitude slower on this chip).  Two such buffers alternate,
// with one barrier per channel.  The global loads run P channels ahead of
// the accumulation, in P register sets of R float4 slots per thread.
template <typename In, int DW, int KS, int WD, int WT, int R, int P>
__global__ __launch_bounds__(64 * WD * WT) void dedisp_tiled(const TiledArgs a) {
  constexpr int NT = 64 * WD * WT;
  constexpr int T = 128 * KS * WT;
  extern __shared__ float4 lds4[];
  const In* __restrict__ in = static_cast<const In*>(a.in);
  const int q = a.cap >> 2;  // float4 per copy

  int dm_tile, t_tile;
  if (!tile_of(a, dm_tile, t_tile)) return;  // padding block of the last group
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int wd = wave % WD;
  const int wt = wave / WD;
  const int64_t t0 = static_cast<int64_t>(t_tile) * T;
  const int dw0 = dm_tile * (DW * WD) + wd * DW;
  const int tw = wt * 128 * KS;
  cint32* wrow = (cint32*)(a.win) + 2 * static_cast<int64_t>(dm_tile) * a.nchans;
  const int nchans = a.nchans;

  auto geo = [&](int c) {
    const int2 mm = make_int2(wrow[2 * c], wrow[2 * c + 1]);
    Geo g;
    const int64_t g0 = static_cast<int64_t>(c) * a.pitch + t0 + mm.x;
    g.a0 = g0 & ~static_cast<int64_t>(3);
    g.mis = static_cast<int>(g0 - g.a0);
    g.n4 = (g.mis + T + (mm.y - mm.x) + 3) >> 2;
    g.lo = mm.x;
    return g;
  };

  // Global loads of one channel's window into a register set.  `live` false
  // issues the same instructions against an empty range (they return zeros
  // without touching memory), so that every iteration issues the same number
  // of loads and the waits stay exact.
  auto issue = [&](const Geo& g, Raw<In>* rs, bool live) {
    const int64_t avail = (a.total - g.a0) * static_cast<int64_t>(sizeof(In));
    const int64_t need = (4 * static_cast<int64_t>(g.n4) + 1) * static_cast<int64_t>(sizeof(In));
    const int num = live ? static_cast<int>(min(avail, need)) : 0;
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<In*>(in + g.a0), 0, num, 0x00020000);
#pragma unroll
    for (int r = 0; r < R; ++r) load_raw(rsrc, tid + r * NT, rs[r]);
  };

  float part[DW][2 * KS];
  float tot[DW][2 * KS];
#pragma unroll
  for (int j = 0; j < DW; ++j)
#pragma unroll
    for (int k = 0; k < 2 * KS; ++k) {
      part[j][k] = 0.f;
      tot[j][k] = 0.f;
    }

  Raw<In> raw[P][R];
  Geo gq[P];
#pragma unroll
  for (int u = 0; u < P; ++u) {
    gq[u] = geo(min(u, nchans - 1));
    issue(gq[u], raw[u], u < nchans);
  }

  for (int cb = 0; cb < nchans; cb += P) {
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const int c = cb + u;
      float4* copy0_4 = lds4 + (c & 1) * 2 * q;
      float4* copy1_4 = copy0_4 + q;
      const Geo g = gq[u];
      // hand the window of channel c to LDS (past the last channel this
      // writes zeros that nobody reads)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = tid + r * NT;
        if (i < g.n4) {
          float4 v;
          float e;
          to_float(raw[u][r], v, e);
          copy0_4[i] = v;
          copy1_4[i] = make_float4(v.y, v.z, v.w, e);
        }
      }
      gq[u] = geo(min(c + P, nchans - 1));
      issue(gq[u], raw[u], c + P < nchans);
      lds_barrier();
      if (c >= nchans) continue;

      const float2* copy0_2 = reinterpret_cast<const float2*>(copy0_4);
      const float2* copy1_2 = reinterpret_cast<const float2*>(copy1_4);
      cint32* srow = (cint32*)(a.shift) + static_cast<int64_t>(c) * a.ndm_pad + dw0;
#pragma unroll
      for (int j = 0; j < DW; ++j) {
        const int s = srow[j];
        const int rr = g.mis + (s - g.lo) + tw;
        const float2* b = (rr & 1) ? (copy1_2 + ((rr - 1) >> 1)) : (copy0_2 + (rr >> 1));
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
  }

  const int64_t nsamp = a.nsamp;
#pragma unroll
  for (int j = 0; j < DW; ++j) {
    const int d = dw0 + j;
    if (d >= a.ndm) break;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int64_t t = t0 + tw + 2 * lane + 128 * k;
      if (t + 1 < nsamp) {
        if constexpr (sizeof(In) == 1) {
          int32_t* o = static_cast<int32_t*>(a.out) + d * nsamp + t;
          const int2 w = make_int2(static_cast<int32_t>(tot[j][2 * k]), static_cast<int32_t>(tot[j][2 * k + 1]));
          __builtin_memcpy(o, &w, 8);
        } else {
          float* o = static_cast<float*>(a.out) + d * nsamp + t;
          const float2 w = make_float2(tot[j][2 * k], tot[j][2 * k + 1]);
          __builtin_memcpy(o, &w, 8);
        }
      } else if (t < nsamp) {
        if constexpr (sizeof(In) == 1)
          static_cast<int32_t*>(a.out)[d * nsamp + t] = static_cast<int32_t>(tot[j][2 * k]);
        else
          static_cast<float*>(a.out)[d * nsamp + t] = tot[j][2 * k];
      }
    }
  }
}

// ----------------------------------------------------------- registry --

struct Variant {
  TileShape shape;
  int r;              // staging float4 slots per thread
  int p;              // channels of prefetch
  const void* fn[3];  // by dtype: U8, F16, F32
};

#define DEDISP_VARIANT(DW, KS, WD, WT, R, P)                                                        \
  Variant {                                                                                        \
    TileShape{DW, KS, WD, WT}, R, P, {                                                             \
      reinterpret_cast<const void*>(&dedisp_tiled<uint8_t, DW, KS, WD, WT, R, P>),                  \
          reinterpret_cast<const void*>(&dedisp_tiled<__half, DW, KS, WD, WT, R, P>),               \
          reinterpret_cast<const void*>(&dedisp_tiled<float, DW, KS, WD, WT, R, P>)                 \
    }                                                                                              \
  }

const Variant kVariants[] = {
    DEDISP_VARIANT(2, 4, 8, 2, 2, 4),  // 16 trials x 1024 samples, 1024 threads
    DEDISP_VARIANT(2, 4, 4, 4, 2, 4),  // 8 x 2048, 1024 threads
    DEDISP_VARIANT(1, 8, 16, 1, 2, 4), // 16 x 1024, 1024 threads
    DEDISP_VARIANT(2, 8, 8, 2, 1, 4),  // 16 x 2048, 1024 threads
    DEDISP_VARIANT(4, 4, 4, 2, 4, 4),  // 16 x 1024, 512 threads
    DEDISP_VARIANT(2, 8, 4, 2, 4, 4),  // 8 x 2048, 512 threads
    DEDISP_VARIANT(4, 4, 8, 1, 4, 4),  // 32 x 512, 512 threads
    DEDISP_VARIANT(2, 4, 16, 1, 2, 4), // 32 x 512, 1024 threads
};
constexpr int kNumTiled = sizeof(kVariants) / sizeof(kVariants[0]);

constexpr size_t kMaxLds = 160 * 1024;

// Floats per LDS copy a tiled variant needs for this plan (4 copies live:
// two alignments x two buffers), or 0 if the plan's delay spread is too wide
// for the variant's LDS or staging registers.
int lds_cap(dedisp_plan p, const Variant& v) {
  const std::vector<int2>& w = host_windows(p, v.shape.dms());
  int spread = 0;
  for (const int2& x : w) spread = std::max(spread, x.y - x.x);
  const int64_t n4 = (3 + static_cast<int64_t>(v.shape.samples()) + spread + 3) / 4;
  if (n4 > static_cast<int64_t>(v.r) * v.shape.threads()) return 0;
  const int64_t cap = 4 * n4;
  if (4 * cap * 4 > static_cast<int64_t>(kMaxLds)) return 0;
  return static_cast<int>(cap);
}

}  // namespace

int variant_count() { return 1 + kNumTiled; }

TileShape variant_shape(int v) { return kVariants[v - 1].shape; }

bool variant_fits(dedisp_plan p, int v) {
  if (v == 0) return true;
  if (v < 0 || v > kNumTiled) return false;
  return lds_cap(p, kVariants[v - 1]) > 0;
}

int default_variant(dedisp_plan p) {
  static const int order[] = {4, 1, 3, 2, 5, 6, 7, 8};
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
  const int cap = lds_cap(p, var);
  if (cap == 0) return DEDISP_ERR_INVALID_ARG;
  const int2* win = nullptr;
  st = device_windows(p, dev, var.shape.dms(), &win);
  if (st != DEDISP_OK) return st;
  TiledArgs a;
  a.in = in;
  a.pitch = pitch;
  a.total = total;
  a.out = out;
  a.nsamp = nsamp;
  a.shift = dt->shift;
  a.win = win;
  a.ndm = p->ndm;
  a.ndm_pad = p->ndm_pad;
  a.nchans = p->nchans;
  a.cap = cap;
  a.n_dm_tiles = (p->ndm + var.shape.dms() - 1) / var.shape.dms();
  const int64_t n_t_tiles = (nsamp + var.shape.samples() - 1) / var.shape.samples();
  if (n_t_tiles > INT32_MAX / 64) return DEDISP_ERR_INVALID_ARG;
  a.n_t_tiles = static_cast<int>(n_t_tiles);
  // groups of up to 8 trial tiles x 4 time tiles (one per CU of an XCD)
  a.gd = std::min(8, a.n_dm_tiles);
  a.gt = std::min(4, a.n_t_tiles);
  a.n_dm_groups = (a.n_dm_tiles + a.gd - 1) / a.gd;
  const int64_t n_groups = static_cast<int64_t>(a.n_dm_groups) * ((a.n_t_tiles + a.gt - 1) / a.gt);
  // a multiple of 8 groups, so that every XCD's run of blocks is whole groups
  const int64_t nblocks = (n_groups + 7) / 8 * 8 * a.gd * a.gt;
  if (nblocks > INT32_MAX) return DEDISP_ERR_INVALID_ARG;
  const size_t lds = 4 * static_cast<size_t>(cap) * 4;
  const void* fn = var.fn[p->dtype];
  if (lds > 64 * 1024) {
    e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kMaxLds));
    if (e != hipSuccess) return hip_status(e);
  }
  void* args[] = {&a};
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

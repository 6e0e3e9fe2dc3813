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
#include <type_traits>

#include "dedisp_internal.h"

namespace dedisp {
namespace {

// Read-only tables are read through the constant address space so that the
// wave-uniform reads become scalar loads (s_load): they then neither occupy
// vector registers nor wait behind the outstanding vector loads of the
// staging pipeline.
typedef __attribute__((address_space(4))) const int32_t cint32;

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
  if constexpr (std::is_integral<In>::value) {  // 8-bit samples, or 8-bit samples staged as 16-bit
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

// Raw (unconverted) staging registers: four consecutive samples.  Kept raw
// until they are written to LDS so that the load latency overlaps the
// accumulation of earlier channels.
template <typename T>
struct Raw;
template <>
struct Raw<float> {
  float4 v;
};
template <>
struct Raw<__half> {
  uint2 v;
};
template <>
struct Raw<uint8_t> {
  uint32_t v;
};

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v2i __attribute__((ext_vector_type(2)));

// Staging loads go through a buffer resource that covers exactly the part of
// the channel's window that lies in whole 4-sample groups of the input: lanes
// past the window read zeros from the range check instead of touching memory.
// Every thread issues the same number of loads per channel whatever the
// window length, so the compiler can count them and wait for exactly the
// channel it is about to consume while later channels stay in flight.
template <typename T>
__device__ __forceinline__ Raw<T> load_raw(__amdgpu_buffer_rsrc_t rs, int i) {
  Raw<T> r;
  if constexpr (sizeof(T) == 4) {
    const v4i v = __builtin_amdgcn_raw_buffer_load_b128(rs, 16 * i, 0, 0);
    r.v = make_float4(__int_as_float(v.x), __int_as_float(v.y), __int_as_float(v.z), __int_as_float(v.w));
  } else if constexpr (sizeof(T) == 2) {
    const v2i v = __builtin_amdgcn_raw_buffer_load_b64(rs, 8 * i, 0, 0);
    r.v = make_uint2(static_cast<uint32_t>(v.x), static_cast<uint32_t>(v.y));
  } else {
    r.v = static_cast<uint32_t>(__builtin_amdgcn_raw_buffer_load_b32(rs, 4 * i, 0, 0));
  }
  return r;
}

__device__ __forceinline__ float h2f(uint32_t bits) {
  return __half2float(__ushort_as_half(static_cast<unsigned short>(bits)));
}

template <typename T>
__device__ __forceinline__ float4 to_float(const Raw<T>& r) {
  if constexpr (sizeof(T) == 4) {
    return r.v;
  } else if constexpr (sizeof(T) == 2) {
    return make_float4(h2f(r.v.x & 0xffffu), h2f(r.v.x >> 16), h2f(r.v.y & 0xffffu), h2f(r.v.y >> 16));
  } else {
    return make_float4(static_cast<float>(r.v & 0xffu), static_cast<float>((r.v >> 8) & 0xffu),
                       static_cast<float>((r.v >> 16) & 0xffu), static_cast<float>(r.v >> 24));
  }
}

// Barrier that orders LDS traffic only: vector loads issued before it stay in
// flight (a full __syncthreads() would also wait for every outstanding load,
// i.e. for the prefetch of the next channels).
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

// LDS byte address of a shared-memory pointer.
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
  return static_cast<uint32_t>(reinterpret_cast<uintptr_t>((__attribute__((address_space(3))) const void*)p));
}

// ------------------------------------------------ LDS read-accumulate --
//
// The accumulation is written in inline assembly so that the compiler neither
// pairs the 64-bit reads into two-address reads (half the bytes per cycle on
// this chip) nor merges the parity paths of a trial into one block joined by
// register copies.  Reads run one trial ahead of the adds; a wait on the LDS
// counter then covers exactly the trial about to be consumed (LDS operations
// complete in order, so extra outstanding ones only make the wait stricter).

typedef uint32_t v2u __attribute__((ext_vector_type(2)));

// Lane l reads the 64-bit word at addr + 504*k (addr already holds 8*l).  One
// read of the wave spans 512 consecutive bytes, conflict free: lanes 0-62 own
// the first 504 bytes, lane 63 reads the first 8 bytes of the next 504-byte
// block (the neighbour that lane 62 needs for an odd-aligned trial).
template <int N>
__device__ __forceinline__ void lds_reads(uint32_t addr, v2u (&v)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) asm volatile("ds_read_b64 %0, %1 offset:%2" : "=v"(v[k]) : "v"(addr), "i"(504 * k));
}

template <int N>
__device__ __forceinline__ void lds_wait() {
  asm volatile("s_waitcnt lgkmcnt(%0)" ::"i"(N));
}

// One trial's adds for one channel, both alignments in one assembly block
// with a scalar branch inside (written as one block so that the two paths
// share their accumulator registers instead of being joined by copies).
//
// Float: x[2k], x[2k+1] are the lane's two samples of read k.  Even window
// position: += lo and hi word of read k.  Odd position: += hi word of read k
// and lo word of the next lane's read k (DPP wave rotation folded into the
// add; the halo lane 63 supplies lane 62).
//
// 8-bit pairs: e[] holds sums of samples (2i, 2i+1) of the lane, o[] the same
// one sample earlier.  Position mod 4 selects the set (bit 0) and whether the
// words are the lane's own or shifted by one word (bit 1).
#define DD_FA(a, x) "v_add_f32 %" #a ", %" #a ", %" #x "\n\t"
#define DD_FD(a, x) "v_add_f32_dpp %" #a ", %" #x ", %" #a " wave_rol:1 row_mask:0xf bank_mask:0xf\n\t"
#define DD_UA(a, x) "v_add_u32 %" #a ", %" #a ", %" #x "\n\t"
#define DD_UD(a, x) "v_add_u32_dpp %" #a ", %" #x ", %" #a " wave_rol:1 row_mask:0xf bank_mask:0xf\n\t"

#define DD_F_EVEN2(a0, a1, x0, x1) DD_FA(a0, x0) DD_FA(a1, x1)
#define DD_F_ODD2(a0, a1, x0, x1) DD_FA(a0, x1) DD_FD(a1, x0)
#define DD_U_AL2(a0, a1, x0, x1) DD_UA(a0, x0) DD_UA(a1, x1)
#define DD_U_SH2(a0, a1, x0, x1) DD_UA(a0, x1) DD_UD(a1, x0)

#define DD_BR2(P, B, EVEN, ODD)                        \
  "s_bitcmp1_b32 %" #P ", " #B "\n\t"                 \
  "s_cbranch_scc1 .Ldd_odd%=\n\t" EVEN "s_branch .Ldd_end%=\n" \
  ".Ldd_odd%=:\n\t"                                    \
  "s_nop 1\n\t" ODD ".Ldd_end%=:"

#define DD_BR4(P, B0, B1, A0, A2, A1, A3)                                              \
  "s_bitcmp1_b32 %" #P ", " #B0 "\n\t"                                               \
  "s_cbranch_scc1 .Ldd_o%=\n\t"                                                       \
  "s_bitcmp1_b32 %" #P ", " #B1 "\n\t"                                               \
  "s_cbranch_scc1 .Ldd_2%=\n\t" A0 "s_branch .Ldd_end%=\n"                            \
  ".Ldd_2%=:\n\t"                                                                      \
  "s_nop 1\n\t" A2 "s_branch .Ldd_end%=\n"                                             \
  ".Ldd_o%=:\n\t"                                                                      \
  "s_bitcmp1_b32 %" #P ", " #B1 "\n\t"                                               \
  "s_cbranch_scc1 .Ldd_3%=\n\t" A1 "s_branch .Ldd_end%=\n"                            \
  ".Ldd_3%=:\n\t"                                                                      \
  "s_nop 1\n\t" A3 ".Ldd_end%=:"

template <int N>
struct TrialAdds;

template <>
struct TrialAdds<8> {
  static __device__ __forceinline__ void f32(float* x, const v2u (&v)[8], int p) {
    asm volatile(DD_BR2(32, 2,
                        DD_F_EVEN2(0, 1, 16, 17) DD_F_EVEN2(2, 3, 18, 19) DD_F_EVEN2(4, 5, 20, 21)
                            DD_F_EVEN2(6, 7, 22, 23) DD_F_EVEN2(8, 9, 24, 25) DD_F_EVEN2(10, 11, 26, 27)
                                DD_F_EVEN2(12, 13, 28, 29) DD_F_EVEN2(14, 15, 30, 31),
                        DD_F_ODD2(0, 1, 16, 17) DD_F_ODD2(2, 3, 18, 19) DD_F_ODD2(4, 5, 20, 21)
                            DD_F_ODD2(6, 7, 22, 23) DD_F_ODD2(8, 9, 24, 25) DD_F_ODD2(10, 11, 26, 27)
                                DD_F_ODD2(12, 13, 28, 29) DD_F_ODD2(14, 15, 30, 31))
                 : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]), "+v"(x[6]),
                   "+v"(x[7]), "+v"(x[8]), "+v"(x[9]), "+v"(x[10]), "+v"(x[11]), "+v"(x[12]), "+v"(x[13]),
                   "+v"(x[14]), "+v"(x[15])
                 : "v"(v[0].x), "v"(v[0].y), "v"(v[1].x), "v"(v[1].y), "v"(v[2].x), "v"(v[2].y), "v"(v[3].x),
                   "v"(v[3].y), "v"(v[4].x), "v"(v[4].y), "v"(v[5].x), "v"(v[5].y), "v"(v[6].x), "v"(v[6].y),
                   "v"(v[7].x), "v"(v[7].y), "s"(p)
                 : "scc");
  }
};

template <>
struct TrialAdds<4> {
  static __device__ __forceinline__ void f32(float* x, const v2u (&v)[4], int p) {
    asm volatile(DD_BR2(16, 2,
                        DD_F_EVEN2(0, 1, 8, 9) DD_F_EVEN2(2, 3, 10, 11) DD_F_EVEN2(4, 5, 12, 13)
                            DD_F_EVEN2(6, 7, 14, 15),
                        DD_F_ODD2(0, 1, 8, 9) DD_F_ODD2(2, 3, 10, 11) DD_F_ODD2(4, 5, 12, 13)
                            DD_F_ODD2(6, 7, 14, 15))
                 : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]), "+v"(x[6]),
                   "+v"(x[7])
                 : "v"(v[0].x), "v"(v[0].y), "v"(v[1].x), "v"(v[1].y), "v"(v[2].x), "v"(v[2].y), "v"(v[3].x),
                   "v"(v[3].y), "s"(p)
                 : "scc");
  }
  // e[0..7], o[0..7]
  static __device__ __forceinline__ void u8(uint32_t* e, uint32_t* o, const v2u (&v)[4], int p) {
    asm volatile(DD_BR4(24, 1, 2,
                        DD_U_AL2(0, 1, 16, 17) DD_U_AL2(2, 3, 18, 19) DD_U_AL2(4, 5, 20, 21)
                            DD_U_AL2(6, 7, 22, 23),
                        DD_U_SH2(0, 1, 16, 17) DD_U_SH2(2, 3, 18, 19) DD_U_SH2(4, 5, 20, 21)
                            DD_U_SH2(6, 7, 22, 23),
                        DD_U_AL2(8, 9, 16, 17) DD_U_AL2(10, 11, 18, 19) DD_U_AL2(12, 13, 20, 21)
                            DD_U_AL2(14, 15, 22, 23),
                        DD_U_SH2(8, 9, 16, 17) DD_U_SH2(10, 11, 18, 19) DD_U_SH2(12, 13, 20, 21)
                            DD_U_SH2(14, 15, 22, 23))
                 : "+v"(e[0]), "+v"(e[1]), "+v"(e[2]), "+v"(e[3]), "+v"(e[4]), "+v"(e[5]), "+v"(e[6]),
                   "+v"(e[7]), "+v"(o[0]), "+v"(o[1]), "+v"(o[2]), "+v"(o[3]), "+v"(o[4]), "+v"(o[5]),
                   "+v"(o[6]), "+v"(o[7])
                 : "v"(v[0].x), "v"(v[0].y), "v"(v[1].x), "v"(v[1].y), "v"(v[2].x), "v"(v[2].y), "v"(v[3].x),
                   "v"(v[3].y), "s"(p)
                 : "scc");
  }
};

template <>
struct TrialAdds<2> {
  static __device__ __forceinline__ void f32(float* x, const v2u (&v)[2], int p) {
    asm volatile(DD_BR2(8, 2, DD_F_EVEN2(0, 1, 4, 5) DD_F_EVEN2(2, 3, 6, 7),
                        DD_F_ODD2(0, 1, 4, 5) DD_F_ODD2(2, 3, 6, 7))
                 : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3])
                 : "v"(v[0].x), "v"(v[0].y), "v"(v[1].x), "v"(v[1].y), "s"(p)
                 : "scc");
  }
  static __device__ __forceinline__ void u8(uint32_t* e, uint32_t* o, const v2u (&v)[2], int p) {
    asm volatile(DD_BR4(12, 1, 2, DD_U_AL2(0, 1, 8, 9) DD_U_AL2(2, 3, 10, 11),
                        DD_U_SH2(0, 1, 8, 9) DD_U_SH2(2, 3, 10, 11),
                        DD_U_AL2(4, 5, 8, 9) DD_U_AL2(6, 7, 10, 11),
                        DD_U_SH2(4, 5, 8, 9) DD_U_SH2(6, 7, 10, 11))
                 : "+v"(e[0]), "+v"(e[1]), "+v"(e[2]), "+v"(e[3]), "+v"(o[0]), "+v"(o[1]), "+v"(o[2]), "+v"(o[3])
                 : "v"(v[0].x), "v"(v[0].y), "v"(v[1].x), "v"(v[1].y), "s"(p)
                 : "scc");
  }
};

// Value of lane (l + 1) mod 64 (DPP wave rotation by one lane).
__device__ __forceinline__ uint32_t from_next_lane(uint32_t x) {
  return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(x), 0x134, 0xF, 0xF, false));
}

// Wait until at most N of this wave's vector memory operations are outstanding.
template <int N>
__device__ __forceinline__ void wait_vm() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"i"(N) : "memory");
}

// Buffer descriptor words for `bytes` bytes from `p` (raw buffer, range
// checked: reads past the end return zero without touching memory; more than
// 2^32 - 1 bytes are clamped to that).
__device__ __forceinline__ v4i buffer_words(const void* p, int64_t bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t n = bytes >= 0xffffffffll ? 0xffffffffu : static_cast<uint32_t>(bytes < 0 ? 0 : bytes);
  v4i w;  // wave-uniform by construction; made explicit for the scalar operands of inline assembly
  w.x = __builtin_amdgcn_readfirstlane(static_cast<int>(a & 0xffffffffu));
  w.y = __builtin_amdgcn_readfirstlane(static_cast<int>((a >> 32) & 0xffffu));
  w.z = __builtin_amdgcn_readfirstlane(static_cast<int>(n));
  w.w = 0x00020000;
  return w;
}

// K runs of 1 KB from the buffer straight into LDS: run m takes 16 bytes per
// lane from byte offset voff + 1024*m to LDS byte lds + 1024*m + 16*lane (the
// instruction's immediate offset moves both addresses, so the runs share one
// M0 and one offset register).
template <int K>
__device__ __forceinline__ void lds_dma_runs(uint32_t lds, uint32_t voff, const v4i& rs) {
  static_assert(K >= 1 && K <= 4, "immediate offsets stay below 4 KB");
  if constexpr (K == 1)
    asm volatile("s_mov_b32 m0, %[lds]\n\ts_nop 0\n\t"
                 "buffer_load_dwordx4 %[vo], %[rs], 0 offen lds"
                 :
                 : [lds] "s"(lds), [vo] "v"(voff), [rs] "s"(rs)
                 : "memory", "m0");
  else if constexpr (K == 2)
    asm volatile("s_mov_b32 m0, %[lds]\n\ts_nop 0\n\t"
                 "buffer_load_dwordx4 %[vo], %[rs], 0 offen lds\n\t"
                 "buffer_load_dwordx4 %[vo], %[rs], 0 offen offset:1024 lds"
                 :
                 : [lds] "s"(lds), [vo] "v"(voff), [rs] "s"(rs)
                 : "memory", "m0");
  else if constexpr (K == 3)
    asm volatile("s_mov_b32 m0, %[lds]\n\ts_nop 0\n\t"
                 "buffer_load_dwordx4 %[vo], %[rs], 0 offen lds\n\t"
                 "buffer_load_dwordx4 %[vo], %[rs], 0 offen offset:1024 lds\n\t"
                 "buffer_load_dwordx4 %[vo], %[rs], 0 offen offset:2048 lds"
                 :
                 : [lds] "s"(lds), [vo] "v"(voff), [rs] "s"(rs)
                 : "memory", "m0");
  else
    asm volatile("s_mov_b32 m0, %[lds]\n\ts_nop 0\n\t"
                 "buffer_load_dwordx4 %[vo], %[rs], 0 offen lds\n\t"
                 "buffer_load_dwordx4 %[vo], %[rs], 0 offen offset:1024 lds\n\t"
                 "buffer_load_dwordx4 %[vo], %[rs], 0 offen offset:2048 lds\n\t"
                 "buffer_load_dwordx4 %[vo], %[rs], 0 offen offset:3072 lds"
                 :
                 : [lds] "s"(lds), [vo] "v"(voff), [rs] "s"(rs)
                 : "memory", "m0");
}

// LDS read address of a (channel, trial) block: the lane's base plus the
// trial's byte position in the slot with its alignment bits cleared (two
// vector operations, so that no scalar instruction is spent on it).
__device__ __forceinline__ uint32_t block_addr(uint32_t vbase, int q) {
  uint32_t r;
  asm volatile("v_and_b32_e64 %0, %1, -8\n\tv_add_u32 %0, %0, %2" : "=&v"(r) : "s"(q), "v"(vbase));
  return r;
}

// Workgroup barrier after this wave's LDS writes have completed.  Writes that
// go to LDS through the vector memory path are waited for explicitly before.
__device__ __forceinline__ void lds_barrier_asm() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Tile kernel body.  The input is staged by loads that write LDS directly
// (no registers).  Float input (and half input widened to float beforehand)
// is staged as float32, 4 bytes per sample; 8-bit input, widened beforehand
// to 16 bits, is staged as pairs of samples in the two 16-bit halves of a
// word, so that one 32-bit add accumulates two samples exactly (a half holds
// 256 channels of 255 before it could carry).
//
// Channels are processed in stages of CG, two stages alternating in LDS (one
// slot per channel).  Channel c0 + g of every stage is loaded by the first
// IW waves of group g (of NW/CG waves), 4 KB in turn: right after the barrier
// that frees its slot each issues its share of the slot's 1 KB loads, and
// before the next barrier it waits for them (it has nothing else in flight),
// so the barrier makes the stage visible.  A slot has room for the widest
// window of the plan; each window takes the 1 KB loads that cover what its
// tile reads.
// The loads of a channel go through a buffer descriptor based at its row
// (rounded down to 16 bytes) that reaches to the end of the input, so offsets
// stay 32-bit however large the input is, and loads past its end return
// zeros.  Two tables built on the host give, per (trial
// tile, channel), the byte offset of the window and its number of loads and,
// per trial, the byte position of its first sample inside the slot, whose low
// bits carry the alignment the adds need.
// Both are padded past the last channel, so reading them a stage ahead needs
// no check; the slots of channels past the last one are zeroed instead of
// loaded, so adding them needs no check either.
//
// A (channel, trial) block reads its samples with aligned 64-bit reads,
// several blocks of reads in flight.  Lanes 0-62 own the output samples; lane
// 63 only supplies its neighbour when the block's window position is not a
// multiple of the word pair.  8-bit blocks have a second alignment, the
// sample within a word: odd positions accumulate into a second set of words
// that holds every sum one sample earlier, and the two sets are combined into
// 32-bit totals every 256 channels.  Float sums: channels ascending, summed in
// blocks of kChanBlock into a partial that is then added to the total (the
// same order in every variant).
template <bool kPairs, int DW, int KS, int WD, int WT, int CG, int IW>
__device__ __forceinline__ void tile_dma(const TiledArgs& a, int dm_tile, int t_tile) {
  constexpr int NW = WD * WT;
  constexpr int SPW = 126 * KS;
  constexpr int T = SPW * WT;
  constexpr int NR = kPairs ? KS / 2 : KS;  // 64-bit LDS reads per lane and block
  constexpr int ES = kPairs ? 2 : 4;        // bytes per staged sample
  constexpr int WPG = NW / CG;              // waves per issuing group
  constexpr int NB = CG * DW;               // (channel, trial) blocks per stage
  constexpr int QS = DW * WD;               // trials per tile (slot-position row length)
  constexpr int D = (3 - 1) * NR <= 15 ? 3 : 2;  // blocks with reads in flight
  constexpr int FLUSH = kPairs ? 256 : kChanBlock;
  static_assert(KS % 2 == 0 && (D - 1) * NR <= 15, "tile shape");
  static_assert(NW % CG == 0 && FLUSH % CG == 0, "stage shape");
  static_assert(IW >= 1 && IW <= WPG, "waves that load a window");
  static_assert((SPW * ES) % 8 == 0, "time offset of a wave keeps the read alignment");
  extern __shared__ float4 lds4[];

  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;
  const int wd = wave % WD;
  const int wt = wave / WD;
  const int grp = wave / WPG;  // channel of a stage this wave loads
  const int gq = wave % WPG;   // rank inside its group
  const int t0 = t_tile * T;   // rows are below 2^32 bytes, so are these indices
  const int dw0 = dm_tile * QS + wd * DW;
  const int nchans = a.nchans;
  const int nstages = (nchans + CG - 1) / CG;
  const uint32_t slot_bytes = 1024u * static_cast<uint32_t>(a.runs);
  const uint32_t lds0 = lds_addr(lds4);
  constexpr int ALIGN = kPairs ? 8 : 4;     // window starts are aligned to 16 bytes
  const uint32_t lane16 = 16u * static_cast<uint32_t>(lane);
  // read base of the lane: its 8 bytes, and the wave's offset along time
  const uint32_t vlane = lds0 + 8u * static_cast<uint32_t>(lane) + static_cast<uint32_t>(ES * SPW * wt);
  const uint32_t t0b = static_cast<uint32_t>(ES * t0);
  cint32* wb = (cint32*)(a.wbase) + 2 * (static_cast<int64_t>(dm_tile) * (nchans + kGeoPad) + grp);
  cint32* sp = (cint32*)(a.spos) + static_cast<int64_t>(dm_tile) * (nchans + kGeoPad) * QS + wd * DW;

  // The last 1-3 samples of a float input (past the last whole group of 4)
  // are read once here; the slot holding them patches them in.  (Widened
  // inputs are padded to whole groups.)
  float tail[3] = {0.f, 0.f, 0.f};
  int c_tail = nchans;  // first channel whose window can reach them
  const bool has_tail = !kPairs && a.ntail > 0;  // the same for the whole launch
  if (has_tail) {
    const float* inf = static_cast<const float*>(a.in);
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (k < a.ntail) tail[k] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(inf[a.total4 + k])));
    // a window ends before c*pitch + t0 + max_shift + T + 10
    const int64_t lim = a.total4 - t0 - a.max_shift - (T + 10);
    c_tail = lim < 0 ? 0 : static_cast<int>(lim / a.pitch) + 1;
  }

  // Byte offset of the aligned start of row c, where its descriptor is based.
  auto row_base = [&](int c) -> int64_t {
    return ES * ((static_cast<int64_t>(c) * a.pitch) & ~static_cast<int64_t>(ALIGN - 1));
  };
  // Loads of channel c (this group's channel of a stage: window offset wbase
  // from its row base, `runs` loads) into the slot at LDS byte offset slot:
  // the group's first IW waves issue them, 4 KB each in turn; a channel past
  // the last one gets zeros (from the first wave) instead.
  auto issue = [&](int c, uint32_t wbase, int runs, uint32_t slot) {
    if (c < nchans) {
      if (gq >= IW || 4 * gq >= runs) return;
      const int64_t rb = row_base(c);
      const v4i rs = buffer_words(static_cast<const char*>(a.in) + rb, a.total4 * ES - rb);
      uint32_t lds = __builtin_amdgcn_readfirstlane(lds0 + slot + 4096u * gq);
      uint32_t voff = wbase + t0b + lane16 + 4096u * gq;
      for (int i = 4 * gq; i < runs; i += 4 * IW, lds += 4096u * IW, voff += 4096u * IW) {
        const int k = runs - i;
        if (k >= 4)
          lds_dma_runs<4>(lds, voff, rs);
        else if (k == 3)
          lds_dma_runs<3>(lds, voff, rs);
        else if (k == 2)
          lds_dma_runs<2>(lds, voff, rs);
        else
          lds_dma_runs<1>(lds, voff, rs);
      }
    } else if (c < nstages * CG && gq == 0) {
      for (int m = 0; m < a.runs; ++m)
        *reinterpret_cast<float4*>(reinterpret_cast<char*>(lds4) + slot + 1024u * m + lane16) =
            make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  // After the loads of channel c landed: the partial last group of a float
  // input, if the slot holds it, is patched in by the lane that loaded its
  // place.
  auto patch = [&](int c, uint32_t wbase, int runs, uint32_t slot) {
    if (kPairs || c >= nchans || c < c_tail) return;
    const int64_t off = static_cast<int64_t>(a.total4) * 4 - (row_base(c) + wbase + t0b);
    if (off < 0 || off >= 1024 * static_cast<int64_t>(runs)) return;
    if ((off >> 12) % IW != gq) return;  // the wave that loaded its 4 KB
    const uint32_t o = static_cast<uint32_t>(off);
    if (lane == ((o >> 4) & 63))
      *reinterpret_cast<float4*>(reinterpret_cast<char*>(lds4) + slot + o) =
          make_float4(tail[0], tail[1], tail[2], 0.f);
  };

  // Accumulators.  Float: acc0 = partial of the current block of channels,
  // tot = total.  8-bit: acc0/acc1 = words of two 16-bit sums (acc1 one
  // sample earlier), tot = 32-bit totals.
  constexpr int NA = 2 * NR;
  typedef typename std::conditional<kPairs, uint32_t, float>::type Acc;
  Acc acc0[DW][NA];
  Acc acc1[DW][kPairs ? NA : 1];
  Acc tot[DW][kPairs ? 4 * NR : NA];
#pragma unroll
  for (int j = 0; j < DW; ++j) {
#pragma unroll
    for (int k = 0; k < NA; ++k) acc0[j][k] = 0;
#pragma unroll
    for (int k = 0; k < (kPairs ? NA : 1); ++k) acc1[j][k] = 0;
#pragma unroll
    for (int k = 0; k < (kPairs ? 4 * NR : NA); ++k) tot[j][k] = 0;
  }
  auto flush = [&]() {
    if constexpr (kPairs) {
#pragma unroll
      for (int j = 0; j < DW; ++j)
#pragma unroll
        for (int k = 0; k < NR; ++k) {
          const uint32_t ex = acc0[j][2 * k], ey = acc0[j][2 * k + 1];
          const uint32_t ox = acc1[j][2 * k], oy = acc1[j][2 * k + 1];
          const uint32_t oxn = from_next_lane(ox);
          tot[j][4 * k + 0] += (ex & 0xffffu) + (ox >> 16);
          tot[j][4 * k + 1] += (ex >> 16) + (oy & 0xffffu);
          tot[j][4 * k + 2] += (ey & 0xffffu) + (oy >> 16);
          tot[j][4 * k + 3] += (ey >> 16) + (oxn & 0xffffu);
          acc0[j][2 * k] = acc0[j][2 * k + 1] = 0u;
          acc1[j][2 * k] = acc1[j][2 * k + 1] = 0u;
        }
    } else {
#pragma unroll
      for (int j = 0; j < DW; ++j)
#pragma unroll
        for (int k = 0; k < NA; ++k) {
          tot[j][k] += acc0[j][k];
          acc0[j][k] = 0.f;
        }
    }
  };

  // Scalar state, read a stage ahead (the tables are padded past the last
  // channel): slot positions of the current and next stage, window offset of
  // this group's channel in the next stage and the one after.
  int q[CG][DW], qn[CG][DW];
#pragma unroll
  for (int u = 0; u < CG; ++u)
#pragma unroll
    for (int j = 0; j < DW; ++j) q[u][j] = sp[u * QS + j];
  sp += CG * QS;
  int wcur = wb[0], rcur = wb[1];                // this group's channel of stage 0
  int wnext = wb[2 * CG], rnext = wb[2 * CG + 1];  // ... of stage 1
  wb += 4 * CG;
  issue(grp, static_cast<uint32_t>(wcur), rcur, grp * slot_bytes);

  for (int s = 0; s < nstages; ++s) {
    const int c0 = s * CG;
    const uint32_t sbase = (s & 1) ? CG * slot_bytes : 0u;
    wait_vm<0>();  // this wave's loads of the stage (if it issued any) are in LDS
    if (has_tail) patch(c0 + grp, static_cast<uint32_t>(wcur), rcur, sbase + grp * slot_bytes);
    lds_barrier_asm();
    // the other stage's slots are free: issue this group's channel of the next stage
    issue(c0 + CG + grp, static_cast<uint32_t>(wnext), rnext, (sbase ^ (CG * slot_bytes)) + grp * slot_bytes);

    // read address of block b (channel c0 + b / DW, trial b % DW), formed right
    // before its reads so that only the blocks in flight hold one
    auto ba = [&](int b) { return block_addr(vlane + sbase + (b / DW) * slot_bytes, q[b / DW][b % DW]); };
    v2u rb[D][NR];
#pragma unroll
    for (int b = 0; b < D && b < NB; ++b) lds_reads<NR>(ba(b), rb[b]);
    // scalar loads for later stages, consumed a stage from now
#pragma unroll
    for (int u = 0; u < CG; ++u)
#pragma unroll
      for (int j = 0; j < DW; ++j) qn[u][j] = sp[u * QS + j];
    sp += CG * QS;
    const int wnn = wb[0], rnn = wb[1];
    wb += 2 * CG;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int ahead = (NB - 1 - b) < (D - 1) ? (NB - 1 - b) : (D - 1);
      if (ahead >= 2)
        lds_wait<2 * NR>();
      else if (ahead == 1)
        lds_wait<NR>();
      else
        lds_wait<0>();
      if constexpr (kPairs)
        TrialAdds<NR>::u8(acc0[b % DW], acc1[b % DW], rb[b % D], q[b / DW][b % DW]);
      else
        TrialAdds<NR>::f32(acc0[b % DW], rb[b % D], q[b / DW][b % DW]);
      if (b + D < NB) lds_reads<NR>(ba(b + D), rb[(b + D) % D]);
    }
    if (((c0 + CG) % FLUSH) == 0) flush();
#pragma unroll
    for (int u = 0; u < CG; ++u)
#pragma unroll
      for (int j = 0; j < DW; ++j) q[u][j] = qn[u][j];
    wcur = wnext;
    rcur = rnext;
    wnext = wnn;
    rnext = rnn;
  }
  flush();       // the channels after the last whole flush block
  wait_vm<0>();  // no load may still be writing LDS when the workgroup ends

  if (lane == 63) return;  // the halo lane owns no output
  const int64_t nsamp = a.nsamp;
#pragma unroll
  for (int j = 0; j < DW; ++j) {
    const int d = dw0 + j;
    if (d >= a.ndm) break;
    if constexpr (kPairs) {
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const int64_t t = static_cast<int64_t>(t0) + wt * SPW + 4 * lane + 252 * k;
        int32_t* o = static_cast<int32_t*>(a.out) + d * nsamp + t;
        if (t + 3 < nsamp) {
          const int4 w4 = make_int4(static_cast<int32_t>(tot[j][4 * k]), static_cast<int32_t>(tot[j][4 * k + 1]),
                                    static_cast<int32_t>(tot[j][4 * k + 2]), static_cast<int32_t>(tot[j][4 * k + 3]));
          __builtin_memcpy(o, &w4, 16);
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (t + i < nsamp) o[i] = static_cast<int32_t>(tot[j][4 * k + i]);
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const int64_t t = static_cast<int64_t>(t0) + wt * SPW + 2 * lane + 126 * k;
        float* o = static_cast<float*>(a.out) + d * nsamp + t;
        if (t + 1 < nsamp) {
          const float2 w2 = make_float2(tot[j][2 * k], tot[j][2 * k + 1]);
          __builtin_memcpy(o, &w2, 8);
        } else if (t < nsamp) {
          *o = tot[j][2 * k];
        }
      }
    }
  }
}


// Widening of 8-bit input to 16 bits and of half input to float, into a
// buffer padded with zeros to npad samples (a multiple of 8): 8 samples per
// thread.
__global__ __launch_bounds__(256) void widen_u8(const uint8_t* __restrict__ in, uint16_t* __restrict__ out,
                                                int64_t n, int64_t npad) {
  const int64_t i = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) * 8;
  if (i >= npad) return;
  if (i + 8 <= n) {
    uint2 w;
    __builtin_memcpy(&w, in + i, 8);
    uint4 o;
    o.x = (w.x & 0xffu) | ((w.x & 0xff00u) << 8);
    o.y = ((w.x >> 16) & 0xffu) | ((w.x >> 8) & 0xff0000u);
    o.z = (w.y & 0xffu) | ((w.y & 0xff00u) << 8);
    o.w = ((w.y >> 16) & 0xffu) | ((w.y >> 8) & 0xff0000u);
    *reinterpret_cast<uint4*>(out + i) = o;
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) out[i + k] = i + k < n ? in[i + k] : 0;
  }
}

__global__ __launch_bounds__(256) void widen_f16(const __half* __restrict__ in, float* __restrict__ out, int64_t n,
                                                 int64_t npad) {
  const int64_t i = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) * 8;
  if (i >= npad) return;
  if (i + 8 <= n) {
    uint4 w;
    __builtin_memcpy(&w, in + i, 16);
    float4 lo = make_float4(h2f(w.x & 0xffffu), h2f(w.x >> 16), h2f(w.y & 0xffffu), h2f(w.y >> 16));
    float4 hi = make_float4(h2f(w.z & 0xffffu), h2f(w.z >> 16), h2f(w.w & 0xffffu), h2f(w.w >> 16));
    reinterpret_cast<float4*>(out + i)[0] = lo;
    reinterpret_cast<float4*>(out + i)[1] = hi;
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) out[i + k] = i + k < n ? __half2float(in[i + k]) : 0.f;
  }
}


// Staged form of a sample: 8-bit samples widen to 16 bits, half to float.
__device__ __forceinline__ uint16_t stage_of(uint8_t x) { return x; }
__device__ __forceinline__ float stage_of(__half x) { return __half2float(x); }
__device__ __forceinline__ float stage_of(float x) { return x; }

// Assembly of one streaming window [nchans][tail + block] in staged form:
// the first `tail` samples of each channel row are the last `tail` of the
// previous window (already staged), or zeros, and the rest is the new block
// ([nchans][block], raw) widened.  Rows are strided over blockIdx.y, the
// samples of a row over blockIdx.x and the lanes, one sample per lane, so
// every wave reads and writes contiguous runs.
template <typename In, typename St>
__global__ __launch_bounds__(256) void assemble_window(const St* __restrict__ prev, const In* __restrict__ blk,
                                                       St* __restrict__ dst, int64_t tail, int64_t block,
                                                       int nchans, int zero_tail) {
  const int64_t pitch = tail + block;
  for (int c = blockIdx.y; c < nchans; c += gridDim.y) {
    St* d = dst + c * pitch;
    const St* h = prev + c * pitch + block;
    const In* b = blk + c * block;
    for (int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; j < pitch;
         j += static_cast<int64_t>(gridDim.x) * 256) {
      St v;
      if (j < tail)
        v = zero_tail ? St(0) : h[j];
      else
        v = stage_of(b[j - tail]);
      d[j] = v;
    }
  }
}

// One launch of a tile variant: 8-bit input (widened to 16 bits) as pairs,
// float and half input (widened to float) as float32.
template <bool kPairs, int DW, int KS, int WD, int WT, int CG, int IW>
__global__ __launch_bounds__(64 * WD * WT) void dedisp_tiled(const TiledArgs a) {
  int dm_tile, t_tile;
  if (!tile_of(a, dm_tile, t_tile)) return;  // padding block of the last group
  tile_dma<kPairs, DW, KS, WD, WT, CG, IW>(a, dm_tile, t_tile);
}

// Widening of the inputs of a batch: blockIdx.y selects the job, the blocks
// of a job stride over its samples, 8 per thread.
__global__ __launch_bounds__(256) void widen_job_kernel(const WidenJob* __restrict__ jobs) {
  const WidenJob j = jobs[blockIdx.y];
  for (int64_t i = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) * 8; i < j.npad;
       i += static_cast<int64_t>(gridDim.x) * 256 * 8) {
    if (j.dtype == DEDISP_U8) {
      const uint8_t* in = static_cast<const uint8_t*>(j.in);
      uint16_t* out = static_cast<uint16_t*>(j.ws);
      if (i + 8 <= j.n) {
        uint2 w;
        __builtin_memcpy(&w, in + i, 8);
        uint4 o;
        o.x = (w.x & 0xffu) | ((w.x & 0xff00u) << 8);
        o.y = ((w.x >> 16) & 0xffu) | ((w.x >> 8) & 0xff0000u);
        o.z = (w.y & 0xffu) | ((w.y & 0xff00u) << 8);
        o.w = ((w.y >> 16) & 0xffu) | ((w.y >> 8) & 0xff0000u);
        *reinterpret_cast<uint4*>(out + i) = o;
      } else {
        for (int k = 0; k < 8; ++k) out[i + k] = i + k < j.n ? in[i + k] : 0;
      }
    } else {
      const __half* in = static_cast<const __half*>(j.in);
      float* out = static_cast<float*>(j.ws);
      for (int k = 0; k < 8; ++k) out[i + k] = i + k < j.n ? __half2float(in[i + k]) : 0.f;
    }
  }
}

// Persistent batch kernel: resident workgroups pull (beam, trial tile, time
// tile) items from atomic counters (one per XCD) until none are left.  Items are
// numbered beam by beam, beams in order of decreasing cost per item (longest
// items first), and inside a beam in the same groups as a single launch.  One
// kernel per staging kind (its beams are all 8-bit, or all float and half),
// so that each carries the registers of one path only.
template <bool kPairs, int DW, int KS, int WD, int WT, int CG, int IW>
__global__ __launch_bounds__(64 * WD * WT) void dedisp_batch_persistent(const BatchArgs b) {
  __shared__ long long item_s;
  // Blocks run on XCD blockIdx.x mod 8.  Items go out in chunks of
  // kBatchChunk consecutive ones (neighbouring tiles of a beam, whose windows
  // overlap), chunk j to counter j mod nx: the workgroups of one XCD share a
  // counter, so a chunk stays in one L2, and every XCD gets the same mix of
  // beams.  (With fewer than 8 workgroups, nx = the grid.)
  const int nx = gridDim.x < 8 ? static_cast<int>(gridDim.x) : 8;
  const int xcd = static_cast<int>(blockIdx.x) % nx;
  for (;;) {
    if (threadIdx.x == 0) item_s = static_cast<long long>(atomicAdd(b.counter + xcd, 1ull));
    lds_barrier();
    const long long k =
        static_cast<long long>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(item_s)))) |
        (static_cast<long long>(__builtin_amdgcn_readfirstlane(static_cast<int>(item_s >> 32))) << 32);
    const long long item = (k / kBatchChunk) * (nx * kBatchChunk) + xcd * kBatchChunk + k % kBatchChunk;
    if (item >= b.n_items) return;  // the counter's later items are further on
    typedef __attribute__((address_space(4))) const int64_t cint64;
    typedef __attribute__((address_space(4))) const TiledArgs ctargs;
    cint64* ends = (cint64*)(b.item_end);
    int beam = 0;
    while (beam + 1 < b.nbeams && item >= ends[beam]) ++beam;
    const int64_t first = beam == 0 ? 0 : ends[beam - 1];
    TiledArgs a;
    __builtin_memcpy(&a, (const void*)((ctargs*)(b.beams) + beam), sizeof(TiledArgs));
    const int l = static_cast<int>(item - first);
    const int bs = a.gd * a.gt;
    const int g = l / bs;
    const int i = l - g * bs;
    // wave-uniform: kept in scalar registers (the divisions above run on the vector unit)
    const int dm_tile = __builtin_amdgcn_readfirstlane((g % a.n_dm_groups) * a.gd + i % a.gd);
    const int t_tile = __builtin_amdgcn_readfirstlane((g / a.n_dm_groups) * a.gt + i / a.gd);
    if (dm_tile < a.n_dm_tiles && t_tile < a.n_t_tiles) tile_dma<kPairs, DW, KS, WD, WT, CG, IW>(a, dm_tile, t_tile);
    lds_barrier();  // every wave is done with this item's LDS before the next
  }
}

__global__ void reset_counter(unsigned long long* c) {
  if (threadIdx.x < kBatchCounters) c[threadIdx.x] = 0ull;
}

// ----------------------------------------------------------- registry --

struct Variant {
  TileShape shape;
  int cg;             // channels per stage
  const void* fn[3];  // by dtype: U8, F16, F32
  const void* batch[2];  // persistent batch kernel: float staging, 16-bit pair staging
};

#define DEDISP_VARIANT(DW, KS, WD, WT, CG, IW)                                                      \
  Variant {                                                                                        \
    TileShape{DW, KS, WD, WT}, CG,                                                                 \
        {reinterpret_cast<const void*>(&dedisp_tiled<true, DW, KS, WD, WT, CG, IW>),                \
         reinterpret_cast<const void*>(&dedisp_tiled<false, DW, KS, WD, WT, CG, IW>),               \
         reinterpret_cast<const void*>(&dedisp_tiled<false, DW, KS, WD, WT, CG, IW>)},              \
        {reinterpret_cast<const void*>(&dedisp_batch_persistent<false, DW, KS, WD, WT, CG, IW>),      \
         reinterpret_cast<const void*>(&dedisp_batch_persistent<true, DW, KS, WD, WT, CG, IW>)}       \
  }

// The last argument is the number of waves of a group that share a window's
// loads (4 KB each in turn): a single loading wave is late to every stage's
// barrier by the time it spends issuing, so groups of 4 or 8 waves share the
// work; with 2 waves a group (4 channels per stage) sharing measured slower.
const Variant kVariants[] = {
    DEDISP_VARIANT(2, 8, 4, 2, 2, 4),  // 8 trials x 2016 samples, 512 threads (several workgroups per CU)
    DEDISP_VARIANT(2, 8, 8, 2, 2, 2),  // 16 x 2016, 1024 threads
    DEDISP_VARIANT(4, 8, 4, 2, 2, 4),  // 16 x 2016, 512 threads
    DEDISP_VARIANT(2, 8, 4, 4, 2, 2),  // 8 x 4032, 1024 threads
    DEDISP_VARIANT(2, 8, 4, 2, 4, 1),  // 8 x 2016, 512 threads, 4 channels per stage
    DEDISP_VARIANT(2, 8, 8, 2, 4, 4),  // 16 x 2016, 1024 threads, 4 channels per stage
    DEDISP_VARIANT(4, 8, 4, 2, 4, 1),  // 16 x 2016, 512 threads, 4 channels per stage
    DEDISP_VARIANT(2, 8, 4, 2, 1, 2),  // 8 x 2016, 512 threads, 1 channel per stage
    DEDISP_VARIANT(4, 8, 8, 1, 2, 4),  // 32 x 1008, 512 threads
    DEDISP_VARIANT(2, 4, 8, 2, 2, 2),  // 16 x 1008, 1024 threads
    DEDISP_VARIANT(2, 8, 8, 1, 8, 1),  // 16 x 1008, 512 threads, 8 channels per stage (small delay spreads)
};
constexpr int kNumTiled = sizeof(kVariants) / sizeof(kVariants[0]);

constexpr size_t kMaxLds = 160 * 1024;

// 1 KB loads per LDS slot (one channel's window) a tiled variant needs for
// this plan, or 0 if the plan's delay spread is too wide for the variant's
// LDS.  A window covers the tile's samples, the delay spread of its trials,
// the alignment of its start (to 4 samples for float staging, 8 for 16-bit
// pairs) and the neighbour word the halo lane reads past the last sample.
// Two stages of `cg` slots are live.
int slot_runs(dedisp_plan p, const Variant& v) {
  const std::vector<int2>& w = host_windows(p, v.shape.dms());
  int spread = 0;
  for (const int2& x : w) spread = std::max(spread, x.y - x.x);
  const int64_t es = staged_size(p->dtype);
  const int64_t align = p->dtype == DEDISP_U8 ? 8 : 4;
  const int64_t bytes = es * (static_cast<int64_t>(spread) + align - 1 + v.shape.samples()) + 8;
  const int64_t runs = (bytes + 1023) / 1024;
  if (2 * v.cg * runs * 1024 > static_cast<int64_t>(kMaxLds) - 256) return 0;  // 256 B for static LDS
  return static_cast<int>(runs);
}

// The tiled kernels address a row (and a window past its end) with 32-bit
// byte offsets from the row's start.
bool offsets_fit(dedisp_plan p, int64_t nsamp) {
  const int64_t pitch = nsamp + p->max_shift;
  return (pitch + 16) * staged_size(p->dtype) + (static_cast<int64_t>(1) << 20) < (static_cast<int64_t>(1) << 32);
}

}  // namespace

int variant_count() { return 1 + kNumTiled; }

TileShape variant_shape(int v) { return kVariants[v - 1].shape; }

int tiled_per_cu(dedisp_plan p, int v) {
  if (v < 1 || v > kNumTiled) return 0;
  const int runs = slot_runs(p, kVariants[v - 1]);
  if (runs == 0) return 0;
  return static_cast<int>((kMaxLds - 256) / (2 * static_cast<size_t>(kVariants[v - 1].cg) * runs * 1024));
}

bool variant_fits(dedisp_plan p, int v) {
  if (v == 0) return true;
  if (v < 0 || v > kNumTiled) return false;
  return slot_runs(p, kVariants[v - 1]) > 0;
}

int default_variant(dedisp_plan p) {
  static const int order[] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11};
  for (int v : order)
    if (v <= kNumTiled && variant_fits(p, v)) return v;
  return 0;
}

namespace {

// The direct kernel over input of sample type In (raw or staged).
template <typename In>
int launch_direct(dedisp_plan p, const DeviceTables* dt, const void* in, void* out, int64_t nsamp, hipStream_t s) {
  const int64_t pitch = nsamp + p->max_shift;
  const int64_t tblocks = (nsamp + 255) / 256;
  const int64_t nblocks = tblocks * p->ndm;
  if (nblocks > INT32_MAX) return DEDISP_ERR_INVALID_ARG;
  hipLaunchKernelGGL(dedisp_direct<In>, dim3(static_cast<unsigned>(nblocks)), dim3(256), 0, s,
                     static_cast<const In*>(in), pitch, out, nsamp, dt->shift, p->ndm_pad, p->nchans, tblocks);
  return DEDISP_HIP_STATUS(hipGetLastError());
}

// A tiled variant over staged input (float input as given, 8-bit and half
// input widened).
int launch_tiled(dedisp_plan p, int v, const void* staged, void* out, int64_t nsamp, hipStream_t s) {
  TiledArgs a;
  size_t lds = 0;
  int64_t nblocks = 0;
  int threads = 0;
  int st = tiled_args(p, v, staged, out, nsamp, &a, &lds, &nblocks, &threads);
  const void* fn = kVariants[v - 1].fn[p->dtype];
  if (st == DEDISP_OK && lds > 64 * 1024) st = allow_large_lds(fn);
  if (st == DEDISP_OK) {
    void* args[] = {&a};
    st = DEDISP_HIP_STATUS(hipLaunchKernel(fn, dim3(static_cast<unsigned>(nblocks)), dim3(threads), args, lds, s));
  }
  return st;
}

// Stream-ordered workspaces come from the device's default memory pool; by
// default the pool hands memory back to the driver at every synchronisation,
// so each call would map its workspace anew.  Keep it instead (once per
// device).
int keep_pool_memory(int dev) {
  static std::mutex mu;
  static std::map<int, bool> done;
  std::lock_guard<std::mutex> g(mu);
  if (done.count(dev)) return DEDISP_OK;
  hipMemPool_t pool = nullptr;
  hipError_t e = hipDeviceGetDefaultMemPool(&pool, dev);
  uint64_t keep = UINT64_MAX;
  if (e == hipSuccess) e = hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  done[dev] = true;
  return DEDISP_OK;
}

}  // namespace

int launch(dedisp_plan p, int v, const void* in, void* out, int64_t nsamp, hipStream_t s, void* ws_given) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  DeviceTables* dt = nullptr;
  int st = device_tables(p, dev, &dt);
  if (st != DEDISP_OK) return st;
  const int64_t total = (nsamp + p->max_shift) * p->nchans;
  // the tiled kernels address each row with 32-bit byte offsets; longer rows
  // take the direct kernel
  if (v > 0 && !offsets_fit(p, nsamp)) v = 0;
  if (v == 0) {
    switch (p->dtype) {
      case DEDISP_U8: return launch_direct<uint8_t>(p, dt, in, out, nsamp, s);
      case DEDISP_F16: return launch_direct<__half>(p, dt, in, out, nsamp, s);
      default: return launch_direct<float>(p, dt, in, out, nsamp, s);
    }
  }
  if (p->dtype == DEDISP_F32) return launch_tiled(p, v, in, out, nsamp, s);
  // 8-bit and half input are widened into a workspace first: the caller's,
  // else a stream-ordered one
  void* ws = ws_given;
  if (ws == nullptr) {
    st = keep_pool_memory(dev);
    if (st != DEDISP_OK) return st;
    e = hipMallocAsync(&ws, staged_bytes(p, nsamp), s);
    if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  }
  st = widen(p->dtype, in, ws, total, s);
  if (st == DEDISP_OK) st = launch_tiled(p, v, ws, out, nsamp, s);
  if (ws_given == nullptr) {
    const int st2 = DEDISP_HIP_STATUS(hipFreeAsync(ws, s));
    if (st == DEDISP_OK) st = st2;
  }
  return st;
}

int launch_staged(dedisp_plan p, int v, const void* staged, void* out, int64_t nsamp, hipStream_t s) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  DeviceTables* dt = nullptr;
  int st = device_tables(p, dev, &dt);
  if (st != DEDISP_OK) return st;
  if (v > 0 && !offsets_fit(p, nsamp)) v = 0;
  if (v == 0) {
    // same channel order and float conversion as on raw input
    if (p->dtype == DEDISP_U8) return launch_direct<uint16_t>(p, dt, staged, out, nsamp, s);
    return launch_direct<float>(p, dt, staged, out, nsamp, s);
  }
  return launch_tiled(p, v, staged, out, nsamp, s);
}

size_t staged_bytes(dedisp_plan p, int64_t nsamp) {
  return static_cast<size_t>(widened_samples((nsamp + p->max_shift) * p->nchans)) * staged_size(p->dtype);
}

int assemble(int dtype, const void* prev, const void* blk, void* dst, int64_t tail, int64_t block, int nchans,
             bool zero_tail, hipStream_t s) {
  if (nchans < 1 || tail < 0 || block < 1) return DEDISP_ERR_INVALID_ARG;
  const int64_t pitch = tail + block;
  const unsigned gx = static_cast<unsigned>(std::min<int64_t>((pitch + 255) / 256, 32));
  const unsigned gy = static_cast<unsigned>(std::min(nchans, 65535));
  const int z = zero_tail ? 1 : 0;
  switch (dtype) {
    case DEDISP_U8:
      hipLaunchKernelGGL((assemble_window<uint8_t, uint16_t>), dim3(gx, gy), dim3(256), 0, s,
                         static_cast<const uint16_t*>(prev), static_cast<const uint8_t*>(blk),
                         static_cast<uint16_t*>(dst), tail, block, nchans, z);
      break;
    case DEDISP_F16:
      hipLaunchKernelGGL((assemble_window<__half, float>), dim3(gx, gy), dim3(256), 0, s,
                         static_cast<const float*>(prev), static_cast<const __half*>(blk), static_cast<float*>(dst),
                         tail, block, nchans, z);
      break;
    case DEDISP_F32:
      hipLaunchKernelGGL((assemble_window<float, float>), dim3(gx, gy), dim3(256), 0, s,
                         static_cast<const float*>(prev), static_cast<const float*>(blk), static_cast<float*>(dst),
                         tail, block, nchans, z);
      break;
    default:
      return DEDISP_ERR_INVALID_ARG;
  }
  return DEDISP_HIP_STATUS(hipGetLastError());
}

int widen_jobs(const WidenJob* jobs, int njobs, hipStream_t s) {
  if (njobs <= 0) return DEDISP_OK;
  hipLaunchKernelGGL(widen_job_kernel, dim3(1024, static_cast<unsigned>(njobs)), dim3(256), 0, s, jobs);
  return DEDISP_HIP_STATUS(hipGetLastError());
}

int64_t widened_samples(int64_t total) { return (total + 7) / 8 * 8; }

int widen(int dtype, const void* in, void* ws, int64_t total, hipStream_t s) {
  const int64_t npad = widened_samples(total);
  const int64_t blocks = (npad / 8 + 255) / 256;
  if (blocks > INT32_MAX) return DEDISP_ERR_INVALID_ARG;
  if (dtype == DEDISP_U8)
    hipLaunchKernelGGL(widen_u8, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<const uint8_t*>(in), static_cast<uint16_t*>(ws), total, npad);
  else if (dtype == DEDISP_F16)
    hipLaunchKernelGGL(widen_f16, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       static_cast<const __half*>(in), static_cast<float*>(ws), total, npad);
  else
    return DEDISP_ERR_INVALID_ARG;
  return DEDISP_HIP_STATUS(hipGetLastError());
}

int tiled_args(dedisp_plan p, int v, const void* in, void* out, int64_t nsamp, TiledArgs* ap, size_t* lds_out,
               int64_t* nblocks_out, int* threads_out) {
  if (v < 1 || v > kNumTiled) return DEDISP_ERR_INVALID_ARG;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  DeviceTables* dt = nullptr;
  int st = device_tables(p, dev, &dt);
  if (st != DEDISP_OK) return st;
  const Variant& var = kVariants[v - 1];
  const int runs = slot_runs(p, var);
  if (runs == 0) return DEDISP_ERR_INVALID_ARG;
  // the tiled kernels address each row with 32-bit byte offsets
  if (!offsets_fit(p, nsamp)) return DEDISP_ERR_INVALID_ARG;
  const int64_t pitch = nsamp + p->max_shift;
  const int64_t total = pitch * p->nchans;
  const int align = p->dtype == DEDISP_U8 ? 8 : 4;
  const int es = static_cast<int>(staged_size(p->dtype));
  const uint32_t* wbase = nullptr;
  st = device_window_base(p, dev, var.shape.dms(), var.shape.samples(), align, es, static_cast<int>(pitch % align), &wbase);
  if (st != DEDISP_OK) return st;
  const int32_t* spos = nullptr;
  st = device_slot_pos(p, dev, var.shape.dms(), align, es, static_cast<int>(pitch % align), &spos);
  if (st != DEDISP_OK) return st;
  TiledArgs& a = *ap;
  a.in = in;
  a.pitch = pitch;
  if (p->dtype == DEDISP_F32) {
    a.total4 = total & ~static_cast<int64_t>(3);
    a.ntail = static_cast<int>(total - a.total4);
  } else {  // widened input, padded with zeros to whole groups of 8
    a.total4 = widened_samples(total);
    a.ntail = 0;
  }
  a.max_shift = p->max_shift;
  a.out = out;
  a.nsamp = nsamp;
  a.wbase = wbase;
  a.spos = spos;
  a.runs = runs;
  a.ndm = p->ndm;
  a.nchans = p->nchans;
  a.n_dm_tiles = (p->ndm + var.shape.dms() - 1) / var.shape.dms();
  const int64_t n_t_tiles = (nsamp + var.shape.samples() - 1) / var.shape.samples();
  if (n_t_tiles > INT32_MAX / 64) return DEDISP_ERR_INVALID_ARG;
  a.n_t_tiles = static_cast<int>(n_t_tiles);
  // groups of up to 16 trial tiles x 1 time tile (16-bit pair staging) or
  // 8 x 3 (float staging), the fastest of a sweep of group shapes on the
  // LOFAR-shaped and MeerKAT-shaped workloads
  const bool pairs = p->dtype == DEDISP_U8;
  a.gd = std::min(pairs ? 16 : 8, a.n_dm_tiles);
  a.gt = std::min(pairs ? 1 : 3, a.n_t_tiles);
  a.n_dm_groups = (a.n_dm_tiles + a.gd - 1) / a.gd;
  const int64_t n_groups = static_cast<int64_t>(a.n_dm_groups) * ((a.n_t_tiles + a.gt - 1) / a.gt);
  // a multiple of 8 groups, so that every XCD's run of blocks is whole groups
  const int64_t nblocks = (n_groups + 7) / 8 * 8 * a.gd * a.gt;
  if (nblocks > INT32_MAX) return DEDISP_ERR_INVALID_ARG;
  *lds_out = 2 * static_cast<size_t>(var.cg) * runs * 1024;
  *nblocks_out = nblocks;
  *threads_out = var.shape.threads();
  return DEDISP_OK;
}

// Lift the default 64 KiB cap on dynamic LDS for a kernel, once per process
// and device (not a stream operation, so it is done before any graph capture
// that launches the kernel).
int allow_large_lds(const void* fn) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, bool> done;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  std::lock_guard<std::mutex> g(mu);
  auto key = std::make_pair(fn, dev);
  if (done.count(key)) return DEDISP_OK;
  // the batch kernel also has a few bytes of static LDS
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kMaxLds) - 256);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  done[key] = true;
  return DEDISP_OK;
}

int prepare(dedisp_plan p, int v, int64_t nsamp) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  DeviceTables* dt = nullptr;
  int st = device_tables(p, dev, &dt);
  if (st != DEDISP_OK || v <= 0) return st;
  const int64_t pitch = nsamp + p->max_shift;
  const int align = p->dtype == DEDISP_U8 ? 8 : 4;
  const int es = static_cast<int>(staged_size(p->dtype));
  const int dms = variant_shape(v).dms();
  const uint32_t* wbase = nullptr;
  st = device_window_base(p, dev, dms, variant_shape(v).samples(), align, es, static_cast<int>(pitch % align), &wbase);
  if (st != DEDISP_OK) return st;
  const int32_t* spos = nullptr;
  st = device_slot_pos(p, dev, dms, align, es, static_cast<int>(pitch % align), &spos);
  if (st != DEDISP_OK) return st;
  return allow_large_lds(kVariants[v - 1].fn[p->dtype]);
}

const void* batch_kernel(int v, bool pairs) {
  return (v >= 1 && v <= kNumTiled) ? kVariants[v - 1].batch[pairs ? 1 : 0] : nullptr;
}

const void* reset_kernel() { return reinterpret_cast<const void*>(&reset_counter); }
int reset_kernel_threads() { return kBatchCounters; }

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

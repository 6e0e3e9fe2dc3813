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
//
// Three staging kinds (how a sample sits in LDS and how it is added):
//  * float: float32 input as given, 128-bit LDS reads (4 samples a lane);
//  * halves: float16 input as given (2 bytes a sample), 64-bit reads, each
//    half added into a float32 accumulator by one mixed-precision FMA with
//    1.0 (exactly the float32 add of the widened value);
//  * pairs: 8-bit input widened to 16 bits beforehand, two samples a 32-bit
//    word, one integer add for two samples.
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

// ------------------------------------------------------------ direct --

// One lane per output sample.  The reference-simple variant, also the
// fallback for plans whose delay spread does not fit any tiled variant.
// Rows may be rings of `ring` samples (0: plain rows) whose window starts
// `start` samples in; start < ring and t + delay < ring, so one wrap at most.
template <typename In>
__global__ __launch_bounds__(256) void dedisp_direct(const In* __restrict__ in, int64_t pitch,
                                                     void* __restrict__ out_v, int64_t nsamp,
                                                     const int32_t* __restrict__ shift, int ndm_pad,
                                                     int nchans, int64_t tblocks, int64_t start, int64_t ring) {
  const int64_t bid = blockIdx.x;
  const int d = static_cast<int>(bid / tblocks);
  const int64_t t = (bid % tblocks) * 256 + threadIdx.x;
  if (t >= nsamp) return;
  const int32_t* sh = shift + d;
  auto at = [&](int c) {
    int64_t i = t + start + sh[static_cast<int64_t>(c) * ndm_pad];
    if (ring > 0 && i >= ring) i -= ring;
    return c * pitch + i;
  };
  if constexpr (std::is_integral<In>::value) {  // 8-bit samples, or 8-bit samples staged as 16-bit
    int32_t acc = 0;
    for (int c = 0; c < nchans; ++c) acc += static_cast<int32_t>(in[at(c)]);
    static_cast<int32_t*>(out_v)[d * nsamp + t] = acc;
  } else {
    float tot = 0.f;
    for (int c0 = 0; c0 < nchans; c0 += kChanBlock) {
      const int c1 = min(nchans, c0 + kChanBlock);
      float part = 0.f;
      for (int c = c0; c < c1; ++c) part += Elem<In>::get(in, at(c));
      tot += part;
    }
    static_cast<float*>(out_v)[d * nsamp + t] = tot;
  }
}

// ------------------------------------------------------------- tiled --

typedef uint32_t v2u __attribute__((ext_vector_type(2)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));

// Staging kinds.  ES: bytes per staged sample; ALIGN: window starts are
// aligned to 16 bytes (ALIGN samples); RB: bytes per lane of one LDS read
// (every read gives a lane 4 samples; lanes 0-62 own 252 samples a read,
// lane 63 only supplies its neighbour).
template <int K>
struct Kind;
template <>
struct Kind<kStageFloat> {
  static constexpr int ES = 4, ALIGN = 4, RB = 16;
};
template <>
struct Kind<kStageHalves> {
  static constexpr int ES = 2, ALIGN = 8, RB = 8;
};
template <>
struct Kind<kStagePairs> {
  static constexpr int ES = 2, ALIGN = 8, RB = 8;
};

// Barrier that orders LDS traffic only: vector loads issued before it stay in
// flight (a full __syncthreads() would also wait for every outstanding load).
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
// pairs the reads into two-address reads nor merges the alignment paths of a
// trial into one block joined by register copies.  Reads run ahead of the
// adds; a wait on the LDS counter then covers exactly the trial about to be
// consumed (LDS operations complete in order, so extra outstanding ones only
// make the wait stricter).

// Lane l reads its RB bytes at addr + 63*RB*k (addr already holds RB*l).
// One read of the wave spans 64*RB consecutive bytes, conflict free.
template <int N>
__device__ __forceinline__ void lds_reads(uint32_t addr, v4u (&v)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) asm volatile("ds_read_b128 %0, %1 offset:%2" : "=v"(v[k]) : "v"(addr), "i"(1008 * k));
}
template <int N>
__device__ __forceinline__ void lds_reads(uint32_t addr, v2u (&v)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) asm volatile("ds_read_b64 %0, %1 offset:%2" : "=v"(v[k]) : "v"(addr), "i"(504 * k));
}

template <int N>
__device__ __forceinline__ void lds_wait() {
  asm volatile("s_waitcnt lgkmcnt(%0)" ::"i"(N));
}

// One trial's adds for one channel, every alignment in one assembly block
// with a scalar branch inside (written as one block so that the paths share
// their accumulator registers instead of being joined by copies).  The
// position p of the trial's first sample in the slot, in bytes, selects the
// path: r = its sample index mod 4 inside the aligned read.
//
// Float (4 samples x0..x3 a lane and read): output i of the lane takes x[i+r]
// from its own read for i + r < 4, else x[i+r-4] of the next lane's read (DPP
// wave rotation folded into the add; the halo lane 63 supplies lane 62).
//
// Halves (words x = (h0, h1), y = (h2, h3)): the same selection, the next
// lane's words rotated into temporaries first; each half is added by
// v_fma_mix_f32 acc = h * 1.0 + acc (the product is exact, so this is the
// float32 add of the widened half).
//
// 8-bit pairs: e[] holds sums of samples (2i, 2i+1) of the lane, o[] the same
// one sample earlier.  Position mod 4 selects the set (bit 0) and whether the
// words are the lane's own or shifted by one word (bit 1).
#define DD_FA(a, x) "v_add_f32 %" #a ", %" #a ", %" #x "\n\t"
#define DD_FD(a, x) "v_add_f32_dpp %" #a ", %" #x ", %" #a " wave_rol:1 row_mask:0xf bank_mask:0xf\n\t"
#define DD_UA(a, x) "v_add_u32 %" #a ", %" #a ", %" #x "\n\t"
#define DD_UD(a, x) "v_add_u32_dpp %" #a ", %" #x ", %" #a " wave_rol:1 row_mask:0xf bank_mask:0xf\n\t"
#define DD_MD(t, x) "v_mov_b32_dpp %" #t ", %" #x " wave_rol:1 row_mask:0xf bank_mask:0xf\n\t"
#define DD_HL(a, x) "v_fma_mix_f32 %" #a ", %" #x ", 1.0, %" #a " op_sel_hi:[1,0,0]\n\t"
#define DD_HH(a, x) "v_fma_mix_f32 %" #a ", %" #x ", 1.0, %" #a " op_sel:[1,0,0] op_sel_hi:[1,0,0]\n\t"

// float, 4 accumulators a0..a3 from x0..x3 at alignment r
#define DD_F4_0(a0, a1, a2, a3, x0, x1, x2, x3) DD_FA(a0, x0) DD_FA(a1, x1) DD_FA(a2, x2) DD_FA(a3, x3)
#define DD_F4_1(a0, a1, a2, a3, x0, x1, x2, x3) DD_FA(a0, x1) DD_FA(a1, x2) DD_FA(a2, x3) DD_FD(a3, x0)
#define DD_F4_2(a0, a1, a2, a3, x0, x1, x2, x3) DD_FA(a0, x2) DD_FA(a1, x3) DD_FD(a2, x0) DD_FD(a3, x1)
#define DD_F4_3(a0, a1, a2, a3, x0, x1, x2, x3) DD_FA(a0, x3) DD_FD(a1, x0) DD_FD(a2, x1) DD_FD(a3, x2)

// halves, 4 accumulators from words x = (h0, h1), y = (h2, h3), temporaries t, u
#define DD_H4_0(a0, a1, a2, a3, x, y, t, u) DD_HL(a0, x) DD_HH(a1, x) DD_HL(a2, y) DD_HH(a3, y)
#define DD_H4_1(a0, a1, a2, a3, x, y, t, u) DD_MD(t, x) DD_HH(a0, x) DD_HL(a1, y) DD_HH(a2, y) DD_HL(a3, t)
#define DD_H4_2(a0, a1, a2, a3, x, y, t, u) DD_MD(t, x) DD_HL(a0, y) DD_HH(a1, y) DD_HL(a2, t) DD_HH(a3, t)
#define DD_H4_3(a0, a1, a2, a3, x, y, t, u) DD_MD(t, x) DD_MD(u, y) DD_HH(a0, y) DD_HL(a1, t) DD_HH(a2, t) DD_HL(a3, u)

#define DD_U_AL2(a0, a1, x0, x1) DD_UA(a0, x0) DD_UA(a1, x1)
#define DD_U_SH2(a0, a1, x0, x1) DD_UA(a0, x1) DD_UD(a1, x0)

// Four-way scalar branch on bits B0 (low) and B1 of SGPR operand P, NOP
// before each path that has DPP adds.  A DPP operation needs two wait states
// after a vector write of a register it reads; every path is reached through
// four scalar instructions (two tests, two branches), which give them, so the
// float and 8-bit paths take no NOP.  The half paths keep one two-state NOP
// (measured 2 % faster with it than without).
#define DD_BR4X(P, B0, B1, NOP, A0, A2, A1, A3)                                       \
  "s_bitcmp1_b32 %" #P ", " #B0 "\n\t"                                               \
  "s_cbranch_scc1 .Ldd_o%=\n\t"                                                       \
  "s_bitcmp1_b32 %" #P ", " #B1 "\n\t"                                               \
  "s_cbranch_scc1 .Ldd_2%=\n\t" A0 "s_branch .Ldd_end%=\n"                            \
  ".Ldd_2%=:\n\t" NOP A2 "s_branch .Ldd_end%=\n"                                       \
  ".Ldd_o%=:\n\t"                                                                      \
  "s_bitcmp1_b32 %" #P ", " #B1 "\n\t"                                               \
  "s_cbranch_scc1 .Ldd_3%=\n\t" NOP A1 "s_branch .Ldd_end%=\n"                         \
  ".Ldd_3%=:\n\t" NOP A3 ".Ldd_end%=:"
#define DD_BR4(P, B0, B1, A0, A2, A1, A3) DD_BR4X(P, B0, B1, "", A0, A2, A1, A3)
#define DD_BR4H(P, B0, B1, A0, A2, A1, A3) DD_BR4X(P, B0, B1, "s_nop 1\n\t", A0, A2, A1, A3)

#define DD_F4ALL(M)                                                                                   \
  M(0, 1, 2, 3, 16, 17, 18, 19) M(4, 5, 6, 7, 20, 21, 22, 23) M(8, 9, 10, 11, 24, 25, 26, 27) \
      M(12, 13, 14, 15, 28, 29, 30, 31)
#define DD_F2ALL(M) M(0, 1, 2, 3, 8, 9, 10, 11) M(4, 5, 6, 7, 12, 13, 14, 15)
#define DD_H4ALL(M)                                                                                           \
  M(0, 1, 2, 3, 18, 19, 16, 17) M(4, 5, 6, 7, 20, 21, 16, 17) M(8, 9, 10, 11, 22, 23, 16, 17) \
      M(12, 13, 14, 15, 24, 25, 16, 17)
#define DD_H2ALL(M) M(0, 1, 2, 3, 10, 11, 8, 9) M(4, 5, 6, 7, 12, 13, 8, 9)
#define DD_H8ALL(M) M(0, 1, 2, 3, 34, 35, 32, 33) M(4, 5, 6, 7, 36, 37, 32, 33) M(8, 9, 10, 11, 38, 39, 32, 33) M(12, 13, 14, 15, 40, 41, 32, 33) M(16, 17, 18, 19, 42, 43, 32, 33) M(20, 21, 22, 23, 44, 45, 32, 33) M(24, 25, 26, 27, 46, 47, 32, 33) M(28, 29, 30, 31, 48, 49, 32, 33)
// 8-bit pairs, 8 reads: e = %0-15, o = %16-31, reads %32-47
#define DD_U8E(F) F(0, 1, 32, 33) F(2, 3, 34, 35) F(4, 5, 36, 37) F(6, 7, 38, 39) F(8, 9, 40, 41) F(10, 11, 42, 43) F(12, 13, 44, 45) F(14, 15, 46, 47)
#define DD_U8O(F) F(16, 17, 32, 33) F(18, 19, 34, 35) F(20, 21, 36, 37) F(22, 23, 38, 39) F(24, 25, 40, 41) F(26, 27, 42, 43) F(28, 29, 44, 45) F(30, 31, 46, 47)

template <int N>
struct TrialAdds;

template <>
struct TrialAdds<4> {
  // a[0..15] += the block of 4 128-bit reads
  static __device__ __forceinline__ void f32(float* x, const v4u (&v)[4], int p) {
    asm volatile(DD_BR4(32, 2, 3, DD_F4ALL(DD_F4_0), DD_F4ALL(DD_F4_2), DD_F4ALL(DD_F4_1), DD_F4ALL(DD_F4_3))
                 : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]), "+v"(x[6]),
                   "+v"(x[7]), "+v"(x[8]), "+v"(x[9]), "+v"(x[10]), "+v"(x[11]), "+v"(x[12]), "+v"(x[13]),
                   "+v"(x[14]), "+v"(x[15])
                 : "v"(v[0].x), "v"(v[0].y), "v"(v[0].z), "v"(v[0].w), "v"(v[1].x), "v"(v[1].y), "v"(v[1].z),
                   "v"(v[1].w), "v"(v[2].x), "v"(v[2].y), "v"(v[2].z), "v"(v[2].w), "v"(v[3].x), "v"(v[3].y),
                   "v"(v[3].z), "v"(v[3].w), "s"(p)
                 : "scc");
  }
  // a[0..15] += the halves of 4 64-bit reads
  static __device__ __forceinline__ void f16(float* x, const v2u (&v)[4], int p) {
    uint32_t t, u;
    asm volatile(DD_BR4H(26, 1, 2, DD_H4ALL(DD_H4_0), DD_H4ALL(DD_H4_2), DD_H4ALL(DD_H4_1), DD_H4ALL(DD_H4_3))
                 : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]), "+v"(x[6]),
                   "+v"(x[7]), "+v"(x[8]), "+v"(x[9]), "+v"(x[10]), "+v"(x[11]), "+v"(x[12]), "+v"(x[13]),
                   "+v"(x[14]), "+v"(x[15]), "=&v"(t), "=&v"(u)
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

// Eight reads a block (16-bit staging, one trial a wave): twice the adds of
// four behind one scalar branch.
template <>
struct TrialAdds<8> {
  // a[0..31] += the halves of 8 64-bit reads
  static __device__ __forceinline__ void f16(float* x, const v2u (&v)[8], int p) {
    uint32_t t, u;
    asm volatile(DD_BR4H(50, 1, 2, DD_H8ALL(DD_H4_0), DD_H8ALL(DD_H4_2), DD_H8ALL(DD_H4_1), DD_H8ALL(DD_H4_3))
                 : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]), "+v"(x[6]),
                   "+v"(x[7]), "+v"(x[8]), "+v"(x[9]), "+v"(x[10]), "+v"(x[11]), "+v"(x[12]), "+v"(x[13]),
                   "+v"(x[14]), "+v"(x[15]), "+v"(x[16]), "+v"(x[17]), "+v"(x[18]), "+v"(x[19]), "+v"(x[20]),
                   "+v"(x[21]), "+v"(x[22]), "+v"(x[23]), "+v"(x[24]), "+v"(x[25]), "+v"(x[26]), "+v"(x[27]),
                   "+v"(x[28]), "+v"(x[29]), "+v"(x[30]), "+v"(x[31]), "=&v"(t), "=&v"(u)
                 : "v"(v[0].x), "v"(v[0].y), "v"(v[1].x), "v"(v[1].y), "v"(v[2].x), "v"(v[2].y), "v"(v[3].x),
                   "v"(v[3].y), "v"(v[4].x), "v"(v[4].y), "v"(v[5].x), "v"(v[5].y), "v"(v[6].x), "v"(v[6].y),
                   "v"(v[7].x), "v"(v[7].y), "s"(p)
                 : "scc");
  }
  // e[0..15], o[0..15]
  static __device__ __forceinline__ void u8(uint32_t* e, uint32_t* o, const v2u (&v)[8], int p) {
    asm volatile(DD_BR4(48, 1, 2, DD_U8E(DD_U_AL2), DD_U8E(DD_U_SH2), DD_U8O(DD_U_AL2), DD_U8O(DD_U_SH2))
                 : "+v"(e[0]), "+v"(e[1]), "+v"(e[2]), "+v"(e[3]), "+v"(e[4]), "+v"(e[5]), "+v"(e[6]),
                   "+v"(e[7]), "+v"(e[8]), "+v"(e[9]), "+v"(e[10]), "+v"(e[11]), "+v"(e[12]), "+v"(e[13]),
                   "+v"(e[14]), "+v"(e[15]), "+v"(o[0]), "+v"(o[1]), "+v"(o[2]), "+v"(o[3]), "+v"(o[4]),
                   "+v"(o[5]), "+v"(o[6]), "+v"(o[7]), "+v"(o[8]), "+v"(o[9]), "+v"(o[10]), "+v"(o[11]),
                   "+v"(o[12]), "+v"(o[13]), "+v"(o[14]), "+v"(o[15])
                 : "v"(v[0].x), "v"(v[0].y), "v"(v[1].x), "v"(v[1].y), "v"(v[2].x), "v"(v[2].y), "v"(v[3].x),
                   "v"(v[3].y), "v"(v[4].x), "v"(v[4].y), "v"(v[5].x), "v"(v[5].y), "v"(v[6].x), "v"(v[6].y),
                   "v"(v[7].x), "v"(v[7].y), "s"(p)
                 : "scc");
  }
};

template <>
struct TrialAdds<2> {
  static __device__ __forceinline__ void f32(float* x, const v4u (&v)[2], int p) {
    asm volatile(DD_BR4(16, 2, 3, DD_F2ALL(DD_F4_0), DD_F2ALL(DD_F4_2), DD_F2ALL(DD_F4_1), DD_F2ALL(DD_F4_3))
                 : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]), "+v"(x[6]),
                   "+v"(x[7])
                 : "v"(v[0].x), "v"(v[0].y), "v"(v[0].z), "v"(v[0].w), "v"(v[1].x), "v"(v[1].y), "v"(v[1].z),
                   "v"(v[1].w), "s"(p)
                 : "scc");
  }
  static __device__ __forceinline__ void f16(float* x, const v2u (&v)[2], int p) {
    uint32_t t, u;
    asm volatile(DD_BR4H(14, 1, 2, DD_H2ALL(DD_H4_0), DD_H2ALL(DD_H4_2), DD_H2ALL(DD_H4_1), DD_H2ALL(DD_H4_3))
                 : "+v"(x[0]), "+v"(x[1]), "+v"(x[2]), "+v"(x[3]), "+v"(x[4]), "+v"(x[5]), "+v"(x[6]),
                   "+v"(x[7]), "=&v"(t), "=&v"(u)
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

// Buffer resource for `bytes` bytes from `p` (raw buffer, range checked: reads
// past the end return zero without touching memory; more than 2^32 - 1 bytes
// are clamped to that).  The address and size are wave-uniform by construction;
// taking them through readfirstlane lets the compiler see that and keep the
// resource in scalar registers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* p, int64_t bytes) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t n = bytes >= 0xffffffffll ? 0xffffffffu : static_cast<uint32_t>(bytes < 0 ? 0 : bytes);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<int>(a & 0xffffffffu));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<int>(a >> 32));
  const int nu = __builtin_amdgcn_readfirstlane(static_cast<int>(n));
  void* base = reinterpret_cast<void*>((static_cast<uint64_t>(hi) << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, nu, 0x00020000);
}

// K runs of 1 KB from the buffer straight into LDS: run m takes 16 bytes per
// lane from byte offset voff + 1024*m to LDS byte lds + 1024*m + 16*lane (the
// instruction's immediate offset moves both addresses, so the runs share one
// M0 value, which the compiler sets, and one offset register).
template <int K>
__device__ __forceinline__ void lds_dma_runs(uint32_t lds, uint32_t voff, __amdgpu_buffer_rsrc_t r) {
  static_assert(K >= 1 && K <= 4, "immediate offsets stay below 4 KB");
  __attribute__((address_space(3))) void* dst =
      (__attribute__((address_space(3))) void*)(static_cast<uintptr_t>(lds));
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, dst, 16, voff, 0, 0, 0);
  if constexpr (K >= 2) __builtin_amdgcn_raw_ptr_buffer_load_lds(r, dst, 16, voff, 0, 1024, 0);
  if constexpr (K >= 3) __builtin_amdgcn_raw_ptr_buffer_load_lds(r, dst, 16, voff, 0, 2048, 0);
  if constexpr (K >= 4) __builtin_amdgcn_raw_ptr_buffer_load_lds(r, dst, 16, voff, 0, 3072, 0);
}

__device__ __forceinline__ void lds_dma_k(int k, uint32_t lds, uint32_t voff, __amdgpu_buffer_rsrc_t rs) {
  if (k >= 4)
    lds_dma_runs<4>(lds, voff, rs);
  else if (k == 3)
    lds_dma_runs<3>(lds, voff, rs);
  else if (k == 2)
    lds_dma_runs<2>(lds, voff, rs);
  else
    lds_dma_runs<1>(lds, voff, rs);
}

// LDS read address of a (channel, trial) block: the lane's base plus the
// trial's byte position in the slot with its alignment bits cleared (two
// vector operations, so that no scalar instruction is spent on it).
template <int RB>
__device__ __forceinline__ uint32_t block_addr(uint32_t vbase, int q) {
  uint32_t r;
  asm volatile("v_and_b32_e64 %0, %1, %3\n\tv_add_u32 %0, %0, %2" : "=&v"(r) : "s"(q), "v"(vbase), "i"(-RB));
  return r;
}

// Workgroup barrier after this wave's LDS writes have completed.  Writes that
// go to LDS through the vector memory path are waited for explicitly before.
__device__ __forceinline__ void lds_barrier_asm() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Tile kernel body.  The input is staged by loads that write LDS directly
// (no registers), in one of three kinds (float, halves, 16-bit pairs of 8-bit
// samples widened beforehand).
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
// zeros.  Rows may also be rings (a streaming beam's history and newest block
// in one buffer row of ring_bytes): a window then starts start_bytes further
// on, modulo the ring, and loads that cross the end of the ring continue at
// its start.  Two tables built on the host give, per (trial tile, channel),
// the byte offset of the window and its number of loads and, per trial, the
// byte position of its first sample inside the slot, whose low bits carry the
// alignment the adds need.  Both are padded past the last channel, so reading
// them a stage ahead needs no check; the slots of channels past the last one
// are zeroed instead of loaded, so adding them needs no check either.
//
// A (channel, trial) block reads its samples with aligned reads, several
// blocks of reads in flight.  Lanes 0-62 own the output samples; lane 63 only
// supplies its neighbour when the block's window position is not a multiple
// of the read.  8-bit blocks have a second alignment, the sample within a
// word: odd positions accumulate into a second set of words that holds every
// sum one sample earlier, and the two sets are combined into 32-bit totals
// every 256 channels.  Float sums (float and half input): channels ascending,
// summed in blocks of kChanBlock into a partial that is then added to the
// total (the same order in every variant).
template <int KIND, int DW, int KS, int WD, int WT, int CG, int IW>
__device__ __forceinline__ void tile_dma(const TiledArgs& a, int dm_tile, int t_tile) {
  typedef Kind<KIND> K;
  constexpr bool kPairs = KIND == kStagePairs;
  constexpr int NW = WD * WT;
  constexpr int SPW = 126 * KS;  // samples per wave
  constexpr int T = SPW * WT;
  constexpr int NR = KS / 2;                // LDS reads per lane and block (4 samples each)
  constexpr int ES = K::ES;                 // bytes per staged sample
  constexpr int RB = K::RB;                 // bytes per lane and read
  constexpr int WPG = NW / CG;              // waves per issuing group
  constexpr int NB = CG * DW;               // (channel, trial) blocks per stage
  constexpr int QS = DW * WD;               // trials per tile (slot-position row length)
  constexpr int D = (3 - 1) * NR <= 15 ? 3 : 2;  // blocks with reads in flight
  constexpr int FLUSH = kPairs ? 256 : kChanBlock;
  static_assert(KS % 2 == 0 && (D - 1) * NR <= 15, "tile shape");
  static_assert(NW % CG == 0 && FLUSH % CG == 0, "stage shape");
  static_assert(IW >= 1 && IW <= WPG, "waves that load a window");
  static_assert((SPW * ES) % 16 == 0, "time offset of a wave keeps the read alignment");
  typedef typename std::conditional<RB == 16, v4u, v2u>::type Rd;
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
  constexpr int ALIGN = K::ALIGN;  // window starts are aligned to 16 bytes
  const uint32_t lane16 = 16u * static_cast<uint32_t>(lane);
  // read base of the lane: its RB bytes, and the wave's offset along time
  const uint32_t vlane = lds0 + RB * static_cast<uint32_t>(lane) + static_cast<uint32_t>(ES * SPW * wt);
  const uint32_t t0b = static_cast<uint32_t>(ES * t0) + a.start_bytes;
  const uint32_t ring = a.ring_bytes;  // 0: plain rows
  cint32* wb = (cint32*)(a.wbase) + 2 * (static_cast<int64_t>(dm_tile) * (nchans + kGeoPad) + grp);
  cint32* sp = (cint32*)(a.spos) + static_cast<int64_t>(dm_tile) * (nchans + kGeoPad) * QS + wd * DW;

  // The samples of a float or half input past its last whole 16 bytes
  // (1-3 floats, 1-7 halves) are read once here; the slot holding them
  // patches them in.  (Widened inputs and rings are whole.)
  uint32_t tailw[4] = {0u, 0u, 0u, 0u};
  int c_tail = nchans;  // first channel whose window can reach them
  const bool has_tail = !kPairs && ring == 0 && a.ntail > 0;  // the same for the whole launch
  if (has_tail) {
    if constexpr (KIND == kStageFloat) {
      const uint32_t* in32 = static_cast<const uint32_t*>(a.in);
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (k < a.ntail) tailw[k] = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(in32[a.total16 + k])));
    } else {
      const uint16_t* in16 = static_cast<const uint16_t*>(a.in);
#pragma unroll
      for (int k = 0; k < 7; ++k)
        if (k < a.ntail)
          tailw[k >> 1] |= static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(in16[a.total16 + k])))
                           << (16 * (k & 1));
    }
    // a window ends before c*pitch + t0 + max_shift + T + 10
    const int64_t lim = a.total16 - t0 - a.max_shift - (T + 10);
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
      const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(static_cast<const char*>(a.in) + rb, ring ? static_cast<int64_t>(ring)
                                                                             : a.total16 * ES - rb);
      uint32_t lds = __builtin_amdgcn_readfirstlane(lds0 + slot + 4096u * gq);
      uint32_t u = wbase + t0b + 4096u * gq;  // wave-uniform byte offset of the chunk in the row
      for (int i = 4 * gq; i < runs; i += 4 * IW, lds += 4096u * IW, u += 4096u * IW) {
        const int k = runs - i;
        if (ring == 0) {
          lds_dma_k(k, lds, u + lane16, rs);
        } else {
          // A window starts below twice the ring; rings hold the history,
          // the block and 4608 more samples, so one subtraction wraps every
          // offset the block's outputs need.  Only the one-trial tile (8064
          // samples) reads further past the block: those offsets wrap once
          // more below, or read zeros through the descriptor's range check,
          // and feed outputs past the block only.  Offsets stay below 2^32
          // (launch_rows takes the direct kernel for longer rings).
          uint32_t w = u >= ring ? u - ring : u;
          if (w + 1024u * static_cast<uint32_t>(k < 4 ? k : 4) <= ring) {
            lds_dma_k(k, lds, w + lane16, rs);
          } else {  // the chunk crosses the end of the ring: run by run, lane by lane
            for (int m = 0; m < 4 && m < k; ++m) {
              uint32_t wm = w + 1024u * m;
              if (wm >= ring) wm -= ring;
              uint32_t vo = wm + lane16;
              if (vo >= ring) vo -= ring;
              lds_dma_runs<1>(lds + 1024u * m, vo, rs);
            }
          }
        }
      }
    } else if (c < nstages * CG && gq == 0) {
      for (int m = 0; m < a.runs; ++m)
        *reinterpret_cast<float4*>(reinterpret_cast<char*>(lds4) + slot + 1024u * m + lane16) =
            make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  // After the loads of channel c landed: the partial last 16 bytes of the
  // input, if the slot holds them, are patched in by the lane that loaded
  // their place.
  auto patch = [&](int c, uint32_t wbase, int runs, uint32_t slot) {
    if (kPairs || c >= nchans || c < c_tail) return;
    const int64_t off = static_cast<int64_t>(a.total16) * ES - (row_base(c) + wbase + t0b);
    if (off < 0 || off >= 1024 * static_cast<int64_t>(runs)) return;
    if ((off >> 12) % IW != gq) return;  // the wave that loaded its 4 KB
    const uint32_t o = static_cast<uint32_t>(off);
    if (lane == ((o >> 4) & 63))
      *reinterpret_cast<uint4*>(reinterpret_cast<char*>(lds4) + slot + o) =
          make_uint4(tailw[0], tailw[1], tailw[2], tailw[3]);
  };

  // Accumulators.  Float: acc0 = partial of the current block of channels,
  // tot = total.  8-bit: acc0/acc1 = words of two 16-bit sums (acc1 one
  // sample earlier), tot = 32-bit totals.
  constexpr int NA = kPairs ? 2 * NR : 4 * NR;
  typedef typename std::conditional<kPairs, uint32_t, float>::type Acc;
  Acc acc0[DW][NA];
  Acc acc1[DW][kPairs ? NA : 1];
  Acc tot[DW][4 * NR];
#pragma unroll
  for (int j = 0; j < DW; ++j) {
#pragma unroll
    for (int k = 0; k < NA; ++k) acc0[j][k] = 0;
#pragma unroll
    for (int k = 0; k < (kPairs ? NA : 1); ++k) acc1[j][k] = 0;
#pragma unroll
    for (int k = 0; k < 4 * NR; ++k) tot[j][k] = 0;
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
    auto ba = [&](int b) { return block_addr<RB>(vlane + sbase + (b / DW) * slot_bytes, q[b / DW][b % DW]); };
    Rd rb[D][NR];
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
      if constexpr (KIND == kStagePairs)
        TrialAdds<NR>::u8(acc0[b % DW], acc1[b % DW], rb[b % D], q[b / DW][b % DW]);
      else if constexpr (KIND == kStageHalves)
        TrialAdds<NR>::f16(acc0[b % DW], rb[b % D], q[b / DW][b % DW]);
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
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int64_t t = static_cast<int64_t>(t0) + wt * SPW + 4 * lane + 252 * k;
      if constexpr (kPairs) {
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
      } else {
        float* o = static_cast<float*>(a.out) + d * nsamp + t;
        if (t + 3 < nsamp) {
          const float4 w4 = make_float4(tot[j][4 * k], tot[j][4 * k + 1], tot[j][4 * k + 2], tot[j][4 * k + 3]);
          __builtin_memcpy(o, &w4, 16);
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (t + i < nsamp) o[i] = tot[j][4 * k + i];
        }
      }
    }
  }
}

// Widening of 8-bit input to 16 bits into a buffer padded with zeros to npad
// samples (a multiple of 8): 8 samples per thread.
__device__ __forceinline__ uint4 widen8(uint2 w) {
  uint4 o;
  o.x = (w.x & 0xffu) | ((w.x & 0xff00u) << 8);
  o.y = ((w.x >> 16) & 0xffu) | ((w.x >> 8) & 0xff0000u);
  o.z = (w.y & 0xffu) | ((w.y & 0xff00u) << 8);
  o.w = ((w.y >> 16) & 0xffu) | ((w.y >> 8) & 0xff0000u);
  return o;
}

__global__ __launch_bounds__(256) void widen_u8(const uint8_t* __restrict__ in, uint16_t* __restrict__ out,
                                                int64_t n, int64_t npad) {
  const int64_t i = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) * 8;
  if (i >= npad) return;
  if (i + 8 <= n) {
    uint2 w;
    __builtin_memcpy(&w, in + i, 8);
    *reinterpret_cast<uint4*>(out + i) = widen8(w);
  } else {
#pragma unroll
    for (int k = 0; k < 8; ++k) out[i + k] = i + k < n ? in[i + k] : 0;
  }
}

// Widening of the 8-bit inputs of a batch: blockIdx.y selects the job, the
// blocks of a job stride over its samples, 8 per thread.
__global__ __launch_bounds__(256) void widen_job_kernel(const WidenJob* __restrict__ jobs) {
  const WidenJob j = jobs[blockIdx.y];
  const uint8_t* in = static_cast<const uint8_t*>(j.in);
  uint16_t* out = static_cast<uint16_t*>(j.ws);
  for (int64_t i = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) * 8; i < j.npad;
       i += static_cast<int64_t>(gridDim.x) * 256 * 8) {
    if (i + 8 <= j.n) {
      uint2 w;
      __builtin_memcpy(&w, in + i, 8);
      *reinterpret_cast<uint4*>(out + i) = widen8(w);
    } else {
      for (int k = 0; k < 8; ++k) out[i + k] = i + k < j.n ? in[i + k] : 0;
    }
  }
}

// A streaming block [nchans][block] (raw) appended to its beam's ring rows
// [nchans][ring] in staged form (8-bit widened to 16 bits; float and half as
// they are), sample j of a row at ring position (pos + j) mod ring.  Rows are
// strided over blockIdx.y, 8 samples per thread over blockIdx.x: with pos,
// block and ring multiples of 8 each thread moves 8 aligned samples (no
// group crosses the end of the ring), otherwise it moves them one by one.
template <typename In, typename St>
__global__ __launch_bounds__(256) void ring_append(const In* __restrict__ blk, St* __restrict__ ring_rows,
                                                   int64_t block, int64_t ring, int64_t pos, int nchans) {
  const bool vec = (pos % 8) == 0 && (block % 8) == 0 && (ring % 8) == 0;
  for (int c = blockIdx.y; c < nchans; c += gridDim.y) {
    const In* src = blk + c * block;
    St* dst = ring_rows + c * ring;
    for (int64_t j = (static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x) * 8; j < block;
         j += static_cast<int64_t>(gridDim.x) * 256 * 8) {
      int64_t p = pos + j;
      if (p >= ring) p -= ring;
      if (vec) {
        if constexpr (sizeof(In) == 1) {
          uint2 w;
          __builtin_memcpy(&w, src + j, 8);
          *reinterpret_cast<uint4*>(dst + p) = widen8(w);
        } else {
          constexpr int NV = sizeof(In) * 8 / 16;  // 16-byte vectors per 8 samples
#pragma unroll
          for (int v = 0; v < NV; ++v)
            reinterpret_cast<uint4*>(dst + p)[v] = reinterpret_cast<const uint4*>(src + j)[v];
        }
      } else {
        for (int k = 0; k < 8 && j + k < block; ++k) {
          int64_t pk = p + k;
          if (pk >= ring) pk -= ring;
          if constexpr (sizeof(In) == 1)
            dst[pk] = static_cast<St>(src[j + k]);
          else
            dst[pk] = src[j + k];
        }
      }
    }
  }
}

// One launch of a tile variant for one staging kind.
template <int KIND, int DW, int KS, int WD, int WT, int CG, int IW>
__global__ __launch_bounds__(64 * WD * WT) void dedisp_tiled(const TiledArgs a) {
  int dm_tile, t_tile;
  if (!tile_of(a, dm_tile, t_tile)) return;  // padding block of the last group
  tile_dma<KIND, DW, KS, WD, WT, CG, IW>(a, dm_tile, t_tile);
}

// Persistent batch kernel: resident workgroups pull (beam, trial tile, time
// tile) items from atomic counters (one per XCD) until none are left.  Items are
// numbered beam by beam, beams in order of decreasing cost per item (longest
// items first), and inside a beam in the same groups as a single launch.  One
// kernel per staging kind, so that each carries the registers of one path
// only.
template <int KIND, int DW, int KS, int WD, int WT, int CG, int IW>
__global__ __launch_bounds__(64 * WD * WT) __attribute__((amdgpu_waves_per_eu(DW <= 2 ? 4 : 2)))
void dedisp_batch_persistent(const BatchArgs b) {
  __shared__ long long item_s[2];
  // Blocks run on XCD blockIdx.x mod 8.  Items go out in chunks of
  // kBatchChunk consecutive ones (neighbouring tiles of a beam, whose windows
  // overlap), chunk j to counter j mod nx: the workgroups of one XCD share a
  // counter, so a chunk stays in one L2, and every XCD gets the same mix of
  // beams.  (With fewer than 8 workgroups, nx = the grid.)  The next item is
  // claimed while the current one runs, so the counter's latency is off the
  // path between items.
  const int nx = gridDim.x < 8 ? static_cast<int>(gridDim.x) : 8;
  const int xcd = static_cast<int>(blockIdx.x) % nx;
  if (threadIdx.x == 0) item_s[0] = static_cast<long long>(atomicAdd(b.counter + xcd, 1ull));
  lds_barrier();
  for (int cur = 0;; cur ^= 1) {
    const long long k =
        static_cast<long long>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(item_s[cur])))) |
        (static_cast<long long>(__builtin_amdgcn_readfirstlane(static_cast<int>(item_s[cur] >> 32))) << 32);
    const long long item = (k / kBatchChunk) * (nx * kBatchChunk) + xcd * kBatchChunk + k % kBatchChunk;
    if (item >= b.n_items) return;  // the counter's later items are further on
    // claimed now, stored at the end of the item: its latency overlaps the tile
    unsigned long long next = 0;
    if (threadIdx.x == 0) next = atomicAdd(b.counter + xcd, 1ull);
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
    if (dm_tile < a.n_dm_tiles && t_tile < a.n_t_tiles) tile_dma<KIND, DW, KS, WD, WT, CG, IW>(a, dm_tile, t_tile);
    if (threadIdx.x == 0) item_s[cur ^ 1] = static_cast<long long>(next);
    // every wave is done with this item's LDS, and the next item's index is visible
    lds_barrier();
  }
}

__global__ void reset_counter(unsigned long long* c) {
  if (threadIdx.x < kBatchCounters) c[threadIdx.x] = 0ull;
}

// ------------------------------------------------------ static scratch --

// Workspace of the allocation-free entry point (dedisp_execute_static): the
// widened copy of an 8-bit input.  Every device the library runs on holds one
// until the process ends; calls on one device share it.
constexpr size_t kStaticScratchBytes = static_cast<size_t>(1) << 30;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

// ----------------------------------------------------------- registry --

struct Variant {
  TileShape shape;
  int cg;                // channels per stage
  int iw;                // waves of a group that load a window
  const void* fn[3];     // by staging kind: float, halves, pairs
  const void* batch[3];  // persistent batch kernel by staging kind
};

#define DEDISP_VARIANT(DW, KS, WD, WT, CG, IW)                                                             \
  Variant {                                                                                               \
    TileShape{DW, KS, WD, WT}, CG, IW,                                                                    \
        {reinterpret_cast<const void*>(&dedisp_tiled<kStageFloat, DW, KS, WD, WT, CG, IW>),               \
         reinterpret_cast<const void*>(&dedisp_tiled<kStageHalves, DW, KS, WD, WT, CG, IW>),              \
         reinterpret_cast<const void*>(&dedisp_tiled<kStagePairs, DW, KS, WD, WT, CG, IW>)},              \
        {reinterpret_cast<const void*>(&dedisp_batch_persistent<kStageFloat, DW, KS, WD, WT, CG, IW>),    \
         reinterpret_cast<const void*>(&dedisp_batch_persistent<kStageHalves, DW, KS, WD, WT, CG, IW>),   \
         reinterpret_cast<const void*>(&dedisp_batch_persistent<kStagePairs, DW, KS, WD, WT, CG, IW>)}    \
  }

// Variants for the 16-bit staging kinds only (halves and 8-bit pairs): no
// float kernel.
#define DEDISP_VARIANT_16(DW, KS, WD, WT, CG, IW)                                                         \
  Variant {                                                                                               \
    TileShape{DW, KS, WD, WT}, CG, IW,                                                                    \
        {nullptr, reinterpret_cast<const void*>(&dedisp_tiled<kStageHalves, DW, KS, WD, WT, CG, IW>),     \
         reinterpret_cast<const void*>(&dedisp_tiled<kStagePairs, DW, KS, WD, WT, CG, IW>)},              \
        {nullptr, reinterpret_cast<const void*>(&dedisp_batch_persistent<kStageHalves, DW, KS, WD, WT, CG, IW>), \
         reinterpret_cast<const void*>(&dedisp_batch_persistent<kStagePairs, DW, KS, WD, WT, CG, IW>)}    \
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
    // one trial a wave, 2016 samples, eight reads a block (16-bit staging only)
    DEDISP_VARIANT_16(1, 16, 8, 1, 4, 2),   // 8 x 2016, 512 threads, 4 channels per stage
    DEDISP_VARIANT_16(1, 16, 8, 1, 8, 1),   // 8 x 2016, 512 threads, 8 channels per stage
    DEDISP_VARIANT_16(1, 16, 16, 1, 8, 2),  // 16 x 2016, 1024 threads, 8 channels per stage
    // few trials a tile, for delay spreads too wide for the tiles above
    DEDISP_VARIANT(1, 8, 2, 4, 1, 4),  // 2 x 4032, 512 threads, 1 channel per stage
    DEDISP_VARIANT(1, 8, 1, 8, 1, 4),  // 1 x 8064, 512 threads, 1 channel per stage (any spread)
};
constexpr int kNumTiled = sizeof(kVariants) / sizeof(kVariants[0]);

// Bumped whenever the tile kernels change in a way that can change which
// variant is fastest (the autotuner's cache keys carry it).
constexpr int kKernelGeneration = 3;

constexpr size_t kMaxLds = 160 * 1024;

// Bytes a lane reads past a block's last sample (the halo lane's read) for a
// staging kind.
inline int halo_bytes(int dtype) { return staged_size(dtype) == 4 ? 16 : 8; }

// 1 KB loads per LDS slot (one channel's window) a tiled variant needs for
// this plan, or 0 if the plan's delay spread is too wide for the variant's
// LDS.  A window covers the tile's samples, the delay spread of its trials,
// the alignment of its start (16 bytes) and the halo lane's read past the
// last sample.  Two stages of `cg` slots are live.
int slot_runs(dedisp_plan p, const Variant& v) {
  const std::vector<int2>& w = host_windows(p, v.shape.dms());
  int spread = 0;
  for (const int2& x : w) spread = std::max(spread, x.y - x.x);
  const int64_t es = staged_size(p->dtype);
  const int64_t align = stage_align(p->dtype);
  const int64_t bytes = es * (static_cast<int64_t>(spread) + align - 1 + v.shape.samples()) + halo_bytes(p->dtype);
  const int64_t runs = (bytes + 1023) / 1024;
  if (2 * v.cg * runs * 1024 > static_cast<int64_t>(kMaxLds) - 256) return 0;  // 256 B for static LDS
  return static_cast<int>(runs);
}

// The tiled kernels address a row (and a window past its end) with 32-bit
// byte offsets from the row's start.
bool offsets_fit(dedisp_plan p, int64_t pitch) {
  return (pitch + 16) * staged_size(p->dtype) + (static_cast<int64_t>(1) << 20) < (static_cast<int64_t>(1) << 32);
}

}  // namespace

int variant_count() { return 1 + kNumTiled; }

TileShape variant_shape(int v) { return kVariants[v - 1].shape; }

uint64_t registry_signature() {
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the registry's parameters
  auto mix = [&h](int x) {
    for (int k = 0; k < 4; ++k) h = (h ^ static_cast<unsigned char>(x >> (8 * k))) * 1099511628211ull;
  };
  mix(kKernelGeneration);
  for (const Variant& v : kVariants) {
    mix(v.shape.dw);
    mix(v.shape.ks);
    mix(v.shape.wd);
    mix(v.shape.wt);
    mix(v.cg);
    mix(v.iw);
  }
  return h;
}

int tiled_per_cu(dedisp_plan p, int v) {
  if (v < 1 || v > kNumTiled) return 0;
  const int runs = slot_runs(p, kVariants[v - 1]);
  if (runs == 0) return 0;
  return static_cast<int>((kMaxLds - 256) / (2 * static_cast<size_t>(kVariants[v - 1].cg) * runs * 1024));
}

bool variant_fits(dedisp_plan p, int v) {
  if (v == 0) return true;
  if (v < 0 || v > kNumTiled) return false;
  return kVariants[v - 1].fn[stage_kind(p->dtype)] != nullptr && slot_runs(p, kVariants[v - 1]) > 0;
}

int default_variant(dedisp_plan p) {
  static const int order[] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16};
  for (int v : order)
    if (v <= kNumTiled && variant_fits(p, v)) return v;
  return 0;
}

namespace {

// The direct kernel over input of sample type In (raw or staged), rows of
// `pitch` samples (rings of `ring` samples whose windows start `start` in,
// or plain rows when ring = 0).
template <typename In>
int launch_direct(dedisp_plan p, const DeviceTables* dt, const void* in, void* out, int64_t nsamp, int64_t pitch,
                  int64_t start, int64_t ring, hipStream_t s) {
  const int64_t tblocks = (nsamp + 255) / 256;
  const int64_t nblocks = tblocks * p->ndm;
  if (nblocks > INT32_MAX) return DEDISP_ERR_INVALID_ARG;
  hipLaunchKernelGGL(dedisp_direct<In>, dim3(static_cast<unsigned>(nblocks)), dim3(256), 0, s,
                     static_cast<const In*>(in), pitch, out, nsamp, dt->shift, p->ndm_pad, p->nchans, tblocks, start,
                     ring);
  return DEDISP_HIP_STATUS(hipGetLastError());
}

// A tiled variant over staged input.
int launch_tiled(dedisp_plan p, int v, const StagedRows& rows, void* out, int64_t nsamp, hipStream_t s,
                 bool no_alloc = false) {
  TiledArgs a;
  size_t lds = 0;
  int64_t nblocks = 0;
  int threads = 0;
  int st = tiled_args_rows(p, v, rows, out, nsamp, &a, &lds, &nblocks, &threads, no_alloc);
  const void* fn = kVariants[v - 1].fn[stage_kind(p->dtype)];
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

int launch(dedisp_plan p, int v, const void* in, void* out, int64_t nsamp, hipStream_t s, void* ws_given,
           bool no_alloc) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  DeviceTables* dt = nullptr;
  int st = device_tables(p, dev, &dt, !no_alloc);
  if (st != DEDISP_OK) return st;
  const int64_t pitch = nsamp + p->max_shift;
  const int64_t total = pitch * p->nchans;
  // the tiled kernels address each row with 32-bit byte offsets; longer rows
  // take the direct kernel
  if (v > 0 && !offsets_fit(p, pitch)) v = 0;
  if (v == 0) {
    switch (p->dtype) {
      case DEDISP_U8: return launch_direct<uint8_t>(p, dt, in, out, nsamp, pitch, 0, 0, s);
      case DEDISP_F16: return launch_direct<__half>(p, dt, in, out, nsamp, pitch, 0, 0, s);
      default: return launch_direct<float>(p, dt, in, out, nsamp, pitch, 0, 0, s);
    }
  }
  if (p->dtype != DEDISP_U8) return launch_tiled(p, v, StagedRows{in, pitch, total, 0, 0}, out, nsamp, s, no_alloc);
  // 8-bit input is widened into a workspace first: the caller's, else a
  // stream-ordered one
  void* ws = ws_given;
  if (ws == nullptr && no_alloc) return DEDISP_ERR_INVALID_ARG;
  if (ws == nullptr) {
    st = keep_pool_memory(dev);
    if (st != DEDISP_OK) return st;
    e = hipMallocAsync(&ws, staged_bytes(p, nsamp), s);
    if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  }
  st = widen(p->dtype, in, ws, total, s);
  if (st == DEDISP_OK)
    st = launch_tiled(p, v, StagedRows{ws, pitch, widened_samples(total), 0, 0}, out, nsamp, s, no_alloc);
  if (ws_given == nullptr) {
    const int st2 = DEDISP_HIP_STATUS(hipFreeAsync(ws, s));
    if (st == DEDISP_OK) st = st2;
  }
  return st;
}

int launch_rows(dedisp_plan p, int v, const StagedRows& rows, void* out, int64_t nsamp, hipStream_t s) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  DeviceTables* dt = nullptr;
  int st = device_tables(p, dev, &dt);
  if (st != DEDISP_OK) return st;
  // ring windows are addressed from the ring's start up to twice its length
  // plus a tile, in 32-bit byte offsets
  if (v > 0 && !offsets_fit(p, rows.ring > 0 ? 2 * rows.pitch + 8192 : rows.pitch)) v = 0;
  if (v == 0) {
    // same channel order and float conversion as on raw input
    switch (p->dtype) {
      case DEDISP_U8: return launch_direct<uint16_t>(p, dt, rows.in, out, nsamp, rows.pitch, rows.start, rows.ring, s);
      case DEDISP_F16: return launch_direct<__half>(p, dt, rows.in, out, nsamp, rows.pitch, rows.start, rows.ring, s);
      default: return launch_direct<float>(p, dt, rows.in, out, nsamp, rows.pitch, rows.start, rows.ring, s);
    }
  }
  return launch_tiled(p, v, rows, out, nsamp, s);
}

size_t staged_bytes(dedisp_plan p, int64_t nsamp) {
  return static_cast<size_t>(widened_samples((nsamp + p->max_shift) * p->nchans)) * staged_size(p->dtype);
}

int ring_append(int dtype, const void* blk, void* ring_rows, int64_t block, int64_t ring, int64_t pos, int nchans,
                hipStream_t s) {
  if (nchans < 1 || block < 1 || ring < block || pos < 0 || pos >= ring) return DEDISP_ERR_INVALID_ARG;
  const unsigned gx = static_cast<unsigned>(std::min<int64_t>((block / 8 + 255) / 256 + 1, 64));
  const unsigned gy = static_cast<unsigned>(std::min(nchans, 65535));
  switch (dtype) {
    case DEDISP_U8:
      hipLaunchKernelGGL((ring_append<uint8_t, uint16_t>), dim3(gx, gy), dim3(256), 0, s,
                         static_cast<const uint8_t*>(blk), static_cast<uint16_t*>(ring_rows), block, ring, pos, nchans);
      break;
    case DEDISP_F16:
      hipLaunchKernelGGL((ring_append<uint16_t, uint16_t>), dim3(gx, gy), dim3(256), 0, s,
                         static_cast<const uint16_t*>(blk), static_cast<uint16_t*>(ring_rows), block, ring, pos,
                         nchans);
      break;
    case DEDISP_F32:
      hipLaunchKernelGGL((ring_append<float, float>), dim3(gx, gy), dim3(256), 0, s, static_cast<const float*>(blk),
                         static_cast<float*>(ring_rows), block, ring, pos, nchans);
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
  if (dtype != DEDISP_U8) return DEDISP_ERR_INVALID_ARG;
  const int64_t npad = widened_samples(total);
  const int64_t blocks = (npad / 8 + 255) / 256;
  if (blocks > INT32_MAX) return DEDISP_ERR_INVALID_ARG;
  hipLaunchKernelGGL(widen_u8, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, static_cast<const uint8_t*>(in),
                     static_cast<uint16_t*>(ws), total, npad);
  return DEDISP_HIP_STATUS(hipGetLastError());
}

int tiled_args_rows(dedisp_plan p, int v, const StagedRows& rows, void* out, int64_t nsamp, TiledArgs* ap,
                    size_t* lds_out, int64_t* nblocks_out, int* threads_out, bool no_alloc) {
  if (v < 1 || v > kNumTiled) return DEDISP_ERR_INVALID_ARG;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  DeviceTables* dt = nullptr;
  int st = device_tables(p, dev, &dt, !no_alloc);
  if (st != DEDISP_OK) return st;
  const Variant& var = kVariants[v - 1];
  if (var.fn[stage_kind(p->dtype)] == nullptr) return DEDISP_ERR_INVALID_ARG;  // no kernel for this staging kind
  const int runs = slot_runs(p, var);
  if (runs == 0) return DEDISP_ERR_INVALID_ARG;
  // the tiled kernels address each row with 32-bit byte offsets
  if (!offsets_fit(p, rows.pitch)) return DEDISP_ERR_INVALID_ARG;
  const int align = stage_align(p->dtype);
  const int es = static_cast<int>(staged_size(p->dtype));
  if (rows.ring > 0 && (rows.ring % align != 0 || rows.pitch != rows.ring || rows.start < 0 || rows.start >= rows.ring))
    return DEDISP_ERR_INVALID_ARG;
  const int pitch_mod = static_cast<int>(rows.pitch % align);
  const int start_mod = static_cast<int>(rows.start % align);
  const uint32_t* wbase = nullptr;
  st = device_window_base(p, dev, var.shape.dms(), var.shape.samples(), align, es, pitch_mod, start_mod,
                          halo_bytes(p->dtype), &wbase, !no_alloc);
  if (st != DEDISP_OK) return st;
  const int32_t* spos = nullptr;
  st = device_slot_pos(p, dev, var.shape.dms(), align, es, pitch_mod, start_mod, &spos, !no_alloc);
  if (st != DEDISP_OK) return st;
  TiledArgs& a = *ap;
  a.in = rows.in;
  a.pitch = rows.pitch;
  // staged samples in whole 16-byte groups, and the samples after them
  a.total16 = rows.total & ~static_cast<int64_t>(16 / es - 1);
  a.ntail = static_cast<int>(rows.total - a.total16);
  a.start_bytes = static_cast<uint32_t>(es * (rows.start - start_mod));
  a.ring_bytes = static_cast<uint32_t>(es * rows.ring);
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
  // groups of up to 16 trial tiles x 1 time tile (16-bit staging) or 8 x 3
  // (float staging), the fastest of a sweep of group shapes on the
  // LOFAR-shaped and MeerKAT-shaped workloads
  const bool narrow = es == 2;
  a.gd = std::min(narrow ? 16 : 8, a.n_dm_tiles);
  a.gt = std::min(narrow ? 1 : 3, a.n_t_tiles);
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

int tiled_args(dedisp_plan p, int v, const void* staged, void* out, int64_t nsamp, TiledArgs* a, size_t* lds,
               int64_t* nblocks, int* threads) {
  const int64_t pitch = nsamp + p->max_shift;
  const int64_t total = pitch * p->nchans;
  const int64_t staged_total = p->dtype == DEDISP_U8 ? widened_samples(total) : total;
  return tiled_args_rows(p, v, StagedRows{staged, pitch, staged_total, 0, 0}, out, nsamp, a, lds, nblocks, threads);
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
  const int align = stage_align(p->dtype);
  const int es = static_cast<int>(staged_size(p->dtype));
  const int dms = variant_shape(v).dms();
  const uint32_t* wbase = nullptr;
  st = device_window_base(p, dev, dms, variant_shape(v).samples(), align, es, static_cast<int>(pitch % align), 0,
                          halo_bytes(p->dtype), &wbase);
  if (st != DEDISP_OK) return st;
  const int32_t* spos = nullptr;
  st = device_slot_pos(p, dev, dms, align, es, static_cast<int>(pitch % align), 0, &spos);
  if (st != DEDISP_OK) return st;
  const void* fn = kVariants[v - 1].fn[stage_kind(p->dtype)];
  if (fn == nullptr) return DEDISP_ERR_INVALID_ARG;
  return allow_large_lds(fn);
}

int static_scratch(void** out) {
  // the array's name is a host-side stand-in: its device address is looked
  // up once per device (with that device current) and kept
  static std::mutex mu;
  static std::map<int, void*> ptrs;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return DEDISP_HIP_STATUS(e);
  std::lock_guard<std::mutex> g(mu);
  auto it = ptrs.find(dev);
  if (it == ptrs.end()) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) return DEDISP_HIP_STATUS(e != hipSuccess ? e : hipErrorInvalidSymbol);
    it = ptrs.emplace(dev, ptr).first;
  }
  *out = it->second;
  return DEDISP_OK;
}

size_t static_scratch_bytes() { return kStaticScratchBytes; }

const void* batch_kernel(int v, int kind) {
  return (v >= 1 && v <= kNumTiled && kind >= 0 && kind < 3) ? kVariants[v - 1].batch[kind] : nullptr;
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

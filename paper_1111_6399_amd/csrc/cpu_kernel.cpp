// The search on the host CPU: the paper's second algorithm, a brute-force
// de-dispersion written for the CPU's vector registers with cache-line reuse
// in mind (section "Comparisons of GPU and CPU algorithms").  Work is cut
// into tiles of kTileDm trials x kTileT output samples; a tile's input
// windows (one per channel: its samples plus the trials' delay spread) stay
// in the core's caches while every trial of the tile reads them.  For each
// trial, the samples of the tile are summed over a block of 32 channels into
// vector registers (the partial), and the partial is added to the tile's
// total: the same order as the GPU kernels, so float results are
// bit-identical to theirs (the build disables contraction, and vector adds
// are element-wise).  8-bit samples are widened to 32 bits and summed
// exactly.  Half samples are widened exactly to float.
//
// Three builds of the inner loop: AVX-512, AVX2, plain C++, chosen at run
// time from the CPU's features.  Threads take tiles from a shared counter.
#include <immintrin.h>

#include <algorithm>
#include <atomic>
#include <new>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

#include "dedisp_internal.h"

namespace {

constexpr int kTileDm = 16;
constexpr int kTileT = 256;
constexpr int kBlock = dedisp::kChanBlock;

inline float half_to_float(uint16_t h) {
  // exact widening of an IEEE binary16 value
  const uint32_t sign = static_cast<uint32_t>(h & 0x8000u) << 16;
  uint32_t exp = (h >> 10) & 0x1fu;
  uint32_t man = h & 0x3ffu;
  uint32_t bits;
  if (exp == 0) {
    if (man == 0) {
      bits = sign;
    } else {  // subnormal: normalise
      int e = -1;
      do {
        ++e;
        man <<= 1;
      } while ((man & 0x400u) == 0);
      bits = sign | static_cast<uint32_t>(127 - 15 - e) << 23 | (man & 0x3ffu) << 13;
    }
  } else if (exp == 31) {
    bits = sign | 0x7f800000u | man << 13;
  } else {
    bits = sign | (exp + 127 - 15) << 23 | man << 13;
  }
  float f;
  std::memcpy(&f, &bits, 4);
  return f;
}

struct Job {
  dedisp_plan p;
  const void* in;
  void* out;
  int64_t nsamp, pitch;
  const int32_t* shift_t;  // [ndm][nchans]
  int n_dm_tiles, n_t_tiles;
};

// ------------------------------------------------------------ plain C++ --
template <typename In>
void tile_plain(const Job& j, int d0, int d1, int64_t t0, int nt) {
  const In* in = static_cast<const In*>(j.in);
  const int nch = j.p->nchans;
  for (int d = d0; d < d1; ++d) {
    const int32_t* sh = j.shift_t + static_cast<int64_t>(d) * nch;
    if constexpr (sizeof(In) == 1) {
      int32_t tot[kTileT] = {0};
      for (int c = 0; c < nch; ++c) {
        const In* src = in + c * j.pitch + t0 + sh[c];
        for (int i = 0; i < nt; ++i) tot[i] += src[i];
      }
      int32_t* o = static_cast<int32_t*>(j.out) + d * j.nsamp + t0;
      for (int i = 0; i < nt; ++i) o[i] = tot[i];
    } else {
      float tot[kTileT] = {0.f}, part[kTileT];
      for (int c0 = 0; c0 < nch; c0 += kBlock) {
        const int c1 = std::min(nch, c0 + kBlock);
        for (int i = 0; i < nt; ++i) part[i] = 0.f;
        for (int c = c0; c < c1; ++c) {
          const In* src = in + c * j.pitch + t0 + sh[c];
          for (int i = 0; i < nt; ++i) {
            if constexpr (sizeof(In) == 2)
              part[i] += half_to_float(src[i]);
            else
              part[i] += src[i];
          }
        }
        for (int i = 0; i < nt; ++i) tot[i] += part[i];
      }
      float* o = static_cast<float*>(j.out) + d * j.nsamp + t0;
      for (int i = 0; i < nt; ++i) o[i] = tot[i];
    }
  }
}

// --------------------------------------------------------------- AVX-512 --
// A full tile (nt == kTileT): 16 vectors of 16 lanes per trial.
__attribute__((target("avx512f,avx512bw"))) void tile512_f32(const Job& j, int d0, int d1, int64_t t0, bool half) {
  const int nch = j.p->nchans;
  for (int d = d0; d < d1; ++d) {
    const int32_t* sh = j.shift_t + static_cast<int64_t>(d) * nch;
    __m512 tot[16];
    for (int k = 0; k < 16; ++k) tot[k] = _mm512_setzero_ps();
    for (int c0 = 0; c0 < nch; c0 += kBlock) {
      const int c1 = std::min(nch, c0 + kBlock);
      __m512 part[16];
      for (int k = 0; k < 16; ++k) part[k] = _mm512_setzero_ps();
      for (int c = c0; c < c1; ++c) {
        const int64_t off = c * j.pitch + t0 + sh[c];
        if (half) {
          const uint16_t* src = static_cast<const uint16_t*>(j.in) + off;
          for (int k = 0; k < 16; ++k)
            part[k] = _mm512_add_ps(part[k], _mm512_cvtph_ps(_mm256_loadu_si256(
                                                 reinterpret_cast<const __m256i*>(src + 16 * k))));
        } else {
          const float* src = static_cast<const float*>(j.in) + off;
          for (int k = 0; k < 16; ++k) part[k] = _mm512_add_ps(part[k], _mm512_loadu_ps(src + 16 * k));
        }
      }
      for (int k = 0; k < 16; ++k) tot[k] = _mm512_add_ps(tot[k], part[k]);
    }
    float* o = static_cast<float*>(j.out) + d * j.nsamp + t0;
    for (int k = 0; k < 16; ++k) _mm512_storeu_ps(o + 16 * k, tot[k]);
  }
}

__attribute__((target("avx512f,avx512bw"))) void tile512_u8(const Job& j, int d0, int d1, int64_t t0) {
  const int nch = j.p->nchans;
  const uint8_t* in = static_cast<const uint8_t*>(j.in);
  for (int d = d0; d < d1; ++d) {
    const int32_t* sh = j.shift_t + static_cast<int64_t>(d) * nch;
    __m512i tot[16];
    for (int k = 0; k < 16; ++k) tot[k] = _mm512_setzero_si512();
    for (int c = 0; c < nch; ++c) {
      const uint8_t* src = in + c * j.pitch + t0 + sh[c];
      for (int k = 0; k < 16; ++k)
        tot[k] = _mm512_add_epi32(
            tot[k], _mm512_cvtepu8_epi32(_mm_loadu_si128(reinterpret_cast<const __m128i*>(src + 16 * k))));
    }
    int32_t* o = static_cast<int32_t*>(j.out) + d * j.nsamp + t0;
    for (int k = 0; k < 16; ++k) _mm512_storeu_si512(o + 16 * k, tot[k]);
  }
}

// ------------------------------------------------------------------ AVX2 --
__attribute__((target("avx2,f16c"))) void tile256_f32(const Job& j, int d0, int d1, int64_t t0, bool half) {
  const int nch = j.p->nchans;
  for (int d = d0; d < d1; ++d) {
    const int32_t* sh = j.shift_t + static_cast<int64_t>(d) * nch;
    for (int h = 0; h < 2; ++h) {  // two halves of 128 samples: 16 registers of 8
      const int64_t tb = t0 + 128 * h;
      __m256 tot[16];
      for (int k = 0; k < 16; ++k) tot[k] = _mm256_setzero_ps();
      for (int c0 = 0; c0 < nch; c0 += kBlock) {
        const int c1 = std::min(nch, c0 + kBlock);
        __m256 part[16];
        for (int k = 0; k < 16; ++k) part[k] = _mm256_setzero_ps();
        for (int c = c0; c < c1; ++c) {
          const int64_t off = c * j.pitch + tb + sh[c];
          if (half) {
            const uint16_t* src = static_cast<const uint16_t*>(j.in) + off;
            for (int k = 0; k < 16; ++k)
              part[k] = _mm256_add_ps(part[k], _mm256_cvtph_ps(_mm_loadu_si128(
                                                   reinterpret_cast<const __m128i*>(src + 8 * k))));
          } else {
            const float* src = static_cast<const float*>(j.in) + off;
            for (int k = 0; k < 16; ++k) part[k] = _mm256_add_ps(part[k], _mm256_loadu_ps(src + 8 * k));
          }
        }
        for (int k = 0; k < 16; ++k) tot[k] = _mm256_add_ps(tot[k], part[k]);
      }
      float* o = static_cast<float*>(j.out) + d * j.nsamp + tb;
      for (int k = 0; k < 16; ++k) _mm256_storeu_ps(o + 8 * k, tot[k]);
    }
  }
}

__attribute__((target("avx2"))) void tile256_u8(const Job& j, int d0, int d1, int64_t t0) {
  const int nch = j.p->nchans;
  const uint8_t* in = static_cast<const uint8_t*>(j.in);
  for (int d = d0; d < d1; ++d) {
    const int32_t* sh = j.shift_t + static_cast<int64_t>(d) * nch;
    for (int h = 0; h < 2; ++h) {
      const int64_t tb = t0 + 128 * h;
      __m256i tot[16];
      for (int k = 0; k < 16; ++k) tot[k] = _mm256_setzero_si256();
      for (int c = 0; c < nch; ++c) {
        const uint8_t* src = in + c * j.pitch + tb + sh[c];
        for (int k = 0; k < 16; ++k)
          tot[k] = _mm256_add_epi32(
              tot[k], _mm256_cvtepu8_epi32(_mm_loadl_epi64(reinterpret_cast<const __m128i*>(src + 8 * k))));
      }
      int32_t* o = static_cast<int32_t*>(j.out) + d * j.nsamp + tb;
      for (int k = 0; k < 16; ++k) _mm256_storeu_si256(reinterpret_cast<__m256i*>(o + 8 * k), tot[k]);
    }
  }
}

// The widest vector code the host runs: 2 AVX-512, 1 AVX2, 0 plain C++.  The
// environment variable DEDISP_CPU_ISA (0, 1 or 2) caps it, so that tests can
// run every path on one machine.
int isa_level() {
  static const int level = [] {
    __builtin_cpu_init();
    int l = 0;
    if (__builtin_cpu_supports("avx512f") && __builtin_cpu_supports("avx512bw"))
      l = 2;
    else if (__builtin_cpu_supports("avx2") && __builtin_cpu_supports("f16c"))
      l = 1;
    const char* cap = std::getenv("DEDISP_CPU_ISA");
    if (cap != nullptr && cap[0] >= '0' && cap[0] <= '2' && cap[1] == '\0') l = std::min(l, cap[0] - '0');
    return l;
  }();
  return level;
}

void run_tile(const Job& j, int level, int dt, int tt) {
  const int d0 = dt * kTileDm, d1 = std::min(j.p->ndm, d0 + kTileDm);
  const int64_t t0 = static_cast<int64_t>(tt) * kTileT;
  const int nt = static_cast<int>(std::min<int64_t>(kTileT, j.nsamp - t0));
  const int dtype = j.p->dtype;
  if (nt == kTileT && level == 2) {
    if (dtype == DEDISP_U8)
      tile512_u8(j, d0, d1, t0);
    else
      tile512_f32(j, d0, d1, t0, dtype == DEDISP_F16);
  } else if (nt == kTileT && level == 1) {
    if (dtype == DEDISP_U8)
      tile256_u8(j, d0, d1, t0);
    else
      tile256_f32(j, d0, d1, t0, dtype == DEDISP_F16);
  } else {  // ragged last tile, or no vector extension
    if (dtype == DEDISP_U8)
      tile_plain<uint8_t>(j, d0, d1, t0, nt);
    else if (dtype == DEDISP_F16)
      tile_plain<uint16_t>(j, d0, d1, t0, nt);
    else
      tile_plain<float>(j, d0, d1, t0, nt);
  }
}

int run_all(dedisp_plan p, const void* in, void* out, int64_t nsamp, int nthreads, int level);

}  // namespace

extern "C" int dedisp_execute_cpu(dedisp_plan p, const void* in, void* out, int64_t nsamp, int nthreads,
                                  int* isa_used) {
  if (p == nullptr || nsamp < 0 || nthreads < 0) return DEDISP_ERR_INVALID_ARG;
  if (nsamp > static_cast<int64_t>(INT32_MAX) - p->max_shift) return DEDISP_ERR_INVALID_ARG;
  const int level = isa_level();
  if (isa_used) *isa_used = level;
  if (nsamp == 0) return DEDISP_OK;
  if (in == nullptr || out == nullptr) return DEDISP_ERR_INVALID_ARG;
  try {
    return run_all(p, in, out, nsamp, nthreads, level);
  } catch (const std::bad_alloc&) {
    return DEDISP_ERR_OUT_OF_MEMORY;
  } catch (...) {  // thread creation
    return DEDISP_ERR_INTERNAL;
  }
}

namespace {

int run_all(dedisp_plan p, const void* in, void* out, int64_t nsamp, int nthreads, int level) {
  // delays trial-major, so a trial's delays over the channels are contiguous
  std::vector<int32_t> shift_t(static_cast<size_t>(p->ndm) * p->nchans);
  for (int c = 0; c < p->nchans; ++c)
    for (int d = 0; d < p->ndm; ++d)
      shift_t[static_cast<size_t>(d) * p->nchans + c] = p->shift[static_cast<size_t>(c) * p->ndm + d];
  Job j{p, in, out, nsamp, nsamp + p->max_shift, shift_t.data(), (p->ndm + kTileDm - 1) / kTileDm,
        static_cast<int>((nsamp + kTileT - 1) / kTileT)};
  const int64_t ntiles = static_cast<int64_t>(j.n_dm_tiles) * j.n_t_tiles;
  int nt = nthreads > 0 ? nthreads : static_cast<int>(std::max(1u, std::thread::hardware_concurrency()));
  nt = static_cast<int>(std::min<int64_t>(nt, ntiles));
  std::atomic<int64_t> next{0};
  auto worker = [&]() {
    for (;;) {
      const int64_t i = next.fetch_add(1);
      if (i >= ntiles) return;
      // time tiles outermost within a stripe of trial tiles: neighbouring
      // tiles of one thread share their windows
      run_tile(j, level, static_cast<int>(i % j.n_dm_tiles), static_cast<int>(i / j.n_dm_tiles));
    }
  };
  std::vector<std::thread> pool;
  for (int i = 1; i < nt; ++i) pool.emplace_back(worker);
  worker();
  for (std::thread& t : pool) t.join();
  return DEDISP_OK;
}

}  // namespace

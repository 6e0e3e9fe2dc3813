// Corner turn of time-major filterbank samples ([t][c], the order sigproc
// files store them in) into the channel rows the search reads ([c][t], one
// row per channel, contiguous in time).  A tile of (time, channel) goes
// through LDS: read along channels (contiguous in the input), written along
// time (contiguous in the output).  8-bit samples with whole groups of 4
// channels take a kernel that moves 4 bytes per lane on the way in and 16 on
// the way out; other inputs move one sample per lane.
#include <hip/hip_runtime.h>

#include "dedisp_internal.h"

namespace dedisp {
namespace {

constexpr int kTile = 64;

template <typename T>
__global__ __launch_bounds__(256) void corner_turn_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                          int64_t nsamp, int nchans, int64_t pitch, int reverse) {
  __shared__ T tile[kTile][kTile + 1];
  const int tx = threadIdx.x & 63;
  const int ty = threadIdx.x >> 6;  // 0..3
  const int64_t t0 = static_cast<int64_t>(blockIdx.x) * kTile;
  const int c0 = blockIdx.y * kTile;
  // read: rows of time, 64 consecutive channels per wave
#pragma unroll
  for (int r = ty; r < kTile; r += 4) {
    const int64_t t = t0 + r;
    const int c = c0 + tx;
    if (t < nsamp && c < nchans) tile[r][tx] = in[t * nchans + c];
  }
  __syncthreads();
  // write: rows of channels, 64 consecutive times per wave
#pragma unroll
  for (int r = ty; r < kTile; r += 4) {
    const int c = c0 + r;
    const int64_t t = t0 + tx;
    if (t < nsamp && c < nchans) {
      const int row = reverse ? nchans - 1 - c : c;
      out[static_cast<int64_t>(row) * pitch + t] = tile[tx][r];
    }
  }
}

// 8-bit tiles: 256 channels x 128 output samples per row.  Each row of the
// output is written in aligned 16-byte pieces: the row's tiles start
// s = (-address of its sample 0) mod 16 samples late, so a tile reads
// 128 + 16 input rows and the first tile (blockIdx.x == 0) covers the
// samples before s.
constexpr int kCtT = 128;                  // output samples per tile and row
constexpr int kCtRows = kCtT + 16;         // input rows a tile reads
constexpr int kCtC = 256;                  // channels per tile (4 per lane)
constexpr int kCtPitch = kCtRows / 4 + 1;  // 32-bit words per channel in LDS (odd, fewer bank conflicts)
static_assert(kCtRows % 16 == 0, "four waves of whole groups of 4 rows");

__global__ __launch_bounds__(256) void corner_turn_u8(const uint32_t* __restrict__ in, uint8_t* __restrict__ out,
                                                      int64_t nsamp, int nchans, int64_t pitch, int reverse) {
  __shared__ uint32_t tile[kCtC * kCtPitch];  // [channel][4 samples], 37.9 KB
  constexpr int kRowsPerWave = kCtRows / 4;  // 36
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t t0 = (static_cast<int64_t>(blockIdx.x) - 1) * kCtT;  // may be negative: the head tile
  const int c0 = blockIdx.y * kCtC;
  const int nw = nchans >> 2;     // 32-bit words per input row
  const int cw = (c0 >> 2) + lane;  // this lane's word of a row: channels 4cw ... 4cw + 3
  // in: every wave reads 36 rows, one word (4 channels) per lane, 4 rows at
  // a time turned into 4 words of 4 consecutive samples of one channel
  uint32_t r[kRowsPerWave];
#pragma unroll
  for (int i = 0; i < kRowsPerWave; ++i) {
    const int64_t t = t0 + kRowsPerWave * wave + i;
    r[i] = (cw < nw && t >= 0 && t < nsamp) ? in[t * nw + cw] : 0u;
  }
#pragma unroll
  for (int g = 0; g < kRowsPerWave / 4; ++g) {
    // byte k of r[4g + i] is channel 4cw + k at sample 4g + i
    const uint32_t lo01 = __builtin_amdgcn_perm(r[4 * g + 1], r[4 * g], 0x05010400u);  // c0 t0, c0 t1, c1 t0, c1 t1
    const uint32_t hi01 = __builtin_amdgcn_perm(r[4 * g + 1], r[4 * g], 0x07030602u);  // c2 .., c3 ..
    const uint32_t lo23 = __builtin_amdgcn_perm(r[4 * g + 3], r[4 * g + 2], 0x05010400u);
    const uint32_t hi23 = __builtin_amdgcn_perm(r[4 * g + 3], r[4 * g + 2], 0x07030602u);
    uint32_t* row = tile + 4 * lane * kCtPitch + kRowsPerWave / 4 * wave + g;
    row[0 * kCtPitch] = __builtin_amdgcn_perm(lo23, lo01, 0x05040100u);  // channel 4cw: samples 4g ... 4g + 3
    row[1 * kCtPitch] = __builtin_amdgcn_perm(lo23, lo01, 0x07060302u);
    row[2 * kCtPitch] = __builtin_amdgcn_perm(hi23, hi01, 0x05040100u);
    row[3 * kCtPitch] = __builtin_amdgcn_perm(hi23, hi01, 0x07060302u);
  }
  __syncthreads();
  // out: 8 consecutive lanes write a channel's 128 samples, 16 bytes each
#pragma unroll
  for (int it = 0; it < kCtC * 8 / 256; ++it) {
    const int i = it * 256 + static_cast<int>(threadIdx.x);
    const int ch = i >> 3;
    const int j = i & 7;
    const int c = c0 + ch;
    if (c >= nchans) continue;
    uint8_t* d = out + static_cast<int64_t>(reverse ? nchans - 1 - c : c) * pitch;
    const int s = static_cast<int>((16u - (static_cast<uint32_t>(reinterpret_cast<uintptr_t>(d)) & 15u)) & 15u);
    const int b = s + 16 * j;  // first byte of the piece in the tile's row (at most 127)
    const uint32_t* src = tile + ch * kCtPitch + (b >> 2);
    uint32_t w[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) w[m] = src[m];
    uint4 v;
    v.x = __builtin_amdgcn_alignbyte(w[1], w[0], b & 3);
    v.y = __builtin_amdgcn_alignbyte(w[2], w[1], b & 3);
    v.z = __builtin_amdgcn_alignbyte(w[3], w[2], b & 3);
    v.w = __builtin_amdgcn_alignbyte(w[4], w[3], b & 3);
    const int64_t t = t0 + b;  // sample of the piece's first byte; its address is 16-aligned
    if (t >= 0 && t + 16 <= nsamp) {
      *reinterpret_cast<uint4*>(d + t) = v;
    } else {  // the row's first or last piece
      const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int e = 0; e < 16; ++e)
        if (t + e >= 0 && t + e < nsamp) d[t + e] = static_cast<uint8_t>(vw[e >> 2] >> (8 * (e & 3)));
    }
  }
}

}  // namespace

int corner_turn(const void* in, void* out, int64_t nsamp, int nchans, int64_t pitch, int dtype, int reverse,
                hipStream_t s) {
  const int64_t tb = (nsamp + kTile - 1) / kTile;
  const int cb = (nchans + kTile - 1) / kTile;
  if (tb > INT32_MAX || cb > 65535) return DEDISP_ERR_INVALID_ARG;
  const dim3 grid(static_cast<unsigned>(tb), static_cast<unsigned>(cb));
  if (dtype == DEDISP_U8 && nchans % 4 == 0 && reinterpret_cast<uintptr_t>(in) % 4 == 0) {
    const int64_t nt = (nsamp + kCtT - 1) / kCtT + 1;  // with the head tile
    const int nc = (nchans + kCtC - 1) / kCtC;
    if (nt > INT32_MAX) return DEDISP_ERR_INVALID_ARG;
    hipLaunchKernelGGL(corner_turn_u8, dim3(static_cast<unsigned>(nt), static_cast<unsigned>(nc)), dim3(256), 0, s,
                       static_cast<const uint32_t*>(in), static_cast<uint8_t*>(out), nsamp, nchans, pitch, reverse);
    return DEDISP_HIP_STATUS(hipGetLastError());
  }
  switch (dtype) {
    case DEDISP_U8:
      hipLaunchKernelGGL(corner_turn_kernel<uint8_t>, grid, dim3(256), 0, s, static_cast<const uint8_t*>(in),
                         static_cast<uint8_t*>(out), nsamp, nchans, pitch, reverse);
      break;
    case DEDISP_F16:
      hipLaunchKernelGGL(corner_turn_kernel<uint16_t>, grid, dim3(256), 0, s, static_cast<const uint16_t*>(in),
                         static_cast<uint16_t*>(out), nsamp, nchans, pitch, reverse);
      break;
    case DEDISP_F32:
      hipLaunchKernelGGL(corner_turn_kernel<float>, grid, dim3(256), 0, s, static_cast<const float*>(in),
                         static_cast<float*>(out), nsamp, nchans, pitch, reverse);
      break;
    default:
      return DEDISP_ERR_INVALID_ARG;
  }
  return DEDISP_HIP_STATUS(hipGetLastError());
}

}  // namespace dedisp

extern "C" int dedisp_corner_turn(const void* in_dev, void* out_dev, int64_t nsamp, int nchans, int64_t out_pitch,
                                  int dtype, int reverse_channels, void* stream) {
  if (in_dev == nullptr || out_dev == nullptr || nsamp < 0 || nchans < 1 || out_pitch < nsamp)
    return DEDISP_ERR_INVALID_ARG;
  if (dtype != DEDISP_U8 && dtype != DEDISP_F16 && dtype != DEDISP_F32) return DEDISP_ERR_INVALID_ARG;
  if (nsamp == 0) return DEDISP_OK;
  return dedisp::corner_turn(in_dev, out_dev, nsamp, nchans, out_pitch, dtype, reverse_channels != 0,
                             static_cast<hipStream_t>(stream));
}

// Corner turn of time-major filterbank samples ([t][c], the order sigproc
// files store them in) into the channel rows the search reads ([c][t], one
// row per channel, "cache lines of constant frequency, contiguous time").
// A 64 x 64 tile of (time, channel) goes through LDS: read along channels
// (contiguous in the input), written along time (contiguous in the output).
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

}  // namespace

int corner_turn(const void* in, void* out, int64_t nsamp, int nchans, int64_t pitch, int dtype, int reverse,
                hipStream_t s) {
  const int64_t tb = (nsamp + kTile - 1) / kTile;
  const int cb = (nchans + kTile - 1) / kTile;
  if (tb > INT32_MAX || cb > 65535) return DEDISP_ERR_INVALID_ARG;
  const dim3 grid(static_cast<unsigned>(tb), static_cast<unsigned>(cb));
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

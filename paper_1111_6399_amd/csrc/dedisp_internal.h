// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/dedisp.h"
#include "shift_table.h"

namespace dedisp {

// Float sums are accumulated in blocks of this many channels (see dedisp.h).
constexpr int kChanBlock = 32;
// Zero entries after each trial tile's row of the staging tables (covers the
// channels a kernel reads ahead past the last one: window offsets two stages
// ahead, up to 3*CG - 2 channels past the last for CG <= 8).
constexpr int kGeoPad = 32;
// Zero rows after the last channel of the device delay table (covers the
// channels a kernel reads ahead past the last one).
constexpr int kShiftPadRows = 16;
// Boxcar widths the detection kernel supports (1 .. 2^11 samples).
constexpr int kMaxDetectWidths = 12;


inline size_t dtype_size(int dtype) { return dtype == DEDISP_U8 ? 1 : dtype == DEDISP_F16 ? 2 : 4; }
// How the tiled kernels stage a plan's samples in LDS: float32 as given,
// float16 as given (halves), 8-bit widened to 16 bits beforehand (pairs of
// samples in a 32-bit word).
enum StageKind { kStageFloat = 0, kStageHalves = 1, kStagePairs = 2 };
inline int stage_kind(int dtype) {
  return dtype == DEDISP_U8 ? kStagePairs : dtype == DEDISP_F16 ? kStageHalves : kStageFloat;
}
// Bytes per staged sample, and the alignment of window starts in samples
// (16 bytes).
inline int64_t staged_size(int dtype) { return dtype == DEDISP_F32 ? 4 : 2; }
inline int stage_align(int dtype) { return dtype == DEDISP_F32 ? 4 : 8; }
inline size_t out_size(int) { return 4; }

// Shape of a tiled kernel variant.
struct TileShape {
  int dw;   // trials per wave
  int ks;   // float input: 64-bit LDS reads per lane and trial (126*ks samples per wave)
  int wd;   // waves along the trial axis
  int wt;   // waves along the time axis
  int dms() const { return dw * wd; }
  int samples() const { return 126 * ks * wt; }
  int threads() const { return 64 * wd * wt; }
};

// Per-device state of a plan: the delay table padded to a multiple of 64
// trials per channel, and the staging tables of the tiled kernels.
struct DeviceTables {
  int32_t* shift = nullptr;  // [nchans + kShiftPadRows][ndm_pad]
  // (trials per tile, samples per tile, align, bytes per staged sample, pitch mod align,
  //  start mod align, halo bytes) -> windows
  std::map<std::tuple<int, int, int, int, int, int, int>, uint32_t*> window_base;
  // (trials per tile, align, bytes per staged sample, pitch mod align, start mod align) -> slot positions
  std::map<std::tuple<int, int, int, int, int>, int32_t*> slot_pos;
};

// Arguments of one tiled launch (one beam); also the per-beam entry of the
// batched launch's table.
struct TiledArgs {
  const void* in;   // staged input: float, half, or 8-bit widened to 16 bits
  int64_t pitch;    // samples per input row (nsamp + max_shift, or the ring length)
  int64_t total16;  // staged samples of the input in whole 16-byte groups
  uint32_t start_bytes;  // rings: byte offset of the windows in every row (16-byte aligned part)
  uint32_t ring_bytes;   // bytes of a ring row; 0 for plain rows
  void* out;
  int64_t nsamp;
  const uint32_t* wbase;  // [n_dm_tiles][nchans + kGeoPad][2] byte offset of each window from its row's aligned start (less t0), 1 KB loads
  const int32_t* spos;    // [n_dm_tiles][nchans + kGeoPad][trials per tile] byte position in the slot
  int ndm, nchans;
  int runs;  // 1 KB loads per LDS slot (one channel of a stage), the most any window needs
  int n_dm_tiles, n_t_tiles;
  int gd, gt;       // tiles per group along trials and time
  int n_dm_groups;  // groups along trials
  int ntail;        // samples past total16 (float 0..3, half 0..7)
  int max_shift;    // largest delay of the plan
};

// One 8-bit input of a batch to widen to 16 bits before the persistent
// kernel (padded with zeros to npad samples).
struct WidenJob {
  const void* in;
  void* ws;
  int64_t n, npad;
  int dtype;
};

// Staged input rows of one launch: `pitch` samples a row, `total` staged
// samples in all.  Plain rows (ring = 0) hold a window at the start of each
// row; ring rows (pitch = ring, a multiple of 8 samples) hold a streaming
// beam's samples at positions modulo the ring, the window starting `start`
// samples into every row (start < ring).
struct StagedRows {
  const void* in;
  int64_t pitch;
  int64_t total;
  int64_t start;
  int64_t ring;
};

// A persistent batch kernel's work counters: one per XCD (chip), items handed
// out in chunks of kBatchChunk consecutive ones.
constexpr int kBatchCounters = 8;
constexpr int kBatchChunk = 32;

struct BatchArgs {
  const TiledArgs* beams;   // [nbeams], all staged alike (16-bit pairs or float)
  const int64_t* item_end;  // [nbeams] inclusive prefix sums of work items
  int nbeams;
  int64_t n_items;
  unsigned long long* counter;  // [kBatchCounters]
};

}  // namespace dedisp

struct dedisp_plan_s {
  int nchans = 0;
  int ndm = 0;
  int ndm_pad = 0;
  int dtype = DEDISP_F32;
  double f_top = 0, df = 0, tsamp = 0;
  std::vector<double> dms;
  std::vector<int32_t> shift;  // [nchans][ndm]
  int32_t max_shift = 0;
  std::atomic<int> variant{-1};  // -1: library default
  std::mutex mu;
  std::map<int, dedisp::DeviceTables> dev;  // per device id
  std::map<int, std::vector<int2>> host_windows;  // dms-per-tile -> [ntiles][nchans]
};

namespace dedisp {

// Device table of a plan on the current device (uploaded on first use; with
// create = false a missing table is an error instead: nothing is allocated).
int device_tables(dedisp_plan p, int device, DeviceTables** out, bool create = true);
const std::vector<int2>& host_windows(dedisp_plan p, int dms_per_tile);
// Staging tables of the tiled kernels for tiles of `dms_per_tile` trials,
// windows aligned to `align` samples (16 bytes) and `es` bytes per staged
// sample.  A tile's window of channel c holds the samples from
// c*pitch + start + t0 + lo - mis on (lo: smallest delay of the tile in that
// channel, mis: alignment of c*pitch + start + lo, t0 a multiple of align;
// `start` is the offset of the windows in every row, 0 except for rings):
// window_base = (es * (((c*pitch + start) mod align) + lo - mis), loads):
// the byte offset of the window from the start of row c rounded down to
// align, less the aligned part of start (add es*t0 for the tile and es times
// the aligned part of start), and the 1 KB loads that cover what the tile's
// reads reach (`samples` samples past the position of every trial, plus the
// halo lane's `halo` bytes), and slot_pos = es * (delay - lo + mis), the
// byte position of a trial's first sample inside the window (its low bits
// give the alignment of the trial).  Both depend on the row length and the
// start only through pitch mod align and start mod align.
int device_window_base(dedisp_plan p, int device, int dms_per_tile, int samples, int align, int es, int pitch_mod,
                       int start_mod, int halo, const uint32_t** out, bool create = true);
int device_slot_pos(dedisp_plan p, int device, int dms_per_tile, int align, int es, int pitch_mod, int start_mod,
                    const int32_t** out, bool create = true);

// Kernel registry (kernels.hip).
int variant_count();
TileShape variant_shape(int v);   // v >= 1
// Largest window (in samples) a tiled variant can stage for this plan, and
// whether the plan fits it.
bool variant_fits(dedisp_plan p, int v);
// Workgroups of tiled variant v that LDS lets share a CU for this plan (0 if
// it does not fit).
int tiled_per_cu(dedisp_plan p, int v);
int default_variant(dedisp_plan p);

// Launch one plan's kernel over the whole problem.  8-bit input is widened
// into `ws` (staged_bytes(p, nsamp) bytes) when given, else into a
// stream-ordered allocation; float and half input are read as they are.
// With no_alloc, nothing is allocated: the 8-bit workspace must be given and
// the plan's device tables must already exist (else DEDISP_ERR_INVALID_ARG).
int launch(dedisp_plan p, int variant, const void* in, void* out, int64_t nsamp, hipStream_t s, void* ws = nullptr,
           bool no_alloc = false);
// The same over input rows already in staged form (8-bit widened to 16 bits,
// float and half as they are), plain or ring rows.
int launch_rows(dedisp_plan p, int variant, const StagedRows& rows, void* out, int64_t nsamp, hipStream_t s);
// Bytes of the staged form of a plan's input for nsamp output samples.
size_t staged_bytes(dedisp_plan p, int64_t nsamp);
// Append a streaming block [nchans][block] (raw samples) to ring rows
// [nchans][ring] in staged form, sample j of a row at ring position
// (pos + j) mod ring (pos < ring, block <= ring).
int ring_append(int dtype, const void* blk, void* ring_rows, int64_t block, int64_t ring, int64_t pos, int nchans,
                hipStream_t s);

// 8-bit input is widened to 16 bits before a tiled launch, into a buffer of
// widened_samples(total) samples padded with zeros.
int64_t widened_samples(int64_t total);
int widen(int dtype, const void* in, void* ws, int64_t total, hipStream_t s);
// Widen every job of a device table (launched from a batch graph).
int widen_jobs(const WidenJob* jobs, int njobs, hipStream_t s);

// Arguments, LDS bytes, block count and threads of a tiled launch of variant
// v >= 1 (device tables are created on the current device if needed).
int tiled_args(dedisp_plan p, int v, const void* in, void* out, int64_t nsamp, TiledArgs* a, size_t* lds,
               int64_t* nblocks, int* threads);
int tiled_args_rows(dedisp_plan p, int v, const StagedRows& rows, void* out, int64_t nsamp, TiledArgs* a,
                    size_t* lds, int64_t* nblocks, int* threads, bool no_alloc = false);
// The library's static device scratch (the allocation-free entry point's
// 8-bit workspace): its address on the current device, and its size.
int static_scratch(void** out);
size_t static_scratch_bytes();
// Hash of the variant registry and the kernels' generation (autotune keys).
uint64_t registry_signature();
// Everything a launch of variant v of plan p needs that must not happen inside
// a graph capture (device tables, kernel attributes), on the current device.
int prepare(dedisp_plan p, int v, int64_t nsamp);
// Allow a kernel more than 64 KiB of dynamic LDS (once per kernel and device).
int allow_large_lds(const void* fn);
// Corner turn [t][c] -> rows [c][t] (ingest.hip); arguments checked by the caller.
int corner_turn(const void* in, void* out, int64_t nsamp, int nchans, int64_t pitch, int dtype, int reverse,
                hipStream_t s);
// Detection on a de-dispersed block (detect.hip); arguments checked by the caller.
size_t detect_lds_bytes(int nwidths);
int detect(dedisp_plan p, const void* out, int64_t nsamp, int nwidths, double threshold, double* stats,
           double* best_snr, int32_t* best_t, dedisp_candidate* cand, int cap, unsigned* count, hipStream_t s);
// Persistent batch kernel of variant v >= 1 for beams of one staging kind,
// and the counter reset kernel.
const void* batch_kernel(int v, int kind);
const void* reset_kernel();
int reset_kernel_threads();  // block size of the reset kernel (zeroes kBatchCounters counters)


// True when the environment variable DEDISP_TRACE is set: failing HIP calls
// are then reported on stderr with their source line.
bool trace_enabled();
void trace_hip_error(hipError_t e, const char* file, int line);

inline int hip_status(hipError_t e) {
  if (e == hipSuccess) return DEDISP_OK;
  if (e == hipErrorOutOfMemory) return DEDISP_ERR_OUT_OF_MEMORY;
  return DEDISP_ERR_DEVICE;
}

inline int hip_status_at(hipError_t e, const char* file, int line) {
  if (e != hipSuccess && trace_enabled()) trace_hip_error(e, file, line);
  return hip_status(e);
}
#define DEDISP_HIP_STATUS(e) ::dedisp::hip_status_at((e), __FILE__, __LINE__)

}  // namespace dedisp

/*
 * dedisp.h -- brute-force incoherent de-dispersion on AMD Instinct MI355X (gfx950).
 *
 * The operation (paper: Armour et al., "A GPU-based survey for millisecond radio
 * transients using ARTEMIS", sections "Searching for radio transients" and
 * "Acceleration via GPU computing"): every frequency channel of a filterbank
 * (channels x time samples of total intensity) is shifted in time by the
 * dispersion delay of a trial dispersion measure (DM), then the channels are
 * summed.  For every trial d and output sample t
 *
 *     out[d][t] = sum over c of in[c][t + shift[c][d]]
 *
 *     shift[c][d] = round_half_up(DM_d * k_c)
 *     k_c         = 4148.808 * (1/(f_c*f_c) - 1/(f_top*f_top)) / tsamp
 *     f_c         = f_top - c*df            (MHz; channel 0 is the highest)
 *
 * The delay table is computed on the host in IEEE binary64 in exactly this
 * order, without fused multiply-add, so it is reproducible bit for bit.
 *
 * Conventions for every call below
 *  - Return value: a dedisp_status code.  On any error the out-parameters are
 *    left untouched.  Arguments are checked before any GPU call, so argument
 *    errors never touch the device.
 *  - "device pointer": memory on the current HIP device (hipMalloc or torch
 *    CUDA/ROCm tensors).  "stream": a hipStream_t passed as void*; NULL means
 *    the default stream.  Launches are asynchronous on that stream; a device
 *    fault surfaces as DEDISP_ERR_DEVICE at a later synchronising call.
 *  - Layouts are row-major and dense: input [nchans][nsamp + max_shift],
 *    output [ndm][nsamp].  Input must be 16-byte aligned.
 *  - Output element type: int32 for DEDISP_U8 input (exact integer sums),
 *    float32 for DEDISP_F16 / DEDISP_F32 input.  Float sums use a fixed
 *    order: channels in ascending order in blocks of 32, each block summed
 *    into a float32 partial that is then added to the running float32 total.
 *    Every kernel variant, the batched launch and the streaming server follow
 *    this order, so their float32 results are identical to each other.
 *  - Ownership: a plan owns its delay table (host copy and one device copy per
 *    device it has run on).  The caller owns every buffer and stream passed in.
 *    Plans are immutable after creation apart from the kernel-variant choice;
 *    concurrent executes of one plan on different streams are allowed, but a
 *    variant change must not race with them.
 */
#ifndef DEDISP_H
#define DEDISP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dedisp_plan_s *dedisp_plan;
typedef struct dedisp_batch_s *dedisp_batch;
typedef struct dedisp_server_s *dedisp_server;

/* Input sample types. */
enum dedisp_dtype {
    DEDISP_U8 = 0,   /* unsigned 8-bit samples, int32 output, exact */
    DEDISP_F16 = 1,  /* IEEE half samples, float32 accumulation and output */
    DEDISP_F32 = 2   /* IEEE single samples, float32 accumulation and output */
};

enum dedisp_status {
    DEDISP_OK = 0,
    DEDISP_ERR_INVALID_ARG = 1,   /* an argument is out of its documented range */
    DEDISP_ERR_OUT_OF_MEMORY = 2, /* host or device allocation failed */
    DEDISP_ERR_DEVICE = 3,        /* a HIP call failed (no device, launch or fault) */
    DEDISP_ERR_AGAIN = 4,         /* not admitted now (memory budget or slots); retry later */
    DEDISP_ERR_NOT_FOUND = 5,     /* unknown ticket or beam */
    DEDISP_ERR_INTERNAL = 6       /* a library invariant failed */
};

/* Human-readable name of a status code (static storage, never NULL). */
const char *dedisp_status_string(int status);

/* ---------------------------------------------------------------- plans -- */

/*
 * Build a plan: the binary64 delay table of every (channel, trial) pair,
 * section "Searching for radio transients" (the quadratic cold-plasma delay,
 * governed by DM alone, removed channel by channel before integrating over
 * frequency).
 *   nchans    >= 1 channels; channel c is centred at f_top_mhz - c*df_mhz
 *   f_top_mhz > 0, df_mhz > 0, and the lowest channel f_top - (nchans-1)*df > 0
 *   tsamp_s   > 0 sampling interval in seconds
 *   dm_list   host array of ndm >= 1 finite, non-negative trial DMs (pc cm^-3),
 *             any order; copied
 *   in_dtype  one of enum dedisp_dtype
 * Fails with DEDISP_ERR_INVALID_ARG if any of these is violated or a delay
 * exceeds INT32_MAX.  Makes no GPU call (the device copy of the table is made
 * on first use on each device).
 */
int dedisp_plan_create(int nchans, double f_top_mhz, double df_mhz, double tsamp_s,
                       const double *dm_list, int ndm, int in_dtype, dedisp_plan *out_plan);

/* Free a plan and its device tables.  NULL is accepted.  The caller must make
 * sure no launch that uses the plan is still running. */
int dedisp_plan_destroy(dedisp_plan plan);

/* Largest entry of the delay table: input rows need nsamp + max_shift samples. */
int dedisp_plan_max_shift(dedisp_plan plan, int32_t *out);

/* Copy the delay table to host memory, layout [nchans][ndm] int32. */
int dedisp_plan_shift_table(dedisp_plan plan, int32_t *host_out);

/* Shape of a plan: any pointer may be NULL. */
int dedisp_plan_dims(dedisp_plan plan, int *nchans, int *ndm, int *in_dtype);

/*
 * Trial DMs equally spaced from 0 to dm_max inclusive, the grid of the
 * paper's timing comparisons (section "Comparisons of GPU and CPU
 * algorithms", Figure 4: as many equally spaced trials as channels, up to a
 * maximum DM): dm_out[d] = dm_max * ((double)d / (ndm - 1)) in binary64 (the
 * quotient first, so the last trial is dm_max exactly), d = 0 .. ndm-1;
 * ndm = 1 gives {0}.
 *   dm_max   finite, >= 0
 *   ndm      >= 1
 *   dm_out   host array of ndm doubles
 * DEDISP_ERR_INVALID_ARG otherwise; nothing is written then.
 */
int dedisp_dm_grid(double dm_max, int ndm, double *dm_out);

/*
 * Device memory one dedisp_execute of a plan touches for nsamp >= 0 output
 * samples: in_bytes = nchans*(nsamp + max_shift) samples of the input type;
 * out_bytes = ndm*nsamp*4; staged_bytes = the widened copy a tiled launch of
 * 8-bit input works from (16-bit samples, padded with zeros to a multiple of
 * 8 samples, allocated stream-ordered by the launch), 0 for half and float
 * input (read as they are).  Any output pointer may be NULL.
 */
int dedisp_plan_footprint(dedisp_plan plan, int64_t nsamp, uint64_t *in_bytes, uint64_t *out_bytes,
                          uint64_t *staged_bytes);

/*
 * Kernel variants.  Variant 0 is the direct kernel (one lane per output
 * sample); variants 1..n-1 are LDS-tiled kernels of different tile shapes.
 * All variants produce identical results.  dedisp_variant_count returns the
 * number of variants compiled into the library; dedisp_variant_describe
 * writes (DMs per tile, samples per tile, threads per block) of a variant.
 * dedisp_plan_set_variant fails with DEDISP_ERR_INVALID_ARG if the variant's
 * on-chip window does not fit this plan's delay spread or the variant has no
 * kernel for the plan's input type (some variants serve only float, or only
 * half and 8-bit input).
 */
int dedisp_variant_count(void);
int dedisp_variant_describe(int variant, int *dms_per_tile, int *samples_per_tile, int *threads);
int dedisp_plan_set_variant(dedisp_plan plan, int variant);
int dedisp_plan_get_variant(dedisp_plan plan, int *variant);

/*
 * Time every variant that fits this plan on nsamp output samples (scratch
 * buffers of the plan's shape are allocated and freed here, on the current
 * device) and keep the fastest.  The result is cached in memory per
 * (shape, device) and, when the environment variable DEDISP_TUNE_CACHE names
 * a file, in that file.  Synchronises the device.  best_ms may be NULL.
 */
int dedisp_autotune(dedisp_plan plan, int64_t nsamp, int *best_variant, double *best_ms);

/* -------------------------------------------------------------- execute -- */

/*
 * De-disperse one block (the paper's brute-force search: every channel shifted
 * for every trial, then integrated over frequency).
 *   in_dev   device pointer, [nchans][nsamp + max_shift] samples of the plan's
 *            dtype, 16-byte aligned
 *   out_dev  device pointer, [ndm][nsamp] int32 (U8) or float32 (F16, F32)
 *   nsamp    number of OUTPUT samples, >= 0 (0 is a no-op)
 *   stream   hipStream_t or NULL
 * Asynchronous.  The first call on a device uploads the delay table
 * (synchronously, once).
 */
int dedisp_execute(dedisp_plan plan, const void *in_dev, void *out_dev, int64_t nsamp, void *stream);

/*
 * dedisp_execute without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and asynchrony as
 * dedisp_execute.  The only workspace a launch needs (the widened copy of
 * 8-bit input, staged_bytes of dedisp_plan_footprint) comes from a static
 * device array of the library, 1 GiB on every device the library runs on,
 * held until the process ends.  Requirements:
 *   - staged_bytes <= 1 GiB, else DEDISP_ERR_INVALID_ARG (float and half
 *     input need no workspace);
 *   - the plan's device tables for this nsamp must already exist on the
 *     current device (any earlier dedisp_execute or dedisp_autotune of the
 *     plan with this nsamp on this device creates them), else
 *     DEDISP_ERR_INVALID_ARG.
 * Calls on one device share the array: two 8-bit calls that overlap in time
 * on one device (different streams) race; order them on one stream.
 */
int dedisp_execute_static(dedisp_plan plan, const void *in_dev, void *out_dev, int64_t nsamp, void *stream);

/* ------------------------------------------------------------- ingestion -- */

/* Fields of a sigproc filterbank header that the search uses. */
typedef struct {
    int32_t nchans, nbits, nifs, data_type, telescope_id, machine_id, nbeams, ibeam, nsamples;
    int32_t dtype;         /* DEDISP_U8 for 8-bit samples, DEDISP_F32 for 32-bit, -1 otherwise */
    double tsamp;          /* seconds */
    double fch1, foff;     /* MHz: centre of the first channel, channel step (negative: descending) */
    double tstart, refdm;
    int64_t header_bytes;  /* offset of the first sample */
    char source_name[80];  /* NUL-terminated, truncated */
} dedisp_sigproc_header;

/*
 * Parse a sigproc filterbank header (the format of the paper's test data,
 * section "Searching for radio transients": simulated with sigproc) from the
 * first len bytes of a host buffer.  The header is a sequence of keywords,
 * each a 32-bit little-endian length and that many characters, between
 * HEADER_START and HEADER_END, each followed by a 32-bit integer, a binary64
 * value or a length-prefixed string according to the keyword.  Keywords not
 * listed above are skipped when their value type is known (telescope
 * coordinates, beam flags, period, raw file name).  Unset fields are 0 (nifs
 * 1).  DEDISP_ERR_INVALID_ARG for a truncated or malformed header, an unknown
 * keyword, nchans < 1, tsamp <= 0, foff = 0, nifs < 1 or nbits not 8, 16 or
 * 32; *out is written only on success.  Samples follow the header in time
 * order, nifs x nchans per time step.
 */
int dedisp_sigproc_parse(const void *buf, size_t len, dedisp_sigproc_header *out);

/*
 * Corner turn: time-major samples in_dev[t][c] (nsamp x nchans, the sample
 * order of a filterbank with nifs = 1) into channel rows,
 * out_dev[row * out_pitch + t], row = c, or nchans - 1 - c with
 * reverse_channels (a band stored with ascending frequency, foff > 0, becomes
 * channel 0 = highest, as plans expect).  out_pitch >= nsamp samples; writing
 * to a plan input's row offset (out_dev + max_shift, pitch nsamp + max_shift)
 * appends a block behind a history.  dtype: DEDISP_U8, DEDISP_F16 or
 * DEDISP_F32 (element size only).  Device pointers; asynchronous on stream.
 */
int dedisp_corner_turn(const void *in_dev, void *out_dev, int64_t nsamp, int nchans, int64_t out_pitch,
                       int dtype, int reverse_channels, void *stream);

/* ------------------------------------------------------------- detection -- */

/* One detection: trial index, boxcar width in samples, start time of the
 * boxcar in output samples, and its S/N. */
typedef struct {
    int32_t dm_index;
    int32_t width;
    int32_t time;
    float snr;
} dedisp_candidate;

/*
 * Detection on a de-dispersed block, the step after the search (section
 * "Introduction": the pipeline ends in detection; Figure 3: the recovered
 * pulse stands out at its trial DM).  For every trial d of the plan, over its
 * nsamp output samples x_d:
 *   mean_d, std_d       mean and population standard deviation, binary64
 *   S/N_{d,w}(t)        (sum_{i<w} x_d[t+i] - w*mean_d) / (std_d*sqrt(w)) for
 *                       w = 1, 2, 4, .. 2^(nwidths-1) and every t with
 *                       t + w <= nsamp (0 where std_d = 0)
 *   best_{d,w}          the largest S/N_{d,w}(t) and the earliest t reaching it;
 *                       -inf and -1 when w > nsamp
 * and every (d, w) whose best S/N is >= threshold is a candidate.
 *   out_dev        device pointer to the block, [ndm][nsamp] int32 (U8 plans)
 *                  or float32, 4-byte aligned; read only
 *   nsamp          1 .. INT32_MAX
 *   nwidths        1 .. 12
 *   threshold      finite
 *   stats_dev      device [ndm][2] doubles (mean, std), or NULL
 *   best_snr_dev   device [ndm][nwidths] doubles
 *   best_t_dev     device [ndm][nwidths] int32
 *   cand_dev       device array of cand_capacity candidates (order unspecified),
 *                  or NULL for none; cand_count_dev (device uint32) then
 *                  receives the number of candidates, which may exceed the
 *                  capacity (only the first cand_capacity are written)
 *   stream         hipStream_t or NULL
 * Values are converted to binary64 before any arithmetic (exact for int32).
 * Asynchronous; all device buffers are the caller's.
 */
int dedisp_detect(dedisp_plan plan, const void *out_dev, int64_t nsamp, int nwidths, double threshold,
                  double *stats_dev, double *best_snr_dev, int32_t *best_t_dev, dedisp_candidate *cand_dev,
                  int cand_capacity, uint32_t *cand_count_dev, void *stream);

/* ------------------------------------------------------------------ host -- */

/*
 * The search on the host CPU, for timing against the GPU: the paper's second
 * algorithm (section "Comparisons of GPU and CPU algorithms": a brute force
 * written for the CPU's vector registers with cache-line reuse in mind), in
 * tiles of 16 trials x 256 samples.  Same plan, layouts and results as
 * dedisp_execute, with host pointers: float sums follow the GPU kernels' order
 * (channels in blocks of 32), so float results are bit-identical to
 * dedisp_execute's; 8-bit sums are exact.
 *   nthreads   >= 0; 0 uses every hardware thread
 *   isa_used   NULL, or receives 2 (AVX-512), 1 (AVX2) or 0 (plain C++)
 * Synchronous.  dedisp_execute never calls it: there is no CPU fallback.
 */
int dedisp_execute_cpu(dedisp_plan plan, const void *in_host, void *out_host, int64_t nsamp, int nthreads,
                       int *isa_used);

/* --------------------------------------------------------------- batches -- */

/*
 * A batch runs many independent beams (plans of any shape and dtype, each with
 * its own output length) in persistent launches (one per group of beams with
 * the same tile variant, staging kind and LDS occupancy), replayed from a HIP
 * graph.
 * Work is cut into (beam, DM tile, time tile) items, ordered longest first, and
 * pulled by resident workgroups from an atomic counter.  Each beam's result is
 * identical to dedisp_execute of that beam alone.
 *   plans   nbeams plans (not owned; they must outlive the batch)
 *   nsamps  nbeams output lengths (>= 1)
 */
int dedisp_batch_create(const dedisp_plan *plans, const int64_t *nsamps, int nbeams,
                        dedisp_batch *out_batch);

/* Run the batch: ins[b] / outs[b] are device pointers laid out as for
 * dedisp_execute.  Asynchronous on stream.  The graph is built on the first
 * call on a stream's device and re-used; new pointers are uploaded before the
 * replay. */
int dedisp_batch_execute(dedisp_batch batch, const void *const *ins, void *const *outs, void *stream);

/* Number of work items and workgroups the batch launches (either may be NULL;
 * both are 0 before the first execute). */
int dedisp_batch_info(dedisp_batch batch, int64_t *work_items, int *workgroups);

/* Tile variant of the persistent kernel that carries the most work (>= 1; -1
 * if no beam runs in one).  Setting v >= 1 runs every beam that variant fits
 * in persistent kernels (the rest on their own); setting 0 splits by each
 * plan's own variant (beams with a tiled variant in persistent kernels of
 * that variant, the others on their own); setting -1 launches every beam on
 * its own with its plan's variant, the launches captured in the graph.
 * Setting rebuilds the graph on the next execute; it synchronises the
 * batch's device. */
int dedisp_batch_get_variant(dedisp_batch batch, int *variant);
int dedisp_batch_set_variant(dedisp_batch batch, int variant);

/* How the graph spreads its kernels over its four branches (concurrent
 * streams forked from and joined to the launch stream): 0 each on the branch
 * with the least work so far (largest first), 1 all on one branch in beam
 * order (the plain per-beam sequence without its launch overheads), 2 one
 * branch for the float beams and one for the 16-bit (half and 8-bit) beams.
 * Setting a layout outside 0-2 is an invalid argument; setting rebuilds the
 * graph on the next execute and synchronises the batch's device;
 * dedisp_batch_set_variant resets it to 0. */
int dedisp_batch_get_layout(dedisp_batch batch, int *layout);
int dedisp_batch_set_layout(dedisp_batch batch, int layout);

/* Time the batch with every tile variant that fits any of its beams; with
 * 8-bit and float beams mixed, also each variant for the 8-bit beams with the
 * float beams' held, then each for the float beams (the two kinds run as
 * separate persistent kernels); the split that follows each plan's own
 * variant (set or tuned with dedisp_autotune); and every beam launched on its
 * own with its plan's variant, the launches captured in the graph in each
 * layout (dedisp_batch_get_layout); the persistent splits are timed in layout
 * 0, whatever layout was set before.  Keeps the fastest; best_variant is then
 * the variant of the persistent kernel that carries the most work (-1 if the
 * per-beam launches won).  Synchronises the
 * stream.  The outputs are overwritten (with correct results).  best_ms may
 * be NULL. */
int dedisp_batch_autotune(dedisp_batch batch, const void *const *ins, void *const *outs, void *stream,
                          int *best_variant, double *best_ms);

int dedisp_batch_destroy(dedisp_batch batch);

/* --------------------------------------------------------------- serving -- */

/*
 * A streaming server: beams send consecutive blocks as they arrive; the server
 * keeps each beam's last max_shift input samples on the device so that block b
 * of a beam yields the de-dispersed series for stream times
 * [b*B - max_shift, (b+1)*B - max_shift) (B = block length; the history before
 * the first block is zero).  Requests are admitted while the device memory
 * they need fits hbm_budget_bytes and fewer than max_inflight are running;
 * admitted requests from different beams run concurrently on a pool of
 * streams.  Blocks of one beam run in submission order.
 *
 * The output of every block equals dedisp_execute on that beam's history plus
 * block, alone or in any mix of beams.
 */
int dedisp_server_create(size_t hbm_budget_bytes, int max_inflight, dedisp_server *out_server);

/* Register a beam: plan (not owned; must outlive the server) and block length
 * B >= 1.  Allocates the beam's device buffers against the budget: one ring of
 * nchans x R samples in the form the kernels read (8-bit samples as 16-bit,
 * half and float as they are; R = max_shift + B + 4608 rounded up to a
 * multiple of 8), which holds the history and the newest block (each block is
 * written once; the history is never copied), and one raw block of
 * nchans x B samples.  DEDISP_ERR_AGAIN if they do not fit.  A request is
 * charged its ndm x B outputs while it runs. */
int dedisp_server_add_beam(dedisp_server server, dedisp_plan plan, int64_t block_nsamp, int *beam_id);

/*
 * Submit the next block of a beam.
 *   block    host or device pointer to [nchans][B] samples; must stay valid and
 *            unchanged until the ticket is done.  Host memory should be pinned
 *            (hipHostMalloc) for the copy to overlap.
 *   out_dev  device pointer to [ndm][B] outputs; must stay allocated until done
 *   ticket   receives an id for dedisp_poll
 * The server's streams do not wait for work the caller queued elsewhere: a
 * block or output buffer that device work of the caller writes (a copy, a
 * fill) must be complete before the submission.
 * DEDISP_ERR_AGAIN: not admitted (budget or slots); nothing was queued.
 */
int dedisp_submit(dedisp_server server, int beam_id, const void *block, void *out_dev, uint64_t *ticket);

/* Query a ticket without blocking: *done = 0 while it runs.  When it has
 * finished, *done = 1 and *latency_s = seconds from submission to the end of
 * its kernel (recorded on the host when the stream reached it), reported once:
 * the ticket is then forgotten and later polls return DEDISP_ERR_NOT_FOUND.  A
 * request whose work failed returns DEDISP_ERR_DEVICE (once) and its beam
 * restarts from a zero history, which the stream's consumer must treat as a
 * discontinuity.  The environment variable DEDISP_FAULT_INJECT=submit:N makes
 * the N-th submission to a server fail that way (a test hook). */
int dedisp_poll(dedisp_server server, uint64_t ticket, int *done, double *latency_s);

/* Block until every submitted request has finished. */
int dedisp_server_drain(dedisp_server server);

/* Latency percentiles over completed requests, and aggregate throughput in
 * DM*channel*samples per second between the first submission and the last
 * completion.  Pointers may be NULL. */
int dedisp_server_stats(dedisp_server server, double *p50_s, double *p99_s, double *dm_ch_samp_per_s);

/* Drain and free a server (NULL accepted).  Plans are not freed. */
int dedisp_server_destroy(dedisp_server server);

#ifdef __cplusplus
}
#endif

#endif /* DEDISP_H */

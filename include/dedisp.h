/*
 * libdedisp — brute-force incoherent de-dispersion for AMD Instinct MI355X (gfx950).
 *
 * Method: Magro et al., "Real-time, fast radio transient searches with GPU
 * de-dispersion" (MNRAS 2011, arXiv 1107.2516).  For every trial DM d and
 * frequency channel c an integer shift delay[d][c] follows from the cold-plasma
 * dispersion law (section 1, dispersion-law equation) split as in section 3
 * ("Shifts"):
 *     t_chan[c]   = 4150 s * (f_c^-2 - f_top^-2)          (f in MHz)
 *     delay[d][c] = round(t_chan[c] * DM_d / t_samp)        (ties away from 0)
 * evaluated on the host in FP64.  De-dispersion (section 3.1) then sums the
 * shifted channels:
 *     out[d][t] = sum over c of in[c][t + delay[d][c]],   0 <= t < nout,
 * with nout = nsamp - max_shift and max_shift the largest table entry, the
 * "maximum shift" extra samples of section 3.
 *
 * Conventions used by every call:
 *  - Channel c has frequency f_c = f_top - c*df (channel 0 at the top, df > 0).
 *  - Frequencies in MHz, times in seconds, DMs in pc cm^-3.
 *  - Filterbank input is channel-major with time contiguous ("channel order",
 *    section 3.1): sample (c, t) is at in[c*in_stride + t], in_stride >= nsamp.
 *  - Output row d (in the caller's DM order) is at out[d*out_stride + t],
 *    out_stride >= nout.
 *  - Supported (input, output) type pairs: (DD_F32, DD_F32), (DD_F16, DD_F32)
 *    with FP32 accumulation, and (DD_U8, DD_I32) with exact integer sums.
 *  - Device pointers are HIP device memory (for example the data pointer of a
 *    torch tensor on a ROCm device); the caller owns them.  `stream` is a
 *    hipStream_t (NULL = the default stream).  Calls that take a stream only
 *    enqueue work and return; errors found while enqueueing are returned,
 *    faults during execution surface at the next synchronisation.
 *  - Every entry point returns a dd_status; none aborts, and no C++ exception
 *    crosses this interface.  dd_last_error() returns a thread-local message
 *    describing the last failure on the calling thread.
 */
#ifndef DEDISP_H
#define DEDISP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dd_status {
  DD_OK = 0,
  DD_ERR_INVALID_ARG = -1,    /* bad sizes, strides, frequencies, DMs, NULL pointers */
  DD_ERR_DTYPE = -2,          /* unsupported (input, output) type pair */
  DD_ERR_NSAMP = -3,          /* nsamp <= max_shift: no complete output sample */
  DD_ERR_OOM = -4,            /* host or device allocation failed */
  DD_ERR_HIP = -5,            /* a HIP runtime call failed (message in dd_last_error) */
  DD_ERR_AGAIN = -6,          /* serving queue full: retry after polling */
  DD_ERR_TOO_LARGE = -7,      /* request larger than the configured budget or limit */
  DD_ERR_NOT_FOUND = -8,      /* unknown beam or ticket */
  DD_ERR_NOT_IMPLEMENTED = -9,
  DD_ERR_STATE = -10          /* call not valid in the object's current state */
} dd_status;

typedef enum dd_dtype { DD_U8 = 1, DD_F16 = 2, DD_F32 = 3, DD_I32 = 4 } dd_dtype;

typedef struct dd_plan dd_plan;

/* A kernel tile shape (see dd_tile_for, dd_execute_tiled, dd_autotune). */
typedef struct dd_tile_config {
  int32_t variant;      /* kernel variant index (implementation-defined) */
  int32_t dms_per_wave; /* DM trials per wavefront */
  int32_t waves;        /* wavefronts per workgroup */
  int32_t tsamp_per_lane; /* output samples per lane */
  int32_t chans_per_stage; /* channels staged in LDS per pipeline step */
} dd_tile_config;

/* ------------------------------------------------------------------------ */
/* Plans                                                                    */
/* ------------------------------------------------------------------------ */

/*
 * Build a plan: the FP64 delay table of section 3 ("Shifts") for `ndms` trial
 * DMs (any order, duplicates allowed) and `nchans` channels.
 *   nchans >= 1, df_mhz > 0, f_top_mhz - (nchans-1)*df_mhz > 0, t_samp_s > 0,
 *   every DM finite and >= 0, ndms >= 1, nchans <= 2^23 (int32 sums of 8-bit
 *   data stay exact).  Otherwise DD_ERR_INVALID_ARG and *out untouched.
 * The plan owns a host copy of the table; its device copy is uploaded lazily,
 * once per device, on first use.  A plan is immutable after creation and may
 * be used from several threads and streams at once.  No GPU work happens here.
 */
dd_status dd_plan_create(int32_t nchans, double f_top_mhz, double df_mhz, double t_samp_s,
                         const double* dm_list, int32_t ndms, dd_plan** out);

/*
 * Build a plan from an explicit host table delays[d*nchans + c] (row-major
 * [ndms][nchans], every entry >= 0).  Lets tests drive the kernels with
 * arbitrary shifts.  DD_ERR_INVALID_ARG for negative entries or bad sizes.
 */
dd_status dd_plan_create_from_delays(int32_t nchans, int32_t ndms, const int32_t* delays,
                                     dd_plan** out);

/* Sizes of a plan; any output pointer may be NULL. */
dd_status dd_plan_info(const dd_plan* plan, int32_t* nchans, int32_t* ndms, int32_t* max_shift);

/* Copy the plan's table to host memory host_out[d*nchans + c] (ndms*nchans int32). */
dd_status dd_delay_table(const dd_plan* plan, int32_t* host_out);

/* Release a plan (NULL is accepted).  The caller must make sure no enqueued
 * work still uses it. */
dd_status dd_plan_destroy(dd_plan* plan);

/* ------------------------------------------------------------------------ */
/* De-dispersion (section 3.1)                                              */
/* ------------------------------------------------------------------------ */

/*
 * Enqueue out[d][t] = sum_c in[c][t + delay[d][c]] for all d < ndms and
 * t < nout = nsamp - max_shift on `stream`.
 *   d_in  device, in_t elements, nchans rows of in_stride (>= nsamp) elements.
 *   d_out device, out_t elements, ndms rows of out_stride (>= nout) elements;
 *         elements t >= nout of each row are not written.
 * Errors: DD_ERR_INVALID_ARG (NULL pointers, strides), DD_ERR_DTYPE (type
 * pair), DD_ERR_NSAMP (nsamp <= max_shift), DD_ERR_TOO_LARGE (the shift
 * spread of 32 neighbouring DMs of the plan at one channel, plus one time
 * tile, does not fit a workgroup's 160 KB of LDS even for the LDS-streaming
 * kernel: about 40000 samples for FP32 input, twice that for f16 and four
 * times for 8-bit; only very coarse DM grids at low frequencies reach it),
 * DD_ERR_HIP (launch failure).
 * Accuracy.  8-bit input gives exact int32 sums.  Float input (f32, or f16
 * converted exactly to FP32) is summed in FP32 one channel at a time in
 * channel order 0..nchans-1 by the default shapes and every variant up to 7
 * and 11, so they, batches and serving give bit-identical FP32 results for one
 * input, and the error against the exact sum obeys the recursive-summation
 * bound
 *     |y - y*| <= (nchans - 1) 2^-24 sum_c |x_c|      (first order),
 * i.e. a scaled error of at most 6.1e-5 at 1024 channels and 1.2e-4 at 2048.
 * Variants 8 (FP32) and 10 (binary16) first add channels in pairs and then
 * the pair sums in order: a different rounding, within (nchans/2) 2^-24
 * sum_c |x_c|.
 * Realised errors are far smaller: ~2e-7 on zero-mean noise and ~2e-6 on
 * noise with a large positive offset; the worst inputs found, constant
 * positive values whose every partial sum rounds the same way, reach
 * 1.5e-5 at 1024 and 3.1e-5 at 2048 channels.
 */
dd_status dd_execute(const dd_plan* plan, const void* d_in, dd_dtype in_t, int64_t nsamp,
                     int64_t in_stride, void* d_out, dd_dtype out_t, int64_t out_stride,
                     void* stream);

/* ------------------------------------------------------------------------ */
/* Batches: many beams, one persistent launch                               */
/* ------------------------------------------------------------------------ */

typedef struct dd_batch dd_batch;

typedef struct dd_batch_item {
  const dd_plan* plan;  /* borrowed; must outlive the batch */
  const void* d_in;     /* device input of this beam */
  int64_t nsamp;        /* samples per channel (> plan max_shift) */
  int64_t in_stride;    /* elements between channel rows (>= nsamp) */
  void* d_out;          /* device output of this beam */
  int64_t out_stride;   /* elements between DM rows (>= nsamp - max_shift) */
} dd_batch_item;

/*
 * Describe `n` beams that share (in_t, out_t) and are processed together by
 * persistent kernels: every (beam, DM tile, time tile) work item is pulled
 * from a device queue by a fixed grid sized to the GPU, each XCD taking an
 * eighth of every beam first.  Each beam's tile shape comes from the
 * autotune cache (dd_autotune) or the built-in defaults.  Beams are grouped
 * into classes by the kernel their shape runs and by the workgroups per CU
 * their own LDS needs allow (a class's workgroups all get the LDS of its
 * largest beam); one persistent kernel per class, run one after the other.
 * At most 16 classes: beyond that, beams are grouped by kernel alone, and
 * more than 16 different kernels give DD_ERR_TOO_LARGE.  The launch is
 * recorded into a HIP graph on first use and replayed afterwards.
 */
dd_status dd_batch_create(const dd_batch_item* items, int32_t n, dd_dtype in_t, dd_dtype out_t,
                          dd_batch** out);

/* Point the batch at new buffers of the same shapes (same plans, nsamp and
 * strides, same n); the captured graphs are kept.  DD_ERR_INVALID_ARG if any
 * shape differs.  The batch keeps two descriptor tables and alternates between
 * them: the update writes the table the latest launch did not use, first
 * waiting (on the host) for that table's own previous launch to complete, so
 * a launch still in flight keeps its old buffers and no host synchronisation
 * with the latest launch is needed. */
dd_status dd_batch_update(dd_batch* batch, const dd_batch_item* items, int32_t n);

/* Enqueue the whole batch on `stream` (graph replay).  Stream-ordered; a
 * launch that uses the same descriptor table as one still in flight on
 * another stream starts after it (they share work counters). */
dd_status dd_batch_launch(dd_batch* batch, void* stream);

/* Use tile shape *cfg for every beam of the batch (its graph is re-recorded
 * on the next launch); a beam whose tables do not suit the shape's kernel
 * runs the kernel that shape falls back to, in its own class.
 * DD_ERR_NOT_IMPLEMENTED for a shape no kernel has, DD_ERR_TOO_LARGE when
 * some beam does not fit it (the batch keeps its previous shapes then). */
dd_status dd_batch_set_tile(dd_batch* batch, const dd_tile_config* cfg);

/* Work items (beam, DM tile, time tile), persistent grid size (of the first
 * class) and the tile shape of a batch (the forced one, or the largest
 * beam's); any output pointer may be NULL. */
dd_status dd_batch_info(const dd_batch* batch, int32_t* work_items, int32_t* grid,
                        dd_tile_config* cfg);

dd_status dd_batch_destroy(dd_batch* batch);

/* ------------------------------------------------------------------------ */
/* Autotuning                                                               */
/* ------------------------------------------------------------------------ */



/*
 * Time the candidate tile shapes for (plan, in_t, nsamp) on `stream` using
 * scratch buffers it allocates and frees (rows pitched to 64 samples), keep
 * the fastest in the process-wide cache (and in the file named by
 * DD_TUNE_CACHE, if set: one line per entry, led by the GPU architecture
 * name, so lines written on another GPU model are not applied), and return
 * it.  Blocks until the timing is done.  best_ms may be NULL.
 */
dd_status dd_autotune(const dd_plan* plan, dd_dtype in_t, int64_t nsamp, void* stream,
                      dd_tile_config* best, float* best_ms);

/*
 * dd_execute with an explicit tile shape (from dd_tile_for or dd_autotune, or
 * chosen by the caller).  DD_ERR_NOT_IMPLEMENTED if no kernel exists for the
 * shape and type pair; DD_ERR_TOO_LARGE if the plan's shift spread inside one
 * DM tile does not fit the shape's LDS staging.  Results equal dd_execute's
 * (bit-exact for 8-bit input, within the FP32 tolerance otherwise).
 */
dd_status dd_execute_tiled(const dd_plan* plan, const void* d_in, dd_dtype in_t, int64_t nsamp,
                           int64_t in_stride, void* d_out, dd_dtype out_t, int64_t out_stride,
                           const dd_tile_config* cfg, void* stream);

/*
 * Time the candidate tile shapes on the batch itself (its output buffers are
 * overwritten): each shape for every beam, and each beam on its own with
 * every shape (the per-beam winners are remembered in the shape cache and
 * timed together); keep the faster configuration and re-record the graph on
 * the next launch.  *best is the chosen uniform shape, or the largest beam's.
 * Blocks until the timing is done.  best_ms may be NULL.
 */
dd_status dd_batch_autotune(dd_batch* batch, void* stream, dd_tile_config* best, float* best_ms);

/* The tile shape dd_execute would use now for (plan, in_t, nsamp). */
dd_status dd_tile_for(const dd_plan* plan, dd_dtype in_t, int64_t nsamp, dd_tile_config* cfg);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of streaming chunks from many beams          */
/* ------------------------------------------------------------------------ */

typedef struct dd_server dd_server;

typedef struct dd_serve_config {
  dd_dtype in_t;           /* input sample type of every beam */
  dd_dtype out_t;          /* output type (pair rules as dd_execute) */
  int32_t max_inflight;    /* chunks on the device at once (>= 1) */
  int32_t queue_capacity;  /* host submit queue length (>= 1) */
  int32_t nstreams;        /* HIP streams used to overlap chunks (1..16) */
  size_t host_staging_bytes; /* pinned host pool for queued chunks (0 = 1 GiB) */
} dd_serve_config;

typedef struct dd_result {
  uint64_t ticket;
  int32_t beam;
  int32_t status;          /* dd_status of this chunk */
  int64_t seq;             /* caller's sequence number */
  int64_t t_first;         /* absolute output sample of row element 0 */
  int64_t nout;            /* output samples per DM row (0 while warming up) */
  void* d_out;             /* device output, ndms rows of out_stride elements */
  int64_t out_stride;
  double t_submit, t_admit, t_done; /* seconds, steady clock of this process */
} dd_result;

/*
 * Create a server that sub-allocates all of its device memory (per-beam
 * overlap carries, chunk staging, outputs) from the caller's arena
 * [d_arena, d_arena + arena_bytes).  A chunk is admitted only when the arena
 * has room for it (the memory rule of section 3, "Processable Samples").
 */
dd_status dd_serve_create(const dd_serve_config* cfg, void* d_arena, size_t arena_bytes,
                          dd_server** out);

/*
 * Register a beam that streams data for `plan`, in chunks of at most
 * max_chunk samples.  Reserves the beam's ring of 2 max_shift + max_chunk
 * (+ up to 127) samples per channel in the arena: the carry, the last samples
 * later outputs need (at most max_shift per channel, section 3, "Maximum
 * shift"), stays on the device between chunks, and is moved to the front of
 * the ring only when the next chunk would pass its end.  DD_ERR_TOO_LARGE if
 * the ring does not fit the arena, or if, with every beam's ring in place,
 * the rest of the arena could not hold one largest chunk of some beam (its
 * device copy plus its ndms x (max_chunk + 3, rounded up to 64) output),
 * since such a chunk could never be admitted.
 */
dd_status dd_serve_add_beam(dd_server* srv, const dd_plan* plan, int64_t max_chunk, int32_t* beam);

/*
 * Queue one chunk: nsamp samples of every channel, host memory laid out
 * [nchans][in_stride] (in_stride >= nsamp elements between the starts of
 * consecutive channel rows; only the first nsamp of each row are read).
 * The chunk is copied into the server's pinned staging pool
 * before this call returns.  seq must increase by one per beam; a gap
 * restarts the beam (its carry is dropped and it warms up again).  Chunks of
 * one beam must be submitted from one thread at a time.
 * DD_ERR_AGAIN when the queue or the staging pool is full (poll, release and
 * retry), DD_ERR_TOO_LARGE when nsamp exceeds the beam's max_chunk or the
 * chunk is larger than the whole staging pool (it could never be queued),
 * DD_ERR_NOT_FOUND for an unknown beam.
 */
dd_status dd_serve_submit(dd_server* srv, int32_t beam, const void* h_chunk, int64_t nsamp,
                          int64_t in_stride, int64_t seq, uint64_t* ticket);

/* Collect up to `max` finished chunks (non-blocking). */
dd_status dd_serve_poll(dd_server* srv, dd_result* out, int32_t max, int32_t* n);

/* Return a finished chunk's output memory to the arena. */
dd_status dd_serve_release(dd_server* srv, uint64_t ticket);

/* Wait until every queued chunk has finished (results stay pollable).  A
 * chunk waiting for arena memory finishes only after results are released,
 * so release what you poll before draining. */
dd_status dd_serve_drain(dd_server* srv);

/* Queue state: chunks waiting for admission, on the device, finished but not
 * released; and the largest free block of the arena.  Any pointer may be NULL. */
dd_status dd_serve_stats(dd_server* srv, int32_t* pending, int32_t* inflight, int32_t* finished,
                         size_t* largest_free);

dd_status dd_serve_destroy(dd_server* srv);

/* ------------------------------------------------------------ detection
 *
 * The stage after de-dispersion (section 3, output thread; the boxcar S/N of
 * Figure 5): every DM row is normalised by its own mean mu_d and population
 * standard deviation sigma_d over its nout samples (FP64); for widths
 * w = 1, 2, 4, ..., 2^max_log2_width the box starting at sample t has
 * S/N (sum_{i<w} x[d][t+i] - w*mu_d) / (sigma_d*sqrt(w)), defined for
 * t + w <= nout; sample (d, t) is an event when its best S/N over those
 * widths is >= nsigma (the smallest width wins ties).  Rows with
 * sigma_d = 0 have no events.
 */
typedef struct dd_event {
  int32_t dm_row;   /* output row (the plan's DM index) */
  int32_t width;    /* boxcar width in samples */
  int64_t t;        /* first output sample of the box */
  float snr;        /* S/N of that box (FP32) */
  int32_t reserved; /* 0 */
} dd_event;

/*
 * Detect events in a de-dispersed buffer d_out (ndms rows of out_stride
 * elements; out_t DD_F32 or DD_I32; nout >= 1 samples per row used).
 *   max_log2_width  0..6 (widths up to 64 samples)
 *   d_stats         device, 2*ndms doubles, written: (mu_d, sigma_d) per row
 *   d_events        device, room for max_events events (order unspecified)
 *   d_count         device, one uint64, written: the number of events found,
 *                   which may exceed max_events (only max_events of them are
 *                   stored)
 * All buffers belong to the caller; the work is queued on `stream` (NULL =
 * default stream) and the results are valid once it completes.
 * DD_ERR_INVALID_ARG for bad sizes or NULL pointers, DD_ERR_DTYPE for other
 * output types.
 */
dd_status dd_detect(const void* d_out, dd_dtype out_t, int32_t ndms, int64_t nout,
                    int64_t out_stride, float nsigma, int32_t max_log2_width, double* d_stats,
                    dd_event* d_events, int64_t max_events, uint64_t* d_count, void* stream);

/*
 * For callers that cannot allocate (code under graph capture, tight serving
 * loops, harnesses that forbid allocation): dd_detect without the d_stats
 * buffer.  The per-row statistics live in a static device array of the
 * library (65535 rows, 1 MB, one per GPU, held until the process ends); this
 * call allocates nothing.  Other arguments, results and errors as dd_detect;
 * ndms > 65535 returns DD_ERR_TOO_LARGE.  Every call on a GPU shares that
 * GPU's array: calls that overlap on one GPU (different streams, no
 * ordering between them) race on it and must be serialised by the caller.
 */
dd_status dd_detect_noalloc(const void* d_out, dd_dtype out_t, int32_t ndms, int64_t nout,
                            int64_t out_stride, float nsigma, int32_t max_log2_width,
                            dd_event* d_events, int64_t max_events, uint64_t* d_count,
                            void* stream);

/* ------------------------------------------------------------ subband
 *
 * Section 3.2's approximate method for large DM ranges, as a survey plan of
 * passes (Table 1).  For a pass {dm_lo, dm_hi, ddm, dsub, bin}:
 *   fine DMs     dm_lo + i*ddm < dm_hi (the output rows of the pass)
 *   nominal DMs  dm_lo + (k + 0.5)*dsub, the centres of the sub-ranges of
 *                width dsub; fine DM d belongs to k = floor((d - dm_lo)/dsub)
 *   binning      the mean of `bin` adjacent samples; shifts of the pass use
 *                the delay law at t_samp*bin
 *   stage 1      channel c is in subband s = c / ceil(nchans/nsub) with top
 *                channel c_s; sub[s][k][t] = sum over its channels of
 *                binned[c][t + delay(D_k, c) - delay(D_k, c_s)]
 *   stage 2      out[d][t] = sum over s of sub[s][k(d)][t + delay(d, c_s)]
 * Stage-1 series are cut to nsamp_b - M1 samples (M1 the pass's largest
 * stage-1 shift, nsamp_b = nsamp / bin) and the pass's rows to
 * nsamp_b - M1 - M2 (M2 its largest stage-2 shift).  FP32 input and output;
 * both stages run the brute-force kernels.
 */
typedef struct dd_subband_plan dd_subband_plan;
typedef struct dd_subband_pass {
  double dm_lo, dm_hi; /* DM range [dm_lo, dm_hi) */
  double ddm;          /* fine DM step */
  double dsub;         /* nominal DM spacing */
  int32_t bin;         /* binning factor >= 1 */
  int32_t reserved;    /* 0 */
} dd_subband_pass;

/* nsub in 1..nchans; passes in increasing DM order.  DD_ERR_INVALID_ARG for
 * bad bands, steps or pass lists. */
dd_status dd_subband_plan_create(int32_t nchans, double f_top, double df, double t_samp,
                                 int32_t nsub, const dd_subband_pass* passes, int32_t npass,
                                 dd_subband_plan** out);
/* Number of output rows (fine DMs over all passes) and passes. */
dd_status dd_subband_plan_info(const dd_subband_plan* plan, int32_t* ndms, int32_t* npass);
/* Host arrays of ndms entries: each row's DM and its pass index (either may
 * be NULL). */
dd_status dd_subband_dms(const dd_subband_plan* plan, double* dms, int32_t* pass_of_row);
/* For nsamp input samples: each pass's output samples per row (npass
 * entries, host) and the device workspace execute needs.  DD_ERR_NSAMP when
 * some pass has no complete output sample. */
dd_status dd_subband_sizes(const dd_subband_plan* plan, int64_t nsamp, int64_t* nout_per_pass,
                           size_t* workspace_bytes);
/* d_in [nchans][in_stride] FP32 (device), d_out [ndms][out_stride] FP32
 * (device; row r holds nout of its pass, out_stride >= the largest), and a
 * device workspace of at least the bytes dd_subband_sizes reported.  Queued
 * on `stream`. */
dd_status dd_subband_execute(const dd_subband_plan* plan, const float* d_in, int64_t nsamp,
                             int64_t in_stride, float* d_out, int64_t out_stride, void* d_workspace,
                             size_t workspace_bytes, void* stream);
dd_status dd_subband_plan_destroy(dd_subband_plan* plan);

/* ------------------------------------------------------------ front end
 *
 * Section 5's real-time front end: complex voltages of nsub coarse subbands
 * (one spectrum per time sample, subband 0 at the top of the band) are
 * channelised by an FFT of nfft consecutive samples per subband and turned
 * into power, written directly in channel order:
 *   out[(s*nfft + j)*out_stride + t] = |X_{s,k}(t)|^2,
 *   X_{s,k}(t) = sum_{n<nfft} v[(t*nfft + n)*in_stride + s] exp(-2 pi i k n / nfft),
 *   k = (nfft/2 - 1 - j) mod nfft   (channels run from high to low frequency)
 * for t < nsamp / nfft.  v is interleaved complex FP32 (re, im), in_stride
 * >= nsub complex elements between time samples; nfft in {2, 4, 8, 16};
 * out_stride >= nsamp / nfft.  FP32 arithmetic.  Queued on `stream`.
 */
dd_status dd_channelise(const float* d_volt, int64_t nsamp, int32_t nsub, int64_t in_stride,
                        int32_t nfft, float* d_out, int64_t out_stride, void* stream);

/* ------------------------------------------------------------ corner turn
 *
 * Telescope data arrive in time order (one spectrum of nchans channels per
 * time sample); the path reads channel order (one time series per channel,
 * section 3.1).  dd_corner_turn converts the first into the second:
 *   out[c*out_stride + t] = in[t*in_stride + c']   (t < nsamp, c < nchans)
 * with c' = c, or c' = nchans-1-c when flip != 0 (spectra stored with the
 * lowest frequency first; the plan's channel 0 is the top of the band).
 * d_in and d_out are device buffers of `type` (DD_U8, DD_F16 or DD_F32)
 * elements, in_stride >= nchans, out_stride >= nsamp; they must not overlap.
 * Queued on `stream`.  DD_ERR_INVALID_ARG for bad sizes or NULL pointers,
 * DD_ERR_DTYPE for other types.
 */
dd_status dd_corner_turn(const void* d_in, dd_dtype type, int64_t nsamp, int32_t nchans,
                         int64_t in_stride, int32_t flip, void* d_out, int64_t out_stride,
                         void* stream);

/* ------------------------------------------------------------------------ */
/* Host test hooks: the FP32 threaded-jump kernel's table                   */
/* ------------------------------------------------------------------------ */

/*
 * The FP32 threaded-jump kernel (tile variant 6) serves each wavefront's dw
 * DMs from one register window per channel: every DM's add run is a block of
 * code whose window offset is fixed, and the host table entry of each
 * (tile, channel, wavefront, DM) names that block, so the kernel jumps
 * through the entries.  An entry outside the block table would be a jump
 * into arbitrary code; the library therefore checks every table before it
 * uploads it, and these two pure host functions expose the builder and the
 * checker so that tests can plant wrong entries.  No GPU is used.
 *
 * dd_jump_table_build: from ngroups groups of dw shifts rel[g*dw + j] (>= 0,
 * relative to the staged window of the group's channel) writes
 * entries[g*2*dw + j] (block byte offset) and entries[g*2*dw + dw + j]
 * (window start, samples, a multiple of 4) for the block table of window
 * `wmax` registers and k adds per block.  dw in {4, 8}, k a multiple of 4,
 * wmax a multiple of 4 and >= k + 4.  wmax = 0 selects instead the layout of
 * the FP32 default kernel (tile variant 7): a window of 4k samples shared
 * between neighbouring lanes, dw in 2..8, k a multiple of 4 up to 64.
 * DD_ERR_INVALID_ARG for other shapes or a negative shift.
 *
 * dd_jump_table_check: DD_OK when every entry names a block of its own DM's
 * slot (the first DM's a window load), every window start is a multiple of 4
 * in [0, rel], and the window the entries load, read at each block's fixed
 * offset, yields exactly rel for every DM; DD_ERR_STATE otherwise
 * (dd_last_error says which rule failed).
 */
dd_status dd_jump_table_build(const int32_t* rel, int64_t ngroups, int32_t dw, int32_t k,
                              int32_t wmax, int32_t* entries);
dd_status dd_jump_table_check(const int32_t* entries, const int32_t* rel, int64_t ngroups,
                              int32_t dw, int32_t k, int32_t wmax);

/* ------------------------------------------------------------------------ */

/*
 * The FP32 pair-sum kernel (tile variant 8) takes channels in groups of g
 * (pairs) and, per DM tile, builds one LDS row per group and delay pattern
 * (the shifts of the group's later channels relative to its first); each DM
 * then adds one run of its pattern's row.  Its table holds, per (tile,
 * group), the patterns (`aux`: count, then g-1 relative shifts per pattern)
 * and, per (tile, group, wavefront), a chain of block offsets through the
 * jump table of the step (`ent`: first block, one next-block offset per DM
 * slot, one window start per slot).  A wrong offset would be a jump into
 * arbitrary code, so the library checks every table before upload; these
 * pure host functions expose the sizes, the builder and the checker so that
 * tests can plant wrong entries.  No GPU is used.
 *
 * dd_pair_table_sizes: words of `ent` and `aux` for tile height td (a
 * multiple of 4, at most 28), group size g (1..8) and pmax pattern rows per
 * group.
 * dd_pair_table_build: fills them for k samples per lane (a multiple of 4),
 * slot floats per staged row (a multiple of 64) and gps groups per stage;
 * DD_ERR_NOT_IMPLEMENTED when some (tile, group) has more than pmax
 * patterns (the library then runs the single-channel kernel).
 * dd_pair_table_check: DD_OK when every chain visits each DM slot once,
 * starts with a first-visit window load, ends at the exit, keeps every
 * window inside the workgroup's LDS, and gives every DM exactly its own
 * pattern row at its own shift; DD_ERR_STATE otherwise (dd_last_error says
 * which rule failed).
 */
dd_status dd_pair_table_sizes(const dd_plan* plan, int32_t td, int32_t g, int32_t pmax,
                              int64_t* ent_words, int64_t* aux_words);
dd_status dd_pair_table_build(const dd_plan* plan, int32_t td, int32_t g, int32_t pmax, int32_t k,
                              int32_t slot, int32_t gps, int32_t* ent, int32_t* aux);
dd_status dd_pair_table_check(const dd_plan* plan, int32_t td, int32_t g, int32_t pmax, int32_t k,
                              int32_t slot, int32_t gps, const int32_t* ent, const int32_t* aux);

const char* dd_status_str(dd_status s);
const char* dd_last_error(void);
/* Library version, "major.minor.patch". */
const char* dd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DEDISP_H */

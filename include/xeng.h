/*
 * xeng.h - C ABI of the MI355X X-engine library (libxeng.so).
 *
 * The X-engine is the O(N^2) stage of an FX correlator (Section 1; Section
 * 2.5; Fig. 2 caption: the X-engines cross-multiply and time-average the
 * channelised voltages of every antenna pair). For every channel f and every
 * pair of inputs i >= j it accumulates
 *
 *     V[f][i][j] = sum_t x_i(t, f) * conj(x_j(t, f))
 *     Re V = sum_t (xr_i xr_j + xi_i xi_j),  Im V = sum_t (xi_i xr_j - xr_i xi_j)
 *
 * exactly, in integers, over the samples of successive xeng_correlate calls
 * (Section 2.5: groups of spectra are cross-multiplied and summed to the dump
 * cadence) until xeng_dump hands the sums out (Section 2.6: the accumulator
 * is read out and zeroed). Sums are returned as sums; dividing by the sample
 * count ("averaging") is left to the caller.
 *
 * Input samples (caller-owned DEVICE memory, layout [time][channel][input],
 * i.e. after the corner turn of Fig. 2):
 *   in_bits = 4 : one byte per complex sample, the F-engine's 4+4-bit output
 *                 (Section 2.2). Real part in bits 7..4, imaginary part in
 *                 bits 3..0, each two's complement in [-8, 7]; -8 is legal.
 *   in_bits = 8 : two bytes per complex sample, int8 real then int8
 *                 imaginary (the 8+8-bit form of Section 2.4), [-128, 127].
 *
 * Output (per subarray): int32 [n_chans][N(N+1)/2][2], the lower triangle
 * i >= j including the autocorrelations, packed row by row at index
 * i(i+1)/2 + j, each entry (re, im). Products XX, YY, XY, YX of dual-
 * polarisation antennas (Table 1, note a) are entries of this matrix when
 * input i = 2 * antenna + polarisation.
 *
 * Exactness: every result is the exact integer sum. The library refuses
 * (XENG_ERANGE, before launching anything) a call that would let any sum
 * leave int32: at most XENG_MAX_DUMP_SAMPLES_4BIT samples per dump for 4-bit
 * input, XENG_MAX_DUMP_SAMPLES_8BIT for 8-bit input. The FP8 engine sums at
 * most XENG_MAX_CALL_SAMPLES_FP8 samples in fp32 at a time (every partial sum
 * stays below 2^24, where fp32 is exact) and adds each such segment into the
 * int32 accumulator, so its calls may be of any length and its dump bound is
 * the 4-bit one.
 *
 * Streams and ownership: xeng_correlate and xeng_dump enqueue work on the
 * context's HIP stream and return; the caller keeps the sample buffers valid
 * until that work has run. The library owns the accumulators; the caller owns
 * sample and output buffers. A context is used from one host thread at a time.
 *
 * Every function returns 0 (XENG_OK) or a positive XENG_E* code; the detail
 * of the last failure on the calling thread is in xeng_last_error().
 */
#ifndef XENG_H
#define XENG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XENG_OK 0
#define XENG_EINVAL 1 /* bad argument: null pointer, size or option out of range */
#define XENG_ERANGE 2 /* the call would break the exactness bound; nothing launched */
#define XENG_ENOMEM 3 /* device allocation failed */
#define XENG_EHIP 4   /* a HIP runtime call failed; see xeng_last_error() */
#define XENG_EBUSY 5  /* non-blocking stream: no free ring slot, the gulp was counted as dropped */

#define XENG_ENGINE_I8 0  /* int8 MFMA, int32 accumulation */
#define XENG_ENGINE_FP8 1 /* FP8 (OCP e4m3) MFMA, fp32 partial sums; in_bits == 4 and N % 16 == 0 */

#define XENG_MAX_DUMP_SAMPLES_4BIT 16777215LL /* floor((2^31 - 1) / 128) */
#define XENG_MAX_DUMP_SAMPLES_8BIT 65535LL    /* floor((2^31 - 1) / 32768) */
#define XENG_MAX_CALL_SAMPLES_FP8 32768LL     /* samples per fp32 partial sum: 450 * 2^15 < 2^24 */

typedef struct xeng_ctx xeng_ctx; /* opaque, library-owned */

/* One subarray: an independent set of inputs correlated with its own shape. */
typedef struct {
    int32_t n_inputs; /* 1 <= N <= 65535 inputs (input i = 2 * antenna + polarisation) */
    int32_t n_chans;  /* F >= 1 channels */
    int32_t n_time;   /* T >= 1 time samples consumed per xeng_correlate call */
    int32_t in_bits;  /* 4 or 8, see above */
    int32_t engine;   /* XENG_ENGINE_I8 or XENG_ENGINE_FP8 */
} xeng_subarray;

/*
 * Create a context for n_subs (1..16) subarrays. Allocates the device
 * accumulators (n_chans * N(N+1)/2 * 8 bytes each) on the current HIP device
 * and plans the launches. hip_stream is a hipStream_t (NULL = the null
 * stream). On success *out receives the context; on failure *out is NULL and
 * nothing stays allocated. Errors: XENG_EINVAL (bad shape, engine/in_bits
 * combination, n_time above the per-call limit of the engine), XENG_ENOMEM,
 * XENG_EHIP.
 */
int xeng_create(const xeng_subarray *subs, int n_subs, void *hip_stream, xeng_ctx **out);

/*
 * Accumulate one call's samples of every subarray. d_samples[s] is a device
 * pointer to subarray s's n_time x n_chans x n_inputs samples in the layout of
 * its in_bits. Checks all bounds before launching anything: XENG_ERANGE if
 * any subarray's samples since the last dump would exceed its dump limit,
 * XENG_EINVAL for a null context or pointer. Enqueues on the context stream.
 */
int xeng_correlate(xeng_ctx *ctx, const void *const *d_samples);

/*
 * Copy every subarray's sums into out[s] (int32 [n_chans][N(N+1)/2][2]).
 * out_is_device != 0: out[s] are device pointers, the copy is enqueued on the
 * context stream and the call returns at once. out_is_device == 0: out[s] are
 * host pointers; the call waits for the stream to finish the copy. reset != 0
 * starts a new integration (the sums restart from zero and the sample count
 * from 0) after the copy. out may be NULL when reset != 0 to discard the sums.
 */
int xeng_dump(xeng_ctx *ctx, void *const *out, int out_is_device, int reset);

/*
 * xeng_correlate(ctx, d_samples) followed by xeng_dump(ctx, out, out_is_device,
 * reset), with the same arguments, checks and results. With device outputs and
 * reset != 0 the two are fused where the kernel allows it (4-bit input on the
 * int8 engine): the last launch writes each subarray's final sums straight
 * into out[s] instead of the accumulator, so the step reads the accumulator
 * at most once and never writes it. Otherwise it is exactly the two calls.
 */
int xeng_correlate_dump(xeng_ctx *ctx, const void *const *d_samples, void *const *out,
                        int out_is_device, int reset);

/* Release the context and its device memory (waits for its stream). NULL is a no-op. */
int xeng_destroy(xeng_ctx *ctx);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one
 * subarray's correlate-and-dump without a context. Writes the exact sums of
 * the n_time samples at d_samples (device, layout and formats as for
 * xeng_correlate) to d_out (device int32 [n_chans][N(N+1)/2][2], 8-byte
 * aligned), enqueued on hip_stream (a hipStream_t; NULL = null stream), and
 * returns. It calls no hipMalloc or hipFree: the tile schedule is rebuilt on
 * the device on every call in a library-owned static device array of
 * 4,210,692 bytes, which each GPU the library runs on holds until the process
 * ends. Calls that overlap on one GPU (on different streams, or from several
 * threads) race on that array; order them. Limits (XENG_EINVAL, nothing
 * launched): the persistent kernel's shapes (N a multiple of 16 for 4-bit
 * input and the FP8 engine, of 8 for 8-bit input), n_time <= 32768 samples
 * (one launch), and n_chans * nb (nb + 1) / 2 <= 524288 tiles with
 * nb = ceil(N / 128). Other errors: XENG_EINVAL (NULL or misaligned
 * pointers, bad shape), XENG_EHIP.
 */
int xeng_correlate_dump_static(const xeng_subarray *sub, const void *d_samples, void *d_out,
                               void *hip_stream);

/* Point the context at another HIP stream (NULL = null stream) for later calls;
 * work already enqueued on the old stream is ordered before them. */
int xeng_set_stream(xeng_ctx *ctx, void *hip_stream);

/* Samples accumulated into subarray sub since its last reset. */
int xeng_samples_since_dump(const xeng_ctx *ctx, int sub, int64_t *out);

/* Largest number of samples subarray sub may accumulate between dumps. */
int xeng_max_dump_samples(const xeng_ctx *ctx, int sub, int64_t *out);

/*
 * Kernel families, for xeng_set_kernel (the plan JSON names them too):
 *   XENG_KERNEL_REGISTER   register-staging tiles of 32 x tile (any shape)
 *   XENG_KERNEL_PERSISTENT persistent 4-wave workgroups over 128 x 128 tiles
 *                          (N % 16 == 0 for 4-bit, N % 8 == 0 for 8-bit; the
 *                          only one for the FP8 engine)
 *                          (the default for other shapes)
 *   XENG_KERNEL_ONE_WAVE   wave-private items of 128 x 64, one wave per SIMD
 *   XENG_KERNEL_TWO_WAVE   wave-private items of 64 x 64, two waves per SIMD
 *                          (both: 4-bit input, int8 engine, N % 16 == 0)
 *   XENG_KERNEL_SMALL_N    one channel per item, 64 x 64 (4-bit input, int8
 *                          engine, N <= 64 and N % 16 == 0: the memory-bound
 *                          regime; the default for such shapes)
 */
#define XENG_KERNEL_REGISTER 0
#define XENG_KERNEL_PERSISTENT 1
#define XENG_KERNEL_ONE_WAVE 2
#define XENG_KERNEL_TWO_WAVE 3
#define XENG_KERNEL_SMALL_N 4

/*
 * Run subarray sub on kernel family `kernel` (tile: 32, 64 or 128 inputs for
 * XENG_KERNEL_REGISTER, ignored otherwise) from the next call on. The choice
 * falls back to the next family down that supports the subarray's shape and
 * engine (as the plan JSON then shows). Discards anything accumulated (all
 * subarrays restart from zero); synchronises the context stream. Errors:
 * XENG_EINVAL, XENG_ENOMEM, XENG_EHIP.
 */
int xeng_set_kernel(xeng_ctx *ctx, int sub, int kernel, int tile);

/*
 * Describe the launch plan (tile sizes, launch counts per call) as a
 * NUL-terminated JSON object in buf (at most len bytes). XENG_EINVAL if buf
 * is too small.
 */
int xeng_plan_describe(const xeng_ctx *ctx, char *buf, size_t len);

/*
 * ---- Fast-cadence autocorrelations (Section 2.6: total power of chosen
 * inputs, e.g. outrigger antennas, integrated and dumped more often than
 * the cross power, by selective dumping and zeroing of accumulator cells).
 *
 * Select the inputs of subarray sub (host array of n indices in [0, N);
 * n = 0 clears the selection). Allocates a small device list; synchronises
 * the context stream. Errors: XENG_EINVAL, XENG_ENOMEM, XENG_EHIP.
 */
int xeng_set_fast_autos(xeng_ctx *ctx, int sub, const int32_t *inputs, int n);

/*
 * For every subarray with a selection, write Re V_ii of the selected inputs
 * to out[s] (device int32 [n_chans][n], in selection order; Im V_ii is
 * identically 0) and, if reset != 0, zero those cells so that they integrate
 * afresh. Every other cell (the cross power, unselected autocorrelations)
 * keeps integrating to the main dump, and the main dump reports the
 * selected autocorrelations since their last fast reset. out may be NULL
 * when reset != 0. Enqueued on the context stream. out_is_device must be 1.
 */
int xeng_dump_fast_autos(xeng_ctx *ctx, void *const *out, int out_is_device, int reset);

/*
 * ---- Autotuning and graph capture (batched subarrays of uneven N in one
 * persistent launch per engine and input width).
 *
 * Time, on the caller's sample buffers d_samples[s] (as for xeng_correlate),
 * every kernel family that can run each subarray (XENG_KERNEL_*: the
 * persistent kernel with 128 x 128 tiles, the wave-private kernels, the
 * small-N kernel, the register-staging kernel with 32, 64 or 128-input
 * tiles), each alone, and keep the fastest; then time the batched launch's
 * schedule options (1 or 2 workgroups per CU, tiles in locality order or
 * costliest first) and keep the fastest, and whole steps with every
 * subarray the persistent kernel can run moved into one launch. A timing is
 * the median of three batches of `reps` runs after untimed runs that let
 * the clock settle; a whole step is timed both as a correlate and as a
 * correlate-and-dump (into scratch outputs the call allocates and frees;
 * if they cannot be allocated, as a correlate only).
 * The choices are applied to ctx and remembered for this process, keyed by
 * (device architecture, n_inputs, n_chans, n_time, in_bits, engine) per
 * subarray and per list of subarrays: later contexts with the same shapes on
 * the same architecture start with them. With the environment variable
 * XENG_TUNING_FILE set, the whole cache is then written to that file (see
 * xeng_tuning_save). Any accumulated sums are discarded (the context is left
 * reset). Blocks until done. Errors: XENG_EINVAL, XENG_EHIP, XENG_ENOMEM.
 */
int xeng_autotune(xeng_ctx *ctx, const void *const *d_samples, int reps);

/*
 * The process's tuning cache as a JSON file: {"format": "xeng-tuning",
 * "version": 1, "subarrays": [...], "batches": [...]}, one entry per tuned
 * shape (keys as above, the kernel family by its plan-JSON name and its tile
 * edge) and per tuned list of shapes (kernels, workgroups per CU, tile
 * order). Entries of every architecture are kept; only the current device's
 * are applied. xeng_tuning_save writes the whole cache to `path` (through a
 * temporary file renamed over it); xeng_tuning_load merges a file into the
 * cache (all or nothing: a file that does not parse changes nothing).
 * *n_entries (if not NULL) receives the number of entries written or read.
 * With XENG_TUNING_FILE set, the first xeng_create of the process loads that
 * file if it exists (and ignores it if it does not parse). These calls touch
 * no device. Errors: XENG_EINVAL (NULL path, unreadable or unwritable file,
 * malformed content).
 */
int xeng_tuning_save(const char *path, int *n_entries);
int xeng_tuning_load(const char *path, int *n_entries);
/* Forget every tuning choice of this process (contexts already created keep
 * theirs). Returns XENG_OK. */
int xeng_tuning_clear(void);

typedef struct xeng_graph xeng_graph; /* opaque, library-owned */

/*
 * Capture one whole step into a HIP graph: xeng_correlate(d_samples), then
 * xeng_dump(out, out_is_device = 1, reset = 1). The context must have nothing
 * accumulated (a fresh or just-reset context; XENG_EINVAL otherwise) and is
 * left so. Each xeng_graph_launch re-runs the step on the same buffers: the
 * caller refills d_samples[s] and reads out[s] (device pointers) around the
 * launches. The graph holds no memset nodes (buffers are cleared by
 * kernels). The graph keeps its own reference to the tile schedule it was
 * captured with, so a later xeng_autotune (which replans ctx) does not
 * invalidate it; it reads and writes ctx's accumulators and so stays valid
 * while ctx lives. Do not interleave its launches with eager calls on ctx
 * without ordering them on one stream.
 */
int xeng_graph_create(xeng_ctx *ctx, const void *const *d_samples, void *const *out,
                      xeng_graph **out_graph);

/* Enqueue one replay of the captured step on hip_stream (a hipStream_t). */
int xeng_graph_launch(xeng_graph *g, void *hip_stream);

/* Release a graph. NULL is a no-op. */
int xeng_graph_destroy(xeng_graph *g);

/*
 * ---- Streaming integration (Section 2.5: spectra arrive in groups that are
 * cross-multiplied and summed until the dump cadence; Section 2.4: the data
 * reach the GPU through ring buffers).
 *
 * A stream owns a device ring of n_slots gulps (each n_time samples of one
 * subarray, in the subarray's input layout), a context that integrates them,
 * and three HIP streams of default priority: ingest (fills slots), compute
 * (correlates, dumps and resets) and output (copies dumps to the host).
 * Every dump_every gulps the sums are dumped, copied to the caller's host
 * buffers if given, and reset. Slot reuse, dump buffers and the host copies
 * are ordered by events, so the host never blocks in next_slot/push unless a
 * slot or dump buffer is still in use.
 */
typedef struct xeng_stream xeng_stream;

/*
 * Create a stream for one subarray on the current device. n_slots >= 2,
 * dump_every >= 1 with dump_every * n_time within the subarray's dump limit.
 * host_dumps: NULL (dumps stay on the device) or n_host_dumps >= 1 caller-
 * owned host buffers of n_chans * N(N+1)/2 * 8 bytes, preferably pinned;
 * dump d is written to host_dumps[d % n_host_dumps], where it stays until
 * the push that completes dump d + n_host_dumps. Errors: XENG_EINVAL,
 * XENG_ERANGE (dump period above the dump limit), XENG_ENOMEM, XENG_EHIP.
 */
int xeng_stream_create(const xeng_subarray *sub, int n_slots, int dump_every,
                       void *const *host_dumps, int n_host_dumps, xeng_stream **out);

/*
 * Slot for the next gulp. Makes the ingest stream wait until the gulp that
 * used the slot before has been correlated, records the gulp's arrival, and
 * returns the slot's device pointer and the ingest stream (a hipStream_t).
 * The caller enqueues the work that fills the slot (a copy, a producer
 * kernel) on that stream and then calls xeng_stream_push. Calling it twice
 * without a push returns the same slot. In non-blocking mode, if that slot's
 * previous gulp has not been correlated yet (the engine is behind), the gulp
 * is dropped instead (as by xeng_stream_drop): *d_slot = NULL and
 * XENG_EBUSY; the caller discards the gulp's data.
 */
int xeng_stream_next_slot(xeng_stream *s, void **d_slot, void **ingest_stream);

/*
 * The slot from xeng_stream_next_slot is filled by the work enqueued on the
 * ingest stream so far: enqueue its correlation on the compute stream and,
 * when it completes a dump period, the dump, the host copy and the reset.
 * Returns at once. *gulp (may be NULL) receives the gulp's index.
 */
int xeng_stream_push(xeng_stream *s, int64_t *gulp);

/*
 * Wait until dump d (0-based) is complete: in the caller's host buffer if
 * host dumps were given, else in the device buffer whose pointer is stored
 * in *d_dump (valid until dump d + 2 is written). d_dump may be NULL.
 */
int xeng_stream_dump_wait(xeng_stream *s, int64_t d, void **d_dump);

/*
 * Wait for gulp g (one of the last 1024 pushed) and report, in milliseconds,
 * the time from its arrival (the next_slot call that asked for its slot,
 * including any wait for that slot to come free) and from its slot being
 * filled to the end of its correlation (and of its dump, when it completes
 * one).
 */
int xeng_stream_gulp_times(xeng_stream *s, int64_t g, float *arrive_ms, float *ready_ms);

/* Number of gulps so far, pushed or dropped. */
int xeng_stream_gulps(const xeng_stream *s, int64_t *out);

/*
 * Overload handling (Section 2.4: lost data is counted, not corrected). The
 * next gulp is lost (for instance, too few of its packets arrived): it is
 * counted, adds nothing to any sum, and still counts towards the dump and
 * fast-autocorrelation cadences, so every dump covers the same span of
 * time. *gulp (may be NULL) receives its index. A slot obtained by
 * xeng_stream_next_slot and not pushed is given back.
 */
int xeng_stream_drop(xeng_stream *s, int64_t *gulp);

/* on != 0: xeng_stream_next_slot drops a gulp whose slot is still busy
 * instead of making the ingest stream wait for it (XENG_EBUSY). */
int xeng_stream_set_nonblocking(xeng_stream *s, int on);

typedef struct {
    int64_t gulps;      /* pushed + dropped */
    int64_t correlated; /* pushed */
    int64_t dropped;    /* dropped (xeng_stream_drop, or no free slot in non-blocking mode) */
    int64_t dumps;      /* dumps enqueued */
    int64_t fast_dumps; /* fast-cadence autocorrelation dumps enqueued */
    int64_t backlog;    /* gulps whose device work has not finished (as xeng_stream_backlog) */
} xeng_stream_counts;

int xeng_stream_stats(xeng_stream *s, xeng_stream_counts *out);

/*
 * Fast-cadence autocorrelations inside the stream (Section 2.6: total power
 * of chosen inputs dumped more often than the cross power). Before the first
 * gulp: select n inputs of the subarray (host array, indices in [0, N)) and
 * dump their autocorrelations every `every` gulps (pushed or dropped) into a
 * device buffer int32 [n_chans][n] (Re V_ii in selection order), copied to
 * host_out[k % n_host] if host buffers (n_chans * n * 4 bytes, preferably
 * pinned) are given; the selected cells are then cleared. The main dump
 * reports the selected autocorrelations since their last fast dump. Errors:
 * XENG_EINVAL, XENG_ENOMEM, XENG_EHIP.
 */
int xeng_stream_set_fast_autos(xeng_stream *s, const int32_t *inputs, int n, int every,
                               void *const *host_out, int n_host);

/* Wait until fast dump k (0-based, one of the last two) is complete; *d_out
 * (may be NULL) receives its device buffer. */
int xeng_stream_fast_wait(xeng_stream *s, int64_t k, void **d_out);

/* Gulps pushed whose correlation (and dump, if they complete one) has not yet
 * finished on the device: 0 while the engine keeps up; a count that grows
 * from push to push means gulps arrive faster than they are integrated. */
int xeng_stream_backlog(xeng_stream *s, int64_t *out);

/* Wait for all work of the stream and release it. NULL is a no-op. */
int xeng_stream_destroy(xeng_stream *s);

/*
 * ---- Packet ingest (Section 2.3: the F-engine boards send UDP packets of a
 * header and a payload of channelised samples to the GPU servers; Section
 * 2.4: the CPU layer captures them and completes the corner turn into the
 * X-engine's [time][channel][input] order; missing packets are counted, not
 * corrected). The paper's payload layout is not recoverable from its text,
 * so the format is this library's own:
 *
 *   header, 16 bytes, little-endian:
 *     uint64 t0       first time sample of the packet (absolute)
 *     uint16 chan0    first channel
 *     uint16 input0   first input
 *     uint32 magic    XENG_PACKET_MAGIC
 *   payload: pkt_time x pkt_chans x pkt_inputs samples, [time][chan][input],
 *   in the subarray's sample format (1 byte per 4+4-bit sample, 2 for 8-bit)
 *   packet stride: 16 + payload bytes rounded up to a multiple of 16.
 *
 * A gulp [gulp_t0, gulp_t0 + n_time) expects one packet per (time block,
 * channel block, input block): n_time / pkt_time x n_chans / pkt_chans x
 * n_inputs / pkt_inputs packets, which must divide exactly. The ingest
 * writes every valid packet's samples into the gulp buffer, zero-fills the
 * blocks whose packet did not arrive (zeros add nothing to any sum), and
 * counts received, missing, duplicate and rejected packets (bad magic, not
 * aligned to the blocks, or outside the gulp). When several packets name
 * the same block, the first in buffer order fills it and the others count
 * as duplicates, whatever their payloads.
 */
#define XENG_PACKET_MAGIC 0x4C454441u /* "LEDA" */

typedef struct {
    int32_t pkt_time;   /* time samples per packet */
    int32_t pkt_chans;  /* channels per packet */
    int32_t pkt_inputs; /* inputs per packet */
} xeng_packet_format;

typedef struct xeng_ingest xeng_ingest; /* opaque, library-owned */

typedef struct {
    int64_t received;   /* packets written into the gulp */
    int64_t missing;    /* expected packets that did not arrive (zero-filled) */
    int64_t duplicate;  /* second and later copies of a block (ignored) */
    int64_t rejected;   /* bad magic, misaligned, or outside the gulp */
} xeng_ingest_stats;

/* Create an ingest engine for gulps of `sub` (n_time samples) and packets of
 * `fmt`. Allocates a device table of 4 bytes per block and counters. Errors: XENG_EINVAL
 * (sizes that do not divide), XENG_ENOMEM, XENG_EHIP. */
int xeng_ingest_create(const xeng_subarray *sub, const xeng_packet_format *fmt, xeng_ingest **out);

/* Bytes between consecutive packets in a packet buffer. */
int xeng_ingest_packet_stride(const xeng_ingest *ig, int64_t *out);

/* Scatter n_packets packets (device buffer, packet stride apart, any order)
 * into the device gulp buffer d_gulp for the gulp starting at absolute
 * time gulp_t0, zero-fill what is missing and update the counters; all
 * enqueued on hip_stream (a hipStream_t). d_gulp is fully written. The
 * engine's table and counters serve one gulp at a time: a call on another
 * stream than the previous call's waits for that call's work. */
int xeng_ingest_gulp(xeng_ingest *ig, const void *d_packets, int64_t n_packets, int64_t gulp_t0,
                     void *d_gulp, void *hip_stream);

/* Wait for the last gulp's ingest and return its counters. */
int xeng_ingest_stats_get(xeng_ingest *ig, xeng_ingest_stats *out);

/* Release the engine (waits for its last stream). NULL is a no-op. */
int xeng_ingest_destroy(xeng_ingest *ig);

/*
 * ---- F-engine (Section 2.2: a 4-tap, 8192-point polyphase filter bank, an
 * FIR filter with a Hamming window and 18-bit coefficients followed by an FFT
 * that halves the data at each stage; one band-average digital gain; the
 * result requantised to 4+4 bits; a contiguous group of channels kept).
 *
 * For input n and spectrum m (samples [8192 m, 8192 (m + 4)) of the input):
 *   c[l]  = clip(rint(2^17 w[l] sinc((l - 16383.5) / 8192)), -2^17, 2^17 - 1),
 *           l < 32768, w the symmetric Hamming window of length 32768;
 *   y[k]  = sum_{tap<4} c[8192 tap + k] x_n[8192 (m + tap) + k], k < 8192
 *           (exact integers);
 *   Y[ch] = gain 2^-17 / 8192 sum_k y[k] exp(-2 pi i k ch / 8192) (fp32);
 *   out[m][ch - chan0][n] = clip(rint(Re Y), -8, 7) << 4
 *                         | (clip(rint(Im Y), -8, 7) & 15),
 * the X-engine's 4+4-bit [time][channel][input] input (rint: half to even).
 * Channel ch covers ch x 24.0 kHz at the paper's 196.608 MHz sample clock.
 */
#define XENG_FENGINE_FFT 8192
#define XENG_FENGINE_TAPS 4
#define XENG_FENGINE_CHANS 4096 /* channels 0 .. 4095 (DC to just below Nyquist) */

typedef struct xeng_fengine xeng_fengine; /* opaque, library-owned */

typedef struct xeng_fengine_config {
    int32_t n_inputs; /* ADC inputs, 1 .. 65535 */
    int32_t chan0;    /* first channel kept, >= 0 */
    int32_t n_chans;  /* channels kept; chan0 + n_chans <= XENG_FENGINE_CHANS */
    float gain;       /* the one band-average digital gain, > 0 and finite */
} xeng_fengine_config;

/* Create an F-engine on the current device: builds the coefficient and
 * twiddle tables in device memory. Errors: XENG_EINVAL (sizes, gain),
 * XENG_ENOMEM. */
int xeng_fengine_create(const xeng_fengine_config *cfg, xeng_fengine **out);

/* Inputs handled by one workgroup (1, 2 or 4: the largest that divides
 * n_inputs; d_out must be aligned to it). Returns it, or XENG_EINVAL
 * (negative) for NULL. */
int xeng_fengine_group(const xeng_fengine *fe);

/* Channelise n_spectra spectra of every input, enqueued on hip_stream (a
 * hipStream_t; NULL = default stream). d_adc: device int8 [n_inputs][adc_stride]
 * samples, row start and adc_stride multiples of 8, adc_stride >=
 * (n_spectra + 3) 8192. d_out: device uint8 [n_spectra][n_chans][n_inputs],
 * fully written. d_spec: NULL, or device float2 [n_spectra][n_chans][n_inputs]
 * (8-byte aligned) that receives (Re Y, Im Y) before rounding. Errors:
 * XENG_EINVAL (NULL pointers, sizes, alignment), XENG_EHIP (launch). */
int xeng_fengine_run(xeng_fengine *fe, const int8_t *d_adc, int64_t adc_stride, int64_t n_spectra,
                     uint8_t *d_out, void *d_spec, void *hip_stream);

/* Release the engine (synchronises the device first). NULL is a no-op. */
int xeng_fengine_destroy(xeng_fengine *fe);

/* Static text for an XENG_* code. */
const char *xeng_strerror(int code);

/* Detail of the last failure on the calling thread ("" if none). */
const char *xeng_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* XENG_H */

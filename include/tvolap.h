/*
 * tvolap.h - C ABI of the MI355X (gfx950) TVOLAP library.
 *
 * Time-Variant Overlap-Add in Partitions (Jaeger, Simmer, Bitzer, Blau,
 * arXiv 2310.00319). Per channel and per block of L new samples the library
 *   - weights the last 2L input samples with a periodic Hann window of
 *     amplitude 1/2 (Sec. 2, eq. 1-2; the windows at hop L sum to one),
 *   - zero pads the block to 4L and transforms it (eq. 4-5),
 *   - keeps the spectra of past blocks in a frequency-domain delay line and
 *     multiplies every second one with the 4L-point spectra of the impulse
 *     response's 2L-tap partitions (eq. 3, 6-8),
 *   - transforms the sum back (eq. 9) and overlap-adds the 4L-sample result at
 *     hop L (eq. 10-13, each block's right half meeting the left half of the
 *     block two hops later).
 * An impulse-response switch exchanges all partition spectra of a channel at a
 * block boundary (end of Sec. 2); many channels run in parallel.
 *
 * Conventions for every entry point:
 *   - Return value: TVOLAP_OK (0) or a negative error code. On an error the
 *     handle's state is unchanged and tvolap_last_error() describes it.
 *     No C++ exception crosses this interface.
 *   - Device pointers are HIP device allocations on the handle's device. All
 *     device work is enqueued on the handle's stream and is asynchronous with
 *     respect to the host unless stated otherwise.
 *   - A handle is used by one host thread at a time.
 *   - Sample and spectrum values are float32 in device memory.
 */
#ifndef TVOLAP_H
#define TVOLAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TVOLAP_OK 0
#define TVOLAP_EINVAL (-1)   /* invalid argument                                   */
#define TVOLAP_ENOMEM (-2)   /* device or host allocation failed                   */
#define TVOLAP_EDEVICE (-3)  /* a HIP call failed; message in tvolap_last_error()  */
#define TVOLAP_ESTATE (-4)   /* call not valid in the handle's current state       */

/* Storage type of the partition spectra and of the delay line. Transforms and
 * accumulation are float32 for every choice; bf16 and f16 are rounded to
 * nearest even from float32 when stored. */
typedef enum { TVOLAP_F32 = 0, TVOLAP_BF16 = 1, TVOLAP_F16 = 2 } tvolap_dtype;

typedef struct tvolap tvolap_t;

typedef struct {
  int32_t hop;                      /* L: block hop in samples, one of 64, 128, 256, 512.
                                       Input blocks and IR partitions are 2L long,
                                       transforms 4L long (Sec. 2).                      */
  int32_t n_channels;               /* C >= 1: convolution channels (outputs).          */
  int32_t n_inputs;                 /* I >= 1: distinct input signals.                   */
  const int32_t* input_of_channel;  /* host [C], values in [0, I); NULL = identity
                                       (then I must equal C). Channels that share an
                                       input share its delay line.                       */
  int32_t max_taps;                 /* >= 1: longest impulse response of any channel.    */
  const int32_t* taps_of_channel;   /* host [C] IR length per channel (all its slots),
                                       1 .. max_taps; NULL = max_taps for every channel.
                                       Channel c has M_c = ceil(taps_c / 2L) partitions. */
  int32_t n_slots;                  /* K >= 1: impulse-response slots per channel.       */
  int32_t spectra_dtype;            /* tvolap_dtype.                                     */
  void* stream;                     /* hipStream_t for all device work; NULL = the null
                                       stream.                                           */
  int32_t max_batch;                /* largest n_blocks of tvolap_process_blocks, 0..1024
                                       (0 = 16). The delay line keeps (max_batch-1)/2
                                       extra spectra per parity.                         */
  int32_t n_outputs;                /* 0: one output per channel. E > 0: a mixdown into E
                                       output buses: the outputs of the parallel
                                       channels (end of Sec. 2) summed per bus.          */
  const int32_t* output_of_channel; /* host [C] bus of each channel (every bus gets at
                                       least one channel); used when n_outputs > 0. The
                                       channels' spectra are summed per bus before one
                                       inverse transform (the transforms are linear).
                                       A mixdown runs the per-block path with fused = 0. */
} tvolap_config;

/* Sizes of a handle, for accounting. Bytes count what one processed block must
 * move at least: every active partition spectrum once, every delay-line
 * spectrum once per input, the new spectra written, the input and output
 * samples. */
typedef struct {
  int32_t hop, n_channels, n_inputs, n_slots, spectra_dtype;
  int32_t bins;                     /* 2L complex values per stored spectrum (the DC and
                                       Nyquist bins, both real, share one complex slot). */
  int64_t sum_partitions;           /* sum over channels of M_c                          */
  int64_t sum_input_partitions;     /* sum over inputs of the delay-line length M_i      */
  int64_t mac_bytes_per_block;      /* spectral MAC: IR + delay-line spectra read        */
  int64_t block_bytes;              /* whole block: MAC + new spectra + samples in/out   */
  int64_t bank_bytes, delay_line_bytes, workspace_bytes;
  int32_t n_work_items;             /* MAC work items per block                          */
  int32_t mac_chunk;                /* partitions per MAC work item                      */
  int32_t mac_waves;                /* waves per MAC workgroup                           */
  int32_t mac_grid;                 /* MAC workgroups launched (each loops over items)   */
  int32_t fused;                    /* launches per block: 1 -> one, 2 -> two, 0 -> three */
  int32_t n_cu;                     /* compute units of the device                       */
  /* batched calls (tvolap_process_blocks): time-blocked MAC schedule          */
  int32_t batch_chunk;              /* partitions per work item                          */
  int32_t batch_vec;                /* complex bins per lane                             */
  int32_t batch_waves;              /* waves per workgroup (each owns 64 vec bins)       */
  int32_t batch_tile_width;         /* bins per work item: 64 vec waves                  */
  int32_t batch_work_items;         /* items per time group (a parity class of up to
                                       batch_time_block blocks of a call)                */
  int32_t batch_rows;               /* partial-spectrum rows per block                   */
  int32_t batch_time_block;         /* blocks of one parity per time group (8 or 16)     */
  int32_t batch_group;              /* channels of one input per work item (1 or 2)      */
  int32_t batch_engine;             /* 1 = vector ALU, 2 = matrix cores                  */
  int32_t n_outputs;                /* output rows: n_channels, or the mixdown buses     */
} tvolap_info;

/* Create a convolver (Sec. 2: partitioned, block-synchronously switchable,
 * multichannel). Allocates on the current HIP device: the IR bank
 * [C][K][M_c][2L], the delay line [I][2][M_i + (max_batch-1)/2][2L] (M_i =
 * max M_c over the channels fed by input i), input history, overlap-add
 * state, and tables
 * (twiddles and window computed in double precision on the host). The bank is
 * zeroed (all slots hold a zero IR), the stream state is reset and every
 * channel selects slot 0. Synchronous. *out receives the handle, or NULL on an
 * error. Errors: EINVAL (bad sizes, hop not supported, map out of range),
 * ENOMEM, EDEVICE. */
int tvolap_create(const tvolap_config* cfg, tvolap_t** out);

/* Free every allocation of the handle after waiting for its stream. NULL is
 * accepted. */
int tvolap_destroy(tvolap_t* h);

/* Load an impulse response into slot `slot` of channel `channel` (Sec. 2,
 * eq. 3, 6-7): the taps are cut into M_c partitions of 2L taps (taps beyond
 * n_taps are zero), each partition is zero padded to 4L and transformed, and
 * the spectra are stored in the bank. `taps` is host memory (copied before
 * the call returns) or, if taps_on_device != 0, a device array read in stream
 * order. If the slot is the channel's active slot the new IR takes effect at
 * the next processed block, for all partitions at once.
 * Errors: EINVAL (channel/slot out of range, n_taps < 0 or > taps of the
 * channel, NULL taps with n_taps > 0). n_taps == 0 stores a zero IR. */
int tvolap_set_ir(tvolap_t* h, int32_t channel, int32_t slot, const float* taps,
                  int32_t n_taps, int32_t taps_on_device);

/* Load slot `slot` of every channel in one launch (Sec. 2, eq. 3, 5, 7, as
 * tvolap_set_ir does per channel): channel c's taps are
 * taps_dev[c*taps_stride + t] (device memory, read in stream order), t <
 * min(taps_stride, taps of channel c); the rest of its partitions are zero.
 * For whole-bank loads and for impulse responses that change at every block
 * (head tracking), followed by a selection of that slot. Asynchronous; may
 * be recorded in a graph. Errors: EINVAL (slot out of range, NULL taps,
 * taps_stride < 1), EDEVICE. */
int tvolap_set_irs(tvolap_t* h, int32_t slot, const float* taps_dev, int64_t taps_stride);

/* Select the active slot of every channel (end of Sec. 2: all partitions of a
 * channel switch together). `slot_of_channel` is a host array [C] with values
 * in [0, K); it is copied before the call returns and applies from the next
 * processed block on. Errors: EINVAL (NULL, value out of range). */
int tvolap_select_ir(tvolap_t* h, const int32_t* slot_of_channel);

/* Process one block (Sec. 2, eq. 1-13; Fig. 2). `in` is a device array holding
 * L new samples of every input, input i at in[i*in_stride + n], n < L; `out`
 * receives L samples of every output (channel, or bus with a mixdown) at
 * out[c*out_stride + n]. Strides are in
 * floats, >= L. Call number c (counting from creation or the last reset)
 * consumes input samples [cL, (c+1)L), completes input block c - 1 (covering
 * [(c-1)L, (c+1)L)) and emits output samples [(c-1)L, cL): the stream is the
 * time-variant convolution delayed by L samples (with the L samples of
 * buffering, an input-to-output latency of 2L, Sec. 3 Table 1).
 * `slot_of_channel_dev` is NULL (use the current selection) or a device array
 * [C] of slots for this block, read in stream order; it also becomes the
 * current selection. Values outside [0, K) are clamped into range.
 * Errors: EINVAL (NULL in/out, stride < L). */
int tvolap_process_block(tvolap_t* h, const float* in, int64_t in_stride, float* out,
                         int64_t out_stride, const int32_t* slot_of_channel_dev);

/* Process n_blocks consecutive blocks at once (1 <= n_blocks <= max_batch):
 * the same results as n_blocks calls of tvolap_process_block (up to the order
 * of floating-point additions in the spectral MAC), block j reading
 * in[i*in_stride + j*L + n] and writing out[c*out_stride + j*L + n] (n < L),
 * with the slots of block j at slots_dev[j*slots_stride + c] (device array,
 * values clamped into [0, K)) or, if slots_dev is NULL, the current selection
 * for all of them. The last block's slots become the selection. Four
 * launches: the input spectra of all blocks (eq. 1-6), the spectral MAC of
 * all blocks (eq. 8) in time groups of same-parity blocks that share
 * delay-line and partition-spectrum reads, the inverse transforms (eq. 9) and
 * the overlap-add in call order (eq. 10-13). No allocation; the call is
 * asynchronous and may be captured in a graph. Errors: EINVAL (NULL in/out,
 * n_blocks out of range, strides too small), EDEVICE. */
int tvolap_process_blocks(tvolap_t* h, const float* in, int64_t in_stride, int32_t n_blocks, float* out,
                          int64_t out_stride, const int32_t* slots_dev, int64_t slots_stride);

/* Zero the delay line, the input history and the overlap-add state and
 * restart the call count (the bank and the selection are kept). Stream
 * ordered. */
int tvolap_reset(tvolap_t* h);

/* Fill *info (host). */
int tvolap_get_info(const tvolap_t* h, tvolap_info* info);

/* Partition count M_c of every channel into the host array m_of_channel [C]. */
int tvolap_get_partitions(const tvolap_t* h, int32_t* m_of_channel);

/* Scheduling of the per-block work (no effect on results beyond the order of
 * floating-point additions). fused == 1: one kernel launch per block in which
 * the work items holding partition 0 also transform the new input block and
 * the last item to finish a channel transforms back and overlap-adds;
 * fused == 2: two launches (transform-in fused into the spectral MAC, then
 * transform-out); fused == 0: three launches (transform-in, spectral MAC,
 * transform-out). chunk:
 * partitions per work item (0 = about four items per compute unit). waves: 4
 * or 8 waves per workgroup splitting a work item's partitions (0 = 4). grid:
 * workgroups launched, each looping over the work items (0 = one per item).
 * Waits for the stream; rebuilds the work list. Errors: EINVAL, ESTATE during
 * capture, ENOMEM/EDEVICE. */
int tvolap_configure(tvolap_t* h, int32_t fused, int32_t chunk, int32_t waves, int32_t grid);

/* Autotuner for the fused schedules: times `iters` blocks (zero input, current
 * bank and selection) for each candidate (fused 1 or 2, chunk, waves, grid),
 * keeps the
 * fastest, caches it for handles of the same shape in this process, and then
 * resets the stream state as tvolap_reset does. *best_us (may be NULL)
 * receives the best time per block in microseconds, or -1 when the choice came
 * from the cache. Synchronous. Errors: EINVAL, ESTATE during capture, EDEVICE;
 * after an error past the argument checks the previous schedule is applied
 * again and the stream state is reset (the timed blocks have advanced it). */
int tvolap_autotune(tvolap_t* h, int32_t iters, float* best_us);

/* Schedule of batched calls (tvolap_process_blocks; no effect on results
 * beyond the order of floating-point additions). The spectral MAC of a call
 * works on time groups: up to time_block blocks of the same parity, which read
 * overlapping delay-line spectra (block l + 2 at partition m + 1 reads what
 * block l reads at partition m, eq. 8) and, where their slots agree, the same
 * partition spectra. chunk: partitions per work item (0 = about one workgroup
 * per compute unit); vec: complex bins per lane (1 or 2; 0 = 2, or 1 with time
 * groups of 16); waves: 1, 2 or 4 waves per workgroup, each owning 64 vec bins
 * (0 = 4, fewer when 2L bins are fewer; the matrix-core engine takes 4 or 8
 * waves of 16 bins); time_block: 8, 16 or 32 (16 needs vec 1, 32 the
 * matrix-core engine; 0 = 16 when max_batch >= 32, else 8); group: channels
 * of one input per work item, 1 or 2 (two channels share the delay-line loads; 0 = 2 when an input
 * feeds several channels); engine: 1 = vector ALU (multiply-adds or packed
 * dot products per complex product), 2 = matrix cores (per bin, the products
 * of a time group and the two channels of an input form one 16-bin MFMA per
 * step: 4x4x1 outer products for f32 spectra, 4x4x4 products over two
 * partitions for bf16/f16; 16 bins per wave, so vec must be 0 or 1; time
 * groups of 16 or 32 blocks, 0 = 32 when max_batch >= 64; time groups whose
 * slots do not alternate by parity go to the vector ALU), 0 = 1. Waits for
 * the stream; rebuilds the batched work list. Errors: EINVAL, ESTATE during
 * capture, ENOMEM/EDEVICE. */
int tvolap_configure_batch(tvolap_t* h, int32_t chunk, int32_t vec, int32_t waves, int32_t time_block,
                           int32_t group, int32_t engine);

/* Autotuner for batched calls: times `iters` calls of max_batch blocks (zero
 * input, current bank, block b of the batch in slot b mod K) for each
 * candidate (engine, group, time_block, vec, waves, chunk), keeps the fastest, caches it for handles of
 * the same shape, slot count and max_batch in this process, then resets the stream state
 * as tvolap_reset does. The selection (tvolap_select_ir) is kept. *best_us
 * (may be NULL) receives the best time per block in microseconds, or -1 when
 * the choice came from the cache. Synchronous. Errors: EINVAL, ESTATE during
 * capture, ENOMEM, EDEVICE; after an error past the argument checks the
 * previous schedule is applied again and the stream state is reset. */
int tvolap_autotune_batch(tvolap_t* h, int32_t iters, float* best_us);

/* HIP graph capture of the handle's stream (which must not be the null
 * stream). Device work enqueued between begin and end (process_block with
 * device slot arrays, set_ir with device taps, reset) is recorded instead of
 * executed; select_ir and host taps are refused with ESTATE during capture.
 * tvolap_graph_launch replays the recording on the stream; the block counter
 * lives in device memory, so every replay continues the stream. */
int tvolap_capture_begin(tvolap_t* h);
int tvolap_capture_end(tvolap_t* h);
int tvolap_graph_launch(tvolap_t* h);

/* Kernel timing. With enable != 0, every process_block / process_blocks call
 * records HIP events on the handle's stream around its kernels.
 * tvolap_get_timing waits for the recorded calls and returns the summed
 * milliseconds of the transform-in, spectral-MAC and transform-out phases and
 * the number of blocks they cover, then clears the sums. Phases that run fused
 * inside one kernel report their time under the MAC (for a batched call the
 * MAC phase is the one kernel that runs the MAC of all its blocks). */
int tvolap_set_timing(tvolap_t* h, int32_t enable);
int tvolap_get_timing(tvolap_t* h, double* ms_in, double* ms_mac, double* ms_out,
                      int64_t* n_blocks);

/* ------------------------------------------------------------------------
 * Offline, differentiable form. A whole signal per channel is processed at
 * once: channel c filters x[c][0 .. N) with its K partition-spectrum sets
 * H[c][s][m][k] (k = 0 .. 2L, complex float32 interleaved re/im, the paper's
 * H(k, m) of eq. 6) under schedule[b][c], the set active at block b (b = 0 ..
 * nblk-1 with nblk = ceil(N/L) + 1; block b is the paper's block l = b - 1,
 * covering samples [(b-1)L, (b+1)L)); NULL schedule = set 0 throughout. The
 * output y[c][0 .. N) is the time-variant convolution of Sec. 2 (equal to the
 * streaming output without its L-sample delay). Imaginary parts of H at
 * k = 0 and k = 2L do not enter (the inverse transform of eq. 9 is real).
 * All arrays are device memory; work is enqueued on `stream` (hipStream_t,
 * NULL = null stream) and the calls return without waiting. The caller
 * provides a device workspace of tvolap_offline_workspace_bytes() bytes,
 * which the call may overwrite; it is not used after the call's work ends.
 * Errors: EINVAL (shape, NULL pointer, small workspace), EDEVICE; the message
 * is in tvolap_offline_last_error(). */
typedef struct {
  int32_t hop;            /* L: 64, 128, 256 or 512                         */
  int32_t n_channels;     /* C, 1 .. 65535                                  */
  int32_t n_partitions;   /* M >= 1                                         */
  int32_t n_slots;        /* K >= 1                                         */
  int64_t n_samples;      /* N >= 1                                         */
} tvolap_offline_shape;

/* Workspace size in bytes, or -1 for an invalid shape. Both calls run the
 * signal in segments of up to 1024 hops, so the workspace grows with the
 * segment and not with N: the packed partition spectra (C K M 2L complex
 * values) plus, per channel, the spectra of 1024 + 2M + 2 blocks twice and
 * 1028 blocks of 4L samples (less for signals shorter than a segment). */
int64_t tvolap_offline_workspace_bytes(const tvolap_offline_shape* shape);

/* H[c][s][m][k] (k = 0 .. 2L) of taps[c][s][0 .. n_taps): partition m holds
 * taps [2Lm, 2Lm + 2L), zero padded to 4L and transformed (eq. 3, 6-7).
 * n_taps in [1, 2LM]. */
int tvolap_offline_ir_spectra(const tvolap_offline_shape* shape, const float* taps, int32_t n_taps, float* H,
                              void* stream);

/* y = TVOLAP(x, H, schedule) (eq. 1-13). */
int tvolap_offline_forward(const tvolap_offline_shape* shape, const float* x, const float* H,
                           const int32_t* schedule, float* y, void* workspace, int64_t workspace_bytes,
                           void* stream);

/* Adjoint of the forward map for a real loss with gradient gy = dLoss/dy
 * ([C][N]): dx[c][t] = dLoss/dx[c][t] and dH[c][s][m][k] = dLoss/dRe H +
 * i dLoss/dIm H (zero imaginary parts at k = 0 and 2L). Either output may be
 * NULL to skip it. The input spectra are recomputed from x, segment by
 * segment, with the 2(M - 1) blocks before each segment recomputed too; dH
 * is summed over the segments. */
int tvolap_offline_backward(const tvolap_offline_shape* shape, const float* x, const float* H,
                            const int32_t* schedule, const float* gy, float* dx, float* dH, void* workspace,
                            int64_t workspace_bytes, void* stream);

/* Working memory of tvolap_offline_forward_noalloc on each GPU (32 MiB). */
#define TVOLAP_NOALLOC_SCRATCH_BYTES (32LL << 20)

/* tvolap_offline_forward without a workspace and without any allocation, for
 * callers that cannot allocate device memory: code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc. The result equals
 * tvolap_offline_forward's bit for bit. Its working memory is one static
 * device array of TVOLAP_NOALLOC_SCRATCH_BYTES per GPU, placed by the loader
 * and held until the process ends; its address is looked up on the first
 * call on each device (`stream` must belong to the current device). The
 * signal is processed in segments of hops sized to that array; each segment
 * recomputes the input spectra of the 2(M - 1) blocks before it. Every call
 * on a GPU shares that GPU's array and overwrites it, so calls whose work
 * overlaps on one GPU (other streams, other host threads) race: order them on
 * one stream. Errors: EINVAL (as tvolap_offline_forward, or a shape whose
 * segments of one hop need more than C (2M + 8) 16L > the array's bytes),
 * EDEVICE. */
int tvolap_offline_forward_noalloc(const tvolap_offline_shape* shape, const float* x, const float* H,
                                   const int32_t* schedule, float* y, void* stream);

/* Message describing the last failed offline call of this thread. */
const char* tvolap_offline_last_error(void);

/* ------------------------------------------------------------------------
 * Non-uniform partitions (Sec. 1 names uniform and non-uniform partitioning;
 * Sec. 2's time-variant method applied to each part): a head of M1 short
 * partitions at hop L1 (latency 2 L1) covers taps [0, D), D = 2 L1 M1, and a
 * tail of long partitions at hop L2 = r L1 covers taps [D, max_taps), its
 * output joining D samples later. y(t) = y_head(t) + y_tail(t - D), each part
 * a TVOLAP output on its own block grid (switches fade over L1 in the head,
 * over L2 in the tail). Tail block l2 starts contributing where head block
 * r l2 + 2 M1 does and takes that block's selection; it is computed in the
 * same call, once every r calls, which needs M1 >= r - 1. With r = 1 the
 * result is uniform TVOLAP at hop L1. The stream is y delayed by L1. */
typedef struct tvolap_nup tvolap_nup_t;
typedef struct {
  tvolap_config base;        /* hop = L1; max_taps = N_IR; taps_of_channel must be
                                NULL and n_outputs 0; max_batch is not used        */
  int32_t tail_ratio;        /* r: power of two, r L1 in {64, 128, 256, 512}        */
  int32_t head_partitions;   /* M1 >= max(1, r - 1)                               */
} tvolap_nup_config;

/* Create: two TVOLAP handles (head and tail) on base.stream plus an input ring
 * and a tail output stage. Errors: EINVAL, ENOMEM, EDEVICE. */
int tvolap_nup_create(const tvolap_nup_config* cfg, tvolap_nup_t** out);
int tvolap_nup_destroy(tvolap_nup_t* h);
/* As tvolap_set_ir: taps [0, D) go to the head, taps [D, n_taps) to the tail. */
int tvolap_nup_set_ir(tvolap_nup_t* h, int32_t channel, int32_t slot, const float* taps, int32_t n_taps,
                      int32_t taps_on_device);
/* As tvolap_select_ir, for both parts. */
int tvolap_nup_select_ir(tvolap_nup_t* h, const int32_t* slot_of_channel);
/* One call of L1 new samples per input (as tvolap_process_block); every r
 * calls it also runs the tail's block. slot_of_channel_dev (device [C] or
 * NULL) is this call's selection; the tail takes the latest one. */
int tvolap_nup_process_block(tvolap_nup_t* h, const float* in, int64_t in_stride, float* out, int64_t out_stride,
                             const int32_t* slot_of_channel_dev);
int tvolap_nup_reset(tvolap_nup_t* h);
/* Autotune both parts (tvolap_autotune), then reset. */
int tvolap_nup_autotune(tvolap_nup_t* h, int32_t iters);
/* Graph capture of the shared stream. The calls are issued with host-side
 * positions in the input ring, so a graph must start at a call count that is
 * a multiple of the period P (tvolap_nup_period) and hold a multiple of P
 * calls; replays then continue the stream. */
int tvolap_nup_period(const tvolap_nup_t* h);
int tvolap_nup_capture_begin(tvolap_nup_t* h);
int tvolap_nup_capture_end(tvolap_nup_t* h);
int tvolap_nup_graph_launch(tvolap_nup_t* h);
const char* tvolap_nup_last_error(const tvolap_nup_t* h);

/* ------------------------------------------------------------------------
 * The comparison algorithms of Sec. 3, offline over whole signals (for the
 * switching and cost comparisons of Figs. 3-5 and Tables 1-2): block
 * convolution by overlap-add (OLA) and overlap-save (OLS) with block B =
 * N_IR, weighted overlap-add (WOLA, hop B/2) with an analysis and a synthesis
 * window, all with 2B-point transforms; and two or more direct time-domain
 * convolutions cross-faded at the output (CF-TDC). Channel c filters
 * x[c][0 .. N) with its K responses taps[c][s][0 .. n_taps); the response
 * active in block b is schedule[b][c] (values clamped into [0, K); NULL =
 * response 0 throughout). Block grids: OLA block b takes x[bB, (b+1)B) and adds
 * 2B output samples at bB; OLS block b transforms x[(b-1)B, (b+1)B) and keeps
 * the last B samples as y[bB, (b+1)B); WOLA block b (b = 0, 1, ...) weights
 * x[(b-1)R, (b-1)R + B) (R = B/2) with the analysis window and adds, weighted
 * by the synthesis window, its output at (b-1)R: a rectangular synthesis
 * keeps all 2B samples, a square-root Hann synthesis weights the first B and
 * drops the rest. Windows are periodic of length B: Hann (1 - cos(2 pi n/B))/2,
 * square-root Hann sin(pi n/B). y is aligned with x (no block delay). Device
 * arrays; work on `stream`, asynchronous. Errors: EINVAL, EDEVICE; message in
 * tvolap_cmp_last_error(). */
typedef enum { TVOLAP_CMP_OLA = 0, TVOLAP_CMP_OLS = 1, TVOLAP_CMP_WOLA = 2 } tvolap_cmp_method;
typedef enum { TVOLAP_WIN_RECT = 0, TVOLAP_WIN_HANN = 1, TVOLAP_WIN_SQRT_HANN = 2 } tvolap_window;
typedef struct {
  int32_t method;       /* tvolap_cmp_method                                   */
  int32_t block;        /* B = 128, 256, 512, 1024 or 2048                     */
  int32_t n_channels;   /* C, 1 .. 65535                                       */
  int32_t n_slots;      /* K >= 1 responses per channel                        */
  int64_t n_samples;    /* N >= 1                                              */
  int32_t n_taps;       /* response length, 1 .. B                             */
  int32_t analysis;     /* WOLA: TVOLAP_WIN_HANN or TVOLAP_WIN_SQRT_HANN         */
  int32_t synthesis;    /* WOLA: TVOLAP_WIN_RECT or TVOLAP_WIN_SQRT_HANN         */
} tvolap_cmp_shape;

/* Rows of the schedule (blocks of the method's grid), or -1 for a bad shape. */
int64_t tvolap_cmp_blocks(const tvolap_cmp_shape* shape);
/* Device workspace bytes of tvolap_cmp_forward, or -1 for a bad shape. */
int64_t tvolap_cmp_workspace_bytes(const tvolap_cmp_shape* shape);
/* y = method(x, taps, schedule). */
int tvolap_cmp_forward(const tvolap_cmp_shape* shape, const float* x, const float* taps, const int32_t* schedule,
                       float* y, void* workspace, int64_t workspace_bytes, void* stream);
/* CF-TDC: y(t) = sum_s c_s(t) (x * h_s)(t) with direct convolutions (FP32
 * sums) and c_s(t) = sum over blocks l = -1, 0, ... with schedule[l + 1][c] =
 * s of w(t - lL), w the Hann window of length 2L (amplitude 1/2): a Hann
 * cross-fade of L samples at every switch, on TVOLAP's block grid of hop L
 * (ceil(N/L) + 1 schedule rows). taps [C][K][n_taps]; any hop >= 1. */
int tvolap_cftdc_forward(int32_t hop, int32_t n_channels, int32_t n_slots, int64_t n_samples, int32_t n_taps,
                         const float* x, const float* taps, const int32_t* schedule, float* y, void* stream);
/* Message describing the last failed comparison call of this thread. */
const char* tvolap_cmp_last_error(void);

/* Message describing the last error of `h`, or of the last failed
 * tvolap_create when h is NULL. Never NULL. */
const char* tvolap_last_error(const tvolap_t* h);

/* Library version string. */
const char* tvolap_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TVOLAP_H */

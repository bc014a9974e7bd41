/*
 * filark.h - C ABI of the MI355X stateful chunked SOS + STA/LTA library.
 *
 * The operators follow the paper's stateful-compatible contract (FiLark,
 * Section 3.4 "Signal processing, pipelines, and algorithm integration"):
 * a call takes one chunk of a channel x time stream, returns an output of the
 * same length and carries the operator state to the next call, so that any
 * split of a record into chunks gives the output of a single call over the
 * whole record.  The first chunk after initialisation carries the start-up
 * transient set by the zero initial condition; later chunks carry none
 * (Section 6.2, "Signal processing performance").
 *
 * Data layout (every entry point): records are FP32, time-major
 * [n_t][n_ch] with row stride n_ch (channel contiguous), the 'nt_nc'
 * convention of the paper's binary tape (Section 3.5).
 *
 * Ownership: the caller owns every data buffer (device memory for signals,
 * host memory for coefficients and state snapshots).  The library owns its
 * state objects, their device state and scan tables, and frees them in the
 * matching *_destroy call.
 *
 * Errors: every call returns a filark_status; nothing aborts or throws across
 * the ABI.  filark_last_error() gives a thread-local message for the last
 * failure on the calling thread.  Argument errors are detected on the host
 * before anything is enqueued.
 *
 * Asynchrony: *_process calls only enqueue work on `stream` (a hipStream_t;
 * NULL is the null stream) and return; the caller synchronises before reading
 * outputs.  Calls that use one state object must be issued in order on one
 * stream: the state is a sequential dependency, updated in place on the
 * device by each call.  filark_state_get/_set and filark_check synchronise
 * `stream` themselves.  The process calls allocate nothing and may be
 * captured in a HIP graph; each replay advances the state like a call.
 */
#ifndef FILARK_H
#define FILARK_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum filark_status {
  FILARK_OK = 0,
  FILARK_EINVAL = 1,     /* bad argument (range, null pointer, aliasing) */
  FILARK_ESHAPE = 2,     /* n_ch differs from the one the state was made for */
  FILARK_ENOMEM = 3,     /* host or device allocation failed */
  FILARK_EHIP = 4,       /* a HIP runtime call failed (message has details) */
  FILARK_EUNSTABLE = 5,  /* a pole on or outside the unit circle */
  FILARK_ETIMEOUT = 6    /* reserved (no kernel of this version waits on another) */
} filark_status;

typedef enum filark_btype {
  FILARK_LOWPASS = 0,
  FILARK_HIGHPASS = 1,
  FILARK_BANDPASS = 2,
  FILARK_BANDSTOP = 3
} filark_btype;

/* State kinds for filark_state_get / _set / _save / _load / _bytes; the
 * tile calls also take the adjoint-kernel kinds. */
enum {
  FILARK_STATE_SOS = 0,
  FILARK_STATE_STALTA = 1,
  FILARK_TILE_SOS_ADJOINT = 2,
  FILARK_TILE_STALTA_ADJOINT = 3
};

/* Modes of filark_sos_stalta_adjoint. */
enum { FILARK_ADJ_GRAD = 0, FILARK_ADJ_MSE = 1 };

typedef struct filark_sos_state *filark_sos_t;
typedef struct filark_stalta_state *filark_stalta_t;
typedef struct filark_batch *filark_batch_t;
typedef struct filark_trigger_state *filark_trigger_t;
typedef struct filark_ema_state *filark_ema_t;
typedef struct filark_fir_state *filark_fir_t;

/* Modes of filark_ema_init. */
enum { FILARK_EMA_DEMEAN = 0, FILARK_EMA_AGC = 1 };

/*
 * Butterworth design by the bilinear transform with pre-warped band edges
 * (the paper's bandpass / lowpass / highpass wrappers of the real-time IIR,
 * Section 3.4; the design method is the textbook one, the paper gives none).
 *   order  total digital order; for FILARK_BANDPASS / FILARK_BANDSTOP it must
 *          be even (prototype order order/2).  1 <= order <= 64.
 *   btype  a filark_btype.  LP/HP use f1; BP/BS use f1 < f2.
 *   f1,f2  band edges in Hz, 0 < f < fs/2.   fs: sample rate in Hz.
 *   sos_out caller-owned host array of ceil(order/2) rows of 6 doubles
 *          {b0, b1, b2, 1, a1, a2}; sections run from the best-damped pole
 *          pair to the one closest to the unit circle; the overall gain sits
 *          in section 1's numerator.
 *   n_sec  receives ceil(order/2).
 * Host only, synchronous.  FILARK_EINVAL on a bad argument,
 * FILARK_EUNSTABLE if a designed pole has |p| >= 1 (numerically).
 */
filark_status filark_sos_design(int order, int btype, double f1, double f2, double fs,
                                double *sos_out, int *n_sec);

/*
 * Create a stateful SOS cascade for n_ch channels (Section 3.4, Table 1
 * "IIR (offline & realtime SOS)", stateful and GPU columns).
 *   sos    host array [n_sec][6] {b0 b1 b2 a0 a1 a2}; rows are normalised by
 *          a0 (which must be nonzero).  1 <= n_sec <= 8.  Copied.
 *   n_ch   channels, >= 1.
 *   flags  0 (reserved).
 * Allocates and zeroes the device state (zero initial condition) and uploads
 * the FP64 scan tables.  Runs on the current HIP device; `stream` orders the
 * upload.  FILARK_EUNSTABLE if a section has a pole with |p| >= 1.
 */
filark_status filark_sos_init(filark_sos_t *st, const double *sos, int n_sec, int64_t n_ch,
                              unsigned flags, hipStream_t stream);

/*
 * Filter one chunk: out = SOS(in) with the state carried in and out
 * (process(chunk, state) -> (output, new_state), Section 3.4).
 *   in, out  device FP32 [n_t][n_ch]; out == in is allowed (in place).
 *   n_ch     must equal the n_ch given to filark_sos_init (else FILARK_ESHAPE).
 *   n_t      samples in this chunk, n_t >= 0; 0 is a no-op.  Chunks whose
 *            padded byte size exceeds 2^31 run as several launches.
 * Asynchronous on `stream`.
 */
filark_status filark_sos_process(filark_sos_t st, const float *in, float *out, int64_t n_ch,
                                 int64_t n_t, hipStream_t stream);

/*
 * Create a recursive STA/LTA characteristic-function state for n_ch channels
 * (energy-detector monitor, Section 3.4).  nsta = round(sta_s * fs),
 * nlta = round(lta_s * fs), both >= 1.  With e = y^2:
 *   sta <- (1 - 1/nsta) sta + e / nsta,   lta <- (1 - 1/nlta) lta + e / nlta,
 *   cf = sta / lta once the global sample index reaches nlta and lta > 0,
 *   else 0.  The state (sta, lta, sample counter) starts at zero.
 */
filark_status filark_stalta_init(filark_stalta_t *st, double sta_s, double lta_s, double fs,
                                 int64_t n_ch, hipStream_t stream);

/*
 * Zero-phase (forward-backward) SOS filtering of a window: the "zero-phase"
 * option of the display filter of Section 3.2 (a non-causal filter of a whole
 * window, not a stream).  The cascade runs forward over in[0 .. n_t) from
 * rest, then backward in time over that output from rest, so the magnitude
 * response is |H|^2 and the phase is zero; no edge padding is added.  Uses
 * the coefficients and tile of `st` (which must have 48-sample blocks, the
 * default); its carried state is neither read nor changed.  in / out: device FP32 [n_t][n_ch] (in == out allowed); n_ch must
 * equal the state's and be below 2^23.  Asynchronous on `stream`.  The
 * passes' own filter state [2K][n_ch] FP64 is a workspace of `st`, allocated
 * on the first call (and grown on a larger one), then cleared by a kernel.
 */
filark_status filark_sos_filtfilt(filark_sos_t st, const float *in, float *out, int64_t n_ch, int64_t n_t,
                                  hipStream_t stream);

/*
 * filark_sos_filtfilt without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and kernels;
 * the passes' filter state lives in a fixed 1 MiB array that each GPU holds
 * for the life of the process, so 2 * n_sec * n_ch must not exceed 131072
 * (FILARK_EINVAL otherwise, before anything is enqueued).  Every call on one
 * GPU uses the same array: calls that overlap on a GPU (other streams, other
 * threads) race.
 */
filark_status filark_sos_filtfilt_noalloc(filark_sos_t st, const float *in, float *out, int64_t n_ch, int64_t n_t,
                                          hipStream_t stream);

/*
 * STA/LTA of one chunk of an already filtered signal.
 *   in  device FP32 [n_t][n_ch];  cf  device FP32 [n_t][n_ch] (may equal in).
 * Asynchronous on `stream`.
 */
filark_status filark_stalta_process(filark_stalta_t st, const float *in, float *cf, int64_t n_ch,
                                    int64_t n_t, hipStream_t stream);

/*
 * Fused chunk: y = SOS(in), cf = STA/LTA(y), both states carried.  Equivalent
 * to filark_sos_process followed by filark_stalta_process on its output, in
 * one pass over HBM.
 *   y_or_null  device FP32 [n_t][n_ch] or NULL (then y is not written);
 *              may equal in.
 *   cf         device FP32 [n_t][n_ch]; must differ from y_or_null.
 * Both states must be for n_ch channels.  Asynchronous on `stream`.
 */
filark_status filark_sos_stalta_process(filark_sos_t sos, filark_stalta_t sl, const float *in,
                                        float *y_or_null, float *cf, int64_t n_ch, int64_t n_t,
                                        hipStream_t stream);

/*
 * Snapshot / restore a state in a canonical FP64 host layout, independent of
 * the device realisation:
 *   FILARK_STATE_SOS:    [n_ch][n_sec][2] doubles, the direct-form-II-
 *                        transposed delay pair (z1, z2) of each section;
 *                        bytes = n_ch * n_sec * 16.
 *   FILARK_STATE_STALTA: [n_ch][2] doubles (sta, lta) followed by one
 *                        int64 global sample counter; bytes = n_ch * 16 + 8.
 * `st` is a filark_sos_t or filark_stalta_t matching `kind`.  Both calls
 * synchronise `stream` (the state is read or written after all work already
 * enqueued on it).  FILARK_EINVAL if bytes does not match.
 */
filark_status filark_state_get(const void *st, int kind, void *host_buf, size_t bytes,
                               hipStream_t stream);
filark_status filark_state_set(void *st, int kind, const void *host_buf, size_t bytes,
                               hipStream_t stream);

/*
 * Tile shape of a state object's kernels (a tuning knob; results do not
 * depend on it beyond FP64 rounding of the carries).  A workgroup of `waves`
 * waves owns `group` consecutive channels and covers a window of
 * waves * 64 / group blocks of `block` samples per lane; longer chunks run
 * window by window.
 *   kind FILARK_STATE_SOS / _STALTA (forward): block 32, 48 or 64, default 48 x 8 x 16;
 *   kind FILARK_TILE_SOS_ADJOINT / _STALTA_ADJOINT: block 8 or 16, default 16 x 4 x 8;
 *   waves 1 .. 8;  group 4, 8, 16, 32 or 64.
 * The SOS and STA/LTA states used together must have equal shapes.  _set
 * synchronises `stream` and rebuilds the scan tables.  FILARK_EINVAL for a
 * shape outside the ranges above.
 */
filark_status filark_tile_set(void *st, int kind, int block, int waves, int group, hipStream_t stream);
filark_status filark_tile_get(const void *st, int kind, int *block, int *waves, int *group);

/*
 * Most adjoint windows that one launch of the adjoint kernel takes (0, the
 * default: no limit; 1: one launch per window).  With the default adjoint
 * tile and a cascade of 2 to 4 sections whose sections after the first
 * have numerators [1, +-2, 1] and |a2| >= 1/4 (every even-order Butterworth
 * design), all windows of a chunk run in one launch, a partial last window
 * first: each workgroup keeps its channels from window to window,
 * hands the adjoint state on through LDS and loads the next window's input
 * while the current one runs.  Other cascades take one launch per window.  Results are bit-identical
 * for every value (the windows' arithmetic and its order do not change); the
 * limit exists to measure and test that.  Takes effect at the next adjoint
 * call.  FILARK_EINVAL for a null state or a negative value.
 */
filark_status filark_adjoint_windows_set(filark_sos_t sos, int max_windows);

/*
 * Tile autotuner: times the forward kernel of a scratch state with the same
 * filter and channel count as `st` on a chunk of n_t rows of synthetic input
 * (allocated and freed by the call) for each candidate tile, with HIP events
 * on `stream`, takes the fastest and applies it to `st` (filark_tile_set).
 *   block   0: search 32, 48 and 64; else keep this block (32, 48 or 64).
 *   waves   0: search 2, 4 and 8 waves per workgroup; else keep this value.
 *   groups  always searched: 4, 8, 16, 32 and 64 channels (those whose
 *           window and LDS fit).
 *   cache   a JSON file (or NULL): an entry for this shape (channels, rows,
 *           sections, block and waves constraints) is applied without
 *           measuring; a new measurement is added to the file.
 * out_*: the tile chosen.  Synchronous.  Errors: FILARK_EINVAL (arguments,
 * no candidate fits, cache not writable), FILARK_EHIP.
 */
filark_status filark_autotune(filark_sos_t st, int64_t n_t, int block, int waves, const char *cache,
                              int *out_block, int *out_waves, int *out_group, hipStream_t stream);

/*
 * Device-side checkpoints of a state (for the adjoint of a chunked run):
 * _bytes gives the size of the opaque device image, _save copies the state
 * into `dev_dst` and _load restores it from `dev_src` (device buffers of that
 * size owned by the caller).  Both are asynchronous copies on `stream`.
 */
filark_status filark_state_bytes(const void *st, int kind, size_t *bytes);
filark_status filark_state_save(const void *st, int kind, void *dev_dst, hipStream_t stream);
filark_status filark_state_load(void *st, int kind, const void *dev_src, hipStream_t stream);

/*
 * Reverse-mode gradient of a loss on the fused path's characteristic
 * function over one chunk (the adjoint of filark_sos_stalta_process: the
 * time-reversed, transposed recurrences of the STA/LTA and of the cascade).
 * The paper gives no gradient; this is the derivative of the forward
 * operation defined above.
 *   sos, sl   hold the forward state at the START of the chunk (restore the
 *             chunk's checkpoint first); they are not modified.
 *   x         device FP32 [n_t][n_ch], the chunk's input.
 *   g         mode FILARK_ADJ_GRAD: dL/dcf [n_t][n_ch];
 *             mode FILARK_ADJ_MSE:  the target cf, with
 *             L = scale * sum (cf - target)^2 over the chunk.
 *   gx        device FP32 [n_t][n_ch], receives dL/dx.
 *   adj       device FP64 [2K + 2][n_ch]: the adjoint of the state after the
 *             chunk on entry (zero after a record's last chunk), the adjoint
 *             of the state before it on return; rows are (dL/dz1, dL/dz2) of
 *             each section, then dL/dsta, dL/dlta.
 *   gsos      device FP64 [K][5], dL/d(b0, b1, b2, a1, a2) of each section,
 *             ADDED to (coefficients normalised by a0).
 * Chunks of a record are processed last to first with their checkpoints,
 * carrying adj.  Results are deterministic.  Asynchronous on `stream`; may
 * allocate its workspace (window checkpoints) on first use.
 */
filark_status filark_sos_stalta_adjoint(filark_sos_t sos, filark_stalta_t sl, const float *x,
                                        const float *g, int mode, double scale, float *gx, double *adj,
                                        double *gsos, int64_t n_ch, int64_t n_t, hipStream_t stream);

/*
 * The adjoint with a tape: the forward call records what the adjoint needs,
 * so the adjoint runs no forward pass of its own and reads no object state.
 *   _tape_bytes  size of the tape of one chunk of n_t rows: the forward
 *                state at the start of every adjoint window of the chunk
 *                (windows of the adjoint tile's rows, 512 by default), each
 *                slot the filter state [2K][n_ch], (sta, lta) [2][n_ch] and
 *                the sample counter [n_ch] (FP64 / int64).  Fails with
 *                FILARK_EINVAL when the adjoint window is not a multiple of
 *                64 rows that divides 2048 (the default adjoint tile is).
 *   _process_tape  filark_sos_stalta_process (cf required, y optional), run
 *                with 64-row blocks, that also writes the chunk's tape into
 *                `tape` (device, caller-owned, `tape_bytes` long: at least
 *                _tape_bytes for this n_t, else FILARK_EINVAL).  The objects' state advances as in the plain call; cf
 *                and the state agree with it to rounding (a different block
 *                length sums in a different order).  Asynchronous on `stream`.
 *   _adjoint_tape  filark_sos_stalta_adjoint over the same chunk from its
 *                tape (arguments as there); the objects only supply the
 *                filter, the windows and the tiles, and their state is
 *                neither read nor written, so no checkpoint needs restoring.
 *                The adjoint tile must be the one the tape was written with
 *                (a tape shorter than the current tile needs is refused).
 * Errors: FILARK_EINVAL, FILARK_ESHAPE, FILARK_EHIP.
 */
filark_status filark_adjoint_tape_bytes(filark_sos_t sos, filark_stalta_t sl, int64_t n_t, size_t *bytes);
filark_status filark_sos_stalta_process_tape(filark_sos_t sos, filark_stalta_t sl, const float *x, float *y,
                                             float *cf, void *tape, size_t tape_bytes, int64_t n_ch, int64_t n_t,
                                             hipStream_t stream);
filark_status filark_sos_stalta_adjoint_tape(filark_sos_t sos, filark_stalta_t sl, const void *tape,
                                             size_t tape_bytes, const float *x, const float *g, int mode,
                                             double scale, float *gx, double *adj, double *gsos, int64_t n_ch,
                                             int64_t n_t, hipStream_t stream);

/*
 * Batched filtering of many independent streams in one launch (the stateful
 * SOS operator of Section 3.4 applied to several records at once; streams
 * may differ in channel count, chunk length and filter).
 *   _create  takes n SOS state objects (one per stream; each keeps its own
 *            state and tables).  All must have 48-sample blocks and the same
 *            waves per workgroup; the channel group may differ per stream
 *            (per-stream tuning, e.g. with filark_autotune).
 *   _bind    records one chunk per stream: in[s], out[s] device FP32
 *            [n_t[s]][n_ch of state s] (host arrays of device pointers;
 *            n_t[s] = 0 skips the stream), builds the work table and uploads
 *            it (synchronous).  An item of work is one channel group of one
 *            stream over every window of its chunk, walked in order by one
 *            workgroup that carries the state from window to window; the
 *            items sit in one queue per XCD (the groups of a stream in
 *            contiguous slabs), longest first.  Rebind when pointers or
 *            lengths change, and after filark_tile_set on any of the states
 *            (a launch after such a change fails with FILARK_EINVAL; bind
 *            refuses a state whose block or waves differ from the batch's).
 *            A bind drops the graph held by _capture.
 *   _launch  enqueues the bound work on `stream`: one persistent kernel
 *            whose workgroups (as many as stay resident, at most the longest
 *            queue) take items until their XCD's queue is empty, the last
 *            one to leave clearing the queue counters for the next launch
 *            (a launch that did not complete leaves the batch unusable:
 *            destroy it); or, after
 *            _capture, one launch of the captured graph.  It allocates
 *            nothing and does not synchronise; every launch advances each
 *            stream's state by its chunk, exactly like filark_sos_process
 *            (bit for bit: the same kernel body and tile).  Launches of one
 *            batch must not overlap (they share the counters and stamps).
 *   _capture captures the launch sequence in a HIP graph owned by the batch
 *            (on a stream of its own; synchronous); later _launch calls
 *            replay it.  Callers that capture _launch into graphs of their
 *            own must capture again after a bind.
 *   _stamps  synchronises `stream` and copies n + 1 uint64 values: the
 *            completion time of each stream's last item and, last, the time
 *            the launch started (its first item was taken), in ticks of the
 *            device's 100 MHz clock; of the last completed launch.
 * SOS only (no STA/LTA).  Errors as elsewhere; FILARK_EINVAL if a stream's
 * tile does not fit the device or the state objects disagree.
 */
filark_status filark_batch_create(filark_batch_t *b, int n, const filark_sos_t *states, hipStream_t stream);
filark_status filark_batch_bind(filark_batch_t b, const float *const *in, float *const *out,
                                const int64_t *n_t, hipStream_t stream);
filark_status filark_batch_launch(filark_batch_t b, hipStream_t stream);
filark_status filark_batch_capture(filark_batch_t b);
filark_status filark_batch_stamps(filark_batch_t b, uint64_t *host, hipStream_t stream);
filark_status filark_batch_destroy(filark_batch_t b);

/*
 * Stateful exponential-average operators (Table 1's running mean and running
 * AGC rows; stateful operators of Section 3.4).  Per channel, with
 * n_win = round(win_s * fs) and c = 1 / n_win:
 *   FILARK_EMA_DEMEAN  m = (1 - c) m + c x;    y = x - m   (running-mean removal)
 *   FILARK_EMA_AGC     p = (1 - c) p + c x^2;  y = x / sqrt(p), 0 where p is 0
 *                      (or below FP32's normal range)
 * The average is carried from call to call (0 at creation), so any chunking
 * gives the one-shot result.
 *   _init     mode, window (s) and rate (Hz) positive, n_ch in [1, 2^24].
 *   _process  in / out: device FP32 [n_t][n_ch] (in == out allowed);
 *             asynchronous on `stream`; n_t = 0 is a no-op.
 *   _state_get / _set  the averages, host FP64 [n_ch].  Synchronous.
 * Errors: FILARK_EINVAL, FILARK_ESHAPE (n_ch mismatch), FILARK_EHIP.
 */
filark_status filark_ema_init(filark_ema_t *st, int mode, double win_s, double fs, int64_t n_ch, hipStream_t stream);
filark_status filark_ema_process(filark_ema_t st, const float *in, float *out, int64_t n_ch, int64_t n_t,
                                 hipStream_t stream);
filark_status filark_ema_state_get(filark_ema_t st, double *avg, hipStream_t stream);
filark_status filark_ema_state_set(filark_ema_t st, const double *avg, hipStream_t stream);
filark_status filark_ema_destroy(filark_ema_t st);

/*
 * Realtime FIR with carried history (Table 1's FIR row; a stateful operator
 * of Section 3.4).  Per channel
 *   y[t] = sum_{k < n_taps} h[k] x[t - k],
 * where the n_taps - 1 samples before a chunk are the previous chunks' last
 * samples (0 at creation), so that any chunking gives the one-shot result;
 * on the GPU the two agree bit for bit (every output takes its taps in
 * ascending order in FP32 FMAs).
 *   _init      taps: host FP64 [n_taps], finite, applied as FP32;
 *              1 <= n_taps <= 1024; n_ch in [1, 2^24], and small enough
 *              that 2 Mp + 81 + 96 w rows of n_ch floats stay below 2 GiB
 *              (Mp: n_taps rounded up to 32; w: waves per workgroup, 1 by
 *              default; checked at _init and _set_tile).
 *   _set_tile  output rows per wave (0: 48 for launch windows of 8192 rows
 *              or more with at most 64 taps, else 32; or 16, 32, 48), waves
 *              per workgroup (1..8)
 *              and workgroup order (0: each XCD walks along time within its
 *              channel groups; 1: each XCD walks its rows across all channel
 *              groups first; 2: each XCD owns an eighth of the channel groups
 *              and sweeps its rows across them); default 0 x 1, order 2.
 *              Any tile gives the same bits.
 *   _process   in / out: device FP32 [n_t][n_ch], time-major; they must not
 *              overlap (neighbouring outputs read the same inputs).
 *              Asynchronous on `stream`; n_t = 0 is a no-op.  Successive
 *              calls must be ordered (one stream, or synchronised), since
 *              each reads the history the previous one wrote.  Which of the
 *              state's two history buffers is current lives on the device,
 *              so a call captured in a HIP graph carries the history from
 *              replay to replay like an eager call.
 *   _state_get / _set  the history, host FP32 [n_taps - 1][n_ch], oldest row
 *              first (nothing when n_taps = 1).  Synchronous.
 * Errors: FILARK_EINVAL (arguments, overlap), FILARK_ESHAPE (n_ch mismatch),
 * FILARK_EHIP.
 */
filark_status filark_fir_init(filark_fir_t *st, const double *taps, int n_taps, int64_t n_ch, hipStream_t stream);
/*
 * Method of a FIR object: FILARK_FIR_DIRECT (the default: direct form, FP32
 * FMAs in ascending tap order, chunked == one-shot bit for bit) or
 * FILARK_FIR_FFT (FFT filtering, Table 1's overlap-add row: blocks of
 * 2049 - n_taps output rows, each the last rows of a 2048-row window's
 * circular convolution with the zero-padded taps (overlap-save, which sums
 * the same products as overlap-add and carries the same input history as the
 * direct form), in FP32 radix-4 transforms of two channels' real samples
 * packed as one complex sequence, 8 channels per workgroup; its error is
 * that of FP32 transforms, O(2^-24 log2 2048 |h| |x|), not bit-reproducible
 * across chunkings).  Both methods keep the same state (the last n_taps - 1
 * input rows), so a stream may switch between calls.  Selecting FFT builds
 * its tables (taps' spectrum in FP64, rounded; synchronous).  Calls with
 * more than 65535 blocks are refused.
 */
#define FILARK_FIR_DIRECT 0
#define FILARK_FIR_FFT 1
filark_status filark_fir_set_method(filark_fir_t st, int method, hipStream_t stream);
filark_status filark_fir_set_tile(filark_fir_t st, int rows, int waves, int order);
filark_status filark_fir_process(filark_fir_t st, const float *in, float *out, int64_t n_ch, int64_t n_t,
                                 hipStream_t stream);
filark_status filark_fir_state_get(filark_fir_t st, float *hist, hipStream_t stream);
filark_status filark_fir_state_set(filark_fir_t st, const float *hist, hipStream_t stream);
filark_status filark_fir_destroy(filark_fir_t st);

/*
 * Two-threshold trigger on a characteristic function: the monitor of
 * Section 3.4 (a window of data in, a list of time-channel events out) as the
 * hysteresis of an energy detector.  Per channel, while closed, the first
 * sample whose cf exceeds `on` opens an event; while open, the first later
 * sample whose cf is below `off` closes it, and the event [t_on, t_off) is
 * emitted.  Comparisons in FP32; NaN neither opens nor closes.  An event open
 * at the end of a call stays in the state (open flag and t_on), so any
 * chunking emits the events of the one-shot run.  Sample indices are global
 * (counted from the state's creation).
 *   _init     thresholds (finite, off <= on), n_ch in [1, 2^24]; all channels
 *             closed, counter 0.
 *   _process  cf: device FP32 [n_t][n_ch] (e.g. the cf of
 *             filark_sos_stalta_process); events: device int64 [cap][3]
 *             (channel, t_on, t_off); count: device uint64, which the call
 *             advances by the number of events that close in this chunk;
 *             event i of the call is stored at position *count + i if that
 *             is below cap (so a zeroed count collects several calls one
 *             after another; events past cap are counted, not stored).  The
 *             order of the events within a call is not specified.
 *             Asynchronous on `stream`; n_t = 0 is a no-op.
 *   _state_get / _set  canonical host form: open_ton [n_ch][2] int64 =
 *             (open flag 0/1, start of the open event or 0), and the global
 *             sample counter.  Synchronous.
 * Errors: FILARK_EINVAL (arguments), FILARK_ESHAPE (n_ch mismatch),
 * FILARK_EHIP.
 */
filark_status filark_trigger_init(filark_trigger_t *st, float on, float off, int64_t n_ch, hipStream_t stream);
filark_status filark_trigger_process(filark_trigger_t st, const float *cf, int64_t n_ch, int64_t n_t,
                                     int64_t *events, int64_t cap, uint64_t *count, hipStream_t stream);
filark_status filark_trigger_state_get(filark_trigger_t st, int64_t *open_ton, int64_t *counter,
                                       hipStream_t stream);
filark_status filark_trigger_state_set(filark_trigger_t st, const int64_t *open_ton, int64_t counter,
                                       hipStream_t stream);
filark_status filark_trigger_destroy(filark_trigger_t st);

/*
 * The monitor chain in one pass over a chunk (the energy-detector monitor of
 * Section 3.4): SOS cascade, STA/LTA characteristic and two-threshold
 * trigger, each with its carried state.  The same outputs, states and events
 * as filark_sos_stalta_process followed by filark_trigger_process on its cf
 * (events as a set: their order in the list depends on timing in either
 * case), without cf going through memory unless asked for.
 *   in          device FP32 [n_t][n_ch].
 *   y_or_null   device FP32 [n_t][n_ch] or NULL (not written).
 *   cf_or_null  device FP32 [n_t][n_ch] or NULL (not written).
 *   events, cap, count  as filark_trigger_process.
 * The states' forward tile must have 48-row blocks (the default).
 * Asynchronous on `stream`.  Errors: FILARK_EINVAL, FILARK_ESHAPE,
 * FILARK_EHIP.
 */
filark_status filark_monitor_process(filark_sos_t sos, filark_stalta_t sl, filark_trigger_t tr, const float *in,
                                     float *y_or_null, float *cf_or_null, int64_t *events, int64_t cap,
                                     uint64_t *count, int64_t n_ch, int64_t n_t, hipStream_t stream);

/*
 * Synchronise `stream` and report an asynchronous HIP error of the work
 * enqueued on it (FILARK_EHIP).  kind as above.
 */
filark_status filark_check(const void *st, int kind, hipStream_t stream);

/* Free a state object and its device memory (NULL is a no-op). */
filark_status filark_sos_destroy(filark_sos_t st);
filark_status filark_stalta_destroy(filark_stalta_t st);

/* Thread-local message describing the last failure on this thread ("" if none). */
const char *filark_last_error(void);

/* Library version string. */
const char *filark_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FILARK_H */

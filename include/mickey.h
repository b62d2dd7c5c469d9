/*
 * mickey.h - C ABI of libmickey.so: bitsliced MICKEY 2.0 keystream generation on
 * AMD Instinct MI355X (gfx950).
 *
 * The operation (paper Sec. II-C-1 and Sec. IV-D): n independent MICKEY 2.0 generator
 * instances, each with its own 80-bit key and an IV of 0..80 bits, are packed one per
 * bit lane of 32-bit words; the two 100-bit registers R and S become 200 words per
 * group of 32 instances, and every clock advances all lanes at once.  Bitslicing only
 * changes the layout: instance i produces exactly the keystream of the MICKEY 2.0
 * definition (the cipher specification the paper cites), bit for bit.
 *
 * Conventions
 *   - Bits of keys and IVs are read MSB first: key bit j is bit (7 - j%8) of byte j/8.
 *   - z_t is keystream bit t of an instance (t = 0 is the first bit after the 100
 *     preclocks of the initialisation).
 *   - n is padded internally to n_pad = 64*ceil(n/64) instances; pad instances run with
 *     an all-zero key and an all-zero 80-bit IV.
 *
 * Output layouts (mickey_generate):
 *   MICKEY_BITSLICED    plane-major bit-planes.  Plane t (t = 0..nbits-1) holds z_t of
 *                       every instance as an LSB-first bit vector of n_pad bits:
 *                       instance i is bit (i % 8) of byte (t*pitch + i/8), where
 *                       pitch = mickey_plane_pitch(n) = n_pad/8 bytes.  The buffer is
 *                       nbits*pitch bytes.  Bits of pad instances hold their (zero
 *                       key) keystream and are not part of the result.
 *   MICKEY_ROWMAJOR_U32 instance-major 32-bit words: word j of instance i is
 *                       out[i*(nbits/32) + j], and bit (31 - b) of it is z_{32j+b}.
 *                       Needs nbits % 32 == 0.  Buffer: n*nbits/8 bytes.
 *   MICKEY_ROWMAJOR_F32 the same words w as floats (w >> 8) * 2^-24, exact, in
 *                       [0, 1 - 2^-24].  Needs nbits % 32 == 0.  Buffer: n*nbits/8 bytes.
 *
 * Ownership and ordering
 *   - The library owns a mickey_state and the device memory behind it.  The caller
 *     owns every key, IV, length and output buffer; inputs may be reused as soon as the
 *     call that reads them has completed on its stream.
 *   - All device pointers are HIP device (or managed) pointers on the current device.
 *   - Work is enqueued on the state's stream (the HIP null stream unless set) and is
 *     asynchronous unless stated; results are valid after that stream synchronises.
 *   - Calls on one state are not thread-safe.  Different states are independent.
 *
 * Errors: functions return MICKEY_OK (0) or a negative code; mickey_init returns NULL
 * on error.  mickey_last_error() gives the calling thread's last code and
 * mickey_last_error_message() a description.  A call on a state that fails leaves its
 * registers and bit counters as they were (a call made of several launches that change
 * the registers first copies them and copies them back if a later launch fails); the
 * contents of its output buffers are then unspecified.  If even that copy cannot be
 * enqueued, or mickey_sync() reports a device failure, the state is poisoned: every
 * later call on it returns MICKEY_EDEVICE, except mickey_free, the queries, a re-key or
 * an import (which replace all registers), and export, which then gives the registers
 * saved before the call that failed when they exist.
 */
#ifndef MICKEY_H
#define MICKEY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MICKEY_OK 0
#define MICKEY_EINVAL (-1)  /* bad argument: NULL pointer, n == 0, IV length > 80, layout */
#define MICKEY_ENOMEM (-2)  /* device allocation failed */
#define MICKEY_EDEVICE (-3) /* a HIP call or kernel launch failed, or the state is poisoned */
#define MICKEY_ERANGE (-4)  /* more than 2^40 keystream bits for one key/IV pair (Sec. II-C-1) */
#define MICKEY_ENOSYS (-5)  /* unsupported combination (e.g. word width) */

#define MICKEY_BITSLICED 0
#define MICKEY_ROWMAJOR_U32 1
#define MICKEY_ROWMAJOR_F32 2

/* Keystream bits allowed per key/IV pair (paper Sec. II-C-1: up to 2^40). */
#define MICKEY_MAX_BITS_PER_IV ((uint64_t)1 << 40)

typedef struct mickey_state mickey_state;

/* Load n instances and run the initialisation of every one: registers cleared, then the
 * IV bits, the 80 key bits and 100 zero bits clocked in with mixing on (the cipher's
 * key/IV loading and preclock procedure; paper Sec. IV-D, bitsliced input handler).
 *   keys    device, n*10 bytes, key of instance i at keys + 10*i
 *   ivs     device, n*10 bytes, IV of instance i at ivs + 10*i (bits past its length
 *           are ignored)
 *   iv_bits device, n bytes, IV length of instance i in 0..80; NULL means 80 for all.
 *           When non-NULL the lengths are validated, which synchronises the stream.
 * Runs on the HIP null stream.  Returns NULL on error (see mickey_last_error). */
mickey_state *mickey_init(const uint8_t *keys, const uint8_t *ivs, const uint8_t *iv_bits, size_t n);

/* As mickey_init, on the given HIP stream (hipStream_t passed as void*), which becomes
 * the state's stream. */
mickey_state *mickey_init_on_stream(const uint8_t *keys, const uint8_t *ivs, const uint8_t *iv_bits,
                                    size_t n, void *hip_stream);

/* Re-run the initialisation of every instance of an existing state with new keys, IVs
 * and IV lengths (same n, same arguments as mickey_init), reusing its device memory; the
 * bit counter restarts at 0.  Asynchronous unless iv_bits is non-NULL. */
int mickey_rekey(mickey_state *st, const uint8_t *keys, const uint8_t *ivs, const uint8_t *iv_bits);

/* Advance every instance by nbits clocks and write the nbits keystream bits each one
 * produced (bit z = r_0 xor s_0 of the state before each clock; paper Sec. IV-D: one
 * word per 32 instances per clock) to `out` in `layout` (see above).  nbits >= 1; for
 * the row-major layouts nbits % 32 == 0.  out: device, size as given by the layout.
 * The next call continues with the following bit.  MICKEY_ERANGE if any instance would
 * pass 2^40 bits in total. */
int mickey_generate(mickey_state *st, uint64_t nbits, void *out, int layout);

/* Row-major delivery of both forms in one pass: out_u32 and/or out_f32 (either may be
 * NULL, not both), each n*nbits/8 bytes on the device, layouts as MICKEY_ROWMAJOR_U32
 * and MICKEY_ROWMAJOR_F32.  nbits % 32 == 0. */
int mickey_generate_rowmajor(mickey_state *st, uint64_t nbits, uint32_t *out_u32, float *out_f32);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
 * loops or harnesses that forbid hipMalloc): mickey_generate_rowmajor with the same
 * arguments, results and errors, that allocates nothing.  The staged transposition's
 * register snapshot and bit-plane chunks live in a library-owned static device array of
 * 256 MiB, which every device that runs the library holds until the process ends; chunks
 * are as many clocks as fit beside the snapshot (at most 8192), and everything runs on the
 * state's stream.  States of more than ~8.1 million instances (200 + 64 planes exceeding
 * the array) get MICKEY_EINVAL.  All calls on one device share the array: calls that
 * overlap on a device (different streams or host threads) race and must be serialised by
 * the caller. */
int mickey_generate_rowmajor_noalloc(mickey_state *st, uint64_t nbits, uint32_t *out_u32, float *out_f32);

/* Per-instance requests (the paper's problem statement, Sec. IV-D: independent instances,
 * each with its own key and IV).  Request k resumes instance reqs[k].instance of `st` for
 * reqs[k].nbits keystream bits (a multiple of 32; 0 is allowed and does nothing) and writes
 * them to reqs[k].out (device, nbits/8 bytes) in reqs[k].layout, which is
 * MICKEY_ROWMAJOR_U32 (bit 31-b of word j is z_{32j+b} of that instance's stream from where
 * it stood) or MICKEY_ROWMAJOR_F32 (the same words as exact floats (w >> 8) * 2^-24).
 * Requests on the same instance are applied in array order: each continues at the bit
 * after the previous one.  Other instances do not move.  Every request is validated
 * before any work is enqueued (MICKEY_EINVAL for an instance >= n, another layout, a
 * length not a multiple of 32 or a NULL output; MICKEY_ERANGE when an instance would pass
 * 2^40 bits in total or 2^37 bits in this call).  Long per-instance streams run in latency
 * mode (four lanes per instance), the rest bitsliced; the output bytes do not depend on
 * that.  Asynchronous on the state's stream; the library's device scratch and a pinned
 * host staging buffer grow on demand and are kept until mickey_free.  reqs (host) may be
 * reused when the call returns. */
typedef struct mickey_req {
    uint64_t instance; /* 0 .. n-1 */
    uint64_t nbits;    /* keystream bits, a multiple of 32 */
    void *out;         /* device, nbits/8 bytes */
    int layout;        /* MICKEY_ROWMAJOR_U32 or MICKEY_ROWMAJOR_F32 */
} mickey_req;
int mickey_generate_batch(mickey_state *st, const mickey_req *reqs, size_t nreq);

/* Release the state (synchronises its streams first).  NULL is allowed. */
void mickey_free(mickey_state *st);

/* Bind the state to a HIP stream (void* hipStream_t; NULL = null stream). */
int mickey_set_stream(mickey_state *st, void *hip_stream);

/* Slicing word width of the generate kernels: 32 (default; 32 instances per lane) or
 * 64 (64 instances per lane, each state bit in a 64-bit word).  The output bytes do
 * not depend on it. */
int mickey_set_word_bits(mickey_state *st, int word_bits);

/* Work split of the generate kernels (the output bytes do not depend on it):
 *   MICKEY_SCHED_ONE_WAVE  one lane keeps all 200 state words of its slice(s);
 *   MICKEY_SCHED_SPLIT     two waves per 64 slices, one keeping the R words and one the
 *                          S words; every clock they exchange the bits that cross
 *                          between the registers (r_33, s_34, s_0) through LDS.  Twice
 *                          the waves for the same work: for calls too small to fill the
 *                          device.  32-bit words only (MICKEY_EINVAL with word_bits 64,
 *                          in either order of the two calls);
 *   MICKEY_SCHED_SPLIT4    four waves per 64 slices, each keeping half of R or half of
 *                          S and computing first the values the others need (10 words
 *                          exchanged per clock); 128 VGPRs per wave.  Bit-planes only:
 *                          the fused row-major path runs SPLIT instead.  32-bit words only;
 *   MICKEY_SCHED_AUTO      (default) with 32-bit words: ONE_WAVE when the one-wave launch
 *                          gives every SIMD two waves (n >= 2^22 on MI355X), SPLIT when it
 *                          gives every SIMD at least one (n >= 2^21), SPLIT4 below; with
 *                          64-bit words ONE_WAVE. */
#define MICKEY_SCHED_AUTO 0
#define MICKEY_SCHED_ONE_WAVE 1
#define MICKEY_SCHED_SPLIT 2
#define MICKEY_SCHED_SPLIT4 3
int mickey_set_schedule(mickey_state *st, int schedule);

/* How the row-major layouts are produced (the output bytes do not depend on it):
 *   MICKEY_TRANSPOSE_FUSED   inside the generate kernel: every 32 clocks each lane
 *                            transposes its 32 x 32 block and stores one word per
 *                            instance (4-byte stores spread over 64 rows per instruction);
 *   MICKEY_TRANSPOSE_STAGED  the keystream goes to library-owned bit-plane buffers in
 *                            chunks of up to 8192 clocks (two buffers of at most 256 MiB,
 *                            allocated on first use, kept until mickey_free), and a tiled
 *                            transpose kernel writes 1024-clock row segments as whole
 *                            lines.  The transposes run on a library-owned second stream,
 *                            overlapping the next chunk; the call's work still completes
 *                            in order on the state's stream (it waits for the last one);
 *   MICKEY_TRANSPOSE_AUTO    (default) STAGED unless one 1024-clock tile of planes
 *                            exceeds 2 GiB (n > 2^24), then FUSED.
 * A failed chunk-buffer allocation makes the generate call return MICKEY_ENOMEM. */
#define MICKEY_TRANSPOSE_AUTO 0
#define MICKEY_TRANSPOSE_FUSED 1
#define MICKEY_TRANSPOSE_STAGED 2
int mickey_set_transpose(mickey_state *st, int mode);

size_t mickey_num_instances(const mickey_state *st);
/* Keystream bits every instance has produced through whole-state calls (mickey_generate,
 * mickey_generate_rowmajor) since the last initialisation or import; instances that
 * mickey_generate_batch advanced further have their own totals (mickey_instance_bits).
 * The 2^40 limit of Sec. II-C-1 applies to each instance's total. */
uint64_t mickey_bits_generated(const mickey_state *st);
/* Keystream bits instance `instance` has produced in total; UINT64_MAX (and
 * MICKEY_EINVAL) for a NULL state or an instance >= n. */
uint64_t mickey_instance_bits(const mickey_state *st, size_t instance);
/* Bytes per bit-plane of the MICKEY_BITSLICED layout for n instances: 8*ceil(n/64). */
size_t mickey_plane_pitch(size_t n);

/* Copy the 200 state bits of every instance into `packed` (device, n*25 bytes):
 * instance i occupies bytes 25*i .. 25*i+24, and bit j of the string
 * r_0..r_99 s_0..s_99 is bit (7 - j%8) of byte 25*i + j/8.  Also returns the bit
 * counter in *bits_generated if that (host) pointer is non-NULL.  Asynchronous. */
int mickey_state_export(const mickey_state *st, uint8_t *packed, uint64_t *bits_generated);

/* Overwrite every instance's registers from `packed` (device, n*25 bytes, layout as in
 * mickey_state_export) and set every instance's bit counter to bits_generated
 * (MICKEY_ERANGE beyond 2^40); generation then resumes from there.  Pad instances are
 * left as they are.  Asynchronous. */
int mickey_state_import(mickey_state *st, const uint8_t *packed, uint64_t bits_generated);

/* Host form of a state, for checkpoints (a state resumes exactly, Sec. II-C-1's per-key/IV
 * budget included): a 32-byte header (8 bytes "MICKEY2\0", uint32 version 1, uint32 25,
 * uint64 n, 8 reserved bytes), then the n packed states of mickey_state_export, then n
 * uint64 bit counters (mickey_instance_bits), all little-endian: mickey_state_host_bytes(st)
 * = 32 + 33*n bytes (0 for NULL).  Export writes it to `host` (cap bytes, host memory; too
 * small: MICKEY_EINVAL) and synchronises the state's stream.  Import checks the header, n,
 * len and every counter before it changes anything (MICKEY_EINVAL / MICKEY_ERANGE), then
 * replaces every instance's registers and counter, and synchronises the copy to the device. */
size_t mickey_state_host_bytes(const mickey_state *st);
int mickey_state_export_host(const mickey_state *st, void *host, size_t cap);
int mickey_state_import_host(mickey_state *st, const void *host, size_t len);

/* Wait for all work enqueued on the state's streams.  A failure poisons the state. */
int mickey_sync(mickey_state *st);

/* Failure injection, for testing the error paths without a faulty device: the k-th launch
 * (kernel or state copy) from now, made by any state of this process, is not made and
 * its call returns MICKEY_EDEVICE as if the launch had failed; k = 0 cancels a pending
 * injection.  MICKEY_EINVAL for k < 0. */
int mickey_debug_fail_launch(int k);

/* ---------------------------------------------------------------------------------
 * Batched generation (one persistent launch for many fresh requests).
 *
 * Each request is a fresh instance: its own key, IV of 0..80 bits and keystream length.
 * The executor sorts the requests longest first into groups of 32 (one bit lane each
 * of one slice), stages every group's input planes, and runs one persistent work-queue
 * kernel whose waves pop groups of groups until the queue is empty.  The launch
 * sequence is captured once as a HIP graph and replayed by mickey_batch_run.  The
 * result of a request does not depend on the other requests of the batch.
 */
typedef struct mickey_batch mickey_batch;

/* Executor for up to max_requests requests per batch, on a HIP stream (NULL: the
 * executor creates and owns a stream; graph capture needs a non-null stream). */
mickey_batch *mickey_batch_create(size_t max_requests, void *hip_stream);

/* Set the requests that the following runs execute.
 *   keys, ivs  device, 10 bytes per request (request r at offset 10*r)
 *   iv_bits    device, one byte per request in 0..80, or NULL for 80 (validated here,
 *              which synchronises the batch's stream)
 *   nbits      host, keystream bits of request r: a multiple of 32, at most 2^37
 *   outs       host array of device pointers: request r's nbits/32 words, laid out as
 *              MICKEY_ROWMAJOR_U32 for one instance (bit 31-b of word j is z_{32j+b})
 * Host arrays may be freed on return; device arrays must stay valid while runs use
 * them.  Builds the sorted metadata and captures the launch graph. */
int mickey_batch_set(mickey_batch *b, const uint8_t *keys, const uint8_t *ivs, const uint8_t *iv_bits,
                     const uint64_t *nbits, uint32_t *const *outs, size_t nreq);

/* Run the current requests: one graph launch (queue reset, input staging, the
 * persistent kernel).  Asynchronous on the batch's stream. */
int mickey_batch_run(mickey_batch *b);
int mickey_batch_sync(mickey_batch *b);
/* The batch's HIP stream (hipStream_t as void*). */
void *mickey_batch_stream(const mickey_batch *b);

/* Kernel variant: clocks per loop iteration (2, 4 or 8) and waves per workgroup (1, 2
 * or 4); 0 keeps the current value.  Re-captures the graph. */
int mickey_batch_set_params(mickey_batch *b, int unroll, int waves_per_block);
int mickey_batch_get_params(const mickey_batch *b, int *unroll, int *waves_per_block);

/* Autotuner: times every built variant on the current requests with lengths capped at
 * cap_bits (a multiple of 32; outputs go to scratch memory), keeps the fastest, times
 * the same capped requests in latency mode to set the routing ratio r, and
 * re-captures.  With cache_path, a JSON record of the choice is read from that file
 * when its signature (architecture, request count, capped lengths) matches, and written
 * there otherwise.  Synchronises the batch's stream. */
int mickey_batch_autotune(mickey_batch *b, uint64_t cap_bits, const char *cache_path);

/* Size-aware routing: requests of at least `bits` bits run in latency mode (one
 * request per four lanes, words of the registers spread over the lanes: ~10x more VALU
 * work per bit, but a lone instance advances several times faster), the rest bitsliced;
 * both run concurrently in the same graph and give identical words.  0 (the default)
 * sets the threshold automatically to 3/4 * L_max * r, r being the tuned ratio of the two
 * engines' clock times, so that the bitsliced part finishes before the longest request;
 * UINT64_MAX turns latency mode off.  At most 16384 requests take latency mode. */
int mickey_batch_set_latency_threshold(mickey_batch *b, uint64_t bits);
/* The threshold in use (UINT64_MAX if none), how many requests take latency mode, and
 * the clock-time ratio r. */
int mickey_batch_get_routing(const mickey_batch *b, uint64_t *threshold, size_t *latency_requests,
                             double *latency_clock_ratio);

void mickey_batch_free(mickey_batch *b);

/* ---------------------------------------------------------------------------------
 * Serving: resident generator states, requests that resume them, continuous batching.
 *
 * The server keeps every state of an initialised mickey_state resident in HBM (25 bytes
 * each, the mickey_state_export layout) and owns `nslices` bitsliced slots of 32 lane
 * bits, a quantum length and an output budget.  mickey_server_step() admits waiting
 * requests in arrival order into free lane bits while their whole output fits in the
 * budget (one request per state at a time, so requests on a state run in arrival
 * order), gathers their states, and runs one quantum on every occupied slot; requests
 * that arrive while others run join at the next quantum.  A request's keystream
 * continues its state exactly where the previous request on that state stopped, and
 * its state is written back at the exact clock where it ends.
 */
typedef struct mickey_server mickey_server;

/* Create a server over the n instances of `init` (their current registers and bit
 * counter become the resident states 0..n-1; `init` may be freed afterwards).
 *   nslices         slot capacity in slices (32 concurrent requests each; rounded up to
 *                   a multiple of 64)
 *   quantum_clocks  clocks per scheduling step, a multiple of 32
 *   budget_bytes    device memory for outputs of admitted requests
 *   hip_stream      stream of the server's work (NULL: the server creates one) */
mickey_server *mickey_server_create(const mickey_state *init, size_t nslices, uint32_t quantum_clocks,
                                    uint64_t budget_bytes, void *hip_stream);

/* Queue a request: resume state `state_id` for nbits keystream bits (a positive multiple
 * of 32, at most 2^40; with whole-request delivery the output must also fit the budget
 * and 2^32 words).  Returns the request id (>= 0) or a negative error code. */
int64_t mickey_server_submit(mickey_server *s, uint32_t state_id, uint64_t nbits);

/* Batched forms: submit n requests (ids[k] gets the id or a negative code), release n
 * completed requests, and read n completed requests' (arrival, admission, completion)
 * times into out[3k..3k+2] (completion 0 for a request refused at 2^40 bits). */
int mickey_server_submit_many(mickey_server *s, const uint32_t *sids, const uint64_t *nbits, size_t n,
                              int64_t *ids);
int mickey_server_release_many(mickey_server *s, const uint64_t *ids, size_t n);
int mickey_server_times_many(const mickey_server *s, const uint64_t *ids, size_t n, uint64_t *out);
/* Words of each of n requests (submitted, not necessarily complete) admitted so far to
 * latency streams (see mickey_server_set_latency) rather than to bit lanes. */
int mickey_server_latency_words_many(const mickey_server *s, const uint64_t *ids, size_t n, uint64_t *out);

/* One scheduling step: wait for the quantum launched by the previous step and retire
 * the requests it completed, admit waiting requests and gather their states, then launch
 * the next quantum and return without waiting for it (the caller's host work overlaps
 * the GPU).  Does nothing on the GPU when no request is running or admitted. */
int mickey_server_step(mickey_server *s);

/* Wait for the in-flight quantum, if any, and retire its requests. */
int mickey_server_wait(mickey_server *s);

/* Ids of requests completed since the last call (at most cap); returns the count. */
int64_t mickey_server_poll(mickey_server *s, uint64_t *ids, size_t cap);

/* Chunked delivery.  After mickey_server_set_chunk(s, c) (c a multiple of 4 bytes that
 * fits the budget; 0 restores whole-request delivery), new submissions are delivered in
 * consecutive chunks of c bytes (the last one shorter).  A request then reserves only
 * one chunk of the budget at a time, so its total size is bounded by the 2^40-bit limit
 * rather than by the budget.  Its state stays reserved for it between chunks, so requests
 * on a state still run in arrival order, and each chunk continues the keystream at the
 * exact bit where the previous one stopped (the state is written back at the end of every
 * chunk, as at the end of a request).
 *
 * mickey_server_poll_chunks() returns the chunks finished since the last call, in
 * completion order (chunks of one request in stream order).  Their words stay valid until
 * the caller gives them back with mickey_server_release_chunks(); until then they count
 * against the budget.  A chunked request also appears in mickey_server_poll() when its
 * last chunk is done; mickey_server_result()/copy()/release() do not apply to it. */
typedef struct mickey_chunk {
    uint64_t request; /* request id */
    uint64_t handle;  /* give back with mickey_server_release_chunks() */
    uint64_t offset;  /* index of the chunk's first word in the request's stream */
    uint64_t words;   /* 32-bit words in the chunk */
    uint32_t *out;    /* device pointer to the words (MICKEY_ROWMAJOR_U32 layout) */
    uint64_t last;    /* nonzero when this chunk completes the request */
} mickey_chunk;

int mickey_server_set_chunk(mickey_server *s, uint64_t chunk_bytes);

/* Kernels of the following quanta (the delivered bytes do not depend on them):
 *   transpose  MICKEY_TRANSPOSE_FUSED: one kernel stores every lane's word per 32 clocks
 *              into its request (one-wave schedule only); MICKEY_TRANSPOSE_STAGED: the
 *              quantum writes bit-planes to server-owned buffers (two of at most 512 MiB,
 *              made at creation; a quantum whose planes exceed one runs as several
 *              launches, alternating between them) and a tiled transpose writes each
 *              request's words as whole lines, beside the next launch when no latency
 *              stream runs;
 *              MICKEY_TRANSPOSE_AUTO: STAGED when the buffer exists (it does unless one
 *              32-clock launch of planes exceeds 512 MiB).
 *   schedule   for staged quanta, MICKEY_SCHED_ONE_WAVE / _SPLIT / _SPLIT4 / _AUTO as
 *              for mickey_set_schedule (AUTO: the four-wave split below two one-wave
 *              waves per SIMD).
 * MICKEY_EINVAL for FUSED with a split schedule, or STAGED / a split without the buffer. */
int mickey_server_set_kernel(mickey_server *s, int schedule, int transpose);

/* Latency streams (the paper's Sec. VI: delay is the GPU's drawback): the part of a
 * request that still has at least threshold_bits to go is admitted, when one is free, to
 * one of `streams` (at most 16384) latency streams instead of a bit lane, while at most
 * half of the bit lanes are busy.  A latency stream is four lanes of one wave holding the
 * request's registers as words; it advances clocks_per_quantum clocks per quantum (a
 * positive multiple of 32), beside the bitsliced quantum on a second stream, at ~27 VALU
 * per clock instead of ~330 per 32 requests: several times faster per request, ~10x the
 * device work per bit.  Output bytes are the same either way.  Defaults at creation:
 * 16384 streams, 2^20 bits, 8 x the quantum.  streams = 0
 * turns routing off.  MICKEY_EINVAL while latency streams or quanta are in flight (call
 * it between mickey_server_wait and new work). */
int mickey_server_set_latency(mickey_server *s, uint32_t streams, uint64_t threshold_bits,
                              uint64_t clocks_per_quantum);
int64_t mickey_server_poll_chunks(mickey_server *s, mickey_chunk *out, size_t cap);
int mickey_server_release_chunks(mickey_server *s, const uint64_t *handles, size_t n);
/* Copy the first nwords words of a delivered, not yet released chunk into dst (device);
 * synchronous. */
int mickey_server_copy_chunk(const mickey_server *s, uint64_t handle, uint32_t *dst, uint64_t nwords);

/* A completed request's output (device, nbits/32 words in the MICKEY_ROWMAJOR_U32 layout
 * of one instance) and its arrival / admission / completion times (ns, steady clock).
 * MICKEY_ERANGE (and *out = NULL) if it was refused for passing 2^40 bits. */
int mickey_server_result(const mickey_server *s, uint64_t id, uint32_t **out, uint64_t times_ns[3]);

/* Copy the first nwords words of a completed request's output into dst (device);
 * synchronous. */
int mickey_server_copy(const mickey_server *s, uint64_t id, uint32_t *dst, uint64_t nwords);

/* Return a completed request's output space to the budget (its words become invalid). */
int mickey_server_release(mickey_server *s, uint64_t id);

/* [0] waiting (including chunked requests between two chunks), [1] running, [2] admitted,
 * [3] finished, [4] steps, [5] quantum time in
 * ns (launch to retirement), [6] keystream bits delivered, [7] free budget in 32-bit
 * words, [8] host ns blocked on quanta, [9] host ns retiring, [10] host ns admitting,
 * [11] device ns of the quanta (each from its first kernel's start to its completion count,
 * timed with HIP events; gaps between quanta are not counted). */
int mickey_server_stats(const mickey_server *s, uint64_t out[12]);

/* Device pointer to resident state `state_id` (25 bytes) and its bit counter. */
int mickey_server_state(const mickey_server *s, uint32_t state_id, const uint8_t **packed, uint64_t *bits);

void *mickey_server_stream(const mickey_server *s);
void mickey_server_free(mickey_server *s);

int mickey_last_error(void);
const char *mickey_last_error_message(void);

/* Per-clock VALU instruction count of the generate clock for 32 instances (the
 * algorithmic op count used for the VALU roofline).  Compile-time constant. */
int mickey_ops_per_clock(void);

#ifdef __cplusplus
}
#endif

#endif /* MICKEY_H */

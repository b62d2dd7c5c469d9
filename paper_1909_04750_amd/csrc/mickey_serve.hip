// Served generation: a pool of resident generator states in HBM, requests that resume
// one state each for a keystream of a given length, and continuous batching.
//
// Resident states are kept packed (25 bytes each: r_0..r_99 s_0..s_99, MSB first, the
// mickey_state_export layout).  The server owns a fixed set of bitsliced slots (slices
// of 32 lane bits, state planes as in the plain path).  Each scheduling step
//   1. retires requests that completed in the last quantum (their state was written
//      back to the pool by the kernel at the exact clock where the request ended),
//   2. admits waiting requests, in arrival order, into free lane bits while the output
//      budget allows (a request reserves its whole output, or in chunked delivery one
//      chunk at a time; a state runs at most one request at a time, so requests on one
//      state run in arrival order),
//   3. flags the admitted lanes (the next quantum gathers their states into its
//      registers), and
//   4. runs one quantum of Q clocks on every occupied slice, writing each request's
//      keystream as row-major words (MICKEY_ROWMAJOR_U32 layout) into its output.
// Requests that arrive while others run join at the next quantum, next to them.
//
// Chunked delivery: a request submitted after mickey_server_set_chunk(c) runs as a
// sequence of admissions of at most c bytes each.  Each admission reserves only its own
// chunk, and its lane writes the state back when the chunk ends (the same exact
// write-back as at the end of a request), so the next chunk resumes at the next bit.  The
// state stays reserved for the request between its chunks, and requests that are
// between chunks are admitted before new ones.  The client reads each finished chunk
// and gives its space back, so the budget bounds the output in flight, not the size of
// a request.
#include "arena.h"
#include "mickey_device.h"
#include "mickey_host.h"
#include "mickey_pack.h"
#include "mickey_split4_loop.h"
#include "mickey_wordpar.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <queue>
#include <unordered_map>
#include <new>
#include <vector>

using namespace mickey;
using namespace mickey_host;

namespace {

constexpr int kServeUnroll = 4;

// One admission: lane bit `lane` (slice lane/32, bit lane%32) takes resident state `sid`.
struct Admit {
    uint32_t lane;
    uint32_t sid;
    uint32_t words;
    uint32_t pad;
    uint32_t *out;
};

// Admission metadata: lane `lane` takes resident state `sid` with an output of `words`
// words at `out`, and is flagged fresh in its slice's mask (one atomic per admission); the
// next quantum gathers the fresh lanes' states into its registers.  Lane ids from nlanes
// on are latency streams (lane - nlanes), flagged fresh in their own word.
__global__ __launch_bounds__(256) void admit_kernel(const Admit *__restrict__ adm, uint32_t nadm, uint32_t nlanes,
                                                    uint32_t **lane_out, uint32_t *lane_left, uint32_t *lane_sid,
                                                    uint32_t *fresh, uint32_t **lat_out, uint32_t *lat_left,
                                                    uint32_t *lat_sid, uint32_t *lat_fresh)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nadm) return;
    const Admit a = adm[k];
    if (a.lane >= nlanes) {
        const uint32_t j = a.lane - nlanes;
        lat_out[j] = a.out;
        lat_left[j] = a.words;
        lat_sid[j] = a.sid;
        lat_fresh[j] = 1u;
        return;
    }
    lane_out[a.lane] = a.out;
    lane_left[a.lane] = a.words;
    lane_sid[a.lane] = a.sid;
    atomicOr(fresh + (a.lane >> 5), 1u << (a.lane & 31u));
}

// One quantum of nblocks*32 clocks on every slice with an occupied lane bit.  Each lane's
// output pointer and remaining words are read once into LDS and are read-only during the
// quantum.  A block's 32 keystream words per lane are transposed in LDS (lane l's word in
// row 31 - l), and during clock c of the next block the word of lane 31 - c is stored: its
// pointer and word are read from LDS at the start of that clock and stored at its end, so
// the LDS latency hides behind the clock's arithmetic (the last block is drained after the
// loop).  One 32-row buffer holds both: at clock c, row c gives up its word and takes the
// keystream plane of clock c.  A lane whose request
// ends at the end of block b has its state packed back into the pool right there and is
// appended to the completion list; the lanes' end blocks are only scanned when the next
// one is reached.  At the end the pointers and counts move on by the blocks done.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void quantum_kernel(
    uint32_t *__restrict__ planes, uint32_t nslices, uint32_t nblocks, uint32_t **lane_out,
    uint32_t *__restrict__ lane_left, const uint32_t *__restrict__ lane_sid, uint8_t *__restrict__ pool,
    uint32_t *__restrict__ fresh, uint32_t *__restrict__ sink, uint32_t *__restrict__ done_list,
    uint32_t *__restrict__ done_count)
{
    __shared__ uint32_t zbuf[32][64];
    __shared__ uint32_t *s_out[32][64];
    const uint32_t tid = threadIdx.x;
    const uint32_t g = blockIdx.x * 64u + tid;
    if (g >= nslices) return;  // no barriers: each lane touches only its own LDS columns
    uint32_t active = 0;             // lanes with words left
    uint32_t next_end = 0xFFFFFFFFu;  // the earliest block count at which a lane's request ends
    for (int l = 0; l < 32; l++) {
        const uint32_t left = lane_left[g * 32u + l];
        s_out[l][tid] = lane_out[g * 32u + l];
        active |= (left ? 1u : 0u) << l;
        if (left && left < next_end) next_end = left;
    }
    if (!active) return;
    const size_t pitch = (size_t)nslices * 4u;
    const uint32_t voff = g * 4u;
    Regs<1> x;
    load_state<1>(x, planes, pitch, voff);
    uint32_t fr = fresh[g];  // lanes admitted since the last quantum: gather their states
    if (fr) {
        fresh[g] = 0u;
        while (fr) {
            const uint32_t l = (uint32_t)__builtin_ctz(fr);
            fr &= fr - 1u;
            gather_lane(x, l, pool + 25ull * lane_sid[g * 32u + l]);
        }
    }
    uint32_t pend = 0;  // lanes with a word of block blk - 1 waiting in zprev
    uint32_t blk = 0;
    for (; blk < nblocks && active; blk++) {
        for (int b0 = 0; b0 < 32; b0 += kServeUnroll) {
#pragma unroll
            for (int u = 0; u < kServeUnroll; u++) {
                const int c = b0 + u, l = 31 - c;
                const uint32_t w = zbuf[c][tid];  // word of lane l from the previous block
                uint32_t *const p = s_out[l][tid];
                zbuf[c][tid] = (x.r[0] ^ x.s[0]).w[0];  // row c now holds clock c
                clock_gen<1>(x);
                // The store goes after the clock's arithmetic (the scheduler may not move
                // anything across the barrier), so the LDS loads above have the whole clock
                // to complete; a lane without a word writes to the slice's sink word.
                uint32_t *const dst = ((pend >> l) & 1u) ? p + (blk - 1u) : sink + g;
                __builtin_amdgcn_sched_barrier(0);
                store_global(dst, w);
            }
        }
#pragma unroll
        for (int h = 0; h < 32; h += 16) {
            uint32_t a[16];
#pragma unroll
            for (int i = 0; i < 16; i++) a[i] = zbuf[31 - (h + i)][tid];  // row 31-r: clock r
            transpose_half(a);
#pragma unroll
            for (int i = 0; i < 16; i++) zbuf[31 - (h + i)][tid] = a[i];
        }
#pragma unroll
        for (int i = 0; i < 16; i++) {
            uint32_t lo = zbuf[31 - i][tid], hi = zbuf[15 - i][tid];
            swap_stage<16>(lo, hi);
            zbuf[31 - i][tid] = lo;  // word of lane i (bit 31 - b = clock b of the block)
            zbuf[15 - i][tid] = hi;  // word of lane i + 16
        }
        pend = active;
        if (blk + 1u == next_end) {  // some lanes end with this block
            uint32_t finished = 0;
            next_end = 0xFFFFFFFFu;
            for (uint32_t l = 0; l < 32; l++) {
                if (!((active >> l) & 1u)) continue;
                const uint32_t left = lane_left[g * 32u + l];
                if (left == blk + 1u)
                    finished |= 1u << l;
                else if (left < next_end)
                    next_end = left;
            }
            for (uint32_t l = 0; l < 32; l++) {
                if ((finished >> l) & 1u) {
                    write_back_lane(x, l, pool + 25ull * lane_sid[g * 32u + l]);
                    done_list[atomicAdd(done_count, 1u)] = g * 32u + l;
                }
            }
            active &= ~finished;
        }
    }
    for (int l = 0; l < 32; l++)  // drain the last block's words
        if ((pend >> l) & 1u) store_global(s_out[l][tid] + (blk - 1u), zbuf[31 - l][tid]);
    store_state<1>(x, planes, pitch, voff);
    for (int l = 0; l < 32; l++) {
        const uint32_t left = lane_left[g * 32u + l];
        if (!left) continue;
        const uint32_t done = left < blk ? left : blk;
        lane_left[g * 32u + l] = left - done;
        lane_out[g * 32u + l] = s_out[l][tid] + done;
    }
}

// ---------------------------------------------------------------------------------
// Latency streams (the paper's Sec. VI names delay as the drawback of GPU generators): a
// request routed here advances one clock per ~27 VALU operations of one wave instead of
// one per bitsliced clock (~330 operations for 32 requests); with one wave issuing at
// most ~0.4 instructions/ns, that is ~70 ns per clock for the request against several
// hundred for a bit lane of a partly filled launch.  One request per quad of lanes: lane
// q keeps word q of R and of S in the word-parallel layout of mickey_wordpar.h (bit i of
// a register is bit i % 32 of word i / 32).  Per clock the quad XOR-reduces each lane's
// share of the four bits that steer the clock (s_34 ^ r_67 = c_R, r_33 ^ s_67 = c_S,
// r_99 = fb_R, s_99 = fb_S) with two DPP swaps, fetches its neighbours' words for the
// shifts with DPP quad permutes, and updates its two words as the word-parallel clock
// does.  (The one-lane word-parallel clock is ~52 operations: half the speed per request.)

constexpr uint32_t kLatStreams = 16384;  // latency stream capacity of a server

// One quantum of the latency streams: every busy stream runs up to nwords x 32 clocks,
// storing one output word per 32 clocks (lane 0), then keeps its words in lat_state; a
// stream whose words end packs its state back into the pool and joins the completion
// list as id_base + stream.  Streams are whole quads, so every DPP stays inside a quad
// whose lanes are all active.
__global__ __launch_bounds__(64) void latency_quantum_kernel(uint32_t *__restrict__ lat_state, uint32_t nstreams,
                                                             uint32_t nwords, uint32_t **lat_out,
                                                             uint32_t *__restrict__ lat_left,
                                                             const uint32_t *__restrict__ lat_sid,
                                                             uint32_t *__restrict__ lat_fresh, uint8_t *__restrict__ pool,
                                                             uint32_t id_base, uint32_t *__restrict__ done_list,
                                                             uint32_t *__restrict__ done_count)
{
    const uint32_t t = blockIdx.x * 64u + threadIdx.x, k = t >> 2, q = t & 3u;
    if (k >= nstreams) return;
    const uint32_t left = lat_left[k];
    if (!left) return;
    uint32_t r, s;
    if (lat_fresh[k]) {
        quad_gather(pool + 25ull * lat_sid[k], q, r, s);
    } else {
        r = lat_state[8u * k + 2u * q];
        s = lat_state[8u * k + 2u * q + 1u];
    }
    const QuadMasks m = quad_masks(q);
    uint32_t *out = lat_out[k];
    const uint32_t nw = left < nwords ? left : nwords;
    for (uint32_t w = 0; w < nw; w++) {
        const uint32_t word = quad_word(r, s, m);
        if (q == 0) store_global(out + w, word);
    }
    if (nw == left) {
        quad_write_back(r, s, q, pool + 25ull * lat_sid[k]);
        if (q == 0) done_list[atomicAdd(done_count, 1u)] = id_base + k;
    }
    if (q == 0) {
        lat_left[k] = left - nw;
        lat_out[k] = out + nw;
        lat_fresh[k] = 0u;
    }
    lat_state[8u * k + 2u * q] = r;
    lat_state[8u * k + 2u * q + 1u] = s;
}

struct Request {
    uint64_t id;
    uint32_t sid;
    uint64_t nbits;
    uint64_t arrival_ns;
    uint64_t admit_ns = 0, first_ns = 0, done_ns = 0;  // first admission, first chunk done, last done
    uint32_t lane = kNoRequest;
    uint32_t chunk_words = 0;  // 0: whole-request delivery
    size_t out_off = 0;        // word offset in the arena of the output (or current chunk)
    size_t out_granted = 0;    // arena words held by it
    uint64_t next_same = ~0ull;  // next request waiting on the same state
    uint64_t words_admitted = 0, words_done = 0;
    uint32_t cur_words = 0;    // words of the admission in flight
    uint64_t lat_words = 0;    // words admitted to latency streams
    bool refused = false;      // passed 2^40 bits
    bool done = false;
    bool released = false;
};

// A delivered chunk's arena block, by handle.
struct ChunkSlot {
    size_t off = 0, granted = 0;  // arena block
    uint64_t words = 0;           // keystream words in it
    uint32_t slice = 0;           // slice of the lane that wrote it
    bool live = false;
};

// Released chunk blocks are kept per slice (up to this many) and handed to the next chunk
// admitted into the same slice, so the 32 lanes of a slice keep writing into a few nearby
// blocks (the blocks first handed out to a slice are adjacent) instead of blocks spread
// over the whole arena: fewer pages touched per store instruction.
constexpr size_t kSliceCache = 48;

uint64_t now_ns()
{
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace

struct mickey_server {
    size_t nstates = 0, nslices = 0, nlanes = 0;
    uint32_t qblocks = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    uint8_t *pool = nullptr;   // [nstates][25]
    uint32_t *planes = nullptr;
    uint32_t **lane_out = nullptr;
    uint32_t *lane_left = nullptr, *lane_sid = nullptr;
    uint32_t *fresh = nullptr;  // per slice: lanes admitted since the last quantum
    uint32_t *sink = nullptr;   // per slice: target of stores by lanes without output
    // staged quanta: keystream planes of one launch, and per lane what it wrote; two
    // buffers, so that a launch's rows are written (on tstream) while the next launch
    // generates into the other buffer
    uint32_t *zplanes[2] = {nullptr, nullptr};
    uint32_t **row_dst[2] = {nullptr, nullptr};
    uint32_t *row_cnt[2] = {nullptr, nullptr};
    uint32_t sub_blocks = 0;  // blocks per staged launch (0: staging not available)
    uint64_t sub_seq = 0;     // staged launches so far: launch j uses buffer j & 1
    hipStream_t tstream = nullptr;  // transposes and the completion counts
    hipEvent_t ev_sub[2] = {nullptr, nullptr};    // launch into buffer k done
    hipEvent_t ev_tdone[2] = {nullptr, nullptr};  // transpose of buffer k done
    bool tdone_rec[2] = {false, false};
    hipEvent_t ev_qend = nullptr;  // the quantum's last kernel on the server's stream
    int schedule = MICKEY_SCHED_AUTO, transpose = MICKEY_TRANSPOSE_AUTO;
    int simds = 1024;
    // latency streams: lane ids nlanes .. nlanes + kLatStreams - 1
    uint32_t *lat_state = nullptr;  // [kLatStreams][4 lanes][r, s]
    uint32_t **lat_out = nullptr;
    uint32_t *lat_left = nullptr, *lat_sid = nullptr, *lat_fresh = nullptr;
    uint32_t lat_streams = 0;          // streams in use (0: routing off)
    uint64_t lat_threshold_words = 0;  // requests with at least this many words left go there
    uint32_t lat_words = 0;            // output words per stream per quantum
    std::vector<uint32_t> lat_free;    // free stream indices
    uint32_t lat_busy = 0;
    hipStream_t side = nullptr;  // latency streams run here, beside the bitsliced quantum
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    uint32_t *done_list = nullptr, *done_count = nullptr;
    uint32_t *arena = nullptr;
    serve_arena::Arena alloc;
    // host side
    // Admissions, in pinned mapped memory that admit_kernel reads directly (the stream holds
    // kernels and events only).  Two buffers: the kernel reading one may still be queued
    // behind the quantum in flight while the next admissions are written to the other.
    Admit *hadm_buf[2] = {nullptr, nullptr};
    Admit *hadm_dev[2] = {nullptr, nullptr};  // device views
    int adm_b = 0;                            // the buffer being filled
    Admit *hadm = nullptr;                    // == hadm_buf[adm_b]
    // Two quanta can be in flight: quantum q uses completion buffer q & 1.
    uint32_t *hcount = nullptr;     // pinned, mapped [2]: completions of each in-flight quantum
    uint32_t *hcount_dev = nullptr; // device view of hcount
    uint32_t *hlist = nullptr;      // pinned, mapped [2][nlanes]: completed lanes
    uint32_t *hlist_dev = nullptr;  // device view of hlist
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t ev_start[2] = {nullptr, nullptr};  // before each quantum's first kernel
    uint64_t launch_ns[2] = {0, 0};
    uint64_t next_q = 0, oldest_q = 0;  // quanta [oldest_q, next_q) are in flight
    uint32_t pending = 0;               // admissions decided, not yet enqueued
    std::vector<uint64_t> state_bits;
    // A state is owned by at most one request that is ready, running or between chunks;
    // later requests on it wait in a chain (per-state FIFO through Request::next_same).
    std::vector<uint8_t> state_owned;
    std::vector<uint64_t> chain_head, chain_tail;
    uint64_t chained = 0;
    std::vector<uint32_t> free_lanes;
    // requests that own their state and wait for a lane and budget, oldest (lowest id) first
    std::priority_queue<uint64_t, std::vector<uint64_t>, std::greater<uint64_t>> ready_q;
    std::vector<Request> reqs;     // by id
    std::vector<uint64_t> lane_req;
    std::vector<uint64_t> completed;  // not yet reported
    uint32_t chunk_words = 0;         // chunk size of new submissions (0: whole requests)
    std::deque<uint64_t> continuing;  // chunked requests between two chunks, oldest first
    std::vector<mickey_chunk> ready;  // delivered chunks not yet polled
    std::vector<ChunkSlot> slots;     // chunk handles
    std::vector<std::vector<std::pair<size_t, size_t>>> slice_blocks;  // per slice: (offset, granted)
    size_t slice_cached = 0;          // words held there
    std::vector<uint64_t> free_slots;
    uint64_t steps = 0, quanta_ns = 0, admitted = 0, finished = 0, bits_done = 0;
    uint64_t ns_wait = 0, ns_retire = 0, ns_admit = 0;  // host time spent in each part
    uint64_t ns_gpu = 0;  // device time of the quanta, first kernel to completion count
};

namespace {

void destroy(mickey_server *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->tstream) (void)hipStreamSynchronize(s->tstream);
    for (void *p : {(void *)s->pool, (void *)s->planes, (void *)s->lane_out, (void *)s->lane_left,
                    (void *)s->lane_sid, (void *)s->fresh, (void *)s->sink, (void *)s->done_list,
                    (void *)s->arena, (void *)s->zplanes[0], (void *)s->row_dst[0], (void *)s->row_cnt[0],
                    (void *)s->zplanes[1], (void *)s->row_dst[1], (void *)s->row_cnt[1],
                    (void *)s->lat_state, (void *)s->lat_out, (void *)s->lat_left, (void *)s->lat_sid,
                    (void *)s->lat_fresh})
        if (p) (void)hipFree(p);
    for (Admit *h : s->hadm_buf)
        if (h) (void)hipHostFree(h);
    if (s->hcount) (void)hipHostFree(s->hcount);
    if (s->hlist) (void)hipHostFree(s->hlist);
    for (hipEvent_t e : {s->ev[0], s->ev[1], s->ev_start[0], s->ev_start[1], s->ev_sub[0], s->ev_sub[1],
                         s->ev_tdone[0], s->ev_tdone[1], s->ev_qend})
        if (e) (void)hipEventDestroy(e);
    if (s->tstream) (void)hipStreamDestroy(s->tstream);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    if (s->side) {
        (void)hipStreamSynchronize(s->side);
        (void)hipStreamDestroy(s->side);
    }
    if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
    if (s->ev_join) (void)hipEventDestroy(s->ev_join);
    delete s;
}

// ---------------------------------------------------------------------------------
// Staged quanta.  The quantum kernels below write the keystream as bit-planes (plane t:
// one word per slice) to a chunk buffer, with coalesced stores, and record per lane the
// output position and word count of the launch (row_dst, row_cnt); serve_transpose_kernel
// then writes each lane's words to its request in whole lines.  A quantum may run as
// several such launch pairs when its planes exceed the chunk buffer.

// Per-lane end-of-launch bookkeeping shared by the staged kernels: what the launch wrote
// for each lane (blk blocks ran) and where the lane continues.
__device__ __forceinline__ void staged_advance(uint32_t g, uint32_t blk, uint32_t **lane_out, uint32_t *lane_left,
                                               uint32_t **row_dst, uint32_t *row_cnt)
{
    for (int l = 0; l < 32; l++) {
        const uint32_t i = g * 32u + l;
        const uint32_t left = lane_left[i];
        const uint32_t done = left < blk ? left : blk;
        uint32_t *const out = lane_out[i];
        row_dst[i] = out;
        row_cnt[i] = done;
        if (left) {
            lane_left[i] = left - done;
            lane_out[i] = out + done;
        }
    }
}

// Lanes with words left, and the earliest block count at which one of them ends.
__device__ __forceinline__ uint32_t scan_lanes(const uint32_t *lane_left, uint32_t g, uint32_t &next_end)
{
    uint32_t active = 0;
    next_end = 0xFFFFFFFFu;
    for (int l = 0; l < 32; l++) {
        const uint32_t left = lane_left[g * 32u + l];
        active |= (left ? 1u : 0u) << l;
        if (left && left < next_end) next_end = left;
    }
    return active;
}

// Lanes whose words end with block blk (blk + 1 == next_end); next_end moves on.
__device__ __forceinline__ uint32_t ending_lanes(const uint32_t *lane_left, uint32_t g, uint32_t active,
                                                 uint32_t blk, uint32_t &next_end)
{
    uint32_t finished = 0;
    next_end = 0xFFFFFFFFu;
    for (uint32_t l = 0; l < 32; l++) {
        if (!((active >> l) & 1u)) continue;
        const uint32_t left = lane_left[g * 32u + l];
        if (left == blk + 1u)
            finished |= 1u << l;
        else if (left < next_end)
            next_end = left;
    }
    return finished;
}

// One-wave staged quantum: the plain generate loop (one plane store per clock) plus the
// lane bookkeeping of quantum_kernel.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void quantum_planes_kernel(
    uint32_t *__restrict__ planes, uint32_t nslices, uint32_t nblocks, uint32_t **lane_out,
    uint32_t *__restrict__ lane_left, const uint32_t *__restrict__ lane_sid, uint8_t *__restrict__ pool,
    uint32_t *__restrict__ fresh, uint32_t *__restrict__ zplanes, uint32_t **row_dst, uint32_t *__restrict__ row_cnt,
    uint32_t *__restrict__ done_list, uint32_t *__restrict__ done_count)
{
    const uint32_t g = blockIdx.x * 64u + threadIdx.x;  // nslices is a multiple of 64
    uint32_t next_end;
    uint32_t active = scan_lanes(lane_left, g, next_end);
    if (!active) {
        for (int l = 0; l < 32; l++) row_cnt[g * 32u + l] = 0u;
        return;
    }
    const size_t pitch = (size_t)nslices * 4u;
    const uint32_t voff = g * 4u;
    Regs<1> x;
    load_state<1>(x, planes, pitch, voff);
    uint32_t fr = fresh[g];
    if (fr) {
        fresh[g] = 0u;
        while (fr) {
            const uint32_t l = (uint32_t)__builtin_ctz(fr);
            fr &= fr - 1u;
            gather_lane(x, l, pool + 25ull * lane_sid[g * 32u + l]);
        }
    }
    char *plane = (char *)zplanes;  // wave-uniform
    uint32_t blk = 0;
    for (; blk < nblocks && active; blk++) {
        for (int b0 = 0; b0 < 32; b0 += kServeUnroll) {
#pragma unroll
            for (int u = 0; u < kServeUnroll; u++) {
                store_plane<1>(plane, voff, x.r[0] ^ x.s[0]);
                plane += pitch;
                clock_gen<1>(x);
            }
        }
        if (blk + 1u == next_end) {
            const uint32_t finished = ending_lanes(lane_left, g, active, blk, next_end);
            for (uint32_t l = 0; l < 32; l++) {
                if ((finished >> l) & 1u) {
                    write_back_lane(x, l, pool + 25ull * lane_sid[g * 32u + l]);
                    done_list[atomicAdd(done_count, 1u)] = g * 32u + l;
                }
            }
            active &= ~finished;
        }
    }
    store_state<1>(x, planes, pitch, voff);
    staged_advance(g, blk, lane_out, lane_left, row_dst, row_cnt);
}

// Split staged quantum: the two-wave schedule of the plain path (wave 0: R words and the
// keystream, wave 1: S words).  Both waves see the same lane_left values throughout (the
// R wave changes them only after a final barrier), so they run the same blocks and the
// same number of barriers; each packs its own half of a finished lane's state.
__global__ __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2, 2))) void quantum_split_kernel(
    uint32_t *__restrict__ planes, uint32_t nslices, uint32_t nblocks, uint32_t **lane_out,
    uint32_t *__restrict__ lane_left, const uint32_t *__restrict__ lane_sid, uint8_t *__restrict__ pool,
    uint32_t *__restrict__ fresh, uint32_t *__restrict__ zplanes, uint32_t **row_dst, uint32_t *__restrict__ row_cnt,
    uint32_t *__restrict__ done_list, uint32_t *__restrict__ done_count)
{
    __shared__ SplitLds xl;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t g = blockIdx.x * 64u + lane;  // nslices is a multiple of 64
    uint32_t next_end;
    uint32_t active = scan_lanes(lane_left, g, next_end);
    if (!active) {  // both waves leave here, before any barrier
        if (wave == 0)
            for (int l = 0; l < 32; l++) row_cnt[g * 32u + l] = 0u;
        return;
    }
    const size_t pitch = (size_t)nslices * 4u;
    const uint32_t voff = g * 4u;
    const uint32_t fr0 = fresh[g];
    Regs<1> x;
    uint32_t blk = 0;
    if (wave == 0) {
#pragma unroll
        for (int j = 0; j < 100; j++) x.r[j] = ld_word<1>((const char *)planes + (size_t)j * pitch + voff);
        for (uint32_t fr = fr0; fr; fr &= fr - 1u) {
            const uint32_t l = (uint32_t)__builtin_ctz(fr);
            gather_lane<0, 100>(x, l, pool + 25ull * lane_sid[g * 32u + l]);
        }
        xl.r33[0][lane] = x.r[kRCut].w[0];
        lds_barrier();
        Word<1> s34 = {{xl.s34[0][lane]}}, s0 = {{xl.s0[0][lane]}};
        __builtin_amdgcn_sched_barrier(0);
        if (fr0) fresh[g] = 0u;  // both waves have read it (before the barrier)
        char *plane = (char *)zplanes;
        for (; blk < nblocks && active; blk++) {
            for (int b0 = 0; b0 < 32; b0 += kServeUnroll) {
#pragma unroll
                for (int u = 0; u < kServeUnroll; u++) {
                    store_plane<1>(plane, voff, x.r[0] ^ s0);
                    plane += pitch;
                    split_r_clock(x, s34, s0, xl, lane, (u + 1) & 1);
                }
            }
            if (blk + 1u == next_end) {
                const uint32_t finished = ending_lanes(lane_left, g, active, blk, next_end);
                for (uint32_t l = 0; l < 32; l++) {
                    if ((finished >> l) & 1u) {
                        write_back_range<0, 100>(x, l, pool + 25ull * lane_sid[g * 32u + l]);
                        done_list[atomicAdd(done_count, 1u)] = g * 32u + l;
                    }
                }
                active &= ~finished;
            }
        }
        lds_barrier();  // the S wave has read lane_left for the last time
        uint32_t v = voff;
        asm volatile("" : "+v"(v));
#pragma unroll
        for (int j = 0; j < 100; j++) st_word<1>((char *)planes + (size_t)j * pitch + v, x.r[j]);
        staged_advance(g, blk, lane_out, lane_left, row_dst, row_cnt);
    } else {
#pragma unroll
        for (int j = 0; j < 100; j++) x.s[j] = ld_word<1>((const char *)planes + (size_t)(100 + j) * pitch + voff);
        for (uint32_t fr = fr0; fr; fr &= fr - 1u) {
            const uint32_t l = (uint32_t)__builtin_ctz(fr);
            gather_lane<100, 200>(x, l, pool + 25ull * lane_sid[g * 32u + l]);
        }
        xl.s34[0][lane] = x.s[kSCut].w[0];
        xl.s0[0][lane] = x.s[0].w[0];
        lds_barrier();
        Word<1> r33 = {{xl.r33[0][lane]}};
        __builtin_amdgcn_sched_barrier(0);
        for (; blk < nblocks && active; blk++) {
            for (int b0 = 0; b0 < 32; b0 += kServeUnroll) {
#pragma unroll
                for (int u = 0; u < kServeUnroll; u++) split_s_clock(x, r33, xl, lane, (u + 1) & 1);
            }
            if (blk + 1u == next_end) {
                const uint32_t finished = ending_lanes(lane_left, g, active, blk, next_end);
                for (uint32_t l = 0; l < 32; l++)
                    if ((finished >> l) & 1u) write_back_range<100, 200>(x, l, pool + 25ull * lane_sid[g * 32u + l]);
                active &= ~finished;
            }
        }
        lds_barrier();
        uint32_t v = voff;
        asm volatile("" : "+v"(v));
#pragma unroll
        for (int j = 0; j < 100; j++) st_word<1>((char *)planes + (size_t)(100 + j) * pitch + v, x.s[j]);
    }
}

// Four-wave staged quantum: the four-wave split of the plain path (wave 0: r_0..r_49 and
// the keystream, wave 1: r_50..r_99, wave 2: s_0..s_49, wave 3: s_50..s_99) with the lane
// bookkeeping of quantum_split_kernel: every wave sees the same lane_left values (wave 0
// changes them only after a final barrier), so all four run the same blocks and pass the
// same barriers; each gathers and packs back its own quarter of a lane's state.
template <int ROLE>
__device__ __forceinline__ void serve4_run(uint32_t *__restrict__ planes, size_t pitch, uint32_t voff, uint32_t g,
                                           uint32_t lane, uint32_t nblocks, uint32_t active, uint32_t next_end,
                                           uint32_t fr0, uint32_t **lane_out, uint32_t *__restrict__ lane_left,
                                           const uint32_t *__restrict__ lane_sid, uint8_t *__restrict__ pool,
                                           uint32_t *__restrict__ fresh, uint32_t *__restrict__ zplanes,
                                           uint32_t **row_dst, uint32_t *__restrict__ row_cnt,
                                           uint32_t *__restrict__ done_list, uint32_t *__restrict__ done_count,
                                           Split4Lds &xl)
{
    constexpr bool kR = ROLE < 2;
    constexpr int j0 = ROLE == 0 || ROLE == 2 ? 0 : 50;  // first position of the quarter
    constexpr int base = kR ? 0 : 100;                  // r or s planes / packed bits
    constexpr int J0 = base + j0, J1 = J0 + 50;        // the quarter's packed bits
    Regs<1> x;
    S4In in;
#pragma unroll
    for (int j = 0; j < 50; j++) {
        const Word<1> v = ld_word<1>((const char *)planes + (size_t)(base + j0 + j) * pitch + voff);
        if constexpr (kR) x.r[j0 + j] = v;
        else x.s[j0 + j] = v;
    }
    for (uint32_t fr = fr0; fr; fr &= fr - 1u) {
        const uint32_t l = (uint32_t)__builtin_ctz(fr);
        gather_lane<J0, J1>(x, l, pool + 25ull * lane_sid[g * 32u + l]);
    }
    if constexpr (ROLE == 0) {
        xl.v[0][kX_R49][lane] = x.r[49].w[0];
        xl.v[0][kX_R33][lane] = x.r[33].w[0];
    } else if constexpr (ROLE == 1) {
        xl.v[0][kX_R99][lane] = x.r[99].w[0];
        xl.v[0][kX_R67][lane] = x.r[67].w[0];
    } else if constexpr (ROLE == 2) {
        xl.v[0][kX_S49][lane] = x.s[49].w[0];
        xl.v[0][kX_S34][lane] = x.s[34].w[0];
        xl.v[0][kX_S0][lane] = x.s[0].w[0];
    } else {
        xl.v[0][kX_S50][lane] = x.s[50].w[0];
        xl.v[0][kX_S99][lane] = x.s[99].w[0];
        xl.v[0][kX_S67][lane] = x.s[67].w[0];
    }
    lds_barrier();
    if constexpr (ROLE == 0) {
        in.a.w[0] = xl.v[0][kX_R99][lane];
        in.b.w[0] = xl.v[0][kX_R67][lane];
        in.c.w[0] = xl.v[0][kX_S34][lane];
        in.d.w[0] = xl.v[0][kX_S0][lane];
    } else if constexpr (ROLE == 1) {
        x.r[49].w[0] = xl.v[0][kX_R49][lane];
        in.a.w[0] = xl.v[0][kX_S34][lane];
    } else if constexpr (ROLE == 2) {
        x.s[50].w[0] = xl.v[0][kX_S50][lane];
        in.a.w[0] = xl.v[0][kX_S99][lane];
        in.b.w[0] = xl.v[0][kX_S67][lane];
        in.c.w[0] = xl.v[0][kX_R33][lane];
    } else {
        x.s[49].w[0] = xl.v[0][kX_S49][lane];
        in.a.w[0] = xl.v[0][kX_R33][lane];
    }
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (ROLE == 0) {
        if (fr0) fresh[g] = 0u;  // every wave read it before the barrier
    }
    char *plane = (char *)zplanes;  // wave-uniform (wave 0)
    uint32_t blk = 0;
    for (; blk < nblocks && active; blk++) {
        // the block's 32 clocks as 16 pairs (clock t writes exchange buffer (t + 1) & 1)
        s4_pairs<ROLE>(x, in, xl, lane, plane, voff, (uint32_t)pitch, 16u);
        plane += 32 * pitch;
        if (blk + 1u == next_end) {
            const uint32_t finished = ending_lanes(lane_left, g, active, blk, next_end);
            for (uint32_t l = 0; l < 32; l++) {
                if ((finished >> l) & 1u) {
                    write_back_range<J0, J1>(x, l, pool + 25ull * lane_sid[g * 32u + l]);
                    if constexpr (ROLE == 0) done_list[atomicAdd(done_count, 1u)] = g * 32u + l;
                }
            }
            active &= ~finished;
        }
    }
    lds_barrier();  // every wave has read lane_left for the last time
    uint32_t v = voff;
    asm volatile("" : "+v"(v));
#pragma unroll
    for (int j = 0; j < 50; j++) {
        if constexpr (kR) st_word<1>((char *)planes + (size_t)(base + j0 + j) * pitch + v, x.r[j0 + j]);
        else st_word<1>((char *)planes + (size_t)(base + j0 + j) * pitch + v, x.s[j0 + j]);
    }
    if constexpr (ROLE == 0) staged_advance(g, blk, lane_out, lane_left, row_dst, row_cnt);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 4))) void quantum_split4_kernel(
    uint32_t *__restrict__ planes, uint32_t nslices, uint32_t nblocks, uint32_t **lane_out,
    uint32_t *__restrict__ lane_left, const uint32_t *__restrict__ lane_sid, uint8_t *__restrict__ pool,
    uint32_t *__restrict__ fresh, uint32_t *__restrict__ zplanes, uint32_t **row_dst, uint32_t *__restrict__ row_cnt,
    uint32_t *__restrict__ done_list, uint32_t *__restrict__ done_count, uint32_t raise_prio)
{
    __shared__ Split4Lds xl;
    // beside a transpose kernel, these waves take issue slots first (every wave of a
    // workgroup waits at each clock's barrier for the slowest)
    if (raise_prio) __builtin_amdgcn_s_setprio(3);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t g = blockIdx.x * 64u + lane;  // nslices is a multiple of 64
    uint32_t next_end;
    const uint32_t active = scan_lanes(lane_left, g, next_end);
    if (!active) {  // all four waves leave here, before any barrier
        if (wave == 0)
            for (int l = 0; l < 32; l++) row_cnt[g * 32u + l] = 0u;
        return;
    }
    const size_t pitch = (size_t)nslices * 4u;
    const uint32_t voff = g * 4u;
    const uint32_t fr0 = fresh[g];
    if (wave == 0)
        serve4_run<0>(planes, pitch, voff, g, lane, nblocks, active, next_end, fr0, lane_out, lane_left, lane_sid,
                      pool, fresh, zplanes, row_dst, row_cnt, done_list, done_count, xl);
    else if (wave == 1)
        serve4_run<1>(planes, pitch, voff, g, lane, nblocks, active, next_end, fr0, lane_out, lane_left, lane_sid,
                      pool, fresh, zplanes, row_dst, row_cnt, done_list, done_count, xl);
    else if (wave == 2)
        serve4_run<2>(planes, pitch, voff, g, lane, nblocks, active, next_end, fr0, lane_out, lane_left, lane_sid,
                      pool, fresh, zplanes, row_dst, row_cnt, done_list, done_count, xl);
    else
        serve4_run<3>(planes, pitch, voff, g, lane, nblocks, active, next_end, fr0, lane_out, lane_left, lane_sid,
                      pool, fresh, zplanes, row_dst, row_cnt, done_list, done_count, xl);
}

// Rows of the staged quantum: lane i's row_cnt[i] words of the launch go to row_dst[i],
// tiles of 16 slices x 1024 clocks as in the plain path's staged transpose.  Tiles whose
// lanes have no word in the tile's clocks skip the plane reads.  The tile's 512 row
// destinations and counts are read once, beside the plane reads, into LDS, so the stores
// do not wait on a pointer load each.  Called by every thread of the workgroup.
__device__ __forceinline__ void serve_tile(uint32_t *lds, uint32_t **dsts, uint32_t *cnts,
                                           const uint32_t *__restrict__ zplanes, uint32_t nslices, uint32_t nclocks,
                                           uint32_t *const *row_dst, const uint32_t *__restrict__ row_cnt,
                                           uint32_t s0, uint32_t t0)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t w0 = t0 / 32u;
    const uint32_t nb = min((uint32_t)kTpBlocks, (nclocks - t0) / 32u);
    const uint32_t c0 = row_cnt[32u * s0 + tid], c1 = row_cnt[32u * s0 + tid + 256u];
    if (!__syncthreads_or(c0 > w0 || c1 > w0)) return;
    uint32_t *const d0 = row_dst[32u * s0 + tid], *const d1 = row_dst[32u * s0 + tid + 256u];
    tile_to_rows(lds, zplanes, nslices, s0, t0, nb, tid, [&] {
        cnts[tid] = c0;
        cnts[tid + 256u] = c1;
        dsts[tid] = d0;
        dsts[tid + 256u] = d1;
    });
    // four consecutive words of a row per thread (8 rows per store instruction) where the
    // row's destination is 16-byte aligned and holds all four, else one word at a time
    const uint32_t q = (tid & 7u) * 4u;
    if (q >= nb) return;
    for (uint32_t i = tid >> 3; i < 32u * kTpSlices; i += 32u) {
        const uint32_t cnt = cnts[i];
        if (w0 + q >= cnt) continue;
        uint32_t *const d = dsts[i] + w0 + q;
        if (q + 4u <= nb && w0 + q + 4u <= cnt && ((uintptr_t)d & 15u) == 0u) {
            u32x4 v;
            v.x = tile_row_word(lds, i, q);
            v.y = tile_row_word(lds, i, q + 1u);
            v.z = tile_row_word(lds, i, q + 2u);
            v.w = tile_row_word(lds, i, q + 3u);
            store_global_x4(d, v);
        } else {
            for (uint32_t k = 0; q + k < nb && w0 + q + k < cnt; k++) store_global(d + k, tile_row_word(lds, i, q + k));
        }
    }
}

// One workgroup per tile.
__global__ __launch_bounds__(256) void serve_transpose_kernel(const uint32_t *__restrict__ zplanes, uint32_t nslices,
                                                              uint32_t nclocks, uint32_t *const *row_dst,
                                                              const uint32_t *__restrict__ row_cnt)
{
    __shared__ uint32_t lds[kTpLdsWords];
    __shared__ uint32_t *dsts[32 * kTpSlices];
    __shared__ uint32_t cnts[32 * kTpSlices];
    const uint2 tb = tile_of_block();
    serve_tile(lds, dsts, cnts, zplanes, nslices, nclocks, row_dst, row_cnt, tb.x * kTpSlices, tb.y * kTpClocks);
}

// The same tiles (ntx slice tiles x nty clock tiles) taken by a fixed number of
// workgroups (a multiple of 8) that loop over them, to run beside the next launch's
// generate kernel with one workgroup on most CUs; workgroup g (on XCD g % 8) takes every
// (grid / 8)-th tile of its XCD's contiguous share.
__global__ __launch_bounds__(256) void serve_transpose_persistent_kernel(const uint32_t *__restrict__ zplanes,
                                                                         uint32_t nslices, uint32_t nclocks,
                                                                         uint32_t *const *row_dst,
                                                                         const uint32_t *__restrict__ row_cnt,
                                                                         uint32_t ntx, uint32_t nty)
{
    __shared__ uint32_t lds[kTpLdsWords];
    __shared__ uint32_t *dsts[32 * kTpSlices];
    __shared__ uint32_t cnts[32 * kTpSlices];
    constexpr uint32_t kXcds = 8;
    const uint32_t ntiles = ntx * nty;
    const uint32_t x = blockIdx.x % kXcds, per = gridDim.x / kXcds;
    const uint32_t hi = (uint32_t)((uint64_t)ntiles * (x + 1u) / kXcds);
    for (uint32_t l = (uint32_t)((uint64_t)ntiles * x / kXcds) + blockIdx.x / kXcds; l < hi; l += per) {
        serve_tile(lds, dsts, cnts, zplanes, nslices, nclocks, row_dst, row_cnt, (l % ntx) * kTpSlices,
                   (l / ntx) * kTpClocks);
        __syncthreads();  // the next tile reuses the LDS
    }
}

// Clear the completion counter (a kernel, so that the sequence stays capturable).
__global__ void reset_count_kernel(uint32_t *c)
{
    if (threadIdx.x == 0) *c = 0u;
}

// Copy the completion counter to the host's mapped word (a system-scope store, seen by the
// host once the event after this kernel has completed).
__global__ void publish_count_kernel(const uint32_t *c, uint32_t *host)
{
    if (threadIdx.x == 0) __hip_atomic_store(host, *c, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The request owning state sid is done: the next request waiting on it (if any) becomes
// ready, otherwise the state is free.
void pass_state(mickey_server *s, uint32_t sid)
{
    const uint64_t nx = s->chain_head[sid];
    if (nx == ~0ull) {
        s->state_owned[sid] = 0;
        return;
    }
    s->chain_head[sid] = s->reqs[nx].next_same;
    if (s->chain_head[sid] == ~0ull) s->chain_tail[sid] = ~0ull;
    s->chained--;
    s->ready_q.push(nx);
}

// Size-aware routing: up to `streams` latency streams, for requests with at least
// threshold_bits left; each stream runs clocks_per_quantum clocks per quantum.
void set_latency(mickey_server *s, uint32_t streams, uint64_t threshold_bits, uint64_t clocks_per_quantum)
{
    s->lat_streams = streams;
    s->lat_threshold_words = (threshold_bits + 31) / 32;
    s->lat_words = (uint32_t)(clocks_per_quantum / 32);
    s->lat_free.clear();
    for (uint32_t k = streams; k-- > 0;) s->lat_free.push_back(k);  // lowest index first
}

// Chunk-block cache of a lane: its slice's, or one shared by the latency streams.
uint32_t cache_index(const mickey_server *s, uint32_t lane)
{
    return lane < s->nlanes ? lane / 32u : (uint32_t)s->nslices;
}

// Wait for the oldest in-flight quantum and retire the requests it completed.
int retire_oldest(mickey_server *s)
{
    if (s->oldest_q == s->next_q) return MICKEY_OK;
    const int b = (int)(s->oldest_q & 1);
    const uint64_t tw = now_ns();
    hipError_t e = hipEventSynchronize(s->ev[b]);
    s->oldest_q++;
    if (e != hipSuccess) return fail(MICKEY_EDEVICE, "quantum: %s", hipGetErrorString(e));
    const uint64_t t1 = now_ns();
    s->ns_wait += t1 - tw;
    s->quanta_ns += t1 - s->launch_ns[b];
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s->ev_start[b], s->ev[b]) == hipSuccess) s->ns_gpu += (uint64_t)(ms * 1e6f);
    const uint32_t ndone = s->hcount[b];
    const uint32_t *list = s->hlist + (size_t)b * (s->nlanes + kLatStreams);
    // the loop's reads are spread over tables of 10^6 entries (lane -> request -> state), so
    // it fetches each level a few completions ahead instead of waiting on every miss
    constexpr uint32_t kAhead = 8;
    for (uint32_t k = 0; k < ndone; k++) {
        if (k + 3 * kAhead < ndone) __builtin_prefetch(&s->lane_req[list[k + 3 * kAhead]]);
        if (k + 2 * kAhead < ndone) {
            const char *q = (const char *)&s->reqs[s->lane_req[list[k + 2 * kAhead]]];
            __builtin_prefetch(q, 1);
            __builtin_prefetch(q + 64, 1);
        }
        if (k + kAhead < ndone) __builtin_prefetch(&s->state_bits[s->reqs[s->lane_req[list[k + kAhead]]].sid], 1);
        const uint32_t lane = list[k];
        Request &r = s->reqs[s->lane_req[lane]];
        s->lane_req[lane] = ~0ull;
        if (lane < s->nlanes) {
            s->free_lanes.push_back(lane);
        } else {
            s->lat_free.push_back(lane - (uint32_t)s->nlanes);
            s->lat_busy--;
        }
        r.lane = kNoRequest;
        r.words_done += r.cur_words;
        s->state_bits[r.sid] += 32ull * r.cur_words;
        s->bits_done += 32ull * r.cur_words;
        if (!r.first_ns) r.first_ns = t1;
        const bool last = r.words_done == r.nbits / 32;
        if (r.chunk_words) {
            uint64_t h;
            if (!s->free_slots.empty()) {
                h = s->free_slots.back();
                s->free_slots.pop_back();
            } else {
                h = s->slots.size();
                s->slots.emplace_back();
            }
            s->slots[h] = ChunkSlot{r.out_off, r.out_granted, r.cur_words, cache_index(s, lane), true};
            s->ready.push_back(mickey_chunk{r.id, h, r.words_done - r.cur_words, r.cur_words, s->arena + r.out_off,
                                            last ? 1ull : 0ull});
        }
        r.cur_words = 0;
        if (!last) {
            s->continuing.push_back(r.id);  // the state stays reserved for this request
            continue;
        }
        r.done = true;
        r.done_ns = t1;
        s->completed.push_back(r.id);
        s->finished++;
        pass_state(s, r.sid);
    }
    s->ns_retire += now_ns() - t1;
    return MICKEY_OK;
}

// Admit the next part of request r (its whole output, or its next chunk) into a free lane
// if a lane and the budget allow; false if either is full.
bool admit_next(mickey_server *s, Request &r, uint64_t t_admit)
{
    const uint64_t left = r.nbits / 32 - r.words_admitted;
    const uint32_t words = r.chunk_words ? (uint32_t)std::min<uint64_t>(left, r.chunk_words) : (uint32_t)left;
    // a chunk always reserves a whole chunk, so that chunk blocks share one size class
    const size_t reserve = r.chunk_words ? r.chunk_words : words;
    // size-aware routing: what is left of a long request takes a latency stream if one is free
    // (only while the bit lanes are at most half busy: a latency stream costs ~5x the
    // device work per bit, which a full launch of bit lanes cannot spare)
    const bool lat = s->lat_streams && left >= s->lat_threshold_words && !s->lat_free.empty() &&
                     2 * s->free_lanes.size() >= s->nlanes;
    if (!lat && s->free_lanes.empty()) return false;
    const uint32_t lane = lat ? (uint32_t)s->nlanes + s->lat_free.back() : s->free_lanes.back();
    size_t off = 0, granted = 0;
    auto &cache = s->slice_blocks[cache_index(s, lane)];
    const size_t cls_words = serve_arena::Arena::class_words(serve_arena::Arena::cls(reserve));
    if (r.chunk_words && !cache.empty() && cache.back().second == cls_words) {
        off = cache.back().first;
        granted = cache.back().second;
        cache.pop_back();
        s->slice_cached -= granted;
    } else if (!s->alloc.alloc(reserve, &off, &granted)) {
        if (!s->slice_cached) return false;
        for (auto &c : s->slice_blocks) {  // give every cached block back and retry once
            for (auto &b : c) s->alloc.release(b.first, b.second);
            c.clear();
        }
        s->slice_cached = 0;
        if (!s->alloc.alloc(reserve, &off, &granted)) return false;
    }
    if (lat) {
        s->lat_free.pop_back();
        s->lat_busy++;
        r.lat_words += words;
    } else {
        s->free_lanes.pop_back();
    }
    r.lane = lane;
    r.out_off = off;
    r.out_granted = granted;
    r.cur_words = words;
    r.words_admitted += words;
    if (!r.admit_ns) r.admit_ns = t_admit;
    s->lane_req[lane] = r.id;
    s->hadm[s->pending++] = Admit{lane, r.sid, words, 0u, s->arena + off};
    s->admitted++;
    return true;
}

// Decide admissions into s->hadm (enqueued by the next step): first the chunked requests
// that are between two chunks (oldest first), then ready requests in arrival order, while
// lanes and budget last.  Each request considered is admitted, refused (2^40 bits) or
// left for later, so the cost is proportional to the admissions.
void decide_admissions(mickey_server *s)
{
    const uint64_t t_admit = now_ns();
    bool full = false;
    constexpr size_t kAhead = 8;
    while (!s->continuing.empty()) {
        // prefetch a few admissions ahead: the request, and the block cache of the lane it
        // will take (the free lanes are taken from the back)
        if (s->continuing.size() > kAhead) {
            const char *q = (const char *)&s->reqs[s->continuing[kAhead]];
            __builtin_prefetch(q, 1);
            __builtin_prefetch(q + 64, 1);
        }
        const size_t nf = s->free_lanes.size();
        if (nf > 2 * kAhead) __builtin_prefetch(&s->slice_blocks[cache_index(s, s->free_lanes[nf - 1 - 2 * kAhead])]);
        if (nf > kAhead) {
            const uint32_t l = s->free_lanes[nf - 1 - kAhead];
            const auto &c = s->slice_blocks[cache_index(s, l)];
            if (!c.empty()) __builtin_prefetch(&c.back());
            __builtin_prefetch(&s->lane_req[l], 1);
        }
        if (!admit_next(s, s->reqs[s->continuing.front()], t_admit)) {
            full = true;
            break;
        }
        s->continuing.pop_front();
    }
    while (!full && !s->ready_q.empty()) {
        Request &r = s->reqs[s->ready_q.top()];
        if (s->state_bits[r.sid] + r.nbits > MICKEY_MAX_BITS_PER_IV) {  // 2^40 per key/IV pair
            s->ready_q.pop();
            r.done = true;
            r.refused = true;
            r.done_ns = t_admit;
            s->completed.push_back(r.id);
            pass_state(s, r.sid);
            continue;
        }
        if (!admit_next(s, r, t_admit)) break;  // slots or budget full
        s->ready_q.pop();
    }
    s->ns_admit += now_ns() - t_admit;
}

}  // namespace

extern "C" {

mickey_server *mickey_server_create(const mickey_state *init, size_t nslices, uint32_t quantum_clocks,
                                    uint64_t budget_bytes, void *hip_stream)
{
    if (!init) {
        fail(MICKEY_EINVAL, "mickey_server_create: NULL initial states");
        return nullptr;
    }
    if (nslices == 0 || nslices > ((size_t)1 << 24) || quantum_clocks == 0 || quantum_clocks % 32 ||
        budget_bytes < 4) {
        fail(MICKEY_EINVAL, "mickey_server_create: bad slots, quantum (multiple of 32) or budget");
        return nullptr;
    }
    mickey_server *s = new (std::nothrow) mickey_server();
    if (!s) {
        fail(MICKEY_ENOMEM, "mickey_server_create: host allocation failed");
        return nullptr;
    }
    s->nstates = mickey_num_instances(init);
    s->nslices = (nslices + 63) / 64 * 64;
    s->nlanes = s->nslices * 32;
    s->qblocks = quantum_clocks / 32;
    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
    } else if (hipStreamCreate(&s->stream) == hipSuccess) {
        s->own_stream = true;
    } else {
        delete s;
        fail(MICKEY_EDEVICE, "mickey_server_create: cannot create a stream");
        return nullptr;
    }
    const size_t budget_words = budget_bytes / 4;
    // Staged quanta: launches of up to 512 MiB of planes, in whole 1024-clock transpose
    // tiles when a launch holds at least one.
    {
        const uint64_t plane_bytes = s->nslices * 4;
        uint64_t sub = std::min<uint64_t>(quantum_clocks, (512ull << 20) / plane_bytes / 32 * 32);
        if (sub >= 1024 && sub < quantum_clocks) sub = sub / 1024 * 1024;
        s->sub_blocks = (uint32_t)(sub / 32);
    }
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            s->simds = 4 * cus;
        (void)hipGetLastError();
    }
    bool okm = (s->sub_blocks == 0 ||
                (hipMalloc(&s->zplanes[0], (size_t)s->sub_blocks * 32 * s->nslices * 4) == hipSuccess &&
                 hipMalloc(&s->zplanes[1], (size_t)s->sub_blocks * 32 * s->nslices * 4) == hipSuccess &&
                 hipMalloc(&s->row_dst[0], s->nlanes * sizeof(uint32_t *)) == hipSuccess &&
                 hipMalloc(&s->row_dst[1], s->nlanes * sizeof(uint32_t *)) == hipSuccess &&
                 hipMalloc(&s->row_cnt[0], s->nlanes * 4) == hipSuccess &&
                 hipMalloc(&s->row_cnt[1], s->nlanes * 4) == hipSuccess)) &&
               hipStreamCreateWithFlags(&s->tstream, hipStreamNonBlocking) == hipSuccess &&
               hipEventCreateWithFlags(&s->ev_sub[0], hipEventDisableTiming) == hipSuccess &&
               hipEventCreateWithFlags(&s->ev_sub[1], hipEventDisableTiming) == hipSuccess &&
               hipEventCreateWithFlags(&s->ev_tdone[0], hipEventDisableTiming) == hipSuccess &&
               hipEventCreateWithFlags(&s->ev_tdone[1], hipEventDisableTiming) == hipSuccess &&
               hipEventCreateWithFlags(&s->ev_qend, hipEventDisableTiming) == hipSuccess &&
               hipMalloc(&s->pool, 25 * s->nstates) == hipSuccess &&
               hipMalloc(&s->planes, 200 * s->nslices * 4) == hipSuccess &&
               hipMalloc(&s->lane_out, s->nlanes * sizeof(uint32_t *)) == hipSuccess &&
               hipMalloc(&s->lane_left, s->nlanes * 4) == hipSuccess &&
               hipMalloc(&s->lane_sid, s->nlanes * 4) == hipSuccess &&
               hipMalloc(&s->fresh, s->nslices * 4) == hipSuccess &&
               hipMalloc(&s->sink, s->nslices * 4) == hipSuccess &&
               hipMalloc(&s->done_list, 256) == hipSuccess &&
               hipMalloc(&s->lat_state, kLatStreams * 8 * 4) == hipSuccess &&
               hipMalloc(&s->lat_out, kLatStreams * sizeof(uint32_t *)) == hipSuccess &&
               hipMalloc(&s->lat_left, kLatStreams * 4) == hipSuccess &&
               hipMalloc(&s->lat_sid, kLatStreams * 4) == hipSuccess &&
               hipMalloc(&s->lat_fresh, kLatStreams * 4) == hipSuccess &&
               hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking) == hipSuccess &&
               hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming) == hipSuccess &&
               hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming) == hipSuccess &&
               hipMalloc(&s->arena, budget_words * 4) == hipSuccess &&
               hipHostMalloc((void **)&s->hadm_buf[0], (s->nlanes + kLatStreams) * sizeof(Admit),
                             hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
               hipHostGetDevicePointer((void **)&s->hadm_dev[0], s->hadm_buf[0], 0) == hipSuccess &&
               hipHostMalloc((void **)&s->hadm_buf[1], (s->nlanes + kLatStreams) * sizeof(Admit),
                             hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
               hipHostGetDevicePointer((void **)&s->hadm_dev[1], s->hadm_buf[1], 0) == hipSuccess &&
               hipHostMalloc((void **)&s->hcount, 64, hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
               hipHostGetDevicePointer((void **)&s->hcount_dev, s->hcount, 0) == hipSuccess &&
               hipHostMalloc((void **)&s->hlist, 2 * (s->nlanes + kLatStreams) * 4, hipHostMallocMapped) == hipSuccess &&
               hipHostGetDevicePointer((void **)&s->hlist_dev, s->hlist, 0) == hipSuccess &&
               hipEventCreate(&s->ev[0]) == hipSuccess && hipEventCreate(&s->ev[1]) == hipSuccess &&
               hipEventCreate(&s->ev_start[0]) == hipSuccess && hipEventCreate(&s->ev_start[1]) == hipSuccess;
    s->hadm = s->hadm_buf[0];
    if (!okm) {
        (void)hipGetLastError();
        destroy(s);
        fail(MICKEY_ENOMEM, "mickey_server_create: cannot allocate the pool, slots or %llu-byte budget",
             (unsigned long long)budget_bytes);
        return nullptr;
    }
    s->done_count = s->done_list;  // device words [2]: completions of each in-flight quantum
    // the initial states: the registers of the given initialised instances
    int rc = mickey_state_export(init, s->pool, nullptr);
    if (rc == MICKEY_OK && (hipMemsetAsync(s->lane_left, 0, s->nlanes * 4) != hipSuccess ||
                            hipMemsetAsync(s->lat_left, 0, kLatStreams * 4) != hipSuccess ||
                            hipMemsetAsync(s->lat_fresh, 0, kLatStreams * 4) != hipSuccess ||
                            hipMemsetAsync(s->fresh, 0, s->nslices * 4) != hipSuccess ||
                            hipMemsetAsync(s->planes, 0, 200 * s->nslices * 4) != hipSuccess ||
                            hipDeviceSynchronize() != hipSuccess))
        rc = check_launch("mickey_server_create");
    if (rc != MICKEY_OK) {
        destroy(s);
        prefix_error("mickey_server_create");
        return nullptr;
    }
    s->alloc.reset(budget_words);
    s->slice_blocks.assign(s->nslices + 1, {});  // + the latency streams' cache
    s->state_bits.assign(s->nstates, mickey_bits_generated(init));
    s->state_owned.assign(s->nstates, 0);
    s->chain_head.assign(s->nstates, ~0ull);
    s->chain_tail.assign(s->nstates, ~0ull);
    s->free_lanes.resize(s->nlanes);
    for (size_t i = 0; i < s->nlanes; i++) s->free_lanes[i] = (uint32_t)(s->nlanes - 1 - i);
    s->lane_req.assign(s->nlanes + kLatStreams, ~0ull);
    set_latency(s, kLatStreams, 1ull << 20, 8ull * quantum_clocks);
    ok();
    return s;
}

int64_t mickey_server_submit(mickey_server *s, uint32_t state_id, uint64_t nbits)
{
    if (!s) return fail(MICKEY_EINVAL, "mickey_server_submit: NULL server");
    if (state_id >= s->nstates) return fail(MICKEY_EINVAL, "mickey_server_submit: state %u out of range", state_id);
    if (nbits == 0 || nbits % 32 || nbits > MICKEY_MAX_BITS_PER_IV)
        return fail(MICKEY_EINVAL, "mickey_server_submit: nbits must be k*32 with 0 < k, at most 2^40");
    if (!s->chunk_words && (nbits / 32 > s->alloc.capacity || nbits / 32 > 0xffffffffull))
        return fail(MICKEY_EINVAL,
                    "mickey_server_submit: a whole-request output must fit the budget and 2^32 words "
                    "(use chunked delivery)");
    Request r;
    r.id = s->reqs.size();
    r.sid = state_id;
    r.nbits = nbits;
    r.chunk_words = s->chunk_words;
    r.arrival_ns = now_ns();
    s->reqs.push_back(r);
    if (!s->state_owned[state_id]) {
        s->state_owned[state_id] = 1;
        s->ready_q.push(r.id);
    } else {  // behind the state's current request
        if (s->chain_tail[state_id] == ~0ull)
            s->chain_head[state_id] = r.id;
        else
            s->reqs[s->chain_tail[state_id]].next_same = r.id;
        s->chain_tail[state_id] = r.id;
        s->chained++;
    }
    ok();
    return (int64_t)r.id;
}

// The quantum's kernels.  Staged (planes, then rows) unless staging is unavailable or
// the fused path was asked for; within staged, the split schedule while the one-wave
// kernel would have at most one wave per SIMD (the plain path's rule).
int launch_quantum(mickey_server *s, int b, bool lat_beside)
{
    const bool staged = s->sub_blocks && s->transpose != MICKEY_TRANSPOSE_FUSED;
    uint32_t *const list = s->hlist_dev + (size_t)b * (s->nlanes + kLatStreams);
    if (!staged) {
        hipLaunchKernelGGL(quantum_kernel, dim3((unsigned)(s->nslices / 64)), dim3(64), 0, s->stream, s->planes,
                           (uint32_t)s->nslices, s->qblocks, s->lane_out, s->lane_left, s->lane_sid, s->pool,
                           s->fresh, s->sink, list, s->done_count + b);
        return check_launch("quantum_kernel");
    }
    // the plain path's rule: the four-wave split below two one-wave waves per SIMD
    const bool split4 = s->schedule == MICKEY_SCHED_SPLIT4 ||
                        (s->schedule == MICKEY_SCHED_AUTO && s->nslices / 64 < 2 * (size_t)s->simds);
    const bool split = s->schedule == MICKEY_SCHED_SPLIT;
    // Launch j generates into buffer j & 1 on the server's stream; its rows are written on
    // tstream, beside launch j + 1 (the next quantum's first launch, for a quantum's last).
    // Beside the four-wave split the transposes run persistent on 7/8 of the CUs and the
    // generator's waves at raised priority (as on the plain staged path).  When latency
    // streams run beside the quantum, their kernel sets the pace and would lose issue slots
    // to both: the transposes then follow each launch on the server's stream.
    const unsigned tp_wgs = lat_beside ? 0u : (unsigned)(s->simds / 4 * 7 / 8) / 8 * 8;
    hipStream_t const ts = lat_beside ? s->stream : s->tstream;
    for (uint32_t b0 = 0; b0 < s->qblocks; b0 += s->sub_blocks) {
        const uint32_t nb = std::min(s->sub_blocks, s->qblocks - b0);
        const int k = (int)(s->sub_seq & 1);
        // the buffer's previous transpose has read it
        if (s->tdone_rec[k] && hipStreamWaitEvent(s->stream, s->ev_tdone[k], 0) != hipSuccess)
            return check_launch("staged buffer wait");
        uint32_t *const zp = s->zplanes[k];
        uint32_t **const rd = s->row_dst[k];
        uint32_t *const rcnt = s->row_cnt[k];
        if (split4)
            hipLaunchKernelGGL(quantum_split4_kernel, dim3((unsigned)(s->nslices / 64)), dim3(256), 0, s->stream,
                               s->planes, (uint32_t)s->nslices, nb, s->lane_out, s->lane_left, s->lane_sid, s->pool,
                               s->fresh, zp, rd, rcnt, list, s->done_count + b, (uint32_t)(tp_wgs > 0));
        else if (split)
            hipLaunchKernelGGL(quantum_split_kernel, dim3((unsigned)(s->nslices / 64)), dim3(128), 0, s->stream,
                               s->planes, (uint32_t)s->nslices, nb, s->lane_out, s->lane_left, s->lane_sid, s->pool,
                               s->fresh, zp, rd, rcnt, list, s->done_count + b);
        else
            hipLaunchKernelGGL(quantum_planes_kernel, dim3((unsigned)(s->nslices / 64)), dim3(64), 0, s->stream,
                               s->planes, (uint32_t)s->nslices, nb, s->lane_out, s->lane_left, s->lane_sid, s->pool,
                               s->fresh, zp, rd, rcnt, list, s->done_count + b);
        int rc = check_launch("quantum kernel");
        if (rc != MICKEY_OK) return rc;
        s->sub_seq++;
        if (ts != s->stream && (hipEventRecord(s->ev_sub[k], s->stream) != hipSuccess ||
                                hipStreamWaitEvent(ts, s->ev_sub[k], 0) != hipSuccess))
            return check_launch("staged launch event");
        const dim3 grid((unsigned)(s->nslices / kTpSlices), (nb * 32 + kTpClocks - 1) / kTpClocks);
        if (split4 && tp_wgs > 0)
            hipLaunchKernelGGL(serve_transpose_persistent_kernel, dim3(tp_wgs), dim3(256), 0, ts, zp,
                               (uint32_t)s->nslices, nb * 32, rd, rcnt, grid.x, grid.y);
        else
            hipLaunchKernelGGL(serve_transpose_kernel, grid, dim3(256), 0, ts, zp, (uint32_t)s->nslices, nb * 32,
                               rd, rcnt);
        rc = check_launch("serve_transpose_kernel");
        if (rc != MICKEY_OK) return rc;
        if (hipEventRecord(s->ev_tdone[k], ts) != hipSuccess) return check_launch("staged transpose event");
        s->tdone_rec[k] = true;
    }
    return MICKEY_OK;
}

int mickey_server_step(mickey_server *s)
{
    if (!s) return fail(MICKEY_EINVAL, "mickey_server_step: NULL server");
    int rc = MICKEY_OK;
    if (s->oldest_q == s->next_q) decide_admissions(s);  // idle: admit before launching
    // 1. gather the admissions decided last time (stream-ordered after the quanta in flight)
    if (s->pending) {
        // the kernel reads this buffer when the stream reaches it, after the quantum in
        // flight, which the host does not wait for before deciding the next admissions: they
        // go to the other buffer, whose reader preceded that quantum
        const Admit *adm = s->hadm_dev[s->adm_b];
        s->adm_b ^= 1;
        s->hadm = s->hadm_buf[s->adm_b];
        hipLaunchKernelGGL(admit_kernel, dim3((s->pending + 255) / 256), dim3(256), 0, s->stream, adm,
                           s->pending, (uint32_t)s->nlanes, s->lane_out, s->lane_left, s->lane_sid, s->fresh,
                           s->lat_out, s->lat_left, s->lat_sid, s->lat_fresh);
        rc = check_launch("admit_kernel");
        if (rc != MICKEY_OK) return rc;
        s->pending = 0;
    }
    // 2. launch the next quantum when any lane is occupied: the latency streams on the side
    //    stream (forked after the admissions, joined before the completion count is read),
    //    the bitsliced lanes on the server's stream, side by side
    const bool any_bs = s->free_lanes.size() < s->nlanes, any_lat = s->lat_busy > 0;
    if (any_bs || any_lat) {
        const int b = (int)(s->next_q & 1);
        // quantum next_q - 2 published this completion buffer's count on tstream
        if (s->next_q >= 2 && hipStreamWaitEvent(s->stream, s->ev[b], 0) != hipSuccess)
            return check_launch("completion buffer wait");
        if (hipEventRecord(s->ev_start[b], s->stream) != hipSuccess) return check_launch("quantum start");
        hipLaunchKernelGGL(reset_count_kernel, dim3(1), dim3(64), 0, s->stream, s->done_count + b);
        rc = check_launch("reset_count_kernel");
        if (rc != MICKEY_OK) return rc;
        s->launch_ns[b] = now_ns();
        if (any_lat) {
            const uint32_t n = s->lat_streams;
            if (hipEventRecord(s->ev_fork, s->stream) != hipSuccess ||
                hipStreamWaitEvent(s->side, s->ev_fork, 0) != hipSuccess)
                return check_launch("latency fork");
            hipLaunchKernelGGL(latency_quantum_kernel, dim3((n * 4 + 63) / 64), dim3(64), 0, s->side, s->lat_state, n,
                               s->lat_words, s->lat_out, s->lat_left, s->lat_sid, s->lat_fresh, s->pool,
                               (uint32_t)s->nlanes, s->hlist_dev + (size_t)b * (s->nlanes + kLatStreams),
                               s->done_count + b);
            rc = check_launch("latency_quantum_kernel");
            if (rc != MICKEY_OK) return rc;
            if (hipEventRecord(s->ev_join, s->side) != hipSuccess) return check_launch("latency join");
        }
        if (any_bs) {
            rc = launch_quantum(s, b, any_lat);
            if (rc != MICKEY_OK) return rc;
        }
        if (any_lat && hipStreamWaitEvent(s->stream, s->ev_join, 0) != hipSuccess) return check_launch("latency join");
        // the completion count goes out on tstream, after the quantum's last transpose and
        // its last kernel on the server's stream, so the next quantum's kernels need not
        // wait for that transpose
        if (hipEventRecord(s->ev_qend, s->stream) != hipSuccess ||
            hipStreamWaitEvent(s->tstream, s->ev_qend, 0) != hipSuccess)
            return check_launch("quantum end");
        hipLaunchKernelGGL(publish_count_kernel, dim3(1), dim3(64), 0, s->tstream, s->done_count + b, s->hcount_dev + b);
        rc = check_launch("publish_count_kernel");
        if (rc != MICKEY_OK) return rc;
        if (hipEventRecord(s->ev[b], s->tstream) != hipSuccess) return check_launch("completion count");
        s->next_q++;
        s->steps++;
    }
    // 3. retire the previous quantum while this one runs (or the last one, if idle), then
    //    decide what the lanes it freed take next
    if (s->next_q - s->oldest_q >= 2 ||
        (s->next_q > s->oldest_q && s->free_lanes.size() == s->nlanes && s->lat_busy == 0)) {
        rc = retire_oldest(s);
        if (rc != MICKEY_OK) return rc;
    }
    decide_admissions(s);
    return ok();
}

// Wait for every quantum in flight and retire its requests (no new work is started).
int mickey_server_wait(mickey_server *s)
{
    if (!s) return fail(MICKEY_EINVAL, "mickey_server_wait: NULL server");
    while (s->oldest_q != s->next_q) {
        int rc = retire_oldest(s);
        if (rc != MICKEY_OK) return rc;
    }
    return ok();
}

// Many submissions at once: ids[k] receives the id of (sids[k], nbits[k]), or a negative
// error code for that entry.  Returns MICKEY_OK, or the first error code.
int mickey_server_submit_many(mickey_server *s, const uint32_t *sids, const uint64_t *nbits, size_t n,
                              int64_t *ids)
{
    if (!s || (n && (!sids || !nbits || !ids))) return fail(MICKEY_EINVAL, "mickey_server_submit_many: bad argument");
    int first = MICKEY_OK;
    for (size_t k = 0; k < n; k++) {
        ids[k] = mickey_server_submit(s, sids[k], nbits[k]);
        if (ids[k] < 0 && first == MICKEY_OK) first = (int)ids[k];
    }
    return first == MICKEY_OK ? ok() : first;
}

// Release many completed requests; returns MICKEY_OK or the first error code.
int mickey_server_release_many(mickey_server *s, const uint64_t *ids, size_t n)
{
    if (!s || (n && !ids)) return fail(MICKEY_EINVAL, "mickey_server_release_many: bad argument");
    int first = MICKEY_OK;
    for (size_t k = 0; k < n; k++) {
        const int rc = mickey_server_release(s, ids[k]);
        if (rc != MICKEY_OK && first == MICKEY_OK) first = rc;
    }
    return first == MICKEY_OK ? ok() : first;
}

// Times of many completed requests: out[3k..3k+2] = arrival, admission, completion (ns);
// refused requests get completion = 0.
int mickey_server_times_many(const mickey_server *s, const uint64_t *ids, size_t n, uint64_t *out)
{
    if (!s || (n && (!ids || !out))) return fail(MICKEY_EINVAL, "mickey_server_times_many: bad argument");
    for (size_t k = 0; k < n; k++) {
        if (ids[k] >= s->reqs.size() || !s->reqs[ids[k]].done)
            return fail(MICKEY_EINVAL, "mickey_server_times_many: request %llu not complete",
                        (unsigned long long)ids[k]);
        const Request &r = s->reqs[ids[k]];
        out[3 * k] = r.arrival_ns;
        out[3 * k + 1] = r.admit_ns;
        out[3 * k + 2] = r.refused ? 0 : r.done_ns;
    }
    return ok();
}

// Completed request ids since the last call (up to cap); returns how many were written.
int mickey_server_latency_words_many(const mickey_server *s, const uint64_t *ids, size_t n, uint64_t *out)
{
    if (!s || (n && (!ids || !out))) return fail(MICKEY_EINVAL, "mickey_server_latency_words_many: bad argument");
    for (size_t k = 0; k < n; k++) {
        if (ids[k] >= s->reqs.size())
            return fail(MICKEY_EINVAL, "mickey_server_latency_words_many: no request %llu",
                        (unsigned long long)ids[k]);
        out[k] = s->reqs[ids[k]].lat_words;
    }
    return ok();
}

int64_t mickey_server_poll(mickey_server *s, uint64_t *ids, size_t cap)
{
    if (!s || (!ids && cap)) return fail(MICKEY_EINVAL, "mickey_server_poll: bad argument");
    const size_t n = std::min(cap, s->completed.size());
    std::copy(s->completed.begin(), s->completed.begin() + n, ids);
    s->completed.erase(s->completed.begin(), s->completed.begin() + n);
    ok();
    return (int64_t)n;
}

// Result of a completed request: device pointer to its nbits/32 words (NULL if it was
// rejected for passing 2^40 bits), its timestamps (ns, steady clock) and status.
int mickey_server_result(const mickey_server *s, uint64_t id, uint32_t **out, uint64_t times_ns[3])
{
    if (!s || id >= s->reqs.size()) return fail(MICKEY_EINVAL, "mickey_server_result: unknown request");
    const Request &r = s->reqs[id];
    if (!r.done) return fail(MICKEY_EINVAL, "mickey_server_result: request %llu not complete", (unsigned long long)id);
    if (r.released) return fail(MICKEY_EINVAL, "mickey_server_result: request %llu was released", (unsigned long long)id);
    if (out) *out = r.refused || r.chunk_words ? nullptr : s->arena + r.out_off;
    if (times_ns) {
        times_ns[0] = r.arrival_ns;
        times_ns[1] = r.admit_ns;
        times_ns[2] = r.done_ns;
    }
    if (r.refused) return fail(MICKEY_ERANGE, "request %llu would pass 2^40 bits", (unsigned long long)id);
    if (r.chunk_words && out)
        return fail(MICKEY_EINVAL, "mickey_server_result: request %llu was delivered in chunks",
                    (unsigned long long)id);
    return ok();
}

// Give a completed request's output space back to the budget.
int mickey_server_release(mickey_server *s, uint64_t id)
{
    if (!s || id >= s->reqs.size()) return fail(MICKEY_EINVAL, "mickey_server_release: unknown request");
    Request &r = s->reqs[id];
    if (!r.done || r.refused || r.released || r.chunk_words)
        return fail(MICKEY_EINVAL, "mickey_server_release: nothing to release");
    s->alloc.release(r.out_off, r.out_granted);
    r.released = true;
    return ok();
}

// Counters: [0] waiting (with chunked requests between two chunks), [1] running,
// [2] admitted, [3] finished, [4] steps,
// [5] total quantum time (ns, launch to retirement), [6] keystream bits delivered,
// [7] free budget words, [8] host ns blocked on quanta, [9] host ns retiring,
// [10] host ns deciding admissions, [11] device ns of the quanta.
int mickey_server_stats(const mickey_server *s, uint64_t out[12])
{
    if (!s || !out) return fail(MICKEY_EINVAL, "mickey_server_stats: bad argument");
    const size_t freew = s->alloc.free_words() + s->slice_cached;
    out[0] = s->ready_q.size() + s->chained + s->continuing.size();
    out[1] = s->nlanes - s->free_lanes.size() + s->lat_busy;
    out[2] = s->admitted;
    out[3] = s->finished;
    out[4] = s->steps;
    out[5] = s->quanta_ns;
    out[6] = s->bits_done;
    out[7] = freew;
    out[8] = s->ns_wait;
    out[9] = s->ns_retire;
    out[10] = s->ns_admit;
    out[11] = s->ns_gpu;
    return ok();
}

// Packed registers of resident state `sid` (25 bytes, device) and its bit counter.
int mickey_server_state(const mickey_server *s, uint32_t sid, const uint8_t **packed, uint64_t *bits)
{
    if (!s || sid >= s->nstates) return fail(MICKEY_EINVAL, "mickey_server_state: bad state");
    if (packed) *packed = s->pool + 25ull * sid;
    if (bits) *bits = s->state_bits[sid];
    return ok();
}

// Copy the first nwords words of a completed request's output into dst (device);
// synchronous.
int mickey_server_copy(const mickey_server *s, uint64_t id, uint32_t *dst, uint64_t nwords)
{
    uint32_t *src = nullptr;
    int rc = mickey_server_result(s, id, &src, nullptr);
    if (rc != MICKEY_OK) return rc;
    if (!dst || nwords > s->reqs[id].nbits / 32) return fail(MICKEY_EINVAL, "mickey_server_copy: bad destination");
    if (hipMemcpyAsync(dst, src, nwords * 4, hipMemcpyDeviceToDevice, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return check_launch("mickey_server_copy");
    return ok();
}

int mickey_server_set_latency(mickey_server *s, uint32_t streams, uint64_t threshold_bits,
                              uint64_t clocks_per_quantum)
{
    if (!s) return fail(MICKEY_EINVAL, "mickey_server_set_latency: NULL server");
    if (streams > kLatStreams || (streams && (clocks_per_quantum == 0 || clocks_per_quantum % 32 ||
                                              clocks_per_quantum / 32 > 0xFFFFFFFFull)))
        return fail(MICKEY_EINVAL, "mickey_server_set_latency: at most %u streams, clocks a positive multiple of 32",
                    kLatStreams);
    if (s->lat_busy || s->oldest_q != s->next_q)
        return fail(MICKEY_EINVAL, "mickey_server_set_latency: latency streams or quanta are in flight");
    set_latency(s, streams, threshold_bits, clocks_per_quantum);
    return ok();
}

int mickey_server_set_kernel(mickey_server *s, int schedule, int transpose)
{
    if (!s) return fail(MICKEY_EINVAL, "mickey_server_set_kernel: NULL server");
    if (schedule != MICKEY_SCHED_AUTO && schedule != MICKEY_SCHED_ONE_WAVE && schedule != MICKEY_SCHED_SPLIT &&
        schedule != MICKEY_SCHED_SPLIT4)
        return fail(MICKEY_EINVAL, "mickey_server_set_kernel: unknown schedule %d", schedule);
    if (transpose != MICKEY_TRANSPOSE_AUTO && transpose != MICKEY_TRANSPOSE_FUSED &&
        transpose != MICKEY_TRANSPOSE_STAGED)
        return fail(MICKEY_EINVAL, "mickey_server_set_kernel: unknown transpose mode %d", transpose);
    const bool any_split = schedule == MICKEY_SCHED_SPLIT || schedule == MICKEY_SCHED_SPLIT4;
    if (transpose == MICKEY_TRANSPOSE_FUSED && any_split)
        return fail(MICKEY_EINVAL, "mickey_server_set_kernel: the fused kernel runs the one-wave schedule");
    if (!s->sub_blocks && (transpose == MICKEY_TRANSPOSE_STAGED || any_split))
        return fail(MICKEY_EINVAL, "mickey_server_set_kernel: staging needs one 32-clock plane chunk per "
                                   "launch within 512 MiB (too many slots)");
    s->schedule = schedule;
    s->transpose = transpose;
    return ok();
}

int mickey_server_set_chunk(mickey_server *s, uint64_t chunk_bytes)
{
    if (!s) return fail(MICKEY_EINVAL, "mickey_server_set_chunk: NULL server");
    if (chunk_bytes % 4 || chunk_bytes / 4 > s->alloc.capacity || chunk_bytes / 4 > 0xffffffffull)
        return fail(MICKEY_EINVAL, "mickey_server_set_chunk: chunk must be whole 32-bit words within the budget");
    s->chunk_words = (uint32_t)(chunk_bytes / 4);
    return ok();
}

int64_t mickey_server_poll_chunks(mickey_server *s, mickey_chunk *out, size_t cap)
{
    if (!s || (!out && cap)) return fail(MICKEY_EINVAL, "mickey_server_poll_chunks: bad argument");
    const size_t n = std::min(cap, s->ready.size());
    std::copy(s->ready.begin(), s->ready.begin() + n, out);
    s->ready.erase(s->ready.begin(), s->ready.begin() + n);
    ok();
    return (int64_t)n;
}

int mickey_server_release_chunks(mickey_server *s, const uint64_t *handles, size_t n)
{
    if (!s || (n && !handles)) return fail(MICKEY_EINVAL, "mickey_server_release_chunks: bad argument");
    int first = MICKEY_OK;
    constexpr size_t kAhead = 8;
    for (size_t k = 0; k < n; k++) {
        if (k + 2 * kAhead < n && handles[k + 2 * kAhead] < s->slots.size())
            __builtin_prefetch(&s->slots[handles[k + 2 * kAhead]], 1);
        if (k + kAhead < n && handles[k + kAhead] < s->slots.size()) {
            const auto &c = s->slice_blocks[s->slots[handles[k + kAhead]].slice];
            __builtin_prefetch(&c);
            __builtin_prefetch(c.data() + c.size(), 1);
        }
        const uint64_t h = handles[k];
        if (h >= s->slots.size() || !s->slots[h].live) {
            if (first == MICKEY_OK)
                first = fail(MICKEY_EINVAL, "mickey_server_release_chunks: handle %llu is not a delivered chunk",
                             (unsigned long long)h);
            continue;
        }
        auto &cache = s->slice_blocks[s->slots[h].slice];
        if (cache.size() < kSliceCache) {
            cache.emplace_back(s->slots[h].off, s->slots[h].granted);
            s->slice_cached += s->slots[h].granted;
        } else {
            s->alloc.release(s->slots[h].off, s->slots[h].granted);
        }
        s->slots[h].live = false;
        s->free_slots.push_back(h);
    }
    return first == MICKEY_OK ? ok() : first;
}

int mickey_server_copy_chunk(const mickey_server *s, uint64_t handle, uint32_t *dst, uint64_t nwords)
{
    if (!s || handle >= s->slots.size() || !s->slots[handle].live)
        return fail(MICKEY_EINVAL, "mickey_server_copy_chunk: not a delivered chunk");
    if (!dst || nwords > s->slots[handle].words) return fail(MICKEY_EINVAL, "mickey_server_copy_chunk: bad destination");
    if (hipMemcpyAsync(dst, s->arena + s->slots[handle].off, nwords * 4, hipMemcpyDeviceToDevice, s->stream) !=
            hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return check_launch("mickey_server_copy_chunk");
    return ok();
}

void *mickey_server_stream(const mickey_server *s) { return s ? (void *)s->stream : nullptr; }

void mickey_server_free(mickey_server *s) { destroy(s); }

}  // extern "C"

// Batched generation: thousands of fresh MICKEY 2.0 requests of uneven keystream lengths
// and IV lengths in one persistent, work-queue kernel launch, captured as a HIP graph.
//
// The requests are sorted longest first and packed 32 to a group (one slice: one bit
// lane each); a task is 64 consecutive groups (one wave).  Waves pop tasks from a
// device counter until the queue is empty, so the longest requests start first and
// every wave exits once the counter passes the last task.  Each lane initialises its
// group (with per-lane IV lengths, Sec. IV-D's input handler) and then runs as many
// 32-clock row-major blocks as the longest request of the group needs; a request's
// lane stops storing when its own words are done.
#include "mickey_device.h"
#include "mickey_host.h"
#include "mickey_wordpar.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

using namespace mickey;
using namespace mickey_host;

namespace {

constexpr uint64_t kMaxBatchBits = (uint64_t)1 << 37;  // per request (32-bit word counts)

__global__ void reset_words_kernel(uint32_t *p, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void check_iv_bits_kernel(const uint8_t *__restrict__ iv_bits, uint32_t n, uint32_t *status)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && iv_bits[i] > 80u) atomicOr(status, 1u);
}

// The persistent work-queue kernel.  Lane l of a wave working on task T owns group
// g = 64T + l: slots 32g .. 32g+31, whose input planes are column g of the staged
// planes (pitch gpitch words), and whose outputs are lane_out[32g + i] (lane_words
// words each).  group_words[g] is the longest of them.
template <int U, int WPB>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(2, 2))) void batch_kernel(
    const uint32_t *__restrict__ in_planes, const uint32_t *__restrict__ mask_planes, uint32_t gpitch,
    uint32_t ngroups, uint32_t ntasks, const uint32_t *__restrict__ group_words,
    uint32_t *const *__restrict__ lane_out, const uint32_t *__restrict__ lane_words, uint32_t *__restrict__ counter)
{
    __shared__ uint32_t zbuf[32][64 * WPB];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    const size_t pitch = (size_t)gpitch * 4u;
    for (;;) {
        uint32_t task = 0;
        if (lane == 0u) task = atomicAdd(counter, 1u);
        task = __shfl(task, 0);
        if (task >= ntasks) break;  // every wave leaves once the queue is drained
        const uint32_t g = task * 64u + lane;  // < gpitch: planes exist for padding groups
        const uint32_t nwords = g < ngroups ? group_words[g] : 0u;
        Regs<1> x;
        init_clocks<true, 4>(x, in_planes, mask_planes, pitch, g * 4u);
        for (uint32_t j = 0; j < nwords; j++) {
            rowmajor_block<U>(x, zbuf, tid, [&](int l, uint32_t w) {
                const uint32_t slot = g * 32u + (uint32_t)l;
                if (j < lane_words[slot]) store_global(lane_out[slot] + j, w);
            });
        }
    }
}

// Latency mode: one request per quad of lanes.  Every lane of quad i runs request
// order[i]'s initialisation with the one-lane word-parallel clock (the same input string
// as the bitsliced staging: IV right-aligned to clock 80, then the key, then 100 zero
// clocks; lanes with IV length L idle for 80 - L clocks); then lane q keeps word q of R
// and S and the quad generates with the four-lane clock, 32 clocks per output word
// (first bit in the MSB, stored by lane 0).
__global__ __launch_bounds__(64) void latency_kernel(const uint8_t *__restrict__ keys, const uint8_t *__restrict__ ivs,
                                                     const uint8_t *__restrict__ iv_bits,
                                                     const uint32_t *__restrict__ order, uint32_t nlanes,
                                                     uint32_t *const *__restrict__ lane_out,
                                                     const uint32_t *__restrict__ lane_words)
{
    const uint32_t t = blockIdx.x * 64u + threadIdx.x, i = t >> 2, q = t & 3u;
    if (i >= nlanes) return;  // whole quads
    const uint32_t req = order[i];
    const uint8_t *k = keys + 10ull * req;
    const uint8_t *v = ivs + 10ull * req;
    uint64_t kh = 0, ih = 0;
#pragma unroll
    for (int b = 0; b < 8; b++) {
        kh = (kh << 8) | k[b];
        ih = (ih << 8) | v[b];
    }
    const uint32_t kl = ((uint32_t)k[8] << 8) | k[9], il = ((uint32_t)v[8] << 8) | v[9];
    uint32_t L = iv_bits ? iv_bits[req] : 80u;
    if (L > 80u) L = 80u;  // lengths are validated on the host before any run
    typedef unsigned __int128 u128;
    const u128 key80 = ((u128)kh << 16) | kl, iv80 = ((u128)ih << 16) | il;
    const u128 ivL = L ? (iv80 >> (80u - L)) : (u128)0;
    const u128 lo = key80 | (ivL << 80);
    const uint32_t w[5] = {(uint32_t)(ivL >> 48), (uint32_t)(lo >> 96), (uint32_t)(lo >> 64), (uint32_t)(lo >> 32),
                           (uint32_t)lo};
    const uint32_t d = 80u - L;
    WState x;
#pragma unroll
    for (int j = 0; j < 4; j++) x.r[j] = x.s[j] = 0u;
#pragma unroll
    for (int c = 0; c < 5; c++) {  // the 160 input clocks, 32 per input word
        for (uint32_t b = 0; b < 32u; b += 4) {
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const uint32_t tt = 32u * c + b + u;
                const uint32_t in_m = (uint32_t)((int32_t)(w[c] << (b + u)) >> 31);
                if (tt >= d) wclock<true>(x, in_m);  // lanes with short IVs start late
            }
        }
    }
    for (uint32_t tt = 0; tt < 100u; tt += 4) {  // preclocks
#pragma unroll
        for (int u = 0; u < 4; u++) wclock<true>(x, 0u);
    }
    uint32_t r = pick4(q, x.r[0], x.r[1], x.r[2], x.r[3]);
    uint32_t s = pick4(q, x.s[0], x.s[1], x.s[2], x.s[3]);
    const QuadMasks m = quad_masks(q);
    uint32_t *out = lane_out[i];
    const uint32_t nw = lane_words[i];
    for (uint32_t j = 0; j < nw; j++) {
        const uint32_t word = quad_word(r, s, m);
        if (q == 0) store_global(out + j, word);
    }
}

typedef void (*BatchKernelFn)(const uint32_t *, const uint32_t *, uint32_t, uint32_t, uint32_t, const uint32_t *,
                              uint32_t *const *, const uint32_t *, uint32_t *);

struct Variant {
    int unroll;
    int wpb;
    BatchKernelFn fn;
};

const Variant kVariants[] = {
    {2, 1, batch_kernel<2, 1>}, {2, 2, batch_kernel<2, 2>}, {2, 4, batch_kernel<2, 4>},
    {4, 1, batch_kernel<4, 1>}, {4, 2, batch_kernel<4, 2>}, {4, 4, batch_kernel<4, 4>},
    {8, 1, batch_kernel<8, 1>}, {8, 2, batch_kernel<8, 2>}, {8, 4, batch_kernel<8, 4>},
};

const Variant *find_variant(int unroll, int wpb)
{
    for (const Variant &v : kVariants)
        if (v.unroll == unroll && v.wpb == wpb) return &v;
    return nullptr;
}

// Resident waves of the batch kernel on the whole GPU (2 per SIMD at 256 VGPRs).
int resident_waves()
{
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    return cus * 4 * 2;
}

}  // namespace

struct mickey_batch {
    size_t max_req = 0;
    size_t max_groups_pad = 0;
    hipStream_t stream = nullptr;  // the batch's stream (bitsliced branch)
    hipStream_t side = nullptr;    // latency branch of the graph
    bool own_stream = false;
    hipEvent_t fork = nullptr, join = nullptr;
    // device buffers (one allocation)
    void *dmem = nullptr;
    uint32_t *order = nullptr;        // [slots] request of each bitsliced slot, kNoRequest for padding
    uint32_t **lane_out = nullptr;    // [slots]
    uint32_t *lane_words = nullptr;   // [slots]
    uint32_t *group_words = nullptr;  // [groups]
    uint32_t *counter = nullptr;      // work queue head
    uint32_t *status = nullptr;       // IV length check
    uint32_t *in_planes = nullptr;    // [160][groups_pad]
    uint32_t *mask_planes = nullptr;  // [96][groups_pad]
    uint32_t *lat_order = nullptr;    // [max_req] request of each latency lane
    uint32_t **lat_out = nullptr;     // [max_req]
    uint32_t *lat_words = nullptr;    // [max_req]
    uint32_t *host_status = nullptr;  // pinned
    // current requests and their routing
    const uint8_t *keys = nullptr, *ivs = nullptr, *iv_bits = nullptr;
    size_t nreq = 0, ngroups = 0, groups_pad = 0, ntasks = 0, nlat = 0;
    std::vector<uint64_t> nbits;
    std::vector<uint32_t *> outs;
    std::vector<uint32_t> host_order, lat_host_order;
    int unroll = 4, wpb = 1;
    uint64_t lat_setting = 0;  // 0: automatic threshold, ~0: latency mode off, else threshold in bits
    double lat_ratio = 0.16;   // latency-lane clock time / bitsliced-slice clock time (tuned)
    uint64_t lat_threshold = ~0ull;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr size_t kMaxLatencyLanes = 16384;  // 1024 waves of four-lane latency requests

void drop_graph(mickey_batch *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Size-aware routing: requests of at least `threshold` bits run in latency mode (one
// quad of lanes each), the others bitsliced (32 per slice), each part sorted longest
// first.  The automatic threshold is 3/4 * L_max * (latency clock / bitsliced clock):
// shorter requests finish in bitsliced mode before the longest request finishes in
// latency mode (at the full ratio the persistent bitsliced kernel, with its task tail,
// measured 8% longer than the longest latency request).  At most kMaxLatencyLanes
// requests take latency mode.
void route(mickey_batch *b, const std::vector<uint64_t> &nbits, uint64_t setting)
{
    const size_t n = nbits.size();
    uint64_t lmax = 0;
    for (uint64_t v : nbits) lmax = std::max(lmax, v);
    uint64_t th = ~0ull;
    if (setting == 0) {
        const uint64_t auto_th = (uint64_t)(0.75 * (double)lmax * b->lat_ratio);
        th = std::max<uint64_t>(auto_th, 1u << 12);
    } else if (setting != ~0ull) {
        th = setting;
    }
    std::vector<uint32_t> idx(n);
    std::iota(idx.begin(), idx.end(), 0u);
    std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t c) { return nbits[a] > nbits[c]; });
    size_t nl = 0;
    while (nl < n && nbits[idx[nl]] >= th && nbits[idx[nl]] > 0 && nl < kMaxLatencyLanes) nl++;
    if (nl < n && nl == kMaxLatencyLanes) th = nbits[idx[nl - 1]];
    b->lat_threshold = nl ? th : ~0ull;
    b->nlat = nl;
    b->lat_host_order.assign(idx.begin(), idx.begin() + nl);
    const size_t nshort = n - nl;
    b->ngroups = (nshort + 31) / 32;
    b->groups_pad = (b->ngroups + 63) / 64 * 64;
    b->ntasks = b->groups_pad / 64;
    b->host_order.assign(b->groups_pad * 32, kNoRequest);
    std::copy(idx.begin() + nl, idx.end(), b->host_order.begin());
}

// Upload both parts' metadata for the given lengths and outputs (routing unchanged).
int upload_meta(mickey_batch *b, const std::vector<uint64_t> &nbits, const std::vector<uint32_t *> &outs)
{
    const size_t nslots = b->groups_pad * 32;
    std::vector<uint32_t> words(nslots, 0u), gwords(b->groups_pad, 0u), lwords(b->nlat);
    std::vector<uint32_t *> lo(nslots, nullptr), llo(b->nlat);
    for (size_t s = 0; s < nslots; s++) {
        const uint32_t r = b->host_order[s];
        if (r == kNoRequest) continue;
        words[s] = (uint32_t)(nbits[r] / 32);
        lo[s] = outs[r];
        gwords[s / 32] = std::max(gwords[s / 32], words[s]);
    }
    for (size_t i = 0; i < b->nlat; i++) {
        lwords[i] = (uint32_t)(nbits[b->lat_host_order[i]] / 32);
        llo[i] = outs[b->lat_host_order[i]];
    }
    bool okc = true;
    if (nslots)
        okc = hipMemcpyAsync(b->order, b->host_order.data(), nslots * 4, hipMemcpyHostToDevice, b->stream) ==
                  hipSuccess &&
              hipMemcpyAsync(b->lane_words, words.data(), nslots * 4, hipMemcpyHostToDevice, b->stream) ==
                  hipSuccess &&
              hipMemcpyAsync(b->lane_out, lo.data(), nslots * sizeof(uint32_t *), hipMemcpyHostToDevice,
                             b->stream) == hipSuccess &&
              hipMemcpyAsync(b->group_words, gwords.data(), b->groups_pad * 4, hipMemcpyHostToDevice, b->stream) ==
                  hipSuccess;
    if (okc && b->nlat)
        okc = hipMemcpyAsync(b->lat_order, b->lat_host_order.data(), b->nlat * 4, hipMemcpyHostToDevice,
                             b->stream) == hipSuccess &&
              hipMemcpyAsync(b->lat_words, lwords.data(), b->nlat * 4, hipMemcpyHostToDevice, b->stream) ==
                  hipSuccess &&
              hipMemcpyAsync(b->lat_out, llo.data(), b->nlat * sizeof(uint32_t *), hipMemcpyHostToDevice,
                             b->stream) == hipSuccess;
    if (!okc || hipStreamSynchronize(b->stream) != hipSuccess) return check_launch("batch metadata upload");
    return MICKEY_OK;
}

int launch_bitsliced(mickey_batch *b, const Variant &v)
{
    hipLaunchKernelGGL(reset_words_kernel, dim3(1), dim3(64), 0, b->stream, b->counter, 2u);
    int rc = check_launch("reset_words_kernel");
    if (rc != MICKEY_OK) return rc;
    const uint32_t nslots = (uint32_t)(b->groups_pad * 32);
    const dim3 sgrid((unsigned)((b->groups_pad + kStageSlices - 1) / kStageSlices));
    if (b->iv_bits)
        hipLaunchKernelGGL((stage_kernel<true, true>), sgrid, dim3(256), 0, b->stream, b->keys, b->ivs, b->iv_bits,
                           b->order, nslots, (uint32_t)b->groups_pad, b->in_planes, b->mask_planes, b->status);
    else
        hipLaunchKernelGGL((stage_kernel<false, true>), sgrid, dim3(256), 0, b->stream, b->keys, b->ivs, b->iv_bits,
                           b->order, nslots, (uint32_t)b->groups_pad, b->in_planes, b->mask_planes, b->status);
    rc = check_launch("stage_kernel");
    if (rc != MICKEY_OK) return rc;
    const int waves = (int)std::min<size_t>(b->ntasks, (size_t)resident_waves());
    const int blocks = (waves + v.wpb - 1) / v.wpb;
    hipLaunchKernelGGL(v.fn, dim3(blocks), dim3(64 * v.wpb), 0, b->stream, b->in_planes, b->mask_planes,
                       (uint32_t)b->groups_pad, (uint32_t)b->ngroups, (uint32_t)b->ntasks, b->group_words,
                       b->lane_out, b->lane_words, b->counter);
    return check_launch("batch_kernel");
}

int launch_latency(mickey_batch *b, hipStream_t s)
{
    hipLaunchKernelGGL(latency_kernel, dim3((unsigned)((4 * b->nlat + 63) / 64)), dim3(64), 0, s, b->keys, b->ivs,
                       b->iv_bits, b->lat_order, (uint32_t)b->nlat, b->lat_out, b->lat_words);
    return check_launch("latency_kernel");
}

// Enqueue the batch on b->stream: the bitsliced part (queue reset, input staging,
// persistent kernel) and, concurrently on the side stream, the latency part.
int enqueue(mickey_batch *b, const Variant &v)
{
    int rc = MICKEY_OK;
    if (b->nlat && b->ngroups) {
        if (hipEventRecord(b->fork, b->stream) != hipSuccess || hipStreamWaitEvent(b->side, b->fork, 0) != hipSuccess)
            return check_launch("fork");
        rc = launch_latency(b, b->side);
        if (rc == MICKEY_OK) rc = launch_bitsliced(b, v);
        if (hipEventRecord(b->join, b->side) != hipSuccess || hipStreamWaitEvent(b->stream, b->join, 0) != hipSuccess)
            return check_launch("join");
        return rc;
    }
    if (b->nlat) return launch_latency(b, b->stream);
    if (b->ngroups) return launch_bitsliced(b, v);
    return MICKEY_OK;
}

int capture(mickey_batch *b)
{
    drop_graph(b);
    const Variant *v = find_variant(b->unroll, b->wpb);
    if (!v) return fail(MICKEY_EINVAL, "no batch kernel for unroll %d, %d waves per block", b->unroll, b->wpb);
    if (hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return check_launch("hipStreamBeginCapture");
    int rc = enqueue(b, *v);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (rc != MICKEY_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(MICKEY_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(b);
        return fail(MICKEY_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return MICKEY_OK;
}

// Route, upload and capture the current requests.
int prepare(mickey_batch *b)
{
    route(b, b->nbits, b->lat_setting);
    int rc = upload_meta(b, b->nbits, b->outs);
    return rc == MICKEY_OK ? capture(b) : rc;
}

void destroy(mickey_batch *b)
{
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->side) (void)hipStreamSynchronize(b->side);
    drop_graph(b);
    if (b->dmem) (void)hipFree(b->dmem);
    if (b->host_status) (void)hipHostFree(b->host_status);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

// Time one enqueue on b->stream (ms), after one warm-up.
int time_enqueue(mickey_batch *b, const Variant &v, hipEvent_t e0, hipEvent_t e1, float *ms)
{
    int rc = enqueue(b, v);
    *ms = 1e30f;
    for (int rep = 0; rep < 2 && rc == MICKEY_OK; rep++) {
        (void)hipEventRecord(e0, b->stream);
        rc = enqueue(b, v);
        (void)hipEventRecord(e1, b->stream);
        if (rc != MICKEY_OK) break;
        if (hipEventSynchronize(e1) != hipSuccess) return check_launch("autotune timing");
        float t = 0;
        (void)hipEventElapsedTime(&t, e0, e1);
        *ms = std::min(*ms, t);
    }
    return rc;
}

}  // namespace

extern "C" {

mickey_batch *mickey_batch_create(size_t max_requests, void *hip_stream)
{
    if (max_requests == 0 || max_requests > ((size_t)1 << 30)) {
        fail(MICKEY_EINVAL, "mickey_batch_create: max_requests must be in 1..2^30");
        return nullptr;
    }
    mickey_batch *b = new (std::nothrow) mickey_batch();
    if (!b) {
        fail(MICKEY_ENOMEM, "mickey_batch_create: host allocation failed");
        return nullptr;
    }
    b->max_req = max_requests;
    const size_t groups = (max_requests + 31) / 32;
    b->max_groups_pad = (groups + 63) / 64 * 64;
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else if (hipStreamCreate(&b->stream) == hipSuccess) {
        b->own_stream = true;
    } else {
        delete b;
        fail(MICKEY_EDEVICE, "mickey_batch_create: cannot create a stream");
        return nullptr;
    }
    const size_t slots = b->max_groups_pad * 32;
    const size_t bytes = slots * (4 + sizeof(uint32_t *) + 4) + b->max_groups_pad * 4 + 256 +
                         (size_t)(kInputPlanes + kMaskPlanes) * b->max_groups_pad * 4 +
                         max_requests * (4 + sizeof(uint32_t *) + 4) + 256;
    if (hipStreamCreate(&b->side) != hipSuccess || hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess || hipMalloc(&b->dmem, bytes) != hipSuccess ||
        hipHostMalloc((void **)&b->host_status, 4, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        destroy(b);
        fail(MICKEY_ENOMEM, "mickey_batch_create: cannot allocate %zu bytes or a stream", bytes);
        return nullptr;
    }
    char *p = (char *)b->dmem;
    b->lane_out = (uint32_t **)p;
    p += slots * sizeof(uint32_t *);
    b->lat_out = (uint32_t **)p;
    p += max_requests * sizeof(uint32_t *);
    b->order = (uint32_t *)p;
    p += slots * 4;
    b->lane_words = (uint32_t *)p;
    p += slots * 4;
    b->lat_order = (uint32_t *)p;
    p += max_requests * 4;
    b->lat_words = (uint32_t *)p;
    p += max_requests * 4;
    p = (char *)(((uintptr_t)p + 255) & ~(uintptr_t)255);
    b->group_words = (uint32_t *)p;
    p += b->max_groups_pad * 4;
    b->counter = (uint32_t *)p;  // counter and status share one 256-byte line
    b->status = b->counter + 1;
    p += 256;
    b->in_planes = (uint32_t *)p;
    p += (size_t)kInputPlanes * b->max_groups_pad * 4;
    b->mask_planes = (uint32_t *)p;
    ok();
    return b;
}

int mickey_batch_set(mickey_batch *b, const uint8_t *keys, const uint8_t *ivs, const uint8_t *iv_bits,
                     const uint64_t *nbits, uint32_t *const *outs, size_t nreq)
{
    if (!b) return fail(MICKEY_EINVAL, "mickey_batch_set: NULL batch");
    if (nreq == 0 || nreq > b->max_req)
        return fail(MICKEY_EINVAL, "mickey_batch_set: %zu requests (capacity %zu)", nreq, b->max_req);
    if (!keys || !ivs || !nbits || !outs) return fail(MICKEY_EINVAL, "mickey_batch_set: NULL argument");
    for (size_t r = 0; r < nreq; r++) {
        if (nbits[r] % 32 != 0) return fail(MICKEY_EINVAL, "request %zu: nbits must be a multiple of 32", r);
        if (nbits[r] > kMaxBatchBits) return fail(MICKEY_ERANGE, "request %zu: more than 2^37 bits", r);
        if (nbits[r] && !outs[r]) return fail(MICKEY_EINVAL, "request %zu: NULL output", r);
    }
    if (iv_bits) {  // validate the IV lengths once, here, so that runs never fail on them
        if (hipMemsetAsync(b->status, 0, 4, b->stream) != hipSuccess) return check_launch("hipMemsetAsync");
        hipLaunchKernelGGL(check_iv_bits_kernel, dim3((unsigned)((nreq + 255) / 256)), dim3(256), 0, b->stream,
                           iv_bits, (uint32_t)nreq, b->status);
        if (hipMemcpyAsync(b->host_status, b->status, 4, hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
            hipStreamSynchronize(b->stream) != hipSuccess)
            return check_launch("IV length check");
        if (*b->host_status) return fail(MICKEY_EINVAL, "mickey_batch_set: an IV length exceeds 80 bits");
    }
    b->keys = keys;
    b->ivs = ivs;
    b->iv_bits = iv_bits;
    b->nreq = nreq;
    b->nbits.assign(nbits, nbits + nreq);
    b->outs.assign(outs, outs + nreq);
    int rc = prepare(b);
    return rc == MICKEY_OK ? ok() : rc;
}

int mickey_batch_run(mickey_batch *b)
{
    if (!b) return fail(MICKEY_EINVAL, "mickey_batch_run: NULL batch");
    if (!b->exec) return fail(MICKEY_EINVAL, "mickey_batch_run: no requests set");
    hipError_t e = hipGraphLaunch(b->exec, b->stream);
    if (e != hipSuccess) return fail(MICKEY_EDEVICE, "hipGraphLaunch: %s", hipGetErrorString(e));
    return ok();
}

int mickey_batch_sync(mickey_batch *b)
{
    if (!b) return fail(MICKEY_EINVAL, "mickey_batch_sync: NULL batch");
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return fail(MICKEY_EDEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return ok();
}

void *mickey_batch_stream(const mickey_batch *b) { return b ? (void *)b->stream : nullptr; }

int mickey_batch_set_params(mickey_batch *b, int unroll, int waves_per_block)
{
    if (!b) return fail(MICKEY_EINVAL, "mickey_batch_set_params: NULL batch");
    const int u = unroll ? unroll : b->unroll, w = waves_per_block ? waves_per_block : b->wpb;
    if (!find_variant(u, w))
        return fail(MICKEY_EINVAL, "mickey_batch_set_params: unroll %d / %d waves per block not built", u, w);
    b->unroll = u;
    b->wpb = w;
    if (b->nreq) {
        int rc = capture(b);
        if (rc != MICKEY_OK) return rc;
    }
    return ok();
}

int mickey_batch_get_params(const mickey_batch *b, int *unroll, int *waves_per_block)
{
    if (!b) return fail(MICKEY_EINVAL, "mickey_batch_get_params: NULL batch");
    if (unroll) *unroll = b->unroll;
    if (waves_per_block) *waves_per_block = b->wpb;
    return ok();
}

int mickey_batch_set_latency_threshold(mickey_batch *b, uint64_t bits)
{
    if (!b) return fail(MICKEY_EINVAL, "mickey_batch_set_latency_threshold: NULL batch");
    b->lat_setting = bits;
    if (b->nreq) {
        int rc = prepare(b);
        if (rc != MICKEY_OK) return rc;
    }
    return ok();
}

int mickey_batch_get_routing(const mickey_batch *b, uint64_t *threshold, size_t *latency_requests,
                             double *latency_clock_ratio)
{
    if (!b) return fail(MICKEY_EINVAL, "mickey_batch_get_routing: NULL batch");
    if (threshold) *threshold = b->lat_threshold;
    if (latency_requests) *latency_requests = b->nlat;
    if (latency_clock_ratio) *latency_clock_ratio = b->lat_ratio;
    return ok();
}

int mickey_batch_autotune(mickey_batch *b, uint64_t cap_bits, const char *cache_path)
{
    if (!b) return fail(MICKEY_EINVAL, "mickey_batch_autotune: NULL batch");
    if (!b->nreq) return fail(MICKEY_EINVAL, "mickey_batch_autotune: no requests set");
    if (cap_bits < 32 || cap_bits % 32) return fail(MICKEY_EINVAL, "mickey_batch_autotune: cap must be k*32, k>0");
    // signature of the tuning problem: architecture, request count, capped length mix
    int dev = 0;
    (void)hipGetDevice(&dev);
    hipDeviceProp_t prop;
    const char *arch = hipGetDeviceProperties(&prop, dev) == hipSuccess ? prop.gcnArchName : "unknown";
    std::vector<uint64_t> capped(b->nreq);
    uint64_t capped_total = 0, capped_max = 0;
    size_t words = 0;
    for (size_t r = 0; r < b->nreq; r++) {
        capped[r] = std::min(b->nbits[r], cap_bits);
        capped_total += capped[r];
        capped_max = std::max(capped_max, capped[r]);
        words += capped[r] / 32;
    }
    char sig[256];
    snprintf(sig, sizeof sig, "%s/nreq=%zu/cap=%llu/total=%llu/max=%llu", arch, b->nreq, (unsigned long long)cap_bits,
             (unsigned long long)capped_total, (unsigned long long)capped_max);
    if (cache_path) {
        if (FILE *f = fopen(cache_path, "r")) {
            char buf[4096];
            const size_t len = fread(buf, 1, sizeof buf - 1, f);
            fclose(f);
            buf[len] = 0;
            int u = 0, w = 0;
            double ratio = 0;
            const char *ps = strstr(buf, "\"signature\": \"");
            const char *pu = strstr(buf, "\"unroll\": ");
            const char *pw = strstr(buf, "\"waves_per_block\": ");
            const char *pr = strstr(buf, "\"latency_clock_ratio\": ");
            if (ps && pu && pw && pr && strncmp(ps + 14, sig, strlen(sig)) == 0 && ps[14 + strlen(sig)] == '"' &&
                sscanf(pu + 10, "%d", &u) == 1 && sscanf(pw + 19, "%d", &w) == 1 && sscanf(pr + 23, "%lf", &ratio) == 1 &&
                find_variant(u, w) && ratio > 0) {
                b->unroll = u;
                b->wpb = w;
                b->lat_ratio = ratio;
                int rc = prepare(b);
                return rc == MICKEY_OK ? ok() : rc;
            }
        }
    }
    uint32_t *scratch = nullptr;
    if (hipMalloc(&scratch, std::max<size_t>(words, 1) * 4) != hipSuccess) {
        (void)hipGetLastError();
        return fail(MICKEY_ENOMEM, "mickey_batch_autotune: cannot allocate %zu bytes of scratch", words * 4);
    }
    std::vector<uint32_t *> souts(b->nreq);
    for (size_t r = 0, w = 0; r < b->nreq; r++) {
        souts[r] = scratch + w;
        w += capped[r] / 32;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = MICKEY_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = check_launch("hipEventCreate");
    // 1. bitsliced variants, every request bitsliced
    float best_ms = 0;
    const Variant *best = nullptr;
    std::string timings;
    if (rc == MICKEY_OK) {
        route(b, capped, ~0ull);
        rc = upload_meta(b, capped, souts);
    }
    for (const Variant &v : kVariants) {
        if (rc != MICKEY_OK) break;
        float ms = 0;
        rc = time_enqueue(b, v, e0, e1, &ms);
        if (rc != MICKEY_OK) break;
        char item[64];
        snprintf(item, sizeof item, "%s\"u%dw%d\": %.4f", timings.empty() ? "" : ", ", v.unroll, v.wpb, ms);
        timings += item;
        if (!best || ms < best_ms) {
            best = &v;
            best_ms = ms;
        }
    }
    // 2. the same requests, every one in latency mode (up to the lane limit): the ratio
    //    of per-clock times of the two engines sets the automatic routing threshold
    float lat_ms = 0;
    if (rc == MICKEY_OK) {
        route(b, capped, 1);
        rc = upload_meta(b, capped, souts);
        if (rc == MICKEY_OK && b->ngroups == 0) rc = time_enqueue(b, *best, e0, e1, &lat_ms);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(b->stream);
    (void)hipFree(scratch);
    if (rc == MICKEY_OK && best) {
        b->unroll = best->unroll;
        b->wpb = best->wpb;
        if (lat_ms > 0 && best_ms > 0) b->lat_ratio = lat_ms / best_ms;
    }
    const int rc2 = prepare(b);  // restore the real requests, routing and graph
    if (rc != MICKEY_OK) return rc;
    if (rc2 != MICKEY_OK) return rc2;
    if (cache_path) {
        if (FILE *f = fopen(cache_path, "w")) {
            fprintf(f,
                    "{\"signature\": \"%s\", \"unroll\": %d, \"waves_per_block\": %d, \"word_bits\": 32, "
                    "\"latency_clock_ratio\": %.5f, \"best_ms\": %.4f, \"latency_ms\": %.4f, \"timings_ms\": {%s}}\n",
                    sig, b->unroll, b->wpb, b->lat_ratio, best_ms, lat_ms, timings.c_str());
            fclose(f);
        }
    }
    return ok();
}

void mickey_batch_free(mickey_batch *b) { destroy(b); }

}  // extern "C"

// Per-instance requests on an existing state: mickey_generate_batch.
//
// The paper's problem statement (Sec. IV-D) is many independent generator instances,
// each with its own key and IV; a whole-state generate advances all of them together.
// Here a caller asks for keystream from individual instances of a state, in any mix:
// request k resumes instance reqs[k].instance for reqs[k].nbits bits, and requests on the
// same instance run in array order, each continuing where the previous one stopped.
//
// Execution: the requests of one instance form one task (their lengths added, their
// outputs a list of segments).  A pack kernel copies every task's 200 register bits out
// of the bit-planes into a packed 25-byte state.  Long tasks run in latency mode (one
// task per four lanes, word-parallel clock: a lone instance advances several times
// faster), the others bitsliced, 32 tasks per lane as in the plain path, longest first;
// the two run concurrently on the state's two streams.  A bitsliced lane delivers its 32
// tasks' words every 32 clocks (LDS transpose) through per-task cursors over their
// segments, and packs a task's registers back at the block where it ends.  A scatter
// kernel then writes the changed register bits back into the planes with atomic XORs
// (tasks are distinct instances, so their bits never collide).  Until that last launch
// the planes are only read, so a failed call leaves the state unchanged.
#include "mickey_device.h"
#include "mickey_host.h"
#include "mickey_pack.h"
#include "mickey_state.h"
#include "mickey_wordpar.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

using namespace mickey;
using namespace mickey_host;

namespace {

// One request's output: `words` row-major words at `out`, as u32 or as exact floats.
struct ResumeSeg {
    uint32_t *out;
    uint32_t words;
    uint32_t f32;
};
static_assert(sizeof(ResumeSeg) == 16, "segment record");

// A bitsliced slot's position in its task's segments: the next word goes to `out`; the
// current segment ends at task word `end`; `words` is the task's total.
struct ResumeCur {
    uint32_t *out;
    uint32_t end;
    uint32_t seg;
    uint32_t words;
    uint32_t f32;
};
static_assert(sizeof(ResumeCur) == 24, "cursor record");

constexpr uint32_t kNoTask = 0xFFFFFFFFu;
constexpr size_t kMaxLatencyTasks = 16384;
constexpr uint64_t kMaxTaskWords = 0xFFFFFFFFull;  // per instance and call (32-bit word counts)
constexpr uint64_t kMinLatencyBits = 1u << 14;     // shorter tasks always run bitsliced
// Routing: latency-mode clock time over the bitsliced slice clock time under load (the
// batch autotuner measured ~0.066 on MI355X); tasks of at least 3/4 * L_max * ratio bits
// take latency mode, so that the bitsliced part finishes before the longest task.
constexpr double kLatencyClockRatio = 1.0 / 16;

__device__ __forceinline__ uint32_t f32_word(uint32_t w) { return __float_as_uint((float)(w >> 8) * 0x1p-24f); }

// Task t's 200 register bits (instance task_inst[t]) from the planes into 25 bytes.
__global__ __launch_bounds__(256) void resume_pack_kernel(const uint32_t *__restrict__ planes, uint32_t nslices,
                                                          const uint32_t *__restrict__ task_inst, uint32_t ntasks,
                                                          uint8_t *__restrict__ packed)
{
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntasks) return;
    const uint32_t inst = task_inst[t], g = inst >> 5, l = inst & 31u;
    for (int byte = 0; byte < 25; byte++) {
        uint32_t v = 0;
        for (int k = 0; k < 8; k++) {
            const int j = 8 * byte + k;
            v = (v << 1) | ((planes[(size_t)j * nslices + g] >> l) & 1u);
        }
        packed[25ull * t + byte] = (uint8_t)v;
    }
}

// Register bits that differ between a task's old and new packed states are flipped in the
// planes; one thread per (task, packed byte).
__global__ __launch_bounds__(256) void resume_scatter_kernel(uint32_t *__restrict__ planes, uint32_t nslices,
                                                             const uint32_t *__restrict__ task_inst, uint64_t nbytes,
                                                             const uint8_t *__restrict__ old_packed,
                                                             const uint8_t *__restrict__ new_packed)
{
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nbytes) return;
    const uint32_t d = old_packed[i] ^ new_packed[i];
    if (!d) return;
    const uint64_t t = i / 25;
    const uint32_t byte = (uint32_t)(i - 25 * t);
    const uint32_t inst = task_inst[t];
    const uint32_t bit = 1u << (inst & 31u);
    for (int k = 0; k < 8; k++)
        if ((d >> (7 - k)) & 1u) atomicXor(planes + (size_t)(8 * byte + k) * nslices + (inst >> 5), bit);
}

// Bitsliced part: lane g holds slots 32g .. 32g+31 (tasks slot_task[], longest first) and
// runs group_words[g] blocks of 32 clocks.  Each block's words are delivered per slot
// through its cursor; a slot whose task ends at this block has its registers packed.
template <int U>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2))) void resume_bitsliced_kernel(
    uint32_t ngroups, const uint32_t *__restrict__ slot_task, const uint32_t *__restrict__ group_words,
    const uint32_t *__restrict__ task_words, const ResumeSeg *__restrict__ segs, ResumeCur *__restrict__ cur,
    const uint8_t *__restrict__ old_packed, uint8_t *__restrict__ new_packed)
{
    __shared__ uint32_t zbuf[32][64];
    const uint32_t tid = threadIdx.x;
    const uint32_t g = blockIdx.x * 64u + tid;
    if (g >= ngroups) return;  // no barriers below: each lane only touches its LDS column
    Regs<1> x;
#pragma unroll
    for (int j = 0; j < 100; j++) {
        x.r[j].w[0] = 0u;
        x.s[j].w[0] = 0u;
    }
    uint32_t next_end = 0xFFFFFFFFu;
    for (uint32_t l = 0; l < 32u; l++) {
        const uint32_t t = slot_task[32u * g + l];
        if (t == kNoTask) continue;
        gather_lane(x, l, old_packed + 25ull * t);
        next_end = min(next_end, task_words[t]);
    }
    const uint32_t nw = group_words[g];
    for (uint32_t j = 0; j < nw; j++) {
        rowmajor_block<U>(x, zbuf, tid, [&](int l, uint32_t w) {
            ResumeCur *c = cur + 32u * g + (uint32_t)l;
            if (j < c->words) {
                uint32_t *o = c->out;
                uint32_t f = c->f32;
                if (j == c->end) {  // the next request of this instance starts here
                    const uint32_t s = c->seg + 1u;
                    const ResumeSeg sg = segs[s];
                    o = sg.out;
                    f = sg.f32;
                    c->seg = s;
                    c->end = j + sg.words;
                    c->f32 = f;
                }
                store_global(o, f ? f32_word(w) : w);
                c->out = o + 1;
            }
        });
        if (j + 1u == next_end) {
            uint32_t ne = 0xFFFFFFFFu;
            for (uint32_t l = 0; l < 32u; l++) {
                const uint32_t t = slot_task[32u * g + l];
                if (t == kNoTask) continue;
                const uint32_t tw = task_words[t];
                if (tw == j + 1u) write_back_lane(x, l, new_packed + 25ull * t);
                else if (tw > j + 1u) ne = min(ne, tw);
            }
            next_end = ne;
        }
    }
}

// Latency part: quad i runs task lat_task[i] with the four-lane word-parallel clock,
// segment by segment, then packs its registers.  Whole quads only (the clock's DPP
// exchanges stay inside a quad whose lanes are all active).
__global__ __launch_bounds__(64) void resume_latency_kernel(uint32_t nlat, const uint32_t *__restrict__ lat_task,
                                                            const uint32_t *__restrict__ task_seg0,
                                                            const uint32_t *__restrict__ task_nseg,
                                                            const ResumeSeg *__restrict__ segs,
                                                            const uint8_t *__restrict__ old_packed,
                                                            uint8_t *__restrict__ new_packed)
{
    const uint32_t t = blockIdx.x * 64u + threadIdx.x, i = t >> 2, q = t & 3u;
    if (i >= nlat) return;
    const uint32_t task = lat_task[i];
    uint32_t r, s;
    quad_gather(old_packed + 25ull * task, q, r, s);
    const QuadMasks m = quad_masks(q);
    const uint32_t s0 = task_seg0[task], ns = task_nseg[task];
    for (uint32_t k = 0; k < ns; k++) {
        const ResumeSeg sg = segs[s0 + k];
        for (uint32_t w = 0; w < sg.words; w++) {
            const uint32_t word = quad_word(r, s, m);
            if (q == 0) store_global(sg.out + w, sg.f32 ? f32_word(word) : word);
        }
    }
    quad_write_back(r, s, q, new_packed + 25ull * task);
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Byte offsets of the call's metadata (identical on the host and the device) and of the
// packed states (device only).
struct Layout {
    size_t task_inst, task_words, task_seg0, task_nseg, segs, cur, slot_task, group_words, lat_task, meta_end;
    size_t old_packed, new_packed, end;
};

Layout plan_layout(size_t ntasks, size_t nseg, size_t nslots, size_t groups_pad, size_t nlat)
{
    Layout L;
    size_t p = 0;
    L.task_inst = p;
    p = align_up(p + 4 * ntasks, 256);
    L.task_words = p;
    p = align_up(p + 4 * ntasks, 256);
    L.task_seg0 = p;
    p = align_up(p + 4 * ntasks, 256);
    L.task_nseg = p;
    p = align_up(p + 4 * ntasks, 256);
    L.segs = p;
    p = align_up(p + sizeof(ResumeSeg) * nseg, 256);
    L.cur = p;
    p = align_up(p + sizeof(ResumeCur) * nslots, 256);
    L.slot_task = p;
    p = align_up(p + 4 * nslots, 256);
    L.group_words = p;
    p = align_up(p + 4 * groups_pad, 256);
    L.lat_task = p;
    p = align_up(p + 4 * nlat, 256);
    L.meta_end = p;
    L.old_packed = p;
    p = align_up(p + 25 * ntasks, 256);
    L.new_packed = p;
    p = align_up(p + 25 * ntasks, 256);
    L.end = p;
    return L;
}

int ensure_host_meta(mickey_state *st, size_t bytes)
{
    if (st->bhost_ev && hipEventSynchronize(st->bhost_ev) != hipSuccess)  // the last upload has read it
        return check_launch("mickey_generate_batch: metadata upload");
    if (!st->bhost_ev && hipEventCreateWithFlags(&st->bhost_ev, hipEventDisableTiming) != hipSuccess)
        return check_launch("hipEventCreate");
    if (st->bhost_bytes >= bytes) return MICKEY_OK;
    if (st->bhost) (void)hipHostFree(st->bhost);
    st->bhost = nullptr;
    st->bhost_bytes = 0;
    const size_t want = bytes < ((size_t)1 << 16) ? ((size_t)1 << 16) : bytes;
    if (hipHostMalloc(&st->bhost, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        st->bhost = nullptr;
        return fail(MICKEY_ENOMEM, "mickey_generate_batch: cannot allocate %zu bytes of pinned host memory", want);
    }
    st->bhost_bytes = want;
    return MICKEY_OK;
}

struct TaskH {
    uint32_t inst;
    uint64_t words;
    uint32_t seg0, nseg;
};

}  // namespace

extern "C" int mickey_generate_batch(mickey_state *st, const mickey_req *reqs, size_t nreq)
{
    if (!st) return fail(MICKEY_EINVAL, "mickey_generate_batch: NULL state");
    if (nreq && !reqs) return fail(MICKEY_EINVAL, "mickey_generate_batch: NULL request array");
    if (st->poisoned)
        return fail(MICKEY_EDEVICE, "mickey_generate_batch: the state was lost to an earlier device failure");
    if (nreq > ((size_t)1 << 31)) return fail(MICKEY_EINVAL, "mickey_generate_batch: more than 2^31 requests");
    for (size_t k = 0; k < nreq; k++) {
        const mickey_req &q = reqs[k];
        if (q.instance >= st->n)
            return fail(MICKEY_EINVAL, "request %zu: instance %llu of %zu", k, (unsigned long long)q.instance, st->n);
        if (q.layout != MICKEY_ROWMAJOR_U32 && q.layout != MICKEY_ROWMAJOR_F32)
            return fail(MICKEY_EINVAL, "request %zu: layout must be MICKEY_ROWMAJOR_U32 or MICKEY_ROWMAJOR_F32", k);
        if (q.nbits % 32 != 0) return fail(MICKEY_EINVAL, "request %zu: nbits must be a multiple of 32", k);
        if (q.nbits > MICKEY_MAX_BITS_PER_IV) return fail(MICKEY_ERANGE, "request %zu: more than 2^40 bits", k);
        if (q.nbits && !q.out) return fail(MICKEY_EINVAL, "request %zu: NULL output", k);
    }
    // the requests of each instance, in array order
    std::vector<uint32_t> idx(nreq);
    std::iota(idx.begin(), idx.end(), 0u);
    std::stable_sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) { return reqs[a].instance < reqs[b].instance; });
    std::vector<TaskH> tasks;
    std::vector<ResumeSeg> segs;
    for (size_t a = 0; a < nreq;) {
        size_t b = a;
        const uint64_t inst = reqs[idx[a]].instance;
        TaskH t{(uint32_t)inst, 0, (uint32_t)segs.size(), 0};
        for (; b < nreq && reqs[idx[b]].instance == inst; b++) {
            const mickey_req &q = reqs[idx[b]];
            if (!q.nbits) continue;
            t.words += q.nbits / 32;  // each at most 2^35, at most 2^31 of them: no overflow
            segs.push_back({(uint32_t *)q.out, (uint32_t)(q.nbits / 32), q.layout == MICKEY_ROWMAJOR_F32 ? 1u : 0u});
            t.nseg++;
        }
        a = b;
        if (!t.words) continue;
        if (t.words > kMaxTaskWords)
            return fail(MICKEY_ERANGE, "instance %llu: more than 2^37 bits in one call", (unsigned long long)inst);
        if (instance_bits(st, inst) > MICKEY_MAX_BITS_PER_IV - 32 * t.words)
            return fail(MICKEY_ERANGE, "instance %llu: %llu + %llu bits exceeds 2^40 per key/IV pair",
                        (unsigned long long)inst, (unsigned long long)instance_bits(st, inst),
                        (unsigned long long)(32 * t.words));
        tasks.push_back(t);
    }
    if (tasks.empty()) return ok();
    const size_t nt = tasks.size();
    // routing: longest first; the longest go to latency mode
    std::vector<uint32_t> order(nt);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return tasks[a].words > tasks[b].words; });
    const uint64_t lmax = 32 * tasks[order[0]].words;
    const uint64_t th = std::max<uint64_t>(kMinLatencyBits, (uint64_t)(0.75 * (double)lmax * kLatencyClockRatio));
    size_t nl = 0;
    while (nl < nt && nl < kMaxLatencyTasks && 32 * tasks[order[nl]].words >= th) nl++;
    const size_t nb = nt - nl;
    const size_t ngroups = (nb + 31) / 32, groups_pad = (ngroups + 63) / 64 * 64, nslots = 32 * groups_pad;
    const Layout L = plan_layout(nt, segs.size(), nslots, groups_pad, nl);
    int rc = ensure_scratch(st, L.end);
    if (rc == MICKEY_OK) rc = ensure_host_meta(st, L.meta_end);
    if (rc != MICKEY_OK) return rc;
    char *h = (char *)st->bhost;
    char *d = (char *)st->bmem;
    {
        uint32_t *ti = (uint32_t *)(h + L.task_inst), *tw = (uint32_t *)(h + L.task_words);
        uint32_t *t0 = (uint32_t *)(h + L.task_seg0), *tn = (uint32_t *)(h + L.task_nseg);
        for (size_t t = 0; t < nt; t++) {
            ti[t] = tasks[t].inst;
            tw[t] = (uint32_t)tasks[t].words;
            t0[t] = tasks[t].seg0;
            tn[t] = tasks[t].nseg;
        }
        memcpy(h + L.segs, segs.data(), segs.size() * sizeof(ResumeSeg));
        ResumeCur *cur = (ResumeCur *)(h + L.cur);
        uint32_t *slot = (uint32_t *)(h + L.slot_task), *gw = (uint32_t *)(h + L.group_words);
        memset(gw, 0, 4 * groups_pad);
        for (size_t sl = 0; sl < nslots; sl++) {
            const size_t k = nl + sl;
            if (sl < nb) {
                const TaskH &t = tasks[order[k]];
                const ResumeSeg &s0 = segs[t.seg0];
                slot[sl] = order[k];
                cur[sl] = {s0.out, s0.words, t.seg0, (uint32_t)t.words, s0.f32};
                gw[sl / 32] = std::max(gw[sl / 32], (uint32_t)t.words);
            } else {
                slot[sl] = kNoTask;
                cur[sl] = {nullptr, 0u, 0u, 0u, 0u};
            }
        }
        uint32_t *lt = (uint32_t *)(h + L.lat_task);
        for (size_t i = 0; i < nl; i++) lt[i] = order[i];
    }
    if (hipMemcpyAsync(d, h, L.meta_end, hipMemcpyHostToDevice, st->stream) != hipSuccess ||
        hipEventRecord(st->bhost_ev, st->stream) != hipSuccess)
        return check_launch("mickey_generate_batch: metadata upload");
    const uint32_t *task_inst = (const uint32_t *)(d + L.task_inst);
    uint8_t *old_packed = (uint8_t *)(d + L.old_packed), *new_packed = (uint8_t *)(d + L.new_packed);
    rc = launch_guard("resume_pack_kernel");
    if (rc != MICKEY_OK) return rc;
    hipLaunchKernelGGL(resume_pack_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st->stream, st->planes,
                       (uint32_t)st->nslices, task_inst, (uint32_t)nt, old_packed);
    rc = check_launch("resume_pack_kernel");
    if (rc != MICKEY_OK) return rc;
    const bool both = nl && nb;
    if (both) {
        rc = ensure_side(st);
        if (rc != MICKEY_OK) return rc;
        if (hipEventRecord(st->ev_fork, st->stream) != hipSuccess ||
            hipStreamWaitEvent(st->side, st->ev_fork, 0) != hipSuccess)
            return check_launch("mickey_generate_batch: fork");
    }
    if (nl) {
        rc = launch_guard("resume_latency_kernel");
        if (rc == MICKEY_OK) {
            hipLaunchKernelGGL(resume_latency_kernel, dim3((unsigned)((4 * nl + 63) / 64)), dim3(64), 0,
                               both ? st->side : st->stream, (uint32_t)nl, (const uint32_t *)(d + L.lat_task),
                               (const uint32_t *)(d + L.task_seg0), (const uint32_t *)(d + L.task_nseg),
                               (const ResumeSeg *)(d + L.segs), old_packed, new_packed);
            rc = check_launch("resume_latency_kernel");
        }
    }
    if (rc == MICKEY_OK && nb) {
        rc = launch_guard("resume_bitsliced_kernel");
        if (rc == MICKEY_OK) {
            hipLaunchKernelGGL(resume_bitsliced_kernel<4>, dim3((unsigned)(groups_pad / 64)), dim3(64), 0,
                               st->stream, (uint32_t)ngroups, (const uint32_t *)(d + L.slot_task),
                               (const uint32_t *)(d + L.group_words), (const uint32_t *)(d + L.task_words),
                               (const ResumeSeg *)(d + L.segs), (ResumeCur *)(d + L.cur), old_packed, new_packed);
            rc = check_launch("resume_bitsliced_kernel");
        }
    }
    if (both) {  // join even after a failure: later work on the state's stream reuses the scratch
        if (hipEventRecord(st->ev_join, st->side) != hipSuccess ||
            hipStreamWaitEvent(st->stream, st->ev_join, 0) != hipSuccess) {
            const int jrc = check_launch("mickey_generate_batch: join");
            if (rc == MICKEY_OK) rc = jrc;
        }
    }
    if (rc != MICKEY_OK) return rc;
    rc = launch_guard("resume_scatter_kernel");
    if (rc != MICKEY_OK) return rc;
    hipLaunchKernelGGL(resume_scatter_kernel, dim3((unsigned)((25 * nt + 255) / 256)), dim3(256), 0, st->stream,
                       st->planes, (uint32_t)st->nslices, task_inst, (uint64_t)(25 * nt), old_packed, new_packed);
    rc = check_launch("resume_scatter_kernel");
    if (rc != MICKEY_OK) return rc;
    if (st->extra.empty()) st->extra.assign(st->n, 0);
    for (const TaskH &t : tasks) {
        st->extra[t.inst] += 32 * t.words;
        st->max_extra = std::max(st->max_extra, st->extra[t.inst]);
    }
    st->snap_valid = false;
    return ok();
}

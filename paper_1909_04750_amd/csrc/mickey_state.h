// The library's state object (opaque in include/mickey.h), shared by the translation units
// that work on it: the whole-state calls (mickey_kernels.hip) and the per-instance
// requests of mickey_generate_batch (mickey_resume.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

struct mickey_state {
    size_t n;
    size_t n_pad;
    size_t nslices;
    uint32_t *planes = nullptr;       // device, 200 * nslices words
    uint32_t *stage = nullptr;        // device, input/mask planes + status word
    uint32_t *host_status = nullptr;  // pinned host word for the IV length check
    hipStream_t stream;
    uint64_t bits;  // keystream bits every instance has produced through whole-state calls
    // Bits instance i produced beyond `bits` through mickey_generate_batch (empty until the
    // first such call), and their maximum.
    std::vector<uint64_t> extra;
    uint64_t max_extra = 0;
    int word_bits;
    int schedule;   // MICKEY_SCHED_*
    int transpose;  // MICKEY_TRANSPOSE_*
    int simds;      // SIMDs of the device (4 per compute unit)
    int device;
    uint32_t *chunk = nullptr;  // device, two bit-plane chunk buffers of the staged row-major path
    uint64_t chunk_clocks = 0;  // capacity of each in clocks (0: not allocated yet)
    uint32_t *snap = nullptr;   // device, 200 * nslices words: the registers before a call of
                                // several state-changing launches (restored if one fails)
    bool snap_valid = false;    // snap holds the registers of the last good state
    bool poisoned = false;      // a failure left the registers unknown (MICKEY_EDEVICE from now on)
    uint32_t *noalloc = nullptr;  // device address of this device's static scratch array
    hipStream_t side = nullptr;  // staged transposes and latency-mode requests run here
    hipEvent_t ev_gen[2] = {nullptr, nullptr}, ev_tp[2] = {nullptr, nullptr};
    // mickey_generate_batch: device scratch (metadata, packed states) and the pinned host
    // buffer its metadata is staged in, with the event of the last upload from it
    void *bmem = nullptr;
    size_t bmem_bytes = 0;
    void *bhost = nullptr;
    size_t bhost_bytes = 0;
    hipEvent_t bhost_ev = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

namespace mickey_host {

// Creates the side stream and its events on first use.
int ensure_side(mickey_state *st);
// The state's device scratch of at least `bytes` (grown on demand, kept until mickey_free).
int ensure_scratch(mickey_state *st, size_t bytes);
// Bits instance i has produced in total.
inline uint64_t instance_bits(const mickey_state *st, size_t i)
{
    return st->bits + (st->extra.empty() ? 0 : st->extra[i]);
}

}  // namespace mickey_host

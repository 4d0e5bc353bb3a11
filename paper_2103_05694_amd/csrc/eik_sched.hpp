// Device-wide soft-priority scheduler shared by the persistent kernels.
//
// The paper's asynchronous marching method (Algorithm "Asynchronous Marching
// Method", section "The Asynchronous Marching Method") pushes work with an
// integer priority floor(t / scale) into a concurrent scheduler that returns an
// approximately earliest item and tolerates priority inversions.  Here the work
// item is a grid tile and the scheduler is a window of NB bucket rings:
//
//  * a tile pushed with time t goes to bucket k = floor(t / delta), clamped to
//    the window [cur, cur + NB); ring k mod NB holds it;
//  * a claimer scans the NB rings from `cur` (one lane per ring, one ballot)
//    and takes from the first non-empty one, advancing `cur` past empty rings;
//  * inversions are allowed (late pushes below `cur`, clamped far pushes):
//    the operator is monotone and causal, so the order never changes results.
//
// Each ring is a bounded MPMC array of (sequence << 32 | tile) slots.  A tile is
// queued at most once at a time (see the tile state machine), so a ring never
// holds more than `ntiles` items and capacity = next_pow2(ntiles) suffices.
// Head/tail counters are never reset, so slot sequence numbers never repeat and
// stale slots from earlier solves are never mistaken for new items.
//
// Tile state word (one uint32 per tile):
//   bit0 Q  queued / needs another run       bit1 R  a workgroup is running it
//   bit2 V  interior of t holds real values  bit3 S  contains a point source
// Activation = fetch_or(Q) after a release fence; whoever turns an idle word
// (no Q, no R) into Q pushes the tile.  A runner turns Q into R with an
// acquiring RMW before it reads any t, and at the end either clears R (idle) or,
// if Q was set meanwhile, keeps Q and pushes the tile again.  So every change
// of a tile's halo or interior is followed by a run that starts after it, and
// at most one workgroup runs a tile at any time.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eik {

constexpr uint32_t kQ = 1u, kR = 2u, kV = 4u, kS = 8u;
constexpr int kMaxRings = 64;
constexpr int kCtrStride = 32;  // uint32 words between ring counters (128 B)

// device status flags
constexpr uint32_t kFlagDomain = 1u, kFlagLimit = 2u, kFlagBadSrc = 4u, kFlagWatchdog = 8u;

struct Sched {
    uint64_t* items;     // [nrings][cap]
    uint32_t* ctr;       // per ring r: ctr[r*kCtrStride + {0 head, 1 tail, 2 count}]
    uint32_t* tstate;    // [ntiles]
    int32_t* cur;        // lowest bucket of the window
    int32_t* pending;    // tiles queued or running
    unsigned long long* counters;  // [0] visits [1] point updates [2] relax passes
    uint32_t* flags;     // device status flags
    int32_t* poisoned;   // set on a watchdog expiry: the next reset re-initialises the rings
    int nrings;
    uint32_t cap_mask;
    double inv_delta;    // 1/delta, 0 => single bucket
    long long max_visits;  // 0 => unlimited
};

__device__ __forceinline__ uint32_t ld_acq(uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_rlx(uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_rlx(int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void set_flag(const Sched& s, uint32_t f) {
    __hip_atomic_fetch_or(s.flags, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (f & kFlagWatchdog)
        __hip_atomic_store(s.poisoned, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int64_t bucket_of(const Sched& s, double t) {
    if (s.inv_delta == 0.0) return 0;
    double k = floor(t * s.inv_delta);
    if (!(k < 1.0e15)) k = 1.0e15;
    return (int64_t)k;
}

// Enqueue `tile` with time key `t`.  The caller has already counted it in
// `pending`.  Single lane.
__device__ __forceinline__ void push_tile(const Sched& s, uint32_t tile, double t) {
    int64_t k = bucket_of(s, t);
    int64_t c = ld_rlx(s.cur);
    if (k < c) k = c;
    if (k > c + s.nrings - 1) k = c + s.nrings - 1;
    int r = (int)(k % s.nrings);
    uint32_t* ctr = s.ctr + r * kCtrStride;
    uint32_t slot = __hip_atomic_fetch_add(ctr + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t item = ((uint64_t)slot << 32) | tile;
    __hip_atomic_store(s.items + (size_t)r * (s.cap_mask + 1) + (slot & s.cap_mask), item,
                       __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(ctr + 2, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Count a newly activated tile and enqueue it.  Single lane.
__device__ __forceinline__ void activate_push(const Sched& s, uint32_t tile, double t) {
    __hip_atomic_fetch_add(s.pending, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    push_tile(s, tile, t);
}

// Mark `tile` as needing a run because data it reads changed (the caller has
// issued an agent-scope release fence after those writes).  Single lane.
__device__ __forceinline__ void activate(const Sched& s, uint32_t tile, double t) {
    uint32_t old = __hip_atomic_fetch_or(s.tstate + tile, kQ, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    if ((old & (kQ | kR)) == 0) activate_push(s, tile, t);
}

// Try to take one item from ring r.  Returns the tile or -1.  Single lane.
__device__ __forceinline__ int try_claim(const Sched& s, int r) {
    uint32_t* ctr = s.ctr + r * kCtrStride;
    int32_t old = (int32_t)__hip_atomic_fetch_sub(ctr + 2, 1u, __ATOMIC_ACQUIRE,
                                                  __HIP_MEMORY_SCOPE_AGENT);
    if (old <= 0) {
        __hip_atomic_fetch_add(ctr + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return -1;
    }
    uint32_t slot = __hip_atomic_fetch_add(ctr + 0, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t* p = s.items + (size_t)r * (s.cap_mask + 1) + (slot & s.cap_mask);
    // The producer that reserved this slot has already advanced the tail and is
    // about to store it; wait for the store with a bounded spin.
    for (long long spin = 0;; ++spin) {
        uint64_t it = __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(it >> 32) == slot) return (int)(uint32_t)it;
        if (spin > (1ll << 24)) {
            set_flag(s, kFlagWatchdog);
            return -2;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Called by all 64 lanes of one wave.  Returns a tile, or -1 when no work is
// left anywhere (pending == 0), or -2 on a watchdog expiry.
__device__ __forceinline__ int claim(const Sched& s) {
    const int lane = threadIdx.x & 63;
    long long idle = 0;
    for (;;) {
        int32_t c = ld_rlx(s.cur);
        int r = lane < s.nrings ? (int)(((int64_t)c + lane) % s.nrings) : 0;
        int32_t cnt = lane < s.nrings ? (int32_t)ld_rlx(s.ctr + r * kCtrStride + 2) : 0;
        unsigned long long mask = __ballot(cnt > 0);
        while (mask) {
            int j = __ffsll((long long)mask) - 1;
            mask &= mask - 1;
            int got = -1;
            if (lane == 0) {
                got = try_claim(s, (int)(((int64_t)c + j) % s.nrings));
                if (got >= 0 && j > 0)
                    __hip_atomic_fetch_max(s.cur, c + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            got = __shfl(got, 0);
            if (got >= 0 || got == -2) return got;
        }
        if (ld_rlx(s.pending) <= 0) return -1;
        if (++idle > (1ll << 22)) {
            if (lane == 0) set_flag(s, kFlagWatchdog);
            return -2;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// End of a run of `tile` by its runner.  Returns true if the tile was re-queued
// (Q was set during the run).  Single lane; caller passes the key for a requeue.
__device__ __forceinline__ bool finish_run(const Sched& s, uint32_t tile, double requeue_t) {
    uint32_t* w = s.tstate + tile;
    uint32_t old = ld_rlx(w);
    for (;;) {
        uint32_t nw = old & ~kR;
        uint32_t seen = old;
        if (__hip_atomic_compare_exchange_strong(w, &seen, nw, __ATOMIC_ACQ_REL, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)) {
            if (old & kQ) {
                push_tile(s, tile, requeue_t);  // stays counted in pending
                return true;
            }
            __hip_atomic_fetch_sub(s.pending, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        old = seen;
    }
}

}  // namespace eik

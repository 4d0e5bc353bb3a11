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
//  * a claimer takes work only from the current bucket `cur`; `cur` moves on
//    (to the next non-empty bucket) only once bucket `cur` is drained: nothing
//    queued in it and no tile claimed from it still running.  This is the
//    bucket discipline of delta-stepping: within a bucket any order and any
//    degree of parallelism, across buckets increasing time, so the number of
//    premature (later lowered again) tile runs stays small;
//  * pushes happen only from tiles running in bucket `cur` (or before the
//    solve starts), so `cur` cannot move while a push computes its ring;
//  * delta = 0 puts everything in one bucket (a plain FIFO worklist);
//  * the operator is monotone and causal, so none of this changes results.
//
// Each ring is a bounded MPMC array of 64-bit cells (sequence << 32 | tile),
// positions taken with fetch-add.  Its queued count and the number of runs
// claimed from it share one 64-bit word (running << 32 | count + 2^31), so a
// claim is one RMW (running + 1, count - 1) and one load shows whether the
// bucket is drained (nothing queued and nothing running at the same instant).  A cell for position p is free when its
// sequence equals p, full when it equals p + 1, and is freed for the next lap
// (sequence p + cap) by the consumer after reading: a producer never overwrites
// a cell whose item has been claimed but not yet read.  A tile is queued at most
// once at a time (tile state machine below), so a ring never holds more than
// `ntiles` items and capacity = next_pow2(max(ntiles, 2)) means no producer waits
// on an unclaimed item.  Positions and counters are never reset between solves
// (a solve ends with every ring drained), only re-initialised after a watchdog
// expiry.
//
// Tile state word (one uint32 per tile):
//   bit0 Q  queued / needs another run       bit1 R  a workgroup is running it
//   bit2 V  interior of t holds real values  bit3 S  contains a point source
// Activation = fetch_or(Q) after the writer's stores completed; whoever turns an idle word
// (no Q, no R) into Q pushes the tile.  A runner turns Q into R with an
// acquiring RMW before it reads any t, and at the end either clears R (idle) or,
// if Q was set meanwhile, keeps Q and pushes the tile again.  So every change
// of a tile's halo or interior is followed by a run that starts after it, and
// at most one workgroup runs a tile at any time.
//
// Memory ordering across the 8 XCDs (each with its own L2).  Every access to
// data another workgroup may touch concurrently -- arrival times, adjoint
// multipliers, tile states, queue cells and counters -- is a device-scope
// (agent) atomic, which gfx950 issues with the device-scope cache policy
// (loads and stores coherent at device scope without any cache maintenance).
// Ordering then only needs completion: a writer waits until its stores have
// been acknowledged (`stores_done`, s_waitcnt vmcnt(0) in every wave, then a
// barrier) before the RMW that hands the data over, and a reader issues its
// loads only after the RMW that took the data over has returned.  This replaces
// agent-scope release/acquire fences, whose L2 write-back / invalidate on every
// tile visit cost far more than the visit itself.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eik {

// Wait until every memory operation this wave issued has completed (device
// scope for the device-scope atomics used for shared data); also a compiler
// barrier.
__device__ __forceinline__ void stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

constexpr uint32_t kQ = 1u, kR = 2u, kV = 4u, kS = 8u;
// statistics words (64-bit, cleared by every reset): [0] visits [1] point
// updates [2] relax passes [3] visit-cap count [4] adjoint reference time
// [5..8] phase clocks [9] unused [10] workgroups [11] bucket advances
// [12] hand-offs [13..15] residual accumulators [16] operator evaluations
// [17] improving evaluations [18] evaluations that set the final value
constexpr int kCounters = 24;
constexpr int kMaxRings = 64;
// Each ring counter (head, tail, count + running) lives in its own 256-byte
// line, so polling one does not slow the atomics on the others.
constexpr int kCtrPad = 64;                 // uint32 words per counter line
constexpr int kCtrStride = 4 * kCtrPad;     // uint32 words per ring
constexpr int kCrWord = 2 * kCtrPad;        // offset of the count + running word
constexpr uint64_t kCountBias = 1ull << 31; // count is stored biased, so it may dip below 0
constexpr uint64_t kRunOne = 1ull << 32;

// device status flags
constexpr uint32_t kFlagDomain = 1u, kFlagLimit = 2u, kFlagBadSrc = 4u, kFlagWatchdog = 8u, kFlagBadStart = 16u;

struct Sched {
    uint64_t* items;     // [nrings][cap]
    uint32_t* ctr;       // ring counters, see ring_head / ring_tail / ring_cr
    uint32_t* tstate;    // [ntiles]
    int32_t* cur;        // lowest bucket of the window
    int32_t* pending;    // tiles queued or running
    unsigned long long* counters;  // statistics: [0] visits [1] point updates [2] relax passes ...
    uint32_t* flags;     // device status flags
    int32_t* poisoned;   // set on a watchdog expiry: the next reset re-initialises the rings
    int nrings;
    uint32_t cap_mask;
    double inv_delta;    // 1/delta, 0 => single bucket
    long long max_visits;  // 0 => unlimited
    int lookahead;       // claims may come from buckets cur .. cur + lookahead
    int horizon;         // 0, or k: a run settles only values below bucket (its bucket + k)
    int track;           // ablation operators: re-activate on any change (else on decrease)
    unsigned long long* timeline;  // NULL, or [0] start, [1] end, then (time, bucket) per advance
    int timeline_cap;    // advances the timeline can hold
};

__device__ __forceinline__ uint32_t* ring_head(const Sched& s, int r) { return s.ctr + r * kCtrStride; }
__device__ __forceinline__ uint32_t* ring_tail(const Sched& s, int r) { return s.ctr + r * kCtrStride + kCtrPad; }
__device__ __forceinline__ unsigned long long* ring_cr(const Sched& s, int r) {
    return (unsigned long long*)(s.ctr + r * kCtrStride + kCrWord);
}
__device__ __forceinline__ int32_t cr_count(uint64_t w) { return (int32_t)((int64_t)(w & 0xffffffffull) - (int64_t)kCountBias); }
__device__ __forceinline__ unsigned long long ld_cr(const Sched& s, int r) {
    return __hip_atomic_load(ring_cr(s, r), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void cr_add(const Sched& s, int r, uint64_t v) {
    __hip_atomic_fetch_add(ring_cr(s, r), (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t ld_acq(uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
// `pending`.  `base` is the bucket the pushing run was claimed from (0 before
// the solve starts): `cur` cannot pass it while that run is live and is at least
// base - lookahead, so buckets in [base, base + nrings - 1 - lookahead] never
// alias a bucket behind `cur`.  With count = false the ring's queued count is
// left to the caller, which must add it after its stores are done and before
// it ends the run (publish folds it into the end-of-run RMW).  Single lane.
__device__ __forceinline__ void push_tile(const Sched& s, uint32_t tile, double t, int64_t base,
                                          bool count = true) {
    int64_t k = bucket_of(s, t);
    if (k < base) k = base;
    if (k > base + s.nrings - 1 - s.lookahead) k = base + s.nrings - 1 - s.lookahead;
    int r = (int)(k % s.nrings);
    uint32_t pos = __hip_atomic_fetch_add(ring_tail(s, r), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t* cell = s.items + (size_t)r * (s.cap_mask + 1) + (pos & s.cap_mask);
    // wait until the previous lap's consumer has read this cell (bounded: that
    // consumer has already claimed it)
    for (long long spin = 0;; ++spin) {
        uint64_t it = __hip_atomic_load(cell, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(it >> 32) == pos) break;
        if (spin > (1ll << 24)) {
            set_flag(s, kFlagWatchdog);
            return;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    __hip_atomic_store(cell, ((uint64_t)(pos + 1u) << 32) | tile, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!count) return;
    // everything this wave did before (the live-work count included) completes
    // before the item becomes claimable
    stores_done();
    cr_add(s, r, 1);
}

// Push bucket of a time key as push_tile computes it.
__device__ __forceinline__ int64_t push_bucket(const Sched& s, double t, int64_t base) {
    int64_t k = bucket_of(s, t);
    if (k < base) k = base;
    if (k > base + s.nrings - 1 - s.lookahead) k = base + s.nrings - 1 - s.lookahead;
    return k;
}

// End of the runs claimed from `bucket` by this workgroup: its pushes were
// counted first (push_tile waits for that), so the bucket never looks drained
// while work it produced is in flight.  Single lane.
__device__ __forceinline__ void end_run(const Sched& s, int64_t bucket) {
    stores_done();
    cr_add(s, (int)(bucket % s.nrings), 0ull - kRunOne);
}

// Count a newly activated tile and enqueue it.  Single lane.
__device__ __forceinline__ void activate_push(const Sched& s, uint32_t tile, double t, int64_t base) {
    __hip_atomic_fetch_add(s.pending, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    push_tile(s, tile, t, base);
}

// Try to take one item from ring r: one RMW counts the claimer as running and
// takes one queued item.  Returns the tile, -1 (empty) or -2 (watchdog).
// Single lane.
__device__ __forceinline__ int try_claim(const Sched& s, int r) {
    const uint64_t old = __hip_atomic_fetch_add(ring_cr(s, r), (unsigned long long)(kRunOne - 1),
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cr_count(old) <= 0) {
        cr_add(s, r, 0ull - (kRunOne - 1));
        return -1;
    }
    uint32_t pos = __hip_atomic_fetch_add(ring_head(s, r), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t* cell = s.items + (size_t)r * (s.cap_mask + 1) + (pos & s.cap_mask);
    // The producer that reserved this position is about to fill the cell.
    for (long long spin = 0;; ++spin) {
        uint64_t it = __hip_atomic_load(cell, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(it >> 32) == pos + 1u) {
            // free the cell for the next lap
            __hip_atomic_store(cell, (uint64_t)(pos + s.cap_mask + 1u) << 32, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            return (int)(uint32_t)it;
        }
        if (spin > (1ll << 24)) {
            set_flag(s, kFlagWatchdog);
            return -2;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// Idle back-off: s_sleep takes an immediate, so sleep in units of 127.
__device__ __forceinline__ void idle_sleep(int units) {
    for (int i = 0; i < units; ++i) __builtin_amdgcn_s_sleep(127);
}

// Called by all 64 lanes of one wave.  Returns a tile and the bucket it came
// from (*bucket), counted as running there, or -1 when no work is left anywhere
// (pending == 0), or -2 on a watchdog expiry.
//
// The watchdog counts consecutive polls that saw no progress anywhere: the
// window's first count word (it changes with every claim, push and end of a
// run in the current bucket), the current bucket and the live-work count are
// compared with the previous poll's, and any change restarts the count.  So it
// fires only when nothing has moved for 2^19 polls (about 14 s with the
// back-off below), however long a valid solve takes.
//
// `cur_hint` is the window's lowest bucket as this workgroup last saw it (0
// before its first claim; `cur` never decreases).  A poll reads the window's
// count words at the hint and `cur` itself together, one round trip, and uses
// them only when `cur` still equals the hint; otherwise it reads again from the
// new value (the cost of the former sequential read).
__device__ __forceinline__ int claim(const Sched& s, int64_t* bucket, int32_t& cur_hint) {
    const int lane = threadIdx.x & 63;
    const int win = s.lookahead + 1;
    long long idle = 0;   // polls so far (sets the back-off)
    long long stall = 0;  // polls since anything last moved (the watchdog)
    unsigned long long seen_w = ~0ull;
    long long seen_cp = -1;
    for (;;) {
        const int32_t c = cur_hint;
        const int r = (int)(((int64_t)c + lane) % s.nrings);
        unsigned long long w = kCountBias;  // nothing queued, nothing running
        if (lane < win) w = ld_cr(s, r);
        const int32_t cnow = ld_rlx(s.cur);
        if (cnow != c) {
            cur_hint = cnow;
            continue;
        }
        const unsigned long long mask = __ballot(cr_count(w) > 0);
        if (mask) {
            // lowest bucket of the window with queued work
            const int j = __ffsll((long long)mask) - 1;
            int got = -1;
            if (lane == 0) got = try_claim(s, (int)(((int64_t)c + j) % s.nrings));
            got = __shfl(got, 0);
            if (got >= 0) {
                *bucket = (int64_t)c + j;
                return got;
            }
            if (got == -2) return -2;
            continue;
        }
        const unsigned long long w0 = __shfl(w, 0);
        int32_t pend_now = -1;
        if (w0 == kCountBias) {
            // bucket `cur` drained: move to the next bucket that has work
            // queued or still running (full scan).  A bucket whose runs (taken
            // through the lookahead window) are still live is not skipped:
            // their pushes may land in it, and its ring must not be reused
            // for a later bucket meanwhile.
            unsigned long long wf = kCountBias;
            if (lane < s.nrings) wf = ld_cr(s, r);
            const unsigned long long m2 = __ballot(wf != kCountBias) & ~1ull;
            if (m2) {
                const int j = __ffsll((long long)m2) - 1;
                if (lane == 0) {
                    int32_t expect = c;
                    if (__hip_atomic_compare_exchange_strong(s.cur, &expect, c + j, __ATOMIC_RELAXED,
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        const unsigned long long i = __hip_atomic_fetch_add(s.counters + 11, 1ull, __ATOMIC_RELAXED,
                                                                            __HIP_MEMORY_SCOPE_AGENT);
                        if (s.timeline && i < (unsigned long long)s.timeline_cap) {
                            __hip_atomic_store(s.timeline + 2 + 2 * i, (unsigned long long)wall_clock64(),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            __hip_atomic_store(s.timeline + 3 + 2 * i, (unsigned long long)(c + j),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        }
                    }
                }
                continue;
            }
            pend_now = ld_rlx(s.pending);
            if (pend_now <= 0) return -1;
        }
        const long long cp = ((long long)c << 32) ^ (long long)(uint32_t)pend_now;
        if (w0 != seen_w || cp != seen_cp) {
            stall = 0;  // something moved since the last poll
            seen_w = w0;
            seen_cp = cp;
        }
        ++idle;
        if (++stall > (1ll << 19)) {
            if (lane == 0) set_flag(s, kFlagWatchdog);
            return -2;
        }
        // exponential back-off, ~0.1 us doubling up to ~25 us, keeps idle
        // workgroups from flooding the counters the busy ones need
        if (idle < 2) __builtin_amdgcn_s_sleep(4);
        else if (idle < 3) __builtin_amdgcn_s_sleep(16);
        else if (idle < 4) __builtin_amdgcn_s_sleep(64);
        else idle_sleep(idle < 5 ? 1 : (idle < 6 ? 2 : (idle < 7 ? 4 : 8)));
    }
}

// End of a run of `tile`, executed by the 64 lanes of wave 0 after every wave
// of the block has written its results and waited for them (stores_done).
//   nb[f]   neighbour f's state word with bit 30 set when it exists,
//   nid[f]  its tile id, face[f] the priority key bits of the lowered values on
//           face f (kInfBits: nothing lowered there),
//   first   the run wrote this tile's interior for the first time (sets V).
// The tile's own state word drops R (and gains V); the RMW's return also says
// whether the tile was activated during the run.  Lanes 0..5 activate the
// neighbours in parallel, after that RMW when neighbours read V (order_v).
// The live-work count changes once, by (#newly queued neighbours + requeue -
// 1), before any push makes new items claimable, so it never under-counts.
// `self_key` (bits of a time, kInfBits for none) requeues the tile itself with
// at most that key: the run left points whose new values lie beyond its
// bucket.
// With `cont`, the lowest-key newly activated neighbour that falls in this
// run's own bucket is not pushed: it is returned (state Q, counted live and
// counted running in `bucket`) for this workgroup to run next, which saves a
// push, a poll and a claim on the front's critical path.  Returns that tile or
// -1 (the run has then ended), uniform across the wave.
__device__ __forceinline__ int publish(const Sched& s, uint64_t* tkey, uint32_t tile, int64_t bucket, bool first,
                                       const uint32_t* nb, const uint32_t* nid,
                                       const unsigned long long* face, bool cont = false,
                                       unsigned long long self_key = kInfBits, bool order_v = true) {
    const int lane = threadIdx.x & 63;
    // lane 0 updates the tile's own word before the activations when readers
    // of the neighbours rely on V (order_v); otherwise lane 6 does it
    // alongside them
    const int ol = order_v ? 0 : 6;
    uint32_t own = 0;
    if (lane == ol) {
        // work of this tile left for a later bucket: activate the tile itself
        // while R still keeps everyone else from pushing it
        if (self_key != kInfBits)
            __hip_atomic_fetch_or(s.tstate + tile, kQ, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        own = __hip_atomic_fetch_xor(s.tstate + tile, kR | (first ? kV : 0u), __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
    }
    // with order_v the RMW has returned here, so V is visible before any
    // neighbour is activated
    if (order_v) own = __shfl(own, 0);
    bool want = false;
    uint32_t n = 0;
    unsigned long long fk = kInfBits;
    if (lane < 6) {
        fk = face[lane];
        if ((nb[lane] & 0x40000000u) && fk != kInfBits) {
            n = nid[lane];
            uint32_t old = __hip_atomic_fetch_or(s.tstate + n, kQ, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((old & (kQ | kR)) == 0) {
                want = true;
            } else if (old & kR) {
                __hip_atomic_fetch_min((unsigned long long*)(tkey + n), fk, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    if (!order_v) own = __shfl(own, ol);
    const bool requeue = (own & kQ) != 0;
    const unsigned long long wm = __ballot(want);
    const int k = __popcll(wm);
    int cl = -1;
    if (cont && wm) {
        const bool cand = want && push_bucket(s, as_f64(fk), bucket) == bucket;
        unsigned long long key = cand ? fk : ~0ull;
        // minimum over lanes 0..7 (the six face lanes)
#pragma unroll
        for (int off = 1; off < 8; off <<= 1) {
            const unsigned long long o = __shfl_xor(key, off);
            key = o < key ? o : key;
        }
        key = __shfl(key, 0);
        const unsigned long long cm = __ballot(cand && fk == key);
        if (cm) cl = __ffsll((long long)cm) - 1;
    }
    if (lane == 0) {
        const int delta = k + (requeue ? 1 : 0) - 1;
        if (delta != 0)
            __hip_atomic_fetch_add(s.pending, delta, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // Pushes into this run's own bucket leave their queued count to the one
    // RMW below, which also ends the run (or, for a hand-on, just adds them):
    // their cells are stored first, and the run stays counted until that RMW,
    // so the bucket never looks drained with work of it uncounted.  Pushes to
    // other buckets count themselves, and that completes before the RMW too.
    const bool pushme = want && lane != cl;
    const bool same = pushme && push_bucket(s, as_f64(fk), bucket) == bucket;
    if (pushme) push_tile(s, n, as_f64(fk), bucket, !same);
    bool rq_same = false;
    if (lane == 0 && requeue) {
        uint64_t kb = __hip_atomic_exchange((unsigned long long*)(tkey + tile), kInfBits, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
        if (self_key < kb) kb = self_key;
        const double key = kb == kInfBits ? 0.0 : as_f64(kb);
        rq_same = push_bucket(s, key, bucket) == bucket;
        push_tile(s, tile, key, bucket, !rq_same);
    }
    const uint64_t nsame = (uint64_t)__popcll(__ballot(same)) + (uint64_t)__popcll(__ballot(rq_same));
    const int ring = (int)(bucket % s.nrings);
    if (cl >= 0) {
        if (lane == 0 && nsame) {
            stores_done();
            cr_add(s, ring, nsame);
        }
        return (int)__shfl(n, cl);
    }
    // this run's own pushes are counted: the bucket it came from may now drain
    if (lane == 0) {
        stores_done();
        cr_add(s, ring, nsame - kRunOne);
    }
    return -1;
}

// Drop a claimed tile without running it (visit cap reached).  Lane 0.
__device__ __forceinline__ void drop_run(const Sched& s, uint32_t tile, int64_t bucket) {
    const uint32_t old = __hip_atomic_fetch_xor(s.tstate + tile, kR, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old & kQ) push_tile(s, tile, 0.0, bucket);
    else __hip_atomic_fetch_sub(s.pending, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    end_run(s, bucket);
}

}  // namespace eik

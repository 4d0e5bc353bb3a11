// Forward kernels: per-solve reset, source placement, the persistent
// soft-priority tile solver, finalisation and the upwind-parent record.
//
// The persistent solver realises the paper's asynchronous marching method
// (Algorithm "Asynchronous Marching Method") with a tile of the grid as the unit
// of work: a workgroup claims the approximately earliest active tile, stages
// its times, the 1-cell halo and the per-point constants in LDS, applies the
// update operator (Algorithm "Eikonal Update Operator" with the exactly monotone
// rounding) to dirty points until nothing in the tile changes, writes the
// lowered points back and activates the face neighbours whose halo changed with
// the priority floor(t / delta).  Theorem 1 (monotone + causal => one fixed
// point for every order) is what makes the racing, out-of-order schedule
// produce the same bits as sequential fast marching.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "eik_op.hpp"
#include "eik_sched.hpp"

namespace eik {

// One problem of a (possibly batched) launch.
struct Prob {
    int32_t nx, ny, nz;      // points per axis
    int32_t ntx, nty, ntz;   // tiles per axis
    int64_t pt_off;          // first point in the packed arrays
    int32_t tile_off;        // first global tile id
    int32_t kind;            // 0 speed (q = h/v), 1 slowness (q = h*s)
    double h;
};

// Problem table of a launch.  A single problem travels by value in the kernel
// arguments (no upload, no host synchronisation); batches read the device table.
struct ProbTable {
    const Prob* probs;       // device table, used when nprob > 1
    const int64_t* src_off;  // device source offsets, used when nprob > 1
    int nprob;
    Prob p0;                 // the problem when nprob == 1
    int64_t nsrc0;           // its source count
};

struct SolveArgs {
    ProbTable pt;
    const double* field;
    double* t;
    uint64_t* tkey;          // [ntiles] pending requeue key (bits of a positive double)
    const double* work_ref;  // NULL, or the final times: classify every evaluation
    // rectilinear grids (OP 4): reciprocal spacings per axis and index, laid
    // out [wm_x (nx), wp_x (nx), wm_y (ny), wp_y (ny), wm_z (nz), wp_z (nz)]
    const double* rw;
    Sched s;
};

__device__ __forceinline__ Prob prob_of_tile(const ProbTable& T, int tile) {
    if (T.nprob == 1) return T.p0;
    int lo = 0, hi = T.nprob - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (T.probs[mid].tile_off <= tile) lo = mid; else hi = mid - 1;
    }
    return T.probs[lo];
}

__device__ __forceinline__ Prob prob_of_point(const ProbTable& T, long long g) {
    if (T.nprob == 1) return T.p0;
    int lo = 0, hi = T.nprob - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (T.probs[mid].pt_off <= g) lo = mid; else hi = mid - 1;
    }
    return T.probs[lo];
}

__device__ __forceinline__ Prob prob_of_source(const ProbTable& T, long long g) {
    if (T.nprob == 1) return T.p0;
    int lo = 0, hi = T.nprob - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (T.src_off[mid] <= g) lo = mid; else hi = mid - 1;
    }
    return T.probs[lo];
}

__device__ __forceinline__ double field_q(double f, double h, int kind, bool& ok) {
    double q = kind == 0 ? h / f : h * f;
    double c = q * q;
    ok = (f > 0.0) && (f < inf64()) && (c > 0.0) && (c < inf64());
    return q;
}

// ---------------------------------------------------------------------------
// per-solve set-up
// ---------------------------------------------------------------------------

// Clears tile states and requeue keys, the window, counters and flags.  When the
// previous solve on this workspace ended abnormally (`poisoned`), or the caller
// asks for it (`force_wipe`: memory whose contents are not known yet), it also
// re-initialises the rings so no stale slot can be taken for a new item.
__global__ void k_reset(Sched s, uint64_t* tkey, int ntiles, int32_t* srclist_count,
                        long long ring_words, int force_wipe) {
    const bool wipe = force_wipe || __hip_atomic_load(s.poisoned, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long i0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (long long i = i0; i < ntiles; i += stride) {
        s.tstate[i] = 0u;
        tkey[i] = kInfBits;
    }
    if (wipe) {
        // cell i of every ring starts free for position i (lap 0)
        const long long cap = (long long)s.cap_mask + 1;
        for (long long i = i0; i < ring_words; i += stride) s.items[i] = (uint64_t)(i % cap) << 32;
        // head = tail = 0; count word = bias (0 queued, 0 running)
        for (long long i = i0; i < (long long)s.nrings * kCtrStride; i += stride)
            s.ctr[i] = (i % kCtrStride) == kCrWord ? (uint32_t)kCountBias : 0u;
    }
    if (i0 == 0) {
        if (s.timeline) {
            s.timeline[0] = wall_clock64();
            s.timeline[1] = 0ull;
        }
        *s.cur = 0;
        *s.pending = 0;
        *s.flags = 0u;
        for (int i = 0; i < kCounters; ++i) s.counters[i] = 0ull;
        *srclist_count = 0;
    }
}

template <int TX, int TY, int TZ>
__device__ __forceinline__ uint32_t tile_of_point(const Prob& P, int64_t local) {
    int64_t x = local % P.nx, y = (local / P.nx) % P.ny, z = local / ((int64_t)P.nx * P.ny);
    return (uint32_t)(P.tile_off + ((z / TZ) * P.nty + (y / TY)) * P.ntx + (x / TX));
}

__device__ __forceinline__ bool src_ok(const Prob& P, int64_t idx, double t0) {
    int64_t n = (int64_t)P.nx * P.ny * P.nz;
    return idx >= 0 && idx < n && t0 >= 0.0 && t0 < inf64() && !signbit(t0);
}

// Marks source tiles (S) and lists each one once.
template <int TX, int TY, int TZ>
__global__ void k_src_mark(ProbTable T, const int64_t* src_idx, const double* src_t0, long long nsrc,
                           Sched s, int32_t* srclist, int32_t* srclist_count) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g == 0) *s.poisoned = 0;  // the reset before this kernel has wiped the rings
    if (g >= nsrc) return;
    const Prob P = prob_of_source(T, g);
    int64_t idx = src_idx[g];
    double t0 = src_t0 ? src_t0[g] : 0.0;
    if (!src_ok(P, idx, t0)) {
        set_flag(s, kFlagBadSrc);
        return;
    }
    uint32_t tile = tile_of_point<TX, TY, TZ>(P, idx);
    uint32_t old = __hip_atomic_fetch_or(s.tstate + tile, kS, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!(old & kS)) {
        int k = __hip_atomic_fetch_add(srclist_count, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        srclist[k] = (int32_t)tile;
    }
}

// t := +inf at every point of the launch (grid-stride), before the sources
// are placed: a solve starts from the upper bound +inf everywhere.
__global__ void k_fill_inf(long long npts_total, double* t) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < npts_total; i += stride)
        t[i] = inf64();
}

// Writes each source as -t0 (the sign bit marks a fixed point during the solve;
// min over duplicates through the signed image, where -0.0 is the smallest) and
// queues its tile.
template <int TX, int TY, int TZ>
__global__ void k_src_place(ProbTable T, const int64_t* src_idx, const double* src_t0, long long nsrc,
                            double* t, Sched s) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nsrc) return;
    const Prob P = prob_of_source(T, g);
    int64_t idx = src_idx[g];
    double t0 = src_t0 ? src_t0[g] : 0.0;
    if (!src_ok(P, idx, t0)) return;
    long long* ti = (long long*)(t + P.pt_off + idx);
    __hip_atomic_fetch_min(ti, (long long)as_u64(-t0), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t tile = tile_of_point<TX, TY, TZ>(P, idx);
    uint32_t old = __hip_atomic_fetch_or(s.tstate + tile, kQ | kV, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    if (!(old & kQ)) activate_push(s, tile, t0, 0);
}

// Restores +t0 at the sources.
__global__ void k_src_unsign(ProbTable T, const int64_t* src_idx, const double* src_t0, long long nsrc,
                             double* t) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nsrc) return;
    const Prob P = prob_of_source(T, g);
    int64_t idx = src_idx[g];
    double t0 = src_t0 ? src_t0[g] : 0.0;
    if (!src_ok(P, idx, t0)) return;
    double* ti = t + P.pt_off + idx;
    *ti = fabs(*ti);
}

// ---------------------------------------------------------------------------
// warm start: resume from an upper bound of the solution
// ---------------------------------------------------------------------------

// Checks a caller-supplied starting state and records each tile's smallest
// value (bits of a non-negative double; kInfBits when the tile is all +inf).
// A value that is NaN or has its sign bit set (the solver's source marker) is
// not a valid upper bound: it raises kFlagBadStart and is replaced by +inf, so
// the solve still runs on a valid state.
template <int TX, int TY, int TZ>
__global__ void k_warm_prep(ProbTable T, int ntiles, double* t, uint64_t* tile_min, Sched s) {
    __shared__ unsigned long long s_m;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const Prob P = prob_of_tile(T, tile);
        const int tl = tile - P.tile_off;
        const int tx = tl % P.ntx, ty = (tl / P.ntx) % P.nty, tz = tl / (P.ntx * P.nty);
        if (threadIdx.x == 0) s_m = kInfBits;
        __syncthreads();
        unsigned long long m = kInfBits;
        for (int i = threadIdx.x; i < TX * TY * TZ; i += blockDim.x) {
            const int lx = i % TX, ly = (i / TX) % TY, lz = i / (TX * TY);
            const int x = tx * TX + lx, y = ty * TY + ly, z = tz * TZ + lz;
            if (x < P.nx && y < P.ny && z < P.nz) {
                double* p = t + P.pt_off + ((int64_t)z * P.ny + y) * P.nx + x;
                const double v = *p;
                if (v != v || signbit(v)) {
                    set_flag(s, kFlagBadStart);
                    *p = inf64();
                } else if (as_u64(v) < m) {
                    m = as_u64(v);
                }
            }
        }
        if (m != kInfBits) atomicMin(&s_m, m);
        __syncthreads();
        if (threadIdx.x == 0) tile_min[tile] = s_m;
        __syncthreads();
    }
}

// Queues every tile that has a finite value in itself or in a face neighbour
// (any other tile can only change once a neighbour lowers its face, which
// activates it), keyed by the smallest of those values.  Tiles already queued
// (the source tiles) are left alone.  Their state words were cleared by the
// reset, so every first run relaxes all of its points.
__global__ void k_warm_push(ProbTable T, int ntiles, const uint64_t* tile_min, Sched s) {
    for (int tile = blockIdx.x * blockDim.x + threadIdx.x; tile < ntiles; tile += gridDim.x * blockDim.x) {
        const Prob P = prob_of_tile(T, tile);
        const int tl = tile - P.tile_off;
        const int t3[3] = {tl % P.ntx, (tl / P.ntx) % P.nty, tl / (P.ntx * P.nty)};
        const int lim[3] = {P.ntx, P.nty, P.ntz};
        uint64_t key = tile_min[tile];
        for (int f = 0; f < 6; ++f) {
            int nt[3] = {t3[0], t3[1], t3[2]};
            nt[f >> 1] += (f & 1) ? 1 : -1;
            if (nt[f >> 1] < 0 || nt[f >> 1] >= lim[f >> 1]) continue;
            const uint64_t k = tile_min[P.tile_off + (nt[2] * P.nty + nt[1]) * P.ntx + nt[0]];
            if (k < key) key = k;
        }
        if (key == kInfBits) continue;
        const uint32_t old = __hip_atomic_fetch_or(s.tstate + tile, kQ, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (!(old & kQ)) activate_push(s, (uint32_t)tile, as_f64(key), 0);
    }
}

// ---------------------------------------------------------------------------
// the persistent solver
// ---------------------------------------------------------------------------

template <int TX, int TY, int TZ, int NT>
struct TileCfg {
    static constexpr bool D3 = TZ > 1;
    static constexpr int SY = TX + 2;
    static constexpr int SZ = (TX + 2) * (TY + 2);
    static constexpr int HZ = D3 ? TZ + 2 : 1;
    static constexpr int ZOFF = D3 ? 1 : 0;
    static constexpr int NLDS = SZ * HZ;
    static constexpr int NP = TX * TY * TZ;
    static constexpr int NPT = NP / NT;
    static_assert(NP % NT == 0, "tile points must be a multiple of the block size");
    static_assert(NT % 64 == 0, "block must be whole waves");
    __device__ static constexpr int lds(int lx, int ly, int lz) {
        return (lz + ZOFF) * SZ + (ly + 1) * SY + (lx + 1);
    }
};

__device__ __forceinline__ double hload(const double* p) {
    // Halo cells belong to tiles other workgroups may be writing right now.
    uint64_t u = __hip_atomic_load((const uint64_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return fabs(as_f64(u));
}

__device__ __forceinline__ void tstore(double* p, double v) {
    __hip_atomic_store((uint64_t*)p, as_u64(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Minimum over the 64 lanes of a wave (every lane gets it).
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = nmin(v, __shfl_xor(v, off));
    return v;
}

// Dirty flags of the in-tile relaxation: one byte per point, stored so that
// the NPT points of one thread (p = tid + j * NT) are adjacent and one LDS
// access reads or clears all of them.
template <int NT, int NPT>
__device__ __forceinline__ int didx(int p) {
    return (p % NT) * NPT + p / NT;
}
template <int NPT>
__device__ __forceinline__ uint32_t ld_flags(const uint8_t* f) {
    if constexpr (NPT == 4) return *(const uint32_t*)f;
    else if constexpr (NPT == 2) return *(const uint16_t*)f;
    else return *f;
}
template <int NPT>
__device__ __forceinline__ void st_flags(uint8_t* f, uint32_t v) {
    if constexpr (NPT == 4) *(uint32_t*)f = v;
    else if constexpr (NPT == 2) *(uint16_t*)f = (uint16_t)v;
    else *f = (uint8_t)v;
}

// OP selects the operator: 0 the exact monotone d-bar (the solver), 1 d-hat,
// 2 d-tilde (two-dimensional precision ablation only; see apply_op).
// COUNT adds the work classification (A.work_ref must then be set).
// Registers are capped for three waves per SIMD with blocks of up to 256
// threads (three blocks per compute unit) and four with larger blocks (two
// 512-thread blocks or one 1024-thread block per compute unit).  Compacted
// passes on 3D tiles also take four (four 256-thread blocks per compute unit
// keep more tiles in flight).  The rectilinear operator on 3D tiles takes four
// with one point a thread and two with two points a thread on 512 threads
// (16x8x8 and larger), where it would spill.  The per-workgroup statistics
// sit in LDS, not in registers, so that these budgets hold without spills.
template <int TX, int TY, int TZ, int NT, int OP = 0, bool COUNT = false, bool PACK = false>
__global__ void __launch_bounds__(NT)
    __attribute__((amdgpu_waves_per_eu(OP == 4 && TZ > 1 && NT == 512 && TX * TY * TZ > NT ? 2 : ((NT > 256 || (PACK && TZ > 1)) ? 4 : 3)))) k_solve(SolveArgs A) {
    using C = TileCfg<TX, TY, TZ, NT>;
    constexpr int NPT = C::NPT;
    static_assert(NPT == 1 || NPT == 2 || NPT == 4, "1, 2 or 4 points per thread");
    constexpr uint32_t kAllDirty = NPT == 4 ? 0x01010101u : (NPT == 2 ? 0x0101u : 0x01u);
    __shared__ double sT[C::NLDS];
    __shared__ double sQ[PACK ? C::NP : 1];        // constants (PACK: any thread may relax a point)
    __shared__ double sTin[PACK ? C::NP : 1];      // PACK: the values staged (not held in registers
                                                   // through the passes)
    __shared__ uint16_t sList[PACK ? C::NP : 1];   // PACK: the pass's dirty points, compacted
    __shared__ int s_cnt[2];                       // PACK: list lengths
    // dirty flags, two buffers (read in one pass, marked for the next); the
    // NT bytes past the NP flags are per-thread sinks that let the marking
    // store without branching
    __shared__ __align__(4) uint8_t sDirty[2][C::NP + NT];
    __shared__ int s_more[3];  // per pass (mod 3): some wave marked a point
    // rectilinear grids: the tile's reciprocal spacings, [wm_x | wp_x | wm_y |
    // wp_y | wm_z | wp_z] over its TX, TY, TZ coordinates
    __shared__ double sW[OP == 4 ? 2 * (TX + TY + TZ) : 1];
    __shared__ int s_tile;
    __shared__ int64_t s_bucket;
    __shared__ uint32_t s_state;
    __shared__ uint32_t s_nb[6];
    __shared__ uint32_t s_nid[6];
    __shared__ unsigned long long s_face[6];
    __shared__ unsigned int s_upd;
    __shared__ unsigned long long s_pend;  // smallest value left beyond the bucket (bits)
    __shared__ int s_next;  // tile handed on by the previous run's publish, or -1
    // per-workgroup statistics, kept by thread 0 in LDS (not in registers
    // through the passes) and flushed once at exit: [0..3] phase times on the
    // 100 MHz wall clock (claim, stage, relax, write + publish), [4] visits,
    // [5] point updates, [6] passes, [7] hand-offs, [8] the last phase mark
    __shared__ unsigned long long s_stat[9];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const unsigned long long lanes_below = (1ull << lane) - 1ull;
    (void)lanes_below;
    const Sched& S = A.s;
    // per-wave work classification (with A.work_ref): operator evaluations,
    // those that lowered the value, those that set the final value
    unsigned long long w_eval = 0, w_imp = 0, w_good = 0;
    if (tid == 0) {
        s_next = -1;
        s_bucket = 0;
        for (int i = 0; i < 8; ++i) s_stat[i] = 0;
        s_stat[8] = wall_clock64();
    }

    int32_t cur_hint = 0;  // wave 0: the window's lowest bucket as last seen
    for (;;) {
        // ---- claim (or take the tile handed on) ----------------------------
        if (tid < 64) {
            int64_t bucket = s_bucket;
            int tile = s_next;
            if (tile < 0) tile = claim(S, &bucket, cur_hint);
            else if (tid == 0) ++s_stat[7];
            if (tid == 0) {
                s_next = -1;
                s_tile = tile;
                s_bucket = bucket;
                if (tile >= 0) {
                    // Q -> R; every load of this run is issued after it returned
                    uint32_t st = __hip_atomic_fetch_xor(S.tstate + tile, kQ | kR, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                    if ((st & (kQ | kR)) != kQ) set_flag(S, kFlagWatchdog);
                    if (S.max_visits > 0) {
                        unsigned long long v = __hip_atomic_fetch_add(S.counters + 3, 1ull, __ATOMIC_RELAXED,
                                                                      __HIP_MEMORY_SCOPE_AGENT);
                        if ((long long)v >= S.max_visits) {
                            set_flag(S, kFlagLimit);
                            st |= 0x80000000u;  // skip marker
                        }
                    }
                    s_state = st;
                }
            }
        }
        __syncthreads();
        const int tile = s_tile;
        if (tile < 0) break;
        const uint32_t st = s_state;
        const Prob P = prob_of_tile(A.pt, tile);
        const int tl = tile - P.tile_off;
        const int tx = tl % P.ntx, ty = (tl / P.ntx) % P.nty, tz = tl / (P.ntx * P.nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
        if (tid == 0) {
            ++s_stat[4];
            const unsigned long long now = wall_clock64();
            s_stat[0] += now - s_stat[8];
            s_stat[8] = now;
        }

        if (st & 0x80000000u) {  // visit cap reached: drop the tile
            if (tid == 0) drop_run(S, (uint32_t)tile, s_bucket);
            __syncthreads();
            continue;
        }
        const bool visited = (st & kV) != 0;

        // face neighbours x-, x+, y-, y+, z-, z+ (bit 30: the tile exists)
        if (tid < 6) {
            int d = tid >> 1, side = tid & 1;
            int nt[3] = {tx, ty, tz};
            int lim[3] = {P.ntx, P.nty, P.ntz};
            nt[d] += side ? 1 : -1;
            uint32_t w = 0, nid = 0;
            if (nt[d] >= 0 && nt[d] < lim[d]) {
                nid = (uint32_t)(P.tile_off + (nt[2] * P.nty + nt[1]) * P.ntx + nt[0]);
                w = 0x40000000u;
            }
            s_nb[tid] = w;
            s_nid[tid] = nid;
            s_face[tid] = kInfBits;
        }
        if (tid == 0) {
            s_upd = 0u;
            s_pend = kInfBits;
            s_more[1] = 0;
            s_more[2] = 0;
            s_cnt[0] = 0;
            s_cnt[1] = 0;
        }
        // Optional bucket horizon (k = S.horizon > 0): a run settles only
        // values with floor(r / delta) < b + k, b its bucket (with k = 1 the
        // bucket discipline of delta-stepping).  A lower value never depends on
        // a higher one (the operator is causal), so nothing below the horizon
        // is lost; larger candidates are left for a later run of this tile,
        // keyed by the smallest of them, instead of being written and
        // propagated now as provisional values.
        const double hz = (double)(s_bucket + S.horizon);

        // ---- stage the tile and its halo in LDS ----------------------------
        // t starts at +inf everywhere, so every in-grid value read here is a
        // valid upper bound.  Every load of the stage (field and t of the
        // thread's points, its halo cells) is issued before any is used, so the
        // stage costs one memory round trip rather than one per load.
        double t_in[NPT];   // the values staged (what the run started from)
        double t_own[NPT];  // the thread's points' current values
        double q_own[NPT];  // and their constants (0: not relaxed)
        if constexpr (OP == 4) {
            // the weights of the tile's coordinates (clamped past the grid's
            // end, where no point is relaxed); read-only, ordered for the
            // relaxation by the barrier that ends the stage
            constexpr int NW = 2 * (TX + TY + TZ);
            for (int w = tid; w < NW; w += NT) {
                int k = w, axis = 0;
                if (k >= 2 * TX) {
                    k -= 2 * TX;
                    axis = 1;
                    if (k >= 2 * TY) {
                        k -= 2 * TY;
                        axis = 2;
                    }
                }
                const int n = axis == 0 ? TX : (axis == 1 ? TY : TZ);
                const int side = k >= n ? 1 : 0;
                const int i = k - side * n;
                const int g0 = axis == 0 ? x0 : (axis == 1 ? y0 : z0);
                const int gn = axis == 0 ? P.nx : (axis == 1 ? P.ny : P.nz);
                const int base = axis == 0 ? 0 : (axis == 1 ? 2 * P.nx : 2 * (P.nx + P.ny));
                sW[w] = A.rw[base + side * gn + min(g0 + i, gn - 1)];
            }
        }
        uint32_t live = 0;  // bit j: point j is in the grid and not a source
        {
            constexpr int NXF = 2 * TY * TZ, NYF = 2 * TX * TZ, NZF = C::D3 ? 2 * TX * TY : 0;
            constexpr int NH = NXF + NYF + NZF;
            constexpr int HPT = (NH + NT - 1) / NT;  // halo cells per thread
            double fv[NPT], tv[NPT], hv[HPT];
            int hl[HPT];
            uint32_t inb = 0;
#pragma unroll
            for (int j = 0; j < NPT; ++j) {
                const int p = tid + j * NT;
                const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
                const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
                fv[j] = 0.0;
                tv[j] = inf64();
                if (x < P.nx && y < P.ny && z < P.nz) {
                    const int64_t gi = P.pt_off + ((int64_t)z * P.ny + y) * P.nx + x;
                    fv[j] = A.field[gi];
                    tv[j] = as_f64(__hip_atomic_load((const uint64_t*)(A.t + gi), __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT));
                    inb |= 1u << j;
                }
            }
#pragma unroll
            for (int k = 0; k < HPT; ++k) {
                const int i = tid + k * NT;
                hl[k] = -1;
                hv[k] = inf64();
                if (i < NH) {
                    int lx, ly, lz;
                    if (i < NXF) {
                        int side = i / (TY * TZ), r = i % (TY * TZ);
                        ly = r % TY; lz = r / TY; lx = side ? TX : -1;
                    } else if (i < NXF + NYF) {
                        int k2 = i - NXF, side = k2 / (TX * TZ), r = k2 % (TX * TZ);
                        lx = r % TX; lz = r / TX; ly = side ? TY : -1;
                    } else {
                        int k2 = i - NXF - NYF, side = k2 / (TX * TY), r = k2 % (TX * TY);
                        lx = r % TX; ly = r / TX; lz = side ? TZ : -1;
                    }
                    hl[k] = C::lds(lx, ly, lz);
                    const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
                    // the sign (a source) is dropped after all loads are out:
                    // an operation on the loaded value inside this branch
                    // would wait for it here
                    if (x >= 0 && x < P.nx && y >= 0 && y < P.ny && z >= 0 && z < P.nz)
                        hv[k] = as_f64(__hip_atomic_load((const uint64_t*)(A.t + P.pt_off +
                                                                           ((int64_t)z * P.ny + y) * P.nx + x),
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                }
            }
#pragma unroll
            for (int j = 0; j < NPT; ++j) {
                const int p = tid + j * NT;
                const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
                double tvj = tv[j], q = 0.0;
                if ((inb >> j) & 1u) {
                    bool ok;
                    q = field_q(fv[j], P.h, P.kind, ok);
                    if (!ok) {
                        set_flag(S, kFlagDomain);
                        q = 0.0;
                    }
                    if (signbit(tvj)) {  // a source: fixed
                        tvj = fabs(tvj);
                        q = 0.0;
                    }
                }
                if (q > 0.0) live |= 1u << j;
                sT[C::lds(lx, ly, lz)] = tvj;
                q_own[j] = q;
                if constexpr (PACK) {
                    sQ[p] = q;
                    sTin[p] = tvj;
                }
                t_in[j] = tvj;
                t_own[j] = tvj;
            }
#pragma unroll
            for (int k = 0; k < HPT; ++k)
                if (hl[k] >= 0) sT[hl[k]] = fabs(hv[k]);
        }
        st_flags<NPT>(sDirty[1] + tid * NPT, 0u);
        __syncthreads();
        // First pass: every point on a first run, in a tile holding a source
        // (placed before its first run, which already counts as visited) and
        // with a horizon (points left beyond it last time); otherwise the
        // interior is still at the fixed point its last run left given the old
        // halo, so only boundary points next to a halo value below their own
        // can improve.
        {
            uint32_t seed = 0;
            if (!visited || (st & kS) || S.horizon > 0) {
                seed = kAllDirty;
            } else {
#pragma unroll
                for (int j = 0; j < NPT; ++j) {
                    const int p = tid + j * NT;
                    const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
                    const int L = C::lds(lx, ly, lz);
                    // the point and its six neighbours, read together
                    const double c = sT[L];
                    const double nxm = sT[L - 1], nxp = sT[L + 1], nym = sT[L - C::SY], nyp = sT[L + C::SY];
                    const double nzm = C::D3 ? sT[L - C::SZ] : inf64(), nzp = C::D3 ? sT[L + C::SZ] : inf64();
                    // smallest halo value next to the point (interior cells
                    // do not count: they have not changed since the last run)
                    double hm = inf64();
                    if (lx == 0 && nxm < hm) hm = nxm;
                    if (lx == TX - 1 && nxp < hm) hm = nxp;
                    if (ly == 0 && nym < hm) hm = nym;
                    if (ly == TY - 1 && nyp < hm) hm = nyp;
                    if (C::D3) {
                        if (lz == 0 && nzm < hm) hm = nzm;
                        if (lz == TZ - 1 && nzp < hm) hm = nzp;
                    }
                    if (hm < c) seed |= 1u << (8 * j);
                }
            }
            st_flags<NPT>(sDirty[0] + tid * NPT, seed);
        }
        if (tid == 0) {
            const unsigned long long now = wall_clock64();
            s_stat[1] += now - s_stat[8];
            s_stat[8] = now;
        }

        // ---- relax until the tile is quiet --------------------------------
        // Two pass structures, same result (any order of monotone updates
        // reaches the same fixed point): PACK compacts each pass's dirty points
        // into a dense list first (fewest operator evaluations per wave: more
        // throughput when the device is full of work, as in a batch of shots);
        // otherwise each thread relaxes its own point (one barrier per pass:
        // lower latency when the front holds few tiles, as in a single solve).
        int cb = 0;
        int passes = 0;
        double pend = inf64();
        if constexpr (PACK) {
            // Each pass first compacts the dirty points into a dense list (every
            // thread reads its points' flags with one LDS access; per-point ballots
            // give each point its place in the wave's segment, one LDS atomic per
            // wave reserves the segment), then applies the operator to the list,
            // so the waves run the operator only as many times as there are dirty
            // points, not once per owned point.  A point whose value drops marks
            // its in-tile neighbours above the new value dirty for the next pass;
            // values read within a pass may already be newer (any order of
            // monotone updates is valid).
            for (;;) {
                {
                    uint8_t* df = sDirty[cb] + tid * NPT;
                    const uint32_t fl = ld_flags<NPT>(df);
                    if (fl) st_flags<NPT>(df, 0u);
                    uint32_t m = 0;
    #pragma unroll
                    for (int j = 0; j < NPT; ++j) m |= ((fl >> (8 * j)) & 1u) << j;
                    m &= live;
                    unsigned long long B[NPT];
                    int tot = 0;
    #pragma unroll
                    for (int j = 0; j < NPT; ++j) {
                        B[j] = __ballot((m >> j) & 1u);
                        tot += __popcll(B[j]);
                    }
                    if (tot) {
                        int base = 0;
                        if (lane == 0) base = atomicAdd(&s_cnt[cb], tot);
                        base = __shfl(base, 0);
    #pragma unroll
                        for (int j = 0; j < NPT; ++j) {
                            if ((m >> j) & 1u) sList[base + __popcll(B[j] & lanes_below)] = (uint16_t)(tid + j * NT);
                            base += __popcll(B[j]);
                        }
                    }
                }
                __syncthreads();
                const int n = s_cnt[cb];
                if (n == 0) break;
                // the other counter was last read before the previous barrier and is
                // next filled after the coming one
                if (tid == 0) s_cnt[cb ^ 1] = 0;
                for (int i = tid; i < n; i += NT) {
                    const int p = sList[i];
                    const double q = sQ[p];
                    const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
                    const int L = C::lds(lx, ly, lz);
                    const double tc = sT[L];
                    const double ax = nmin(sT[L - 1], sT[L + 1]);
                    const double ay = nmin(sT[L - C::SY], sT[L + C::SY]);
                    const double az = C::D3 ? nmin(sT[L - C::SZ], sT[L + C::SZ]) : inf64();
                    bool ch, mark;
                    double r;
                    if constexpr (OP == 0) {
                        r = update<C::D3>(ax, ay, az, q, q * q, tc, ch);
                        // held back: its bucket lies at or beyond the horizon (a
                        // value whose bucket index overflows the range is settled
                        // at once, so the requeue can never repeat forever)
                        const double rb = r * S.inv_delta;
                        if (S.horizon > 0 && ch && rb >= hz && rb < 1.0e15) {
                            pend = fmin(pend, r);
                            ch = false;
                        }
                        mark = ch;
                    } else {
                        // the ablation operators assign (their value may rise) and
                        // re-activate on a drop, or on any change when tracking
                        r = apply_op<OP>(ax, ay, az, q);
                        ch = r != tc && r == r;
                        mark = S.track ? ch : (ch && r < tc);
                    }
                    if constexpr (COUNT) {
                        bool good = false;
                        if (ch) {
                            const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
                            good = r == A.work_ref[P.pt_off + ((int64_t)gz * P.ny + gy) * P.nx + gx];
                        }
                        w_eval += __popcll(__ballot(true));
                        w_imp += __popcll(__ballot(ch));
                        w_good += __popcll(__ballot(good));
                    }
                    if (ch) sT[L] = r;
                    if (mark) {
                        // with d-bar only neighbours above the new value can depend
                        // on it (the operator is causal), so only they need another
                        // look; the ablation operators mark every neighbour.  Six
                        // unconditional stores, unwanted ones into this thread's
                        // sink byte (no divergent branches).
                        constexpr bool kAll = OP != 0;
                        uint8_t* nd = sDirty[cb ^ 1];
                        const int sink = C::NP + tid;
                        nd[(lx > 0 && (kAll || sT[L - 1] > r)) ? didx<NT, NPT>(p - 1) : sink] = 1;
                        nd[(lx < TX - 1 && (kAll || sT[L + 1] > r)) ? didx<NT, NPT>(p + 1) : sink] = 1;
                        nd[(ly > 0 && (kAll || sT[L - C::SY] > r)) ? didx<NT, NPT>(p - TX) : sink] = 1;
                        nd[(ly < TY - 1 && (kAll || sT[L + C::SY] > r)) ? didx<NT, NPT>(p + TX) : sink] = 1;
                        if (C::D3) {
                            nd[(lz > 0 && (kAll || sT[L - C::SZ] > r)) ? didx<NT, NPT>(p - TX * TY) : sink] = 1;
                            nd[(lz < TZ - 1 && (kAll || sT[L + C::SZ] > r)) ? didx<NT, NPT>(p + TX * TY) : sink] = 1;
                        }
                    }
                }
                ++passes;
                __syncthreads();
                cb ^= 1;
                if (OP != 0 && OP != 4 && passes >= (1 << 16)) {  // an ablation operator may not settle
                    if (tid == 0) set_flag(S, kFlagLimit);
                    break;
                }
                if (passes > (1 << 20)) {
                    if (tid == 0) set_flag(S, kFlagWatchdog);
                    break;
                }
            }
        } else {
            // Every thread relaxes its own points (p = tid + j * NT), whose time
            // and constant it keeps in registers; only the neighbours come from
            // LDS.  A pass evaluates each dirty point once and marks the in-tile
            // neighbours that may now improve in the other flag buffer, so the
            // pass's reads (buffer cb) and marks (buffer cb ^ 1) never touch the
            // same bytes, and ONE barrier per pass suffices: it orders this pass's
            // marks before the next pass's reads.  A flag byte of slot s_more says
            // whether any wave marked anything; if none did, every flag is clear
            // and the tile is quiet.  Values read within a pass may already be
            // newer (any order of monotone updates is valid, Theorem 1).
            uint32_t dirty = 0;  // bit j: point j is to be evaluated in this pass
            {
                const uint32_t fl = ld_flags<NPT>(sDirty[0] + tid * NPT);
    #pragma unroll
                for (int j = 0; j < NPT; ++j) dirty |= ((fl >> (8 * j)) & 1u) << j;
                st_flags<NPT>(sDirty[0] + tid * NPT, 0u);
                dirty &= live;
            }
            for (;;) {
                if (tid == 0) s_more[(passes + 1) % 3] = 0;  // written next pass; last read two barriers ago
                bool marked = false;
                uint8_t* nd = sDirty[cb ^ 1];
                const int sink = C::NP + tid;
    #pragma unroll
                for (int j = 0; j < NPT; ++j) {
                    if (!__ballot((dirty >> j) & 1u)) continue;
                    bool ch = false, good = false;  // for the work classification
                    if ((dirty >> j) & 1u) {
                        const int p = tid + j * NT;
                        const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
                        const int L = C::lds(lx, ly, lz);
                        const double q = q_own[j];
                        const double tc = t_own[j];
                        const double nxm = sT[L - 1], nxp = sT[L + 1], nym = sT[L - C::SY], nyp = sT[L + C::SY];
                        const double nzm = C::D3 ? sT[L - C::SZ] : inf64(), nzp = C::D3 ? sT[L + C::SZ] : inf64();
                        const double ax = nmin(nxm, nxp), ay = nmin(nym, nyp), az = nmin(nzm, nzp);
                        bool mark;
                        double r;
                        if constexpr (OP == 0 || OP == 4) {
                            if constexpr (OP == 0) {
                                r = update<C::D3>(ax, ay, az, q, q * q, tc, ch);
                            } else {
                                const double nb6[6] = {nxm, nxp, nym, nyp, nzm, nzp};
                                const double w6[6] = {sW[lx], sW[TX + lx], sW[2 * TX + ly], sW[2 * TX + TY + ly],
                                                      C::D3 ? sW[2 * (TX + TY) + lz] : 1.0,
                                                      C::D3 ? sW[2 * (TX + TY) + TZ + lz] : 1.0};
                                r = update_rect<C::D3>(nb6, w6, q * q, tc, ch);
                            }
                            // held back: its bucket lies at or beyond the horizon (a
                            // value whose bucket index overflows the range is settled
                            // at once, so the requeue can never repeat forever)
                            const double rb = r * S.inv_delta;
                            if (S.horizon > 0 && ch && rb >= hz && rb < 1.0e15) {
                                pend = fmin(pend, r);
                                ch = false;
                            }
                            mark = ch;
                        } else {
                            // the ablation operators assign (their value may rise) and
                            // re-activate on a drop, or on any change when tracking
                            r = apply_op<OP>(ax, ay, az, q);
                            ch = r != tc && r == r;
                            mark = S.track ? ch : (ch && r < tc);
                        }
                        if constexpr (COUNT) {
                            if (ch) {
                                const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
                                good = r == A.work_ref[P.pt_off + ((int64_t)gz * P.ny + gy) * P.nx + gx];
                            }
                        }
                        if (ch) {
                            t_own[j] = r;
                            sT[L] = r;
                        }
                        if (mark) {
                            // with d-bar only neighbours above the new value can depend
                            // on it (the operator is causal); the values loaded above
                            // can only have dropped since, so a neighbour loaded at or
                            // below r needs no look.  The ablation operators mark every
                            // neighbour.  Six unconditional stores, unwanted ones into
                            // this thread's sink byte (no divergent branches).
                            // (the targets fold the tile's edge into the sink, so a
                            // mark is one compare and one select)
                            constexpr bool kAll = OP != 0 && OP != 4;
                            const int txm = lx > 0 ? didx<NT, NPT>(p - 1) : sink;
                            const int txp = lx < TX - 1 ? didx<NT, NPT>(p + 1) : sink;
                            const int tym = ly > 0 ? didx<NT, NPT>(p - TX) : sink;
                            const int typ = ly < TY - 1 ? didx<NT, NPT>(p + TX) : sink;
                            nd[(kAll || nxm > r) ? txm : sink] = 1;
                            nd[(kAll || nxp > r) ? txp : sink] = 1;
                            nd[(kAll || nym > r) ? tym : sink] = 1;
                            nd[(kAll || nyp > r) ? typ : sink] = 1;
                            if (C::D3) {
                                const int tzm = lz > 0 ? didx<NT, NPT>(p - TX * TY) : sink;
                                const int tzp = lz < TZ - 1 ? didx<NT, NPT>(p + TX * TY) : sink;
                                nd[(kAll || nzm > r) ? tzm : sink] = 1;
                                nd[(kAll || nzp > r) ? tzp : sink] = 1;
                            }
                            marked = true;
                        }
                    }
                    if constexpr (COUNT) {
                        // every lane of the wave takes part, so lane 0's totals are the wave's
                        w_eval += __popcll(__ballot((dirty >> j) & 1u));
                        w_imp += __popcll(__ballot(ch));
                        w_good += __popcll(__ballot(good));
                    }
                }
                if (__ballot(marked) && lane == 0) s_more[passes % 3] = 1;
                __syncthreads();
                // the pass flag and the thread's next flags are read together
                // (one LDS round trip); when nothing was marked the flags are
                // all clear and the read is simply unused
                uint8_t* df = sDirty[cb ^ 1] + tid * NPT;
                const int more = s_more[passes % 3];
                const uint32_t fl = ld_flags<NPT>(df);
                asm volatile("" ::"v"(fl));  // keeps the flag read ahead of the branch
                ++passes;
                if (!more) break;
                cb ^= 1;
                {
                    dirty = 0;
    #pragma unroll
                    for (int j = 0; j < NPT; ++j) dirty |= ((fl >> (8 * j)) & 1u) << j;
                    if (fl) st_flags<NPT>(df, 0u);
                    dirty &= live;
                }
                if (OP != 0 && OP != 4 && passes >= (1 << 16)) {  // an ablation operator may not settle
                    if (tid == 0) set_flag(S, kFlagLimit);
                    break;
                }
                if (passes > (1 << 20)) {
                    if (tid == 0) set_flag(S, kFlagWatchdog);
                    break;
                }
            }
        }

        if (tid == 0) {
            const unsigned long long now = wall_clock64();
            s_stat[2] += now - s_stat[8];
            s_stat[8] = now;
        }
        // ---- write back lowered points, gather lowered face minima ---------
        uint32_t chg = 0;  // bit j: point j was stored
        double fmin_[6] = {inf64(), inf64(), inf64(), inf64(), inf64(), inf64()};
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int p = tid + j * NT;
            const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
            const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
            // the point and the six cells next to it, read together
            const int L = C::lds(lx, ly, lz);
            const double v = sT[L];
            const double nxm = sT[L - 1], nxp = sT[L + 1], nym = sT[L - C::SY], nyp = sT[L + C::SY];
            const double nzm = C::D3 ? sT[L - C::SZ] : inf64(), nzp = C::D3 ? sT[L + C::SZ] : inf64();
            const double tin = PACK ? sTin[p] : t_in[j];
            if (x < P.nx && y < P.ny && z < P.nz) {
                if (v < tin) {
                    tstore(A.t + P.pt_off + ((int64_t)z * P.ny + y) * P.nx + x, v);
                    chg |= 1u << j;
                    // a lowered face value matters to the neighbour only where
                    // it is below the neighbour's own value there (its halo
                    // cell here, as staged; values only decrease): the
                    // operator ignores a neighbour above the point it updates
                    constexpr bool kAny = OP != 0 && OP != 4;  // not causal: every lowered face value
                    if (lx == 0 && (kAny || v < nxm)) fmin_[0] = nmin(fmin_[0], v);
                    if (lx == TX - 1 && (kAny || v < nxp)) fmin_[1] = nmin(fmin_[1], v);
                    if (ly == 0 && (kAny || v < nym)) fmin_[2] = nmin(fmin_[2], v);
                    if (ly == TY - 1 && (kAny || v < nyp)) fmin_[3] = nmin(fmin_[3], v);
                    if (C::D3) {
                        if (lz == 0 && (kAny || v < nzm)) fmin_[4] = nmin(fmin_[4], v);
                        if (lz == TZ - 1 && (kAny || v < nzp)) fmin_[5] = nmin(fmin_[5], v);
                    }
                } else if (OP != 0 && OP != 4 && v != tin) {
                    // an ablation operator raised the value: store it, and with
                    // change tracking activate the neighbours across its faces
                    tstore(A.t + P.pt_off + ((int64_t)z * P.ny + y) * P.nx + x, v);
                    chg |= 1u << j;
                    if (S.track) {
                        if (lx == 0) fmin_[0] = nmin(fmin_[0], v);
                        if (lx == TX - 1) fmin_[1] = nmin(fmin_[1], v);
                        if (ly == 0) fmin_[2] = nmin(fmin_[2], v);
                        if (ly == TY - 1) fmin_[3] = nmin(fmin_[3], v);
                    }
                }
            }
        }
        // block-wide minima and counts: reduced within each wave first, then
        // one LDS atomic per wave (per-lane atomics on one LDS word would be
        // serialised lane by lane)
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            if (__ballot(fmin_[f] < inf64())) {
                const double m = wave_min(fmin_[f]);
                if (lane == 0) atomicMin(&s_face[f], (unsigned long long)as_u64(m));
            }
        }
        {
            int cnt = 0;
#pragma unroll
            for (int j = 0; j < NPT; ++j) cnt += __popcll(__ballot((chg >> j) & 1u));
            if (cnt && lane == 0) atomicAdd(&s_upd, (unsigned int)cnt);
        }
        if (__ballot(pend < inf64())) {
            const double m = wave_min(pend);
            if (lane == 0) atomicMin(&s_pend, (unsigned long long)as_u64(m));
        }
        // every wave's stores complete before the block hands the tile's faces
        // to the neighbours
        stores_done();
        __syncthreads();

        // ---- publish: activate neighbours, end the run or hand on ----------
        if (tid < 64) {
            // runs of this kernel read halos without looking at V (t starts at
            // +inf), so V needs no ordering against the activations
            const int nxt = publish(S, A.tkey, (uint32_t)tile, s_bucket, !visited, s_nb, s_nid, s_face, true,
                                    s_pend, false);
            if (tid == 0) s_next = nxt;
        }
        if (tid == 0) {
            s_stat[5] += s_upd;
            s_stat[6] += (unsigned long long)passes;
            const unsigned long long now = wall_clock64();
            s_stat[3] += now - s_stat[8];
            s_stat[8] = now;
        }
        __syncthreads();
    }
    if (COUNT && lane == 0) {
        __hip_atomic_fetch_add(S.counters + 16, w_eval, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(S.counters + 17, w_imp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(S.counters + 18, w_good, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid == 0) {
        s_stat[0] += wall_clock64() - s_stat[8];
        for (int i = 0; i < 4; ++i)
            __hip_atomic_fetch_add(S.counters + 5 + i, s_stat[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(S.counters + 10, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(S.counters + 12, s_stat[7], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (S.timeline)
            __hip_atomic_fetch_max(S.timeline + 1, (unsigned long long)wall_clock64(), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(S.counters + 0, s_stat[4], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(S.counters + 1, s_stat[5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(S.counters + 2, s_stat[6], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// ---------------------------------------------------------------------------
// residual of a solution (the error metric of Table "tab:error")
// ---------------------------------------------------------------------------

__global__ void k_fill_u8(long long n, uint8_t* a, uint8_t v) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = v;
}

// Clears the residual accumulators: out[0] count, out[1] max, out[2] flags.
__global__ void k_clear_residual(unsigned long long* out) {
    if (threadIdx.x < 3) out[threadIdx.x] = 0ull;
}

__global__ void k_mark_points(const int64_t* idx, long long n, long long npts, uint8_t* mask) {
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int64_t i = idx[g];
    if (i >= 0 && i < npts) mask[i] = 1;
}

// Counts the non-source points whose time differs from the operator applied
// to their final neighbours, and the largest relative difference (bits of a
// non-negative double, atomic max): out[0] count, out[1] max.  Field values
// that are not positive and finite raise the domain flag.
template <int OP>
__global__ void k_residual(Prob P, const double* field, const double* t, const uint8_t* fixed,
                           unsigned long long* out, uint32_t* flags) {
    const long long n = (long long)P.nx * P.ny * P.nz;
    const long long stride = (long long)gridDim.x * blockDim.x;
    unsigned long long cnt = 0, worst = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (fixed[i]) continue;
        bool ok;
        const double q = field_q(field[i], P.h, P.kind, ok);
        if (!ok) {
            __hip_atomic_fetch_or(flags, kFlagDomain, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            continue;
        }
        const long long x = i % P.nx, y = (i / P.nx) % P.ny, z = i / ((long long)P.nx * P.ny);
        const long long sy = P.nx, sz = (long long)P.nx * P.ny;
        double lo = x > 0 ? t[i - 1] : inf64(), hi = x < P.nx - 1 ? t[i + 1] : inf64();
        const double ax = lo < hi ? lo : hi;
        lo = y > 0 ? t[i - sy] : inf64();
        hi = y < P.ny - 1 ? t[i + sy] : inf64();
        const double ay = lo < hi ? lo : hi;
        double az = inf64();
        if (P.nz > 1) {
            lo = z > 0 ? t[i - sz] : inf64();
            hi = z < P.nz - 1 ? t[i + sz] : inf64();
            az = lo < hi ? lo : hi;
        }
        const double r = apply_op<OP>(ax, ay, az, q);
        const double ti = t[i];
        if (r != ti) {
            ++cnt;
            const unsigned long long rb = as_u64(fabs(r - ti) / fabs(ti)) & ~kSignBit;
            if (rb > worst) worst = rb;
        }
    }
    if (cnt) __hip_atomic_fetch_add(out, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (worst) __hip_atomic_fetch_max(out + 1, worst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// upwind-parent record
// ---------------------------------------------------------------------------

// One thread per point over all problems.  Reads |t| (a set sign bit marks a
// source while the solve's encoding is still in place: then bit 7 is written).
__global__ void k_parents(ProbTable T, long long npts_total, const double* t, uint8_t* par) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x; g < npts_total; g += stride) {
        const Prob P = prob_of_point(T, g);
        const int64_t i = g - P.pt_off;
        const double* tp = t + P.pt_off;
        const double ti = tp[i];
        if (signbit(ti)) {
            par[g] = 0x80;
            continue;
        }
        const int64_t x = i % P.nx, y = (i / P.nx) % P.ny, z = i / ((int64_t)P.nx * P.ny);
        const int64_t sy = P.nx, sz = (int64_t)P.nx * P.ny;
        uint8_t b = 0;
        {
            double l = x > 0 ? fabs(tp[i - 1]) : inf64();
            double r = x < P.nx - 1 ? fabs(tp[i + 1]) : inf64();
            if (fmin(l, r) < ti) b |= (l <= r) ? 1 : 2;
        }
        {
            double l = y > 0 ? fabs(tp[i - sy]) : inf64();
            double r = y < P.ny - 1 ? fabs(tp[i + sy]) : inf64();
            if (fmin(l, r) < ti) b |= ((l <= r) ? 1 : 2) << 2;
        }
        if (P.nz > 1) {
            double l = z > 0 ? fabs(tp[i - sz]) : inf64();
            double r = z < P.nz - 1 ? fabs(tp[i + sz]) : inf64();
            if (fmin(l, r) < ti) b |= ((l <= r) ? 1 : 2) << 4;
        }
        par[g] = b;
    }
}

// Marks sources in a parent record computed from final (unsigned) times.
__global__ void k_parents_mark_src(ProbTable T, const int64_t* src_idx, long long nsrc, uint8_t* par) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nsrc) return;
    const Prob P = prob_of_source(T, g);
    int64_t idx = src_idx[g];
    if (idx < 0 || idx >= (int64_t)P.nx * P.ny * P.nz) return;
    par[P.pt_off + idx] = 0x80;
}

}  // namespace eik

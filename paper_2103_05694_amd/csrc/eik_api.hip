// C ABI of the Eikonal library (declared in include/eik.h): argument checks,
// per-(device, stream) workspaces and the kernel sequence of each entry point.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "eik.h"

#ifndef EIK_SOLVE_THREADS
#define EIK_SOLVE_THREADS 1024
#endif
#include "eik_adjoint.hpp"

using namespace eik;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(EIK_EHIP, std::string(#expr " failed: ") + hipGetErrorString(e_)); \
    } while (0)

constexpr int kThreads = 256;
// Workgroup size of the persistent tile kernels: one thread per point up to
// 256 (tiles of 64 or 128 points run as one or two waves).
template <int TX, int TY, int TZ>
constexpr int tile_threads() { return TX * TY * TZ < kThreads ? TX * TY * TZ : kThreads; }
// Workgroup size of the forward solver: one thread per point (up to 1024), so
// a relaxation pass applies the operator at most once per thread (the
// operator's latency sets the cost of a pass).
constexpr int kSolveThreads = EIK_SOLVE_THREADS;
template <int TX, int TY, int TZ>
constexpr int solve_threads() { return TX * TY * TZ < kSolveThreads ? TX * TY * TZ : kSolveThreads; }
constexpr int kRings = 32;
// A push from a run claimed from bucket b lands at most nrings - 1 - lookahead
// buckets above b; 16 leaves a push range of 15 buckets.
constexpr int kMaxLookahead = 16;
static_assert(kMaxLookahead < kRings && kMaxLookahead < 64, "the claim window is read by one wave");
constexpr int kScalWords = 192;
constexpr int kTimelineCap = 1 << 16;
constexpr int kSCur = 0, kSPending = 64, kSFlags = 128, kSPoisoned = 129, kSSrcCount = 130;

// One uploaded batch layout: the problem table (tile shape and offsets
// included) and the source offsets, as on the host and on the device.
struct Table {
    std::vector<Prob> probs;
    std::vector<int64_t> src_off;   // empty for a table uploaded by the adjoint
    Prob* d_probs = nullptr;
    int64_t* d_src_off = nullptr;
};
constexpr size_t kMaxTables = 64;

struct Workspace {
    int device = -1;
    hipStream_t stream = nullptr;
    // scheduler
    uint64_t* items = nullptr;
    uint32_t* ctr = nullptr;
    uint8_t* mask = nullptr;       // per-point byte mask (residual: fixed points)
    int64_t mask_cap = 0;
    unsigned long long* timeline = nullptr;  // bucket advance record (EIK_FLAG_TIMELINE)
    uint32_t* tstate = nullptr;
    uint64_t* tkey = nullptr;
    int64_t tiles_cap = 0;
    uint32_t ring_cap = 0;
    // scalars, on separate 256-byte lines: cur, pending, then flags / poisoned /
    // source-list count (see the kS* offsets)
    int32_t* scal = nullptr;
    unsigned long long* counters = nullptr;
    int32_t* srclist = nullptr;
    int64_t srclist_cap = 0;
    // device problem tables of batched calls (problem list + source offsets),
    // one per distinct layout, kept until eik_release
    std::vector<Table> tables;
    // rectilinear grids: reciprocal spacings on the device, and what they are
    double* rw = nullptr;
    int64_t rw_cap = 0;
    std::vector<double> rw_host;
    // adjoint scratch
    double* mu = nullptr;
    int64_t mu_cap = 0;
    uint64_t* tile_tmax = nullptr;     // per-tile largest time (adjoint priorities)
    int last_kind = 0;                 // 0 none, 1 forward, 2 adjoint
    int64_t last_ntiles = 0;
    uint64_t last_seq = 0;             // order of the last call among all calls (status lookup)
    std::vector<hipEvent_t> ev;        // event pairs bracketing timed persistent kernels
    size_t ev_used = 0;                // pairs recorded since the last eik_status
};

int timing_begin(Workspace& w, const eik_opts* o) {
    if (!o || !(o->flags & EIK_FLAG_TIME_KERNELS)) return EIK_OK;
    if (w.ev_used * 2 + 2 > w.ev.size()) {
        if (w.ev_used >= 4096) return fail(EIK_EINVAL, "more than 4096 timed launches without eik_status");
        for (int i = 0; i < 2; ++i) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            w.ev.push_back(e);
        }
    }
    HIP_TRY(hipEventRecord(w.ev[2 * w.ev_used], w.stream));
    return EIK_OK;
}

int timing_end(Workspace& w, const eik_opts* o) {
    if (!o || !(o->flags & EIK_FLAG_TIME_KERNELS)) return EIK_OK;
    HIP_TRY(hipEventRecord(w.ev[2 * w.ev_used + 1], w.stream));
    ++w.ev_used;
    return EIK_OK;
}

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;
std::atomic<uint64_t> g_seq{0};
uint64_t next_seq() { return ++g_seq; }

template <class T>
int grow(T** p, int64_t* cap, int64_t need, hipStream_t st) {
    if (*cap >= need) return EIK_OK;
    int64_t n = need + need / 4 + 64;
    if (*p) {
        HIP_TRY(hipStreamSynchronize(st));
        HIP_TRY(hipFree(*p));
        *p = nullptr;
        *cap = 0;
    }
    hipError_t e = hipMalloc((void**)p, sizeof(T) * (size_t)n);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(EIK_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    *cap = n;
    return EIK_OK;
}

int get_ws(hipStream_t st, Workspace** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    auto key = std::make_pair(dev, st);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) {
        *out = it->second;
        return EIK_OK;
    }
    Workspace* w = new Workspace();
    w->device = dev;
    w->stream = st;
    hipError_t e = hipMalloc((void**)&w->scal, kScalWords * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc((void**)&w->counters, kCounters * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc((void**)&w->ctr, sizeof(uint32_t) * kRings * kCtrStride);
    if (e == hipSuccess) e = hipMalloc((void**)&w->timeline, sizeof(unsigned long long) * (2 + 2 * kTimelineCap));
    if (e != hipSuccess) {
        delete w;
        return fail(EIK_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    int32_t init[kScalWords] = {0};
    init[kSPoisoned] = 1;  // the first reset initialises the rings
    HIP_TRY(hipMemcpy(w->scal, init, sizeof(init), hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(w->ctr, 0, sizeof(uint32_t) * kRings * kCtrStride));
    HIP_TRY(hipMemset(w->counters, 0, kCounters * sizeof(unsigned long long)));
    HIP_TRY(hipMemset(w->timeline, 0, sizeof(unsigned long long) * (2 + 2 * kTimelineCap)));
    g_ws[key] = w;
    *out = w;
    return EIK_OK;
}

uint32_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return (uint32_t)p;
}

int ensure_tiles(Workspace& w, int64_t ntiles) {
    if (ntiles > (int64_t)1 << 30) return fail(EIK_ENOTSUP, "more than 2^30 tiles");
    int rc;
    if ((rc = grow(&w.tstate, &w.tiles_cap, ntiles, w.stream))) return rc;
    const uint32_t need_ring = next_pow2((uint64_t)std::max<int64_t>(w.tiles_cap, 2));
    if (need_ring > w.ring_cap) {
        HIP_TRY(hipStreamSynchronize(w.stream));
        if (w.items) HIP_TRY(hipFree(w.items));
        if (w.tkey) HIP_TRY(hipFree(w.tkey));
        if (w.tile_tmax) HIP_TRY(hipFree(w.tile_tmax));
        w.items = nullptr;
        w.tkey = nullptr;
        w.tile_tmax = nullptr;
        w.ring_cap = 0;
        hipError_t e = hipMalloc((void**)&w.items, sizeof(uint64_t) * (size_t)kRings * need_ring);
        if (e == hipSuccess) e = hipMalloc((void**)&w.tkey, sizeof(uint64_t) * (size_t)need_ring);
        if (e == hipSuccess) e = hipMalloc((void**)&w.tile_tmax, sizeof(uint64_t) * (size_t)need_ring);
        if (e != hipSuccess) return fail(EIK_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
        w.ring_cap = need_ring;
        // fresh ring memory: the next reset must initialise it
        int32_t one = 1;
        HIP_TRY(hipMemcpy(w.scal + kSPoisoned, &one, sizeof(one), hipMemcpyHostToDevice));
    }
    return EIK_OK;
}

bool same_probs(const std::vector<Prob>& a, const std::vector<Prob>& b) {
    return a.size() == b.size() && std::memcmp(a.data(), b.data(), sizeof(Prob) * a.size()) == 0;
}

// Finds or uploads the device table of a batch layout.  Each distinct layout
// (problems with their tile geometry, and the source offsets when `src_off` is
// given) is uploaded once and kept, so the forward and the adjoint of a batch
// may use different tile shapes and repeated calls enqueue nothing but
// kernels: HIP graph capture of a call relies on this after one warm-up call
// with each layout.  The adjoint (src_off == NULL) reuses any table with the
// same problems.  Uploading synchronises the stream; past kMaxTables layouts
// the oldest is freed (after a synchronisation) to make room.
int upload_table(Workspace& w, const std::vector<Prob>& probs, const std::vector<int64_t>* src_off,
                 const Table** out) {
    for (const Table& tb : w.tables) {
        if (!same_probs(tb.probs, probs)) continue;
        if (src_off && tb.src_off != *src_off) continue;
        *out = &tb;
        return EIK_OK;
    }
    HIP_TRY(hipStreamSynchronize(w.stream));
    if (w.tables.size() >= kMaxTables) {
        HIP_TRY(hipFree(w.tables.front().d_probs));
        HIP_TRY(hipFree(w.tables.front().d_src_off));
        w.tables.erase(w.tables.begin());
    }
    Table tb;
    tb.probs = probs;
    if (src_off) tb.src_off = *src_off;
    std::vector<int64_t> so = src_off ? *src_off : std::vector<int64_t>(probs.size() + 1, 0);
    hipError_t e = hipMalloc((void**)&tb.d_probs, sizeof(Prob) * probs.size());
    if (e == hipSuccess) e = hipMalloc((void**)&tb.d_src_off, sizeof(int64_t) * so.size());
    if (e != hipSuccess) {
        (void)hipFree(tb.d_probs);
        return fail(EIK_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    // synchronous copies: the host vectors may be gone before the stream runs
    HIP_TRY(hipMemcpy(tb.d_probs, probs.data(), sizeof(Prob) * probs.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(tb.d_src_off, so.data(), sizeof(int64_t) * so.size(), hipMemcpyHostToDevice));
    w.tables.push_back(std::move(tb));
    *out = &w.tables.back();
    return EIK_OK;
}

// Kernel-side problem table: a single problem travels by value (nothing to
// upload, no synchronisation); a batch uses its device copy.
int make_table(Workspace& w, const std::vector<Prob>& probs, const std::vector<int64_t>* src_off,
               ProbTable* T) {
    T->probs = nullptr;
    T->src_off = nullptr;
    T->nprob = (int)probs.size();
    T->p0 = probs[0];
    T->nsrc0 = src_off ? (*src_off)[1] - (*src_off)[0] : 0;
    if (probs.size() == 1) return EIK_OK;
    const Table* tb = nullptr;
    int rc = upload_table(w, probs, src_off, &tb);
    if (rc) return rc;
    T->probs = tb->d_probs;
    T->src_off = tb->d_src_off;
    return EIK_OK;
}

// ---------------------------------------------------------------------------
// tile configurations
// ---------------------------------------------------------------------------

struct TileShape {
    int x, y, z;
};

#define EIK_TILES_3D(X) X(32, 8, 4) X(16, 8, 8) X(8, 8, 8) X(64, 4, 4) X(16, 8, 4) X(8, 8, 4) X(8, 4, 4)
#define EIK_TILES_2D(X) X(32, 32, 1) X(64, 16, 1) X(128, 8, 1) X(16, 16, 1) X(16, 8, 1)

bool tile_supported(int ndim, int x, int y, int z) {
#define EIK_MATCH(a, b, c) \
    if (x == a && y == b && z == c) return (ndim == 3) == (c > 1);
    EIK_TILES_3D(EIK_MATCH)
    EIK_TILES_2D(EIK_MATCH)
#undef EIK_MATCH
    return false;
}

TileShape pick_tile(int ndim, const eik_opts* o) {
    if (o && (o->tile[0] || o->tile[1] || o->tile[2])) return {o->tile[0], o->tile[1], o->tile[2]};
    if (ndim == 3) return {16, 8, 8};
    return {32, 32, 1};
}

int check_grid(const eik_grid* g) {
    if (!g) return fail(EIK_EINVAL, "grid is NULL");
    if (g->ndim != 2 && g->ndim != 3) return fail(EIK_EINVAL, "ndim must be 2 or 3");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return fail(EIK_EINVAL, "dims must be >= 1");
    if (g->ndim == 2 && g->nz != 1) return fail(EIK_EINVAL, "2D grids need nz == 1");
    if (!(g->h > 0.0) || !std::isfinite(g->h)) return fail(EIK_EINVAL, "h must be positive and finite");
    if (g->field_kind != EIK_SPEED && g->field_kind != EIK_SLOWNESS)
        return fail(EIK_EINVAL, "field_kind must be EIK_SPEED or EIK_SLOWNESS");
    if ((int64_t)g->nx * g->ny * g->nz > ((int64_t)1 << 40)) return fail(EIK_ENOTSUP, "grid too large");
    return EIK_OK;
}

int check_opts(const eik_opts* o) {
    if (!o) return EIK_OK;
    if (!(o->delta >= 0.0) || std::isnan(o->delta)) return fail(EIK_EINVAL, "delta must be >= 0");
    // bucket keys are floor(t / delta) through 1 / delta: a width whose
    // reciprocal overflows (subnormal) would put every value beyond any bucket
    if (o->delta > 0.0 && !std::isfinite(1.0 / o->delta))
        return fail(EIK_EINVAL, "delta too small (its reciprocal overflows)");
    if (o->grid_blocks < 0) return fail(EIK_EINVAL, "grid_blocks must be >= 0");
    if (o->max_tile_visits < 0) return fail(EIK_EINVAL, "max_tile_visits must be >= 0");
    if (o->flags & ~(EIK_FLAG_TIME_KERNELS | EIK_FLAG_TIMELINE | EIK_FLAG_TRACK_CHANGE | EIK_FLAG_WARM_START |
                     EIK_FLAG_PACKED))
        return fail(EIK_EINVAL, "unknown flags");
    if ((o->flags & EIK_FLAG_PACKED) && o->op != EIK_OP_DBAR)
        return fail(EIK_ENOTSUP, "compacted passes run with d-bar only");
    if (o->lookahead < 0 || o->lookahead > kMaxLookahead)
        return fail(EIK_EINVAL, "lookahead must be in 0..16");
    if (o->op < EIK_OP_DBAR || o->op > EIK_OP_NEWTON) return fail(EIK_EINVAL, "unknown operator");
    if ((o->flags & EIK_FLAG_TRACK_CHANGE) && o->op == EIK_OP_DBAR)
        return fail(EIK_EINVAL, "change tracking applies to the ablation operators only");
    if (o->horizon < 0 || o->horizon > 4) return fail(EIK_EINVAL, "horizon must be in 0..4");
    if (o->work_ref && o->op != EIK_OP_DBAR)
        return fail(EIK_ENOTSUP, "work classification runs with d-bar only");
    if ((o->flags & EIK_FLAG_WARM_START) && o->op != EIK_OP_DBAR)
        return fail(EIK_ENOTSUP, "a warm start needs the monotone operator (d-bar)");
    return EIK_OK;
}

Prob make_prob(const eik_grid& g, TileShape ts, int64_t pt_off, int64_t tile_off) {
    Prob p;
    p.nx = g.nx;
    p.ny = g.ny;
    p.nz = g.nz;
    p.ntx = (g.nx + ts.x - 1) / ts.x;
    p.nty = (g.ny + ts.y - 1) / ts.y;
    p.ntz = (g.nz + ts.z - 1) / ts.z;
    p.pt_off = pt_off;
    p.tile_off = (int32_t)tile_off;
    p.kind = g.field_kind;
    p.h = g.h;
    return p;
}

int64_t tiles_of(const Prob& p) { return (int64_t)p.ntx * p.nty * p.ntz; }

// The device buffers one forward or adjoint launch sequence works in: the
// stream's workspace, or (eik_solve_noalloc) the library's static scratch.
struct Bufs {
    hipStream_t stream = nullptr;
    uint64_t* items = nullptr;
    uint32_t* ctr = nullptr;
    uint32_t* tstate = nullptr;
    uint64_t* tkey = nullptr;
    uint64_t* tile_aux = nullptr;   // per-tile min (warm start) or max (adjoint) time
    int32_t* scal = nullptr;
    unsigned long long* counters = nullptr;
    int32_t* srclist = nullptr;
    unsigned long long* timeline = nullptr;
    uint32_t ring_cap = 0;
    int force_wipe = 0;             // re-initialise the rings in this call's reset
};

Bufs bufs_of(Workspace& w) {
    Bufs b;
    b.stream = w.stream;
    b.items = w.items;
    b.ctr = w.ctr;
    b.tstate = w.tstate;
    b.tkey = w.tkey;
    b.tile_aux = w.tile_tmax;
    b.scal = w.scal;
    b.counters = w.counters;
    b.srclist = w.srclist;
    b.timeline = w.timeline;
    b.ring_cap = w.ring_cap;
    return b;
}

Sched make_sched(const Bufs& w, const eik_opts* o) {
    Sched s;
    s.items = w.items;
    s.ctr = w.ctr;
    s.tstate = w.tstate;
    s.cur = w.scal + kSCur;
    s.pending = w.scal + kSPending;
    s.flags = (uint32_t*)(w.scal + kSFlags);
    s.poisoned = w.scal + kSPoisoned;
    s.counters = w.counters;
    s.nrings = kRings;
    s.cap_mask = w.ring_cap - 1;
    double d = o ? o->delta : 0.0;
    s.inv_delta = (d > 0.0 && std::isfinite(d)) ? 1.0 / d : 0.0;
    s.max_visits = o ? (long long)o->max_tile_visits : 0;
    s.lookahead = o ? o->lookahead : 0;
    s.horizon = o ? o->horizon : 0;
    s.track = (o && (o->flags & EIK_FLAG_TRACK_CHANGE)) ? 1 : 0;
    const bool tl = o && (o->flags & EIK_FLAG_TIMELINE) && w.timeline;
    s.timeline = tl ? w.timeline : nullptr;
    s.timeline_cap = tl ? kTimelineCap : 0;
    return s;
}

// Persistent workgroups that fit on the device at once.  With `cached`, the
// per-kernel occupancy is remembered (a host map); the allocation-free entry
// point asks the runtime every time instead.
int occupancy_grid(const void* kernel, int threads, int* out, bool cached = true) {
    static std::map<const void*, int> cache;
    static std::mutex m;
    int per_cu = 0;
    if (cached) {
        std::lock_guard<std::mutex> lk(m);
        auto it = cache.find((const void*)kernel);
        if (it != cache.end()) {
            per_cu = it->second;
        } else {
            HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0));
            if (per_cu < 1) per_cu = 1;
            cache[(const void*)kernel] = per_cu;
        }
    } else {
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0));
        if (per_cu < 1) per_cu = 1;
    }
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    *out = per_cu * cus;
    return EIK_OK;
}

int blocks_for(int64_t n, int threads, int cap = 65536) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

// The forward launch sequence for one tile shape, on buffers that already
// exist (no allocation, no host synchronisation).  `tw` receives the timing
// events (NULL: no timing); `cached` as for occupancy_grid.
template <int TX, int TY, int TZ, int OP = 0>
int forward_seq(const Bufs& b, const ProbTable& T, int64_t nsrc, int64_t ntiles, int64_t npts_total,
                const double* field, const int64_t* src_idx, const double* src_t0, double* t, uint8_t* par,
                const eik_opts* o, Workspace* tw, bool cached, const double* rw = nullptr) {
    int rc;
    const bool warm = o && (o->flags & EIK_FLAG_WARM_START);
    hipStream_t st = b.stream;
    Sched s = make_sched(b, o);
    // the ablation operators need not settle: cap the runs unless the caller did
    if (OP != EIK_OP_DBAR && s.max_visits == 0) s.max_visits = 256 * (long long)ntiles;
    int32_t* srccnt = b.scal + kSSrcCount;

    hipLaunchKernelGGL(k_reset, dim3(blocks_for(std::max<int64_t>(ntiles, (int64_t)kRings * b.ring_cap), kThreads, 4096)),
                       dim3(kThreads), 0, st, s, b.tkey, (int)ntiles, srccnt,
                       (long long)kRings * b.ring_cap, b.force_wipe);
    hipLaunchKernelGGL((k_src_mark<TX, TY, TZ>), dim3(blocks_for(nsrc, kThreads)), dim3(kThreads), 0, st,
                       T, src_idx, src_t0, (long long)nsrc, s, b.srclist, srccnt);
    if (warm)
        hipLaunchKernelGGL((k_warm_prep<TX, TY, TZ>), dim3((unsigned)std::min<int64_t>(ntiles, 65536)),
                           dim3(kThreads), 0, st, T, (int)ntiles, t, b.tile_aux, s);
    else
        hipLaunchKernelGGL(k_fill_inf, dim3(blocks_for(npts_total, kThreads, 8192)), dim3(kThreads), 0, st,
                           (long long)npts_total, t);
    hipLaunchKernelGGL((k_src_place<TX, TY, TZ>), dim3(blocks_for(nsrc, kThreads)), dim3(kThreads), 0, st,
                       T, src_idx, src_t0, (long long)nsrc, t, s);
    if (warm)
        hipLaunchKernelGGL(k_warm_push, dim3(blocks_for(ntiles, kThreads, 4096)), dim3(kThreads), 0, st, T,
                           (int)ntiles, (const uint64_t*)b.tile_aux, s);
    HIP_TRY(hipGetLastError());

    SolveArgs a;
    a.pt = T;
    a.field = field;
    a.t = t;
    a.tkey = b.tkey;
    a.work_ref = o ? o->work_ref : nullptr;
    a.rw = rw;
    a.s = s;
    // the two pass structures of k_solve: one thread per point (default) or
    // compacted pass lists on 256-thread blocks (EIK_FLAG_PACKED, d-bar only)
    constexpr int nt = solve_threads<TX, TY, TZ>();
    constexpr int ntp = tile_threads<TX, TY, TZ>();
    const bool count = a.work_ref != nullptr;
    const bool pack = o && (o->flags & EIK_FLAG_PACKED);
    const void* kern = nullptr;
    int threads = nt;
    if constexpr (OP == EIK_OP_DBAR) {
        if (pack) {
            threads = ntp;
            kern = count ? (const void*)k_solve<TX, TY, TZ, ntp, OP, true, true>
                         : (const void*)k_solve<TX, TY, TZ, ntp, OP, false, true>;
        } else {
            kern = count ? (const void*)k_solve<TX, TY, TZ, nt, OP, true>
                         : (const void*)k_solve<TX, TY, TZ, nt, OP>;
        }
    } else if constexpr (OP == 4) {
        // the rectilinear operator holds both neighbours and weights of each
        // axis: in 3D it does not fit the 128 registers of a 1024-thread
        // block, so 3D tiles run on blocks of at most 512 threads with the
        // register budget of two waves per SIMD
        constexpr int ntr = (TZ > 1 && nt > 512) ? 512 : nt;
        threads = ntr;
        kern = (const void*)k_solve<TX, TY, TZ, ntr, OP>;
    } else {
        kern = (const void*)k_solve<TX, TY, TZ, nt, OP>;
    }
    int grid = 0;
    if ((rc = occupancy_grid(kern, threads, &grid, cached))) return rc;
    if (o && o->grid_blocks > 0) grid = std::min(grid, o->grid_blocks);
    if ((int64_t)grid > ntiles) grid = (int)ntiles;
    if (grid < 1) grid = 1;
    if (tw && (rc = timing_begin(*tw, o))) return rc;
    void* kargs[] = {(void*)&a};
    HIP_TRY(hipLaunchKernel(kern, dim3(grid), dim3(threads), kargs, 0, st));
    if (tw && (rc = timing_end(*tw, o))) return rc;

    if (par)
        hipLaunchKernelGGL(k_parents, dim3(blocks_for(npts_total, kThreads, 1 << 16)), dim3(kThreads), 0,
                           st, T, (long long)npts_total, (const double*)t, par);
    hipLaunchKernelGGL(k_src_unsign, dim3(blocks_for(nsrc, kThreads)), dim3(kThreads), 0, st, T, src_idx,
                       src_t0, (long long)nsrc, t);
    HIP_TRY(hipGetLastError());
    return EIK_OK;
}

// The full forward sequence on the stream's workspace (grown as needed).
template <int TX, int TY, int TZ, int OP = 0>
int forward(Workspace& w, const std::vector<Prob>& probs, const std::vector<int64_t>& src_off,
            int64_t ntiles, int64_t npts_total, const double* field, const int64_t* src_idx,
            const double* src_t0, double* t, uint8_t* par, const eik_opts* o, const double* rw = nullptr) {
    int rc;
    const int64_t nsrc = src_off.back();
    if ((rc = ensure_tiles(w, ntiles))) return rc;
    if ((rc = grow(&w.srclist, &w.srclist_cap, nsrc, w.stream))) return rc;
    ProbTable T;
    if ((rc = make_table(w, probs, &src_off, &T))) return rc;
    if ((rc = forward_seq<TX, TY, TZ, OP>(bufs_of(w), T, nsrc, ntiles, npts_total, field, src_idx, src_t0, t,
                                          par, o, &w, true, rw)))
        return rc;
    w.last_kind = 1;
    w.last_ntiles = ntiles;
    w.last_seq = next_seq();
    return EIK_OK;
}

int dispatch_forward(TileShape ts, Workspace& w, const std::vector<Prob>& probs,
                     const std::vector<int64_t>& src_off, int64_t ntiles, int64_t npts,
                     const double* field, const int64_t* src_idx, const double* src_t0, double* t,
                     uint8_t* par, const eik_opts* o) {
#define EIK_CASE(a, b, c)                                                                      \
    if (ts.x == a && ts.y == b && ts.z == c)                                                   \
        return forward<a, b, c>(w, probs, src_off, ntiles, npts, field, src_idx, src_t0, t, par, o);
#define EIK_HCASE(a, b, c)                                                                     \
    if (ts.x == a && ts.y == b && ts.z == c)                                                   \
        return forward<a, b, c, 1>(w, probs, src_off, ntiles, npts, field, src_idx, src_t0, t, par, o);
#define EIK_TCASE(a, b, c)                                                                     \
    if (ts.x == a && ts.y == b && ts.z == c)                                                   \
        return forward<a, b, c, 2>(w, probs, src_off, ntiles, npts, field, src_idx, src_t0, t, par, o);
#define EIK_NCASE(a, b, c)                                                                     \
    if (ts.x == a && ts.y == b && ts.z == c)                                                   \
        return forward<a, b, c, 3>(w, probs, src_off, ntiles, npts, field, src_idx, src_t0, t, par, o);
    const int op = o ? o->op : EIK_OP_DBAR;
    if (op == EIK_OP_DHAT) {
        EIK_TILES_2D(EIK_HCASE)
    } else if (op == EIK_OP_DTILDE) {
        EIK_TILES_2D(EIK_TCASE)
    } else if (op == EIK_OP_NEWTON) {
        EIK_TILES_2D(EIK_NCASE)
    } else {
        EIK_TILES_3D(EIK_CASE)
        EIK_TILES_2D(EIK_CASE)
    }
#undef EIK_CASE
#undef EIK_HCASE
#undef EIK_TCASE
#undef EIK_NCASE
    return fail(EIK_ENOTSUP, "unsupported tile shape");
}

template <int TX, int TY, int TZ>
int adjoint(Workspace& w, const std::vector<Prob>& probs, int64_t ntiles, int64_t npts,
            const double* field, const double* t, const uint8_t* par, const double* g, double* grad,
            double* mu, const eik_opts* o) {
    int rc;
    if ((rc = ensure_tiles(w, ntiles))) return rc;
    if (!mu) {
        if ((rc = grow(&w.mu, &w.mu_cap, npts, w.stream))) return rc;
        mu = w.mu;
    }
    ProbTable T;
    if ((rc = make_table(w, probs, nullptr, &T))) return rc;
    hipStream_t st = w.stream;
    Sched s = make_sched(bufs_of(w), o);
    s.max_visits = 0;
    unsigned long long* tref = w.counters + 4;
    hipLaunchKernelGGL(k_reset, dim3(blocks_for(std::max<int64_t>(ntiles, (int64_t)kRings * w.ring_cap), kThreads, 4096)),
                       dim3(kThreads), 0, st, s, w.tkey, (int)ntiles, w.scal + kSSrcCount,
                       (long long)kRings * w.ring_cap, 0);
    // mu := NaN (not done): a tile that has not run yet reads as not done
    hipLaunchKernelGGL(k_fill_nan, dim3(blocks_for(npts, kThreads, 8192)), dim3(kThreads), 0, st, (long long)npts, mu);
    hipLaunchKernelGGL((k_adj_prep<TX, TY, TZ>), dim3((unsigned)std::min<int64_t>(ntiles, 65536)), dim3(kThreads),
                       0, st, T, (int)ntiles, t, w.tile_tmax, tref);
    hipLaunchKernelGGL(k_adj_push_all, dim3(blocks_for(ntiles, kThreads, 4096)), dim3(kThreads), 0, st,
                       (int)ntiles, (const uint64_t*)w.tile_tmax, (const unsigned long long*)tref, s);
    HIP_TRY(hipGetLastError());
    AdjArgs a;
    a.pt = T;
    a.t = t;
    a.par = par;
    a.g = g;
    a.mu = mu;
    a.tkey = w.tkey;
    a.tref_bits = tref;
    a.s = s;
    // two pass structures as in the forward solver: one thread per point
    // (default) or compacted pass lists on 256-thread blocks (EIK_FLAG_PACKED)
    constexpr int nt = solve_threads<TX, TY, TZ>();
    constexpr int ntp = tile_threads<TX, TY, TZ>();
    const bool pack = o && (o->flags & EIK_FLAG_PACKED);
    const void* kern = pack ? (const void*)k_adjoint<TX, TY, TZ, ntp, true> : (const void*)k_adjoint<TX, TY, TZ, nt>;
    const int threads = pack ? ntp : nt;
    int grid = 0;
    if ((rc = occupancy_grid(kern, threads, &grid))) return rc;
    if (o && o->grid_blocks > 0) grid = std::min(grid, o->grid_blocks);
    if ((int64_t)grid > ntiles) grid = (int)ntiles;
    if (grid < 1) grid = 1;
    if ((rc = timing_begin(w, o))) return rc;
    void* kargs[] = {(void*)&a};
    HIP_TRY(hipLaunchKernel(kern, dim3(grid), dim3(threads), kargs, 0, st));
    if ((rc = timing_end(w, o))) return rc;
    // the gradient from the final multipliers (the sweep never reads the field)
    hipLaunchKernelGGL((k_adj_grad<TX, TY, TZ>), dim3((unsigned)std::min<int64_t>(ntiles, 65536)), dim3(kThreads),
                       0, st, T, (int)ntiles, field, par, (const double*)mu, grad, s.flags);
    HIP_TRY(hipGetLastError());
    w.last_kind = 2;
    w.last_ntiles = ntiles;
    w.last_seq = next_seq();
    return EIK_OK;
}

int adjoint_run(Workspace& w, TileShape ts, const std::vector<Prob>& probs, int64_t ntiles, int64_t npts,
                const double* field, const double* t, const uint8_t* par, const double* g, double* grad,
                double* mu, const eik_opts* o) {
#define EIK_CASE(a, b, c) \
    if (ts.x == a && ts.y == b && ts.z == c) return adjoint<a, b, c>(w, probs, ntiles, npts, field, t, par, g, grad, mu, o);
    EIK_TILES_3D(EIK_CASE)
    EIK_TILES_2D(EIK_CASE)
#undef EIK_CASE
    return fail(EIK_ENOTSUP, "unsupported tile shape");
}

// Rectilinear grids: the reciprocal spacings of the coordinates (the same
// definition the operator is stated with, w = fl(1 / fl(x_i - x_{i-1})), and
// 1 at the ends, where the neighbour is off the grid), laid out
// [wm_x, wp_x, wm_y, wp_y, wm_z, wp_z].  EIK_EINVAL unless every axis is
// strictly increasing and finite with finite reciprocal spacings.
int rect_weights(const eik_grid& g, const double* xs, const double* ys, const double* zs, std::vector<double>* out) {
    const int64_t n[3] = {g.nx, g.ny, g.nz};
    const double* c[3] = {xs, ys, g.ndim == 3 ? zs : nullptr};
    out->assign((size_t)(2 * (n[0] + n[1] + n[2])), 1.0);
    size_t off = 0;
    for (int k = 0; k < 3; ++k) {
        double* wm = out->data() + off;
        double* wp = wm + n[k];
        off += (size_t)(2 * n[k]);
        if (k >= g.ndim) continue;
        if (!c[k]) return fail(EIK_EINVAL, "coordinates missing for an axis");
        for (int64_t i = 0; i < n[k]; ++i) {
            if (!std::isfinite(c[k][i])) return fail(EIK_EINVAL, "coordinates must be finite");
            if (i == 0) continue;
            const double h = c[k][i] - c[k][i - 1];
            const double w = 1.0 / h;
            if (!(h > 0.0) || !std::isfinite(w))
                return fail(EIK_EINVAL, "coordinates must increase strictly (with finite reciprocal spacings)");
            wm[i] = w;
            wp[i - 1] = w;
        }
    }
    return EIK_OK;
}

// Puts the weights on the device (synchronising the stream) unless the same
// ones are there already, so repeated calls on one grid enqueue only kernels.
int upload_weights(Workspace& w, const std::vector<double>& rw) {
    if (w.rw && w.rw_host == rw) return EIK_OK;
    w.rw_host.clear();  // the device copy is stale until the upload below completes
    int rc;
    if ((rc = grow(&w.rw, &w.rw_cap, (int64_t)rw.size(), w.stream))) return rc;
    HIP_TRY(hipStreamSynchronize(w.stream));
    HIP_TRY(hipMemcpy(w.rw, rw.data(), sizeof(double) * rw.size(), hipMemcpyHostToDevice));
    w.rw_host = rw;
    return EIK_OK;
}

int dispatch_rect(TileShape ts, Workspace& w, const std::vector<Prob>& probs, const std::vector<int64_t>& src_off,
                  int64_t ntiles, int64_t npts, const double* field, const int64_t* src_idx, const double* src_t0,
                  double* t, const eik_opts* o) {
#define EIK_RCASE(a, b, c)                                                                                    \
    if (ts.x == a && ts.y == b && ts.z == c)                                                                  \
        return forward<a, b, c, 4>(w, probs, src_off, ntiles, npts, field, src_idx, src_t0, t, nullptr, o, w.rw);
    EIK_TILES_3D(EIK_RCASE)
    EIK_TILES_2D(EIK_RCASE)
#undef EIK_RCASE
    return fail(EIK_ENOTSUP, "unsupported tile shape");
}

int build_problems(int32_t nprob, const eik_grid* grids, const int64_t* offsets, TileShape ts,
                   std::vector<Prob>* probs, int64_t* ntiles, int64_t* npts) {
    int64_t tile_off = 0;
    for (int i = 0; i < nprob; ++i) {
        int rc = check_grid(&grids[i]);
        if (rc) return rc;
        if (grids[i].ndim != grids[0].ndim) return fail(EIK_EINVAL, "all problems must share ndim");
        int64_t n = (int64_t)grids[i].nx * grids[i].ny * grids[i].nz;
        if (offsets[i + 1] - offsets[i] != n) return fail(EIK_EINVAL, "offsets do not match grid sizes");
        if (offsets[i] < 0) return fail(EIK_EINVAL, "negative offset");
        Prob p = make_prob(grids[i], ts, offsets[i], tile_off);
        tile_off += tiles_of(p);
        if (tile_off > ((int64_t)1 << 30)) return fail(EIK_ENOTSUP, "more than 2^30 tiles");
        probs->push_back(p);
    }
    *ntiles = tile_off;
    *npts = offsets[nprob];
    return EIK_OK;
}

// ---------------------------------------------------------------------------
// allocation-free forward solve (eik_solve_noalloc)
// ---------------------------------------------------------------------------

// Layout of the static scratch array, in bytes (each part 256-byte aligned):
// the 32 bucket rings at full capacity for kNaMaxTiles tiles, their counters,
// tile states, requeue keys, per-tile minima (warm start), the scalars, the
// statistics words and the source-tile list.
constexpr int64_t kNaMaxTiles = 1 << 16;
constexpr int64_t kNaMaxSrc = 1 << 16;
constexpr size_t na_round(size_t x) { return (x + 255) / 256 * 256; }
constexpr size_t kNaItems = 0;
constexpr size_t kNaCtr = kNaItems + na_round(sizeof(uint64_t) * kRings * kNaMaxTiles);
constexpr size_t kNaTstate = kNaCtr + na_round(sizeof(uint32_t) * kRings * kCtrStride);
constexpr size_t kNaTkey = kNaTstate + na_round(sizeof(uint32_t) * kNaMaxTiles);
constexpr size_t kNaTmin = kNaTkey + na_round(sizeof(uint64_t) * kNaMaxTiles);
constexpr size_t kNaScal = kNaTmin + na_round(sizeof(uint64_t) * kNaMaxTiles);
constexpr size_t kNaCounters = kNaScal + na_round(sizeof(int32_t) * kScalWords);
constexpr size_t kNaSrclist = kNaCounters + na_round(sizeof(unsigned long long) * kCounters);
constexpr size_t kNaBytes = kNaSrclist + na_round(sizeof(int32_t) * kNaMaxSrc);

}  // namespace

// The allocation-free entry point's workspace: one copy per GPU the library
// runs on, held until the process ends (about 17.6 MiB).  Host code never
// uses this name as an address: it asks the runtime for each device's copy
// (hipGetSymbolAddress) and passes that pointer to the kernels.
static __device__ __align__(256) unsigned char scratch[kNaBytes];

namespace {

constexpr int kNaMaxDevices = 64;
struct NaDevice {
    unsigned char* ptr = nullptr;   // this device's `scratch`
    bool wiped = false;             // its rings have been initialised once
    hipStream_t last_stream = nullptr;
    uint64_t last_seq = 0;          // order of its last call among all calls
    int64_t last_ntiles = 0;
};
NaDevice g_na[kNaMaxDevices];
std::mutex g_na_mu;

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
int na_device(int* dev_out, NaDevice** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNaMaxDevices) return fail(EIK_ENOTSUP, "device index beyond 63");
    NaDevice& d = g_na[dev];
    if (!d.ptr) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(EIK_EHIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        d.ptr = (unsigned char*)p;
    }
    *dev_out = dev;
    *out = &d;
    return EIK_OK;
}

Bufs na_bufs(const NaDevice& d, hipStream_t st) {
    Bufs b;
    b.stream = st;
    b.items = (uint64_t*)(d.ptr + kNaItems);
    b.ctr = (uint32_t*)(d.ptr + kNaCtr);
    b.tstate = (uint32_t*)(d.ptr + kNaTstate);
    b.tkey = (uint64_t*)(d.ptr + kNaTkey);
    b.tile_aux = (uint64_t*)(d.ptr + kNaTmin);
    b.scal = (int32_t*)(d.ptr + kNaScal);
    b.counters = (unsigned long long*)(d.ptr + kNaCounters);
    b.srclist = (int32_t*)(d.ptr + kNaSrclist);
    b.timeline = nullptr;
    b.ring_cap = (uint32_t)kNaMaxTiles;
    // the first call on a device initialises the rings (their memory has
    // never been written by this library); later calls find them drained
    b.force_wipe = d.wiped ? 0 : 1;
    return b;
}

int na_dispatch(TileShape ts, const Bufs& b, const ProbTable& T, int64_t nsrc, int64_t ntiles, int64_t npts,
                const double* field, const int64_t* src_idx, const double* src_t0, double* t, uint8_t* par,
                const eik_opts* o) {
#define EIK_NA(a, b_, c, OPV)                                                                             \
    if (ts.x == a && ts.y == b_ && ts.z == c)                                                             \
        return forward_seq<a, b_, c, OPV>(b, T, nsrc, ntiles, npts, field, src_idx, src_t0, t, par, o, nullptr, \
                                          false);
#define EIK_NA0(a, b_, c) EIK_NA(a, b_, c, 0)
#define EIK_NA1(a, b_, c) EIK_NA(a, b_, c, 1)
#define EIK_NA2(a, b_, c) EIK_NA(a, b_, c, 2)
#define EIK_NA3(a, b_, c) EIK_NA(a, b_, c, 3)
    const int op = o ? o->op : EIK_OP_DBAR;
    if (op == EIK_OP_DHAT) {
        EIK_TILES_2D(EIK_NA1)
    } else if (op == EIK_OP_DTILDE) {
        EIK_TILES_2D(EIK_NA2)
    } else if (op == EIK_OP_NEWTON) {
        EIK_TILES_2D(EIK_NA3)
    } else {
        EIK_TILES_3D(EIK_NA0)
        EIK_TILES_2D(EIK_NA0)
    }
#undef EIK_NA
#undef EIK_NA0
#undef EIK_NA1
#undef EIK_NA2
#undef EIK_NA3
    return fail(EIK_ENOTSUP, "unsupported tile shape");
}

}  // namespace

// ---------------------------------------------------------------------------
// exported entry points
// ---------------------------------------------------------------------------

extern "C" {

const char* eik_version(void) { return "eik-mi355x 0.1 (gfx950)"; }

const char* eik_strerror(int code) {
    switch (code) {
        case EIK_OK: return "ok";
        case EIK_EINVAL: return "invalid argument";
        case EIK_EDOMAIN: return "field value not positive and finite";
        case EIK_ENOMEM: return "out of device memory";
        case EIK_EHIP: return "HIP runtime error";
        case EIK_ELIMIT: return "tile visit limit reached (output is an upper bound)";
        case EIK_ENOTSUP: return "not supported";
        case EIK_EBADSRC: return "invalid source index or start time";
        case EIK_EHANG: return "device watchdog expired";
        default: return "unknown error";
    }
}

const char* eik_last_error(void) { return g_last_error.c_str(); }

int64_t eik_num_tiles(const eik_grid* g, const eik_opts* o) {
    if (check_grid(g)) return -1;
    TileShape ts = pick_tile(g->ndim, o);
    if (!tile_supported(g->ndim, ts.x, ts.y, ts.z)) return -1;
    return tiles_of(make_prob(*g, ts, 0, 0));
}

int eik_solve_batched(int32_t nprob, const eik_grid* grids_host, const int64_t* offsets_host,
                      const double* field_packed, const int64_t* src_off_host, const int64_t* src_idx,
                      const double* src_t0, double* t_packed, uint8_t* parents_packed,
                      const eik_opts* opts, void* stream) {
    if (nprob < 1 || !grids_host || !offsets_host || !src_off_host)
        return fail(EIK_EINVAL, "nprob, grids, offsets and src offsets are required");
    if (!field_packed || !src_idx || !t_packed) return fail(EIK_EINVAL, "NULL device pointer");
    if (offsets_host[0] != 0 || src_off_host[0] != 0) return fail(EIK_EINVAL, "offsets must start at 0");
    int rc = check_opts(opts);
    if (rc) return rc;
    std::vector<int64_t> soff(src_off_host, src_off_host + nprob + 1);
    for (int i = 0; i < nprob; ++i)
        if (soff[i + 1] - soff[i] < 1) return fail(EIK_EINVAL, "every problem needs at least one source");
    if (soff[nprob] > ((int64_t)1 << 31)) return fail(EIK_ENOTSUP, "too many sources");
    TileShape ts = pick_tile(grids_host[0].ndim, opts);
    if (!tile_supported(grids_host[0].ndim, ts.x, ts.y, ts.z))
        return fail(EIK_ENOTSUP, "unsupported tile shape for this ndim");
    if (opts && opts->op != EIK_OP_DBAR && grids_host[0].ndim != 2)
        return fail(EIK_ENOTSUP, "the ablation operators are two-dimensional");
    std::vector<Prob> probs;
    int64_t ntiles = 0, npts = 0;
    if ((rc = build_problems(nprob, grids_host, offsets_host, ts, &probs, &ntiles, &npts))) return rc;
    Workspace* w = nullptr;
    if ((rc = get_ws((hipStream_t)stream, &w))) return rc;
    return dispatch_forward(ts, *w, probs, soff, ntiles, npts, field_packed, src_idx, src_t0, t_packed,
                            parents_packed, opts);
}

int eik_solve(const eik_grid* g, const double* field, int64_t nsrc, const int64_t* src_idx,
              const double* src_t0, double* t_out, uint8_t* parents_out, const eik_opts* opts,
              void* stream) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (nsrc < 1) return fail(EIK_EINVAL, "nsrc must be >= 1");
    int64_t offs[2] = {0, (int64_t)g->nx * g->ny * g->nz};
    int64_t soff[2] = {0, nsrc};
    return eik_solve_batched(1, g, offs, field, soff, src_idx, src_t0, t_out, parents_out, opts, stream);
}

int eik_solve_noalloc(const eik_grid* g, const double* field, int64_t nsrc, const int64_t* src_idx,
                      const double* src_t0, double* t_out, uint8_t* parents_out, const eik_opts* opts,
                      void* stream) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (nsrc < 1) return fail(EIK_EINVAL, "nsrc must be >= 1");
    if (nsrc > kNaMaxSrc) return fail(EIK_ENOTSUP, "eik_solve_noalloc: more than 65536 sources");
    if (!field || !src_idx || !t_out) return fail(EIK_EINVAL, "NULL device pointer");
    if ((rc = check_opts(opts))) return rc;
    if (opts && (opts->flags & (EIK_FLAG_TIME_KERNELS | EIK_FLAG_TIMELINE)))
        return fail(EIK_ENOTSUP, "eik_solve_noalloc: no kernel timing or timeline (they need memory)");
    const TileShape ts = pick_tile(g->ndim, opts);
    if (!tile_supported(g->ndim, ts.x, ts.y, ts.z)) return fail(EIK_ENOTSUP, "unsupported tile shape for this ndim");
    if (opts && opts->op != EIK_OP_DBAR && g->ndim != 2)
        return fail(EIK_ENOTSUP, "the ablation operators are two-dimensional");
    ProbTable T;
    T.probs = nullptr;
    T.src_off = nullptr;
    T.nprob = 1;
    T.p0 = make_prob(*g, ts, 0, 0);
    T.nsrc0 = nsrc;
    const int64_t ntiles = tiles_of(T.p0);
    if (ntiles > kNaMaxTiles)
        return fail(EIK_ENOTSUP, "eik_solve_noalloc: more than 65536 tiles (use eik_solve)");
    int dev = 0;
    NaDevice* d = nullptr;
    std::lock_guard<std::mutex> lk(g_na_mu);
    if ((rc = na_device(&dev, &d))) return rc;
    const hipStream_t st = (hipStream_t)stream;
    const Bufs b = na_bufs(*d, st);
    const int64_t npts = (int64_t)g->nx * g->ny * g->nz;
    if ((rc = na_dispatch(ts, b, T, nsrc, ntiles, npts, field, src_idx, src_t0, t_out, parents_out, opts)))
        return rc;
    d->wiped = true;
    d->last_stream = st;
    d->last_ntiles = ntiles;
    d->last_seq = next_seq();
    return EIK_OK;
}

int eik_solve_rect(const eik_grid* g, const double* xs_host, const double* ys_host, const double* zs_host,
                   const double* field, int64_t nsrc, const int64_t* src_idx, const double* src_t0, double* t_out,
                   const eik_opts* opts, void* stream) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (nsrc < 1) return fail(EIK_EINVAL, "nsrc must be >= 1");
    if (!field || !src_idx || !t_out) return fail(EIK_EINVAL, "NULL device pointer");
    if ((rc = check_opts(opts))) return rc;
    if (opts && (opts->op != EIK_OP_DBAR || opts->work_ref || (opts->flags & (EIK_FLAG_PACKED | EIK_FLAG_TRACK_CHANGE))))
        return fail(EIK_ENOTSUP, "rectilinear grids run the exact operator, per-thread passes, no work classification");
    std::vector<double> rw;
    if ((rc = rect_weights(*g, xs_host, ys_host, zs_host, &rw))) return rc;
    const TileShape ts = pick_tile(g->ndim, opts);
    if (!tile_supported(g->ndim, ts.x, ts.y, ts.z)) return fail(EIK_ENOTSUP, "unsupported tile shape for this ndim");
    eik_grid gu = *g;
    gu.h = 1.0;  // the spacing lives in the weights; q = 1 / v or s
    std::vector<Prob> probs{make_prob(gu, ts, 0, 0)};
    std::vector<int64_t> soff{0, nsrc};
    const int64_t ntiles = tiles_of(probs[0]);
    const int64_t npts = (int64_t)g->nx * g->ny * g->nz;
    Workspace* w = nullptr;
    if ((rc = get_ws((hipStream_t)stream, &w))) return rc;
    if ((rc = upload_weights(*w, rw))) return rc;
    return dispatch_rect(ts, *w, probs, soff, ntiles, npts, field, src_idx, src_t0, t_out, opts);
}

int eik_parents(const eik_grid* g, const double* t, int64_t nsrc, const int64_t* src_idx,
                uint8_t* parents_out, void* stream) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!t || !parents_out || (nsrc > 0 && !src_idx)) return fail(EIK_EINVAL, "NULL device pointer");
    if (nsrc < 0) return fail(EIK_EINVAL, "nsrc must be >= 0");
    Workspace* w = nullptr;
    if ((rc = get_ws((hipStream_t)stream, &w))) return rc;
    TileShape ts = pick_tile(g->ndim, nullptr);
    std::vector<Prob> probs{make_prob(*g, ts, 0, 0)};
    std::vector<int64_t> soff{0, nsrc};
    ProbTable T;
    if ((rc = make_table(*w, probs, &soff, &T))) return rc;
    int64_t n = (int64_t)g->nx * g->ny * g->nz;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k_parents, dim3(blocks_for(n, kThreads, 1 << 16)), dim3(kThreads), 0, st, T,
                       (long long)n, t, parents_out);
    if (nsrc > 0)
        hipLaunchKernelGGL(k_parents_mark_src, dim3(blocks_for(nsrc, kThreads)), dim3(kThreads), 0, st,
                           T, src_idx, (long long)nsrc, parents_out);
    HIP_TRY(hipGetLastError());
    return EIK_OK;
}

int eik_residual(const eik_grid* g, const double* field, int64_t nsrc, const int64_t* src_idx, const double* t,
                 int32_t op, int64_t* count_host, double* maxrel_host, void* stream) {
    int rc = check_grid(g);
    if (rc) return rc;
    if (!field || !t || (nsrc > 0 && !src_idx)) return fail(EIK_EINVAL, "NULL device pointer");
    if (nsrc < 0) return fail(EIK_EINVAL, "nsrc must be >= 0");
    if (op < EIK_OP_DBAR || op > EIK_OP_NEWTON) return fail(EIK_EINVAL, "unknown operator");
    if (op != EIK_OP_DBAR && g->ndim != 2) return fail(EIK_ENOTSUP, "the ablation operators are two-dimensional");
    Workspace* w = nullptr;
    if ((rc = get_ws((hipStream_t)stream, &w))) return rc;
    const int64_t n = (int64_t)g->nx * g->ny * g->nz;
    if ((rc = grow(&w->mask, &w->mask_cap, n, w->stream))) return rc;
    hipStream_t st = w->stream;
    const Prob P = make_prob(*g, pick_tile(g->ndim, nullptr), 0, 0);
    unsigned long long* out = w->counters + 13;  // [13] count, [14] max rel bits, [15] flags
    uint32_t* flags = (uint32_t*)(w->counters + 15);
    hipLaunchKernelGGL(k_fill_u8, dim3(blocks_for(n, kThreads, 8192)), dim3(kThreads), 0, st, (long long)n,
                       w->mask, (uint8_t)0);
    hipLaunchKernelGGL(k_clear_residual, dim3(1), dim3(64), 0, st, out);
    if (nsrc > 0)
        hipLaunchKernelGGL(k_mark_points, dim3(blocks_for(nsrc, kThreads)), dim3(kThreads), 0, st, src_idx,
                           (long long)nsrc, (long long)n, w->mask);
    const dim3 gr(blocks_for(n, kThreads, 8192)), bl(kThreads);
    if (op == EIK_OP_DHAT) hipLaunchKernelGGL(k_residual<1>, gr, bl, 0, st, P, field, t, w->mask, out, flags);
    else if (op == EIK_OP_DTILDE) hipLaunchKernelGGL(k_residual<2>, gr, bl, 0, st, P, field, t, w->mask, out, flags);
    else if (op == EIK_OP_NEWTON) hipLaunchKernelGGL(k_residual<3>, gr, bl, 0, st, P, field, t, w->mask, out, flags);
    else hipLaunchKernelGGL(k_residual<0>, gr, bl, 0, st, P, field, t, w->mask, out, flags);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    unsigned long long res[2];
    uint32_t fl = 0;
    HIP_TRY(hipMemcpy(res, out, sizeof(res), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&fl, flags, sizeof(fl), hipMemcpyDeviceToHost));
    if (fl & kFlagDomain) return fail(EIK_EDOMAIN, "field value not positive and finite");
    if (count_host) *count_host = (int64_t)res[0];
    if (maxrel_host) {
        double d;
        std::memcpy(&d, &res[1], sizeof(d));
        *maxrel_host = d;
    }
    return EIK_OK;
}

int eik_adjoint_batched(int32_t nprob, const eik_grid* grids_host, const int64_t* offsets_host,
                        const double* field_packed, const double* t_packed,
                        const uint8_t* parents_packed, const double* dL_dt_packed, double* dL_ds_packed,
                        double* mu_packed, const eik_opts* opts, void* stream) {
    if (nprob < 1 || !grids_host || !offsets_host) return fail(EIK_EINVAL, "nprob, grids, offsets required");
    if (!field_packed || !t_packed || !parents_packed || !dL_dt_packed || !dL_ds_packed)
        return fail(EIK_EINVAL, "NULL device pointer");
    if (offsets_host[0] != 0) return fail(EIK_EINVAL, "offsets must start at 0");
    int rc = check_opts(opts);
    if (rc) return rc;
    TileShape ts = pick_tile(grids_host[0].ndim, opts);
    if (!tile_supported(grids_host[0].ndim, ts.x, ts.y, ts.z))
        return fail(EIK_ENOTSUP, "unsupported tile shape for this ndim");
    std::vector<Prob> probs;
    int64_t ntiles = 0, npts = 0;
    if ((rc = build_problems(nprob, grids_host, offsets_host, ts, &probs, &ntiles, &npts))) return rc;
    Workspace* w = nullptr;
    if ((rc = get_ws((hipStream_t)stream, &w))) return rc;
    return adjoint_run(*w, ts, probs, ntiles, npts, field_packed, t_packed, parents_packed, dL_dt_packed,
                       dL_ds_packed, mu_packed, opts);
}

int eik_adjoint(const eik_grid* g, const double* field, const double* t, const uint8_t* parents,
                const double* dL_dt, double* dL_dslowness, double* mu_out, const eik_opts* opts,
                void* stream) {
    int rc = check_grid(g);
    if (rc) return rc;
    int64_t offs[2] = {0, (int64_t)g->nx * g->ny * g->nz};
    return eik_adjoint_batched(1, g, offs, field, t, parents, dL_dt, dL_dslowness, mu_out, opts, stream);
}

int eik_reserve(int64_t ntiles, int64_t npts, void* stream) {
    if (ntiles < 0 || npts < 0) return fail(EIK_EINVAL, "sizes must be >= 0");
    Workspace* w = nullptr;
    int rc;
    if ((rc = get_ws((hipStream_t)stream, &w))) return rc;
    if ((rc = ensure_tiles(*w, std::max<int64_t>(ntiles, 1)))) return rc;
    if ((rc = grow(&w->mu, &w->mu_cap, std::max<int64_t>(npts, 1), w->stream))) return rc;
    return EIK_OK;
}

int eik_status(void* stream, eik_stats* out) {
    const hipStream_t st = (hipStream_t)stream;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    Workspace* w = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_ws.find(std::make_pair(dev, st));
        if (it != g_ws.end()) w = it->second;
    }
    // The last call on this stream may have been eik_solve_noalloc, whose
    // status words live in this device's scratch array; then nothing is
    // allocated here either.
    const int32_t* scal_src = nullptr;
    const unsigned long long* ctr_src = nullptr;
    int64_t last_ntiles = 0;
    {
        std::lock_guard<std::mutex> lk(g_na_mu);
        if (dev >= 0 && dev < kNaMaxDevices) {
            const NaDevice& d = g_na[dev];
            if (d.ptr && d.last_seq > 0 && d.last_stream == st && (!w || d.last_seq > w->last_seq)) {
                scal_src = (const int32_t*)(d.ptr + kNaScal);
                ctr_src = (const unsigned long long*)(d.ptr + kNaCounters);
                last_ntiles = d.last_ntiles;
            }
        }
    }
    int rc;
    if (!scal_src) {
        if (!w && (rc = get_ws(st, &w))) return rc;
        scal_src = w->scal;
        ctr_src = w->counters;
        last_ntiles = w->last_ntiles;
    }
    HIP_TRY(hipStreamSynchronize(st));
    int32_t sc[kScalWords];
    unsigned long long ctr[kCounters];
    HIP_TRY(hipMemcpy(sc, scal_src, sizeof(sc), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ctr, ctr_src, sizeof(ctr), hipMemcpyDeviceToHost));
    uint32_t flags = (uint32_t)sc[kSFlags];
    int code = EIK_OK;
    if (flags & kFlagWatchdog) code = EIK_EHANG;
    else if (flags & kFlagBadSrc) code = EIK_EBADSRC;
    else if (flags & kFlagBadStart) code = EIK_EINVAL;
    else if (flags & kFlagDomain) code = EIK_EDOMAIN;
    else if (flags & kFlagLimit) code = EIK_ELIMIT;
    if (out) {
        out->tile_visits = (int64_t)ctr[0];
        out->point_updates = (int64_t)ctr[1];
        out->relax_passes = (int64_t)ctr[2];
        out->ntiles = last_ntiles;
        out->flags = flags;
        out->status = code;
        out->kernel_ms = -1.0;
        out->kernel_launches = w ? (int64_t)w->ev_used : 0;
        for (int i = 0; i < 4; ++i) out->phase_us[i] = (double)ctr[5 + i] / 100.0;  // 100 MHz clock
        out->workgroups = (int64_t)ctr[10];
        out->bucket_advances = (int64_t)ctr[11];
        out->handoffs = (int64_t)ctr[12];
        out->evaluations = (int64_t)ctr[16];
        out->improving = (int64_t)ctr[17];
        out->final_updates = (int64_t)ctr[18];
        if (w && w->ev_used) {
            double sum = 0.0;
            for (size_t i = 0; i < w->ev_used; ++i) {
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, w->ev[2 * i], w->ev[2 * i + 1]));
                sum += ms;
            }
            out->kernel_ms = sum / (double)w->ev_used;
        }
    }
    if (w) w->ev_used = 0;
    if (code != EIK_OK)
        g_last_error = code == EIK_EINVAL ? "warm-start times must be >= +0 and not NaN" : eik_strerror(code);
    return code;
}

int eik_timeline(void* stream, int32_t cap, double* t_us_host, int64_t* bucket_host, double* span_us_host) {
    if (cap < 0 || (cap > 0 && (!t_us_host || !bucket_host))) return fail(EIK_EINVAL, "bad timeline buffers");
    Workspace* w = nullptr;
    int rc;
    if ((rc = get_ws((hipStream_t)stream, &w))) return rc;
    HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
    unsigned long long ctr[kCounters];
    HIP_TRY(hipMemcpy(ctr, w->counters, sizeof(ctr), hipMemcpyDeviceToHost));
    const int64_t n = std::min<int64_t>((int64_t)ctr[11], kTimelineCap);
    std::vector<unsigned long long> tl((size_t)(2 + 2 * n));
    HIP_TRY(hipMemcpy(tl.data(), w->timeline, sizeof(unsigned long long) * tl.size(), hipMemcpyDeviceToHost));
    const unsigned long long t0 = tl[0];
    if (span_us_host) span_us_host[0] = tl[1] > t0 ? (double)(tl[1] - t0) / 100.0 : 0.0;
    const int64_t m = std::min<int64_t>(n, cap);
    for (int64_t i = 0; i < m; ++i) {
        const unsigned long long ti = tl[2 + 2 * i];
        t_us_host[i] = ti > t0 ? (double)(ti - t0) / 100.0 : 0.0;
        bucket_host[i] = (int64_t)tl[3 + 2 * i];
    }
    return (int)n;
}

void eik_release(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& kv : g_ws) {
        Workspace* w = kv.second;
        int cur = 0;
        if (hipGetDevice(&cur) == hipSuccess && cur != w->device) (void)hipSetDevice(w->device);
        (void)hipStreamSynchronize(w->stream);
        (void)hipFree(w->items);
        (void)hipFree(w->ctr);
        (void)hipFree(w->timeline);
        (void)hipFree(w->mask);
        (void)hipFree(w->tstate);
        (void)hipFree(w->tkey);
        (void)hipFree(w->scal);
        (void)hipFree(w->counters);
        (void)hipFree(w->srclist);
        (void)hipFree(w->rw);
        for (Table& tb : w->tables) {
            (void)hipFree(tb.d_probs);
            (void)hipFree(tb.d_src_off);
        }
        (void)hipFree(w->mu);
        (void)hipFree(w->tile_tmax);
        for (hipEvent_t e : w->ev) (void)hipEventDestroy(e);
        if (cur != w->device) (void)hipSetDevice(cur);
        delete w;
    }
    g_ws.clear();
}

}  // extern "C"

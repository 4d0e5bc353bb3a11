/*
 * eik.h -- C ABI of the MI355X (gfx950) Eikonal travel-time library.
 *
 * What is computed
 * ----------------
 * First-arrival times t on a structured 2D or 3D grid with spacing h and a
 * positive speed (or slowness) field, from point sources with given start
 * times.  The discrete equations are the first-order upwind scheme of the
 * paper's Eq. (finite_difference): at every non-source point the upwind
 * differences per axis, taken from the smaller neighbour on that axis, have a
 * 2-norm equal to the local slowness (Eq. difference_as_root, and the one-sided
 * case of Algorithm "Eikonal Update Operator").  Rounding follows the paper's
 * exactly monotone semantics (section "Achieving Exact Monotonicity with Finite
 * Precision Arithmetic"): with a_k the smaller axis-k neighbour (+inf off the
 * grid), q = fl(h/v) or fl(h*s), c = fl(q*q), T_k(r) = fl(fl(r-a_k)^2) when
 * r > a_k else +0, and S(r) the T_k summed largest first, each point's value is
 * the smallest binary64 r >= min_k a_k with S(r) >= c.  That operator is
 * monotone and causal in floating point, so by the paper's Theorem 1 every
 * update order reaches the same fixed point: results are bit-identical to a
 * sequential fast-marching solve and across runs.
 *
 * Conventions
 * -----------
 *  - Layout: C-order [nz][ny][nx] float64, x fastest; 2D grids use nz = 1.
 *  - All array arguments are DEVICE pointers on the current HIP device unless
 *    their name ends in _host.  The caller owns every input and output buffer;
 *    the library only reads/writes them inside work enqueued on `stream`.
 *  - All work is enqueued on `stream` (a hipStream_t, NULL = default stream);
 *    only eik_status(), eik_residual() and eik_timeline() synchronise the host
 *    (and the first call with a given batch layout -- problems, tile shape,
 *    source offsets -- which uploads its table; up to 64 layouts are kept per
 *    workspace).
 *  - The library owns a workspace per (device, stream) (tile states, priority
 *    queues, counters), allocated on first use, grown on demand and freed by
 *    eik_release().  Two calls on the same stream are ordered; calls on
 *    different streams use different workspaces.
 *  - Return codes: EIK_OK (0) or a negative EIK_E* code.  Errors detectable on
 *    the host return immediately without enqueuing work.  Errors found on the
 *    device (bad field values, bad sources, the visit cap) are reported by
 *    eik_status() for the last call on that stream.  eik_last_error() gives a
 *    thread-local message for the last failing call.
 */
#ifndef EIK_H
#define EIK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EIK_OK 0
#define EIK_EINVAL (-1)   /* bad argument (dims, h, pointers, options) */
#define EIK_EDOMAIN (-2)  /* a field value is <= 0, NaN or Inf, or c over/underflows */
#define EIK_ENOMEM (-3)   /* workspace allocation failed */
#define EIK_EHIP (-4)     /* HIP runtime error; eik_last_error() has the text */
#define EIK_ELIMIT (-5)   /* max_tile_visits reached: output is an upper bound */
#define EIK_ENOTSUP (-6)  /* shape / tile / size combination not supported */
#define EIK_EBADSRC (-7)  /* a source index was out of range or a t0 invalid */
#define EIK_EHANG (-8)    /* a device-side watchdog expired (internal error) */

#define EIK_FLAG_TIME_KERNELS 1u  /* eik_opts.flags: time the persistent kernel with HIP events */
                                  /* bit value 2 is unused (rejected as unknown) */
#define EIK_FLAG_TIMELINE 4u      /* eik_opts.flags: record when the lowest open priority bucket
                                     moves on (read back with eik_timeline) */
#define EIK_FLAG_TRACK_CHANGE 8u  /* eik_opts.flags, ablation operators only: re-activate the
                                     neighbours when a value changes, not only when it decreases
                                     (the precision section's change tracking) */
#define EIK_FLAG_PACKED 32u       /* eik_opts.flags, forward solves with EIK_OP_DBAR and
                                     adjoints: each relaxation (adjoint: readiness) pass
                                     first compacts the tile's dirty points into a dense
                                     list (256-thread workgroups); without it every thread
                                     handles its own point (one thread per point, up to
                                     1024).  Same result either way; the packed form does
                                     fewer evaluations per wave and can win when the device
                                     is full of work (batches of shots), the default has
                                     lower latency per pass (single solves). */
#define EIK_FLAG_WARM_START 16u   /* eik_opts.flags, forward solves with EIK_OP_DBAR: resume from
                                     the times already in t_out instead of +inf.  They must be
                                     an upper bound of the solution at every point (>= +0, not
                                     NaN; +inf allowed), e.g. the output of a call on the same
                                     problem that stopped with EIK_ELIMIT.  The operator is
                                     monotone and causal, so from any such state every update
                                     order reaches the same fixed point as a cold solve (the
                                     argument of Theorem 1): the result is bit-identical.
                                     Sources are fixed at their t0 again; every tile with a
                                     finite value in itself or a face neighbour is queued.  A
                                     NaN or negative (sign bit set) input value is replaced by
                                     +inf and reported by eik_status as EIK_EINVAL. */

#define EIK_OP_DBAR 0     /* eik_opts.op: smallest double with S(r) >= c (section "Achieving
                             Exact Monotonicity with Finite Precision Arithmetic") */
#define EIK_OP_DHAT 1     /* the reordered explicit formula of Table "tab:prec_2" */
#define EIK_OP_DTILDE 2   /* the textbook explicit formula of Table "tab:prec_1" */
#define EIK_OP_NEWTON 3   /* Newton's method on the root function from the d-hat guess (the
                             precision section's practical variant; up to 8 steps) */

#define EIK_SPEED 0       /* field holds speed v:    q = h / v */
#define EIK_SLOWNESS 1    /* field holds slowness s: q = h * s */

typedef struct {
    int32_t ndim;        /* 2 or 3 */
    int32_t nx, ny, nz;  /* points per axis; nz must be 1 when ndim == 2 */
    double h;            /* grid spacing, > 0 and finite */
    int32_t field_kind;  /* EIK_SPEED or EIK_SLOWNESS */
} eik_grid;

typedef struct {
    double delta;            /* priority bucket width in time units; 0 => one bucket (FIFO);
                                EIK_EINVAL when negative, NaN or so small that 1/delta
                                overflows */
    int32_t tile[3];         /* tile shape (x, y, z); zeros => default for ndim (3D 16x8x8,
                                2D 32x32).  Supported: 3D 32x8x4, 16x8x8, 8x8x8, 64x4x4,
                                16x8x4, 8x8x4, 8x4x4; 2D 32x32, 64x16, 128x8, 16x16, 16x8 */
    int32_t grid_blocks;     /* persistent workgroups; 0 => fill the device */
    int64_t max_tile_visits; /* 0 => unlimited; else stop after this many tile visits (ELIMIT) */
    uint32_t flags;          /* EIK_FLAG_* bits.  EIK_FLAG_TIME_KERNELS: record HIP events
                                around the persistent kernel (solve or adjoint) on `stream`;
                                eik_status then reports the mean duration of the kernels timed
                                since the previous eik_status (at most 4096 launches in
                                between).  EIK_FLAG_TIMELINE, EIK_FLAG_TRACK_CHANGE,
                                EIK_FLAG_WARM_START, EIK_FLAG_PACKED: above */
    int32_t lookahead;       /* 0..16: work may be taken from the lowest non-drained bucket
                                and this many buckets above it (0 = strict bucket order) */
    int32_t horizon;         /* 0 => off; k in 1..4: a run of a tile claimed from bucket b
                                settles only values r with floor(r / delta) < b + k and requeues
                                the tile for the rest (no effect when delta == 0) */
    int32_t op;              /* update operator: EIK_OP_DBAR (0, the exact monotone rounding;
                                the only one with a schedule-independent result), or, for 2D
                                grids and block tiles only (precision ablation), EIK_OP_DHAT /
                                EIK_OP_DTILDE (the paper's explicit formulas) or EIK_OP_NEWTON.
                                These assign the operator's value (it may rise: they are not
                                monotone) and re-activate neighbours when it drops (or changes,
                                with EIK_FLAG_TRACK_CHANGE); since termination is then not
                                guaranteed, max_tile_visits == 0 means 256 runs per tile and a
                                run stops after 65536 relaxation passes (both: EIK_ELIMIT) */
    const double* work_ref;  /* NULL, or (device, block tiles) the final times of this very
                                solve: every operator evaluation is then classified as empty
                                (no change), good (sets the final value) or bad (lowers the
                                value to something not yet final), the update classes of the
                                paper's work-efficiency analysis; see eik_stats */
} eik_opts;

typedef struct {
    int64_t tile_visits;     /* tiles claimed and processed by the persistent solve */
    int64_t point_updates;   /* points whose value decreased, summed over visits */
    int64_t ntiles;          /* tiles in the problem(s) */
    int64_t relax_passes;    /* in-tile relaxation passes (adjoint: readiness passes), summed
                                over visits */
    uint32_t flags;          /* raw device flags (bit0 domain, bit1 limit, bit2 bad source, bit3 watchdog,
                                bit4 invalid warm-start value) */
    int32_t status;          /* the EIK_* code these flags map to */
    double kernel_ms;        /* mean duration of the timed persistent kernels, or -1 */
    int64_t kernel_launches; /* how many launches kernel_ms averages */
    double phase_us[4];      /* last solve or adjoint, summed over workgroups (microseconds of
                                wall clock): [0] claiming / waiting for work, [1] staging a
                                tile and its halo in LDS, [2] relaxing (adjoint: readiness
                                passes), [3] write-back + publish */
    int64_t workgroups;      /* persistent workgroups of the last launch */
    int64_t bucket_advances; /* times the lowest open priority bucket moved on */
    int64_t handoffs;        /* runs that started on a neighbour handed on by the previous run */
    int64_t evaluations;     /* with eik_opts.work_ref: operator evaluations in the solve */
    int64_t improving;       /*   ... of which lowered the value (the rest were empty) */
    int64_t final_updates;   /*   ... of which set the final value (good; the rest were bad) */
} eik_stats;

/* Forward solve.
 *   g        grid description (host struct).
 *   field    [nz][ny][nx] speed or slowness (device).
 *   nsrc     number of point sources, >= 1.
 *   src_idx  nsrc flat indices (iz*ny+iy)*nx+ix (device int64).  Duplicates are
 *            allowed (the smallest start time wins).
 *   src_t0   nsrc start times >= +0.0 and finite (device), or NULL for all +0.0.
 *   t_out    [nz][ny][nx] arrival times (device, written entirely; with
 *            EIK_FLAG_WARM_START also read first: the starting upper bound).
 *   parents_out  NULL, or [nz][ny][nx] uint8 upwind-parent record computed from
 *            the final times: per axis k (bits 2k..2k+1) 0 = axis not upwind,
 *            1 = minus-side neighbour, 2 = plus-side neighbour (ties: minus);
 *            bit 7 set (other bits 0) marks a source point.
 *   opts     NULL for defaults.
 *   stream   hipStream_t or NULL.
 * Returns EIK_OK when the work was enqueued. */
int eik_solve(const eik_grid* g, const double* field, int64_t nsrc, const int64_t* src_idx,
              const double* src_t0, double* t_out, uint8_t* parents_out,
              const eik_opts* opts, void* stream);

/* Forward solve on a rectilinear grid: the spacing varies per axis and per
 * index, given by the points' coordinates.  The scheme is the first-order
 * upwind one with, per axis, the larger of the two one-sided differences
 * (t - t_minus)/h_minus and (t - t_plus)/h_plus (when positive); rounding
 * follows the exactly monotone construction of the section "Achieving Exact
 * Monotonicity with Finite Precision Arithmetic", applied to this scheme (the
 * irregular-grid case the paper's conclusion points to): with
 * w = fl(1 / fl(x_i - x_{i-1})) per side, m_k(r) = max(fl(fl(r - am)*wm),
 * fl(fl(r - ap)*wp)), T_k = fl(m_k^2) when m_k > 0 else +0, S(r) the T_k summed
 * largest first (fl(fl(T_hi + T_mid) + T_lo)) and c = fl(s^2) for
 * the slowness s = 1/v (speed field) or s, each point's value is the smallest
 * binary64 r >= min of its neighbours with S(r) >= c.  The operator is monotone
 * and causal, so the result is schedule-independent (Theorem 1); with unit
 * spacing it equals eik_solve with h = 1 bit for bit.
 *   xs_host, ys_host, zs_host  host arrays of nx, ny, nz coordinates, strictly
 *            increasing and finite (zs_host ignored for 2D grids); g->h is
 *            ignored.  EIK_EINVAL otherwise.  The first call with given
 *            coordinates on a stream uploads their reciprocal spacings
 *            (synchronising the stream).
 *   field, nsrc, src_idx, src_t0, t_out, stream: as for eik_solve.
 *   opts     as for eik_solve, except: op must be EIK_OP_DBAR, and
 *            EIK_FLAG_PACKED, EIK_FLAG_TRACK_CHANGE and work_ref are not
 *            available (EIK_ENOTSUP).  EIK_FLAG_WARM_START works as for
 *            eik_solve.  No parent record (the adjoint is for uniform grids). */
int eik_solve_rect(const eik_grid* g, const double* xs_host, const double* ys_host, const double* zs_host,
                   const double* field, int64_t nsrc, const int64_t* src_idx, const double* src_t0,
                   double* t_out, const eik_opts* opts, void* stream);

/* Allocation-free forward solve.  For callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results (bit for bit), options and errors
 * as eik_solve, for one problem; but every work buffer (bucket rings, tile
 * states, counters, status words) lives in a static array of the library, one
 * copy per GPU it runs on (about 17.6 MiB, held until the process ends), so
 * the call allocates nothing and uses no per-stream workspace.  Its device
 * address is looked up once per device, on the first call there.
 * Limits, checked before anything is enqueued (EIK_ENOTSUP): at most 65536
 * tiles (see eik_num_tiles) and 65536 sources; EIK_FLAG_TIME_KERNELS and
 * EIK_FLAG_TIMELINE are not available.
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents: each call clears what it needs, but calls whose work may overlap
 * on one GPU (different streams, or different host threads on one stream
 * without ordering) race and give wrong results; serialise them.  The device
 * status of the call is read with eik_status(stream), as for eik_solve. */
int eik_solve_noalloc(const eik_grid* g, const double* field, int64_t nsrc, const int64_t* src_idx,
                      const double* src_t0, double* t_out, uint8_t* parents_out,
                      const eik_opts* opts, void* stream);

/* Upwind-parent record (same encoding as parents_out above) from final times t
 * of a finished solve.  src_idx as for eik_solve. */
int eik_parents(const eik_grid* g, const double* t, int64_t nsrc, const int64_t* src_idx,
                uint8_t* parents_out, void* stream);

/* Adjoint: gradient of a loss L(t) with respect to slowness, given dL/dt.
 * Linearises the discrete equations sum_k (t_n - t_{p_k})^2 = (q_n)^2 over the
 * recorded upwind parents p_k (implicit differentiation; the paper is silent on
 * gradients).  With w_{n,k} = fl(t_n - t_{p_k}), W_n = fl(fl(w_x + w_y) + w_z):
 *   lambda_n = dL/dt_n + sum over children m (neighbour order x-,x+,y-,y+,z-,z+)
 *              of fl(mu_m * w_{m,k}),   mu_n = fl(lambda_n / W_n),
 *   dL/ds_n  = fl(fl(mu_n * q_n) * h),  0 at sources,
 * evaluated children-first (decreasing t), so results are deterministic.
 *   t, parents   outputs of a finished eik_solve on the same grid and field.
 *   dL_dt        [nz][ny][nx] (device).
 *   dL_dslowness [nz][ny][nx] output (device).  For a speed field the gradient
 *                is still with respect to slowness s = 1/v.
 *   mu_out       NULL or [nz][ny][nx] scratch output receiving mu (device);
 *                when NULL the library uses workspace memory.  It is filled
 *                with NaN ("not done") first; on return it holds mu at every
 *                point (0 at sources).  Its previous contents are not read.
 * Errors as eik_solve (EIK_EINVAL for NULL pointers or a bad grid, EIK_EDOMAIN
 * from the device for a bad field value, reported by eik_status). */
int eik_adjoint(const eik_grid* g, const double* field, const double* t, const uint8_t* parents,
                const double* dL_dt, double* dL_dslowness, double* mu_out,
                const eik_opts* opts, void* stream);

/* Batched forward solve of nprob independent problems in ONE persistent launch.
 *   grids_host    nprob grid descriptions (all the same ndim).
 *   offsets_host  nprob+1 point offsets into the packed arrays (offsets_host[0] == 0,
 *                 offsets_host[i+1] - offsets_host[i] == nx*ny*nz of problem i).
 *   field_packed, t_packed, parents_packed (NULL ok): concatenated per-problem arrays.
 *   src_off_host  nprob+1 offsets into src_idx / src_t0 (sources of problem i are
 *                 src_off_host[i] .. src_off_host[i+1]-1, each problem >= 1 source).
 *   src_idx       local flat indices within each problem (device int64).
 *   src_t0        device start times or NULL (all +0.0).
 * The call enqueues a fixed sequence of kernels with no host synchronisation and
 * no allocation once the workspace has grown to this size, so it may be captured
 * into a HIP graph after one warm-up call with the same sizes. */
int eik_solve_batched(int32_t nprob, const eik_grid* grids_host, const int64_t* offsets_host,
                      const double* field_packed, const int64_t* src_off_host,
                      const int64_t* src_idx, const double* src_t0, double* t_packed,
                      uint8_t* parents_packed, const eik_opts* opts, void* stream);

/* Batched adjoint with the same packing (mu_packed NULL => workspace). */
int eik_adjoint_batched(int32_t nprob, const eik_grid* grids_host, const int64_t* offsets_host,
                        const double* field_packed, const double* t_packed,
                        const uint8_t* parents_packed, const double* dL_dt_packed,
                        double* dL_ds_packed, double* mu_packed, const eik_opts* opts,
                        void* stream);

/* Pre-grow the workspace of `stream` for up to `ntiles` tiles and `npts`
 * points so that later calls of that size allocate nothing (e.g. before HIP
 * graph capture). */
int eik_reserve(int64_t ntiles, int64_t npts, void* stream);

/* Number of tiles a problem of this grid uses with these options (host only). */
int64_t eik_num_tiles(const eik_grid* g, const eik_opts* opts);

/* Synchronises `stream`, copies the device status of the last call on it into
 * *out_host (may be NULL) and returns its EIK_* code. */
int eik_status(void* stream, eik_stats* out_host);

/* Residual of a solution, the error metric of Table "tab:error": applies the
 * operator `op` (EIK_OP_*; the explicit formulas for 2D grids only) once at
 * every point that is not one of the nsrc sources (device src_idx), using the
 * neighbours' values in t (device, C-order), and counts the points whose value
 * would change (*count_host) and the largest relative change |r - t| / |t|
 * (*maxrel_host; either pointer may be NULL).  0 for every d-bar solution of
 * eik_solve.  Synchronises `stream`.  EIK_EDOMAIN if a field value is not
 * positive and finite. */
int eik_residual(const eik_grid* g, const double* field, int64_t nsrc, const int64_t* src_idx,
                 const double* t, int32_t op, int64_t* count_host, double* maxrel_host, void* stream);

/* Schedule record of the last persistent launch on `stream` that ran with
 * EIK_FLAG_TIMELINE (the soft-priority bucket order of the section "The
 * Asynchronous Marching Method"): synchronises `stream`, writes for the first
 * min(cap, n) bucket advances the time since the launch's reset (t_us_host,
 * microseconds) and the bucket the window moved to (bucket_host), and the time
 * from reset to the last workgroup's exit (*span_us_host, may be NULL).
 * Returns n, the number of advances (the record holds at most 65536), or a
 * negative EIK_* code. */
int eik_timeline(void* stream, int32_t cap, double* t_us_host, int64_t* bucket_host, double* span_us_host);

const char* eik_strerror(int code);
const char* eik_last_error(void);

/* Frees every cached workspace on every device. */
void eik_release(void);

/* Library version string. */
const char* eik_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EIK_H */

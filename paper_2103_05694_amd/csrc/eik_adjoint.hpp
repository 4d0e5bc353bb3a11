// Adjoint (reverse) sweep: gradient of a travel-time loss with respect to
// slowness through the recorded upwind dependency graph.
//
// The paper gives no gradient; it is the implicit derivative of the discrete
// equations of Eq. (difference_as_root) -- sum over upwind axes of
// (t_n - t_{p_k})^2 = q_n^2 with q_n = h * s_n -- over the upwind parents p_k
// the forward pass recorded.  Writing w_{n,k} = fl(t_n - t_{p_k}) and
// W_n = fl(fl(w_x + w_y) + w_z):
//   lambda_n = g_n + sum over children m (n is m's axis-k parent) of
//              fl(mu_m * w_{m,k}), summed in neighbour order x-,x+,y-,y+,z-,z+,
//   mu_n     = fl(lambda_n / W_n),
//   dL/ds_n  = fl(fl(mu_n * q_n) * h),  sources: 0
// (the last line in a separate elementwise pass, k_adj_grad, once every mu is
// final: the sweep itself never reads the field).
// A child always has a strictly larger time than its parent, so the graph is
// acyclic and mu can be evaluated children-first.
//
// The sweep reuses the forward scheduler with tiles as work items, but is
// readiness-driven: a point is evaluated exactly once, when every child (in the
// tile or in the halo) is done, so each mu is a fixed function of final values
// and the result is deterministic whatever the visit order.  "Not done" is a
// NaN in mu, which is filled with NaN before the sweep; a point's mu goes from
// NaN to its final value once, so any read returns one or the other.  Tiles are
// prioritised by decreasing time (key tref - t), and a finished face point
// activates the neighbour tile holding its parent.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "eik_kernels.hpp"

namespace eik {

__device__ __forceinline__ double qnan64() { return as_f64(0x7FF8000000000000ull); }

// mu := NaN ("not done") everywhere before the sweep, so a point of a tile that
// has not run yet reads as not done without looking at the tile's state.
__global__ void k_fill_nan(long long npts_total, double* mu) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < npts_total; i += stride)
        mu[i] = qnan64();
}

// Per tile: largest time (key source) and the problem-wide largest time.
template <int TX, int TY, int TZ>
__global__ void k_adj_prep(ProbTable T, int ntiles, const double* t, uint64_t* tile_tmax,
                           unsigned long long* tref_bits) {
    __shared__ unsigned long long s_m;
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const Prob P = prob_of_tile(T, tile);
        int tl = tile - P.tile_off;
        int tx = tl % P.ntx, ty = (tl / P.ntx) % P.nty, tz = tl / (P.ntx * P.nty);
        if (threadIdx.x == 0) s_m = 0ull;
        __syncthreads();
        unsigned long long m = 0ull;
        for (int i = threadIdx.x; i < TX * TY * TZ; i += blockDim.x) {
            int lx = i % TX, ly = (i / TX) % TY, lz = i / (TX * TY);
            int x = tx * TX + lx, y = ty * TY + ly, z = tz * TZ + lz;
            if (x < P.nx && y < P.ny && z < P.nz) {
                double v = t[P.pt_off + ((int64_t)z * P.ny + y) * P.nx + x];
                if (v < inf64()) {
                    unsigned long long b = as_u64(fabs(v));
                    m = b > m ? b : m;
                }
            }
        }
        if (m) atomicMax(&s_m, m);
        __syncthreads();
        if (threadIdx.x == 0) {
            tile_tmax[tile] = s_m;
            __hip_atomic_fetch_max(tref_bits, s_m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

// Queue every tile, latest first.
__global__ void k_adj_push_all(int ntiles, const uint64_t* tile_tmax,
                               const unsigned long long* tref_bits, Sched s) {
    const double tref = as_f64(*tref_bits);
    if (blockIdx.x == 0 && threadIdx.x == 0) *s.poisoned = 0;  // rings were wiped by the reset
    for (int tile = blockIdx.x * blockDim.x + threadIdx.x; tile < ntiles; tile += gridDim.x * blockDim.x) {
        s.tstate[tile] = kQ;
        __hip_atomic_fetch_add(s.pending, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        push_tile(s, (uint32_t)tile, tref - as_f64(tile_tmax[tile]), 0);
    }
}

// dL/ds from the final multipliers: fl(fl(mu * q) * h) at non-sources, 0 at
// sources (mu is 0 there); a field value outside the domain raises the flag.
// One block per tile, as k_adj_prep.
template <int TX, int TY, int TZ>
__global__ void k_adj_grad(ProbTable T, int ntiles, const double* field, const uint8_t* par, const double* mu,
                           double* grad, uint32_t* flags) {
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const Prob P = prob_of_tile(T, tile);
        const int tl = tile - P.tile_off;
        const int tx = tl % P.ntx, ty = (tl / P.ntx) % P.nty, tz = tl / (P.ntx * P.nty);
        for (int i = threadIdx.x; i < TX * TY * TZ; i += blockDim.x) {
            const int x = tx * TX + i % TX, y = ty * TY + (i / TX) % TY, z = tz * TZ + i / (TX * TY);
            if (!(x < P.nx && y < P.ny && z < P.nz)) continue;
            const int64_t gi = P.pt_off + ((int64_t)z * P.ny + y) * P.nx + x;
            bool ok;
            const double q = field_q(field[gi], P.h, P.kind, ok);
            if (!ok) __hip_atomic_fetch_or(flags, kFlagDomain, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            grad[gi] = (par[gi] & 0x80) ? 0.0 : (mu[gi] * (ok ? q : 0.0)) * P.h;
        }
    }
}

struct AdjArgs {
    ProbTable pt;
    const double* t;
    const uint8_t* par;
    const double* g;
    double* mu;
    uint64_t* tkey;
    const unsigned long long* tref_bits;
    Sched s;
};

// Registers are capped for three waves per SIMD with blocks of up to 256
// threads (with the staging loads all in flight at once the largest tiles would
// otherwise drop to two) and four with larger blocks (the direct form: one
// thread per point).
template <int TX, int TY, int TZ, int NT, bool PACK = false>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT > 256 ? 4 : 3))) k_adjoint(AdjArgs A) {
    using C = TileCfg<TX, TY, TZ, NT>;
    constexpr int NPT = C::NPT;
    __shared__ double sT[C::NLDS];
    __shared__ double sM[C::NLDS];
    __shared__ uint8_t sP[C::NLDS];
    __shared__ double sG[C::NP];               // dL/dt of the tile's points
    __shared__ uint16_t sList[PACK ? C::NP : 1];  // PACK: the pass's dirty points, compacted
    __shared__ __align__(4) uint8_t sDirty[2][C::NP];  // layout of didx()
    __shared__ int s_cnt[2];
    __shared__ int s_more[3];  // direct form, per pass (mod 3): some point completed with an in-tile parent
    __shared__ int s_tile;
    __shared__ int64_t s_bucket;
    __shared__ uint32_t s_state;
    __shared__ uint32_t s_nb[6];
    __shared__ uint32_t s_nid[6];
    __shared__ unsigned long long s_face[6];
    __shared__ unsigned int s_done;
    __shared__ int s_next;  // tile handed on by the previous run's publish, or -1
    // per-workgroup statistics, kept by thread 0 in LDS (not in registers) and
    // flushed once at exit: [0..3] phase times on the 100 MHz wall clock, as in
    // the forward solver (claim, stage, readiness passes, write + publish),
    // [4] visits, [5] points done, [6] passes, [7] hand-offs, [8] the last
    // phase mark
    __shared__ unsigned long long s_stat[9];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const unsigned long long lanes_below = (1ull << lane) - 1ull;
    (void)lanes_below;
    const Sched& S = A.s;
    const double tref = as_f64(*A.tref_bits);
    constexpr int PSTEP[3] = {1, TX, TX * TY};
    constexpr int LSTEP[3] = {1, C::SY, C::SZ};
    constexpr int NAX = C::D3 ? 3 : 2;
    if (tid == 0) {
        s_next = -1;
        s_bucket = 0;
        for (int i = 0; i < 8; ++i) s_stat[i] = 0;
        s_stat[8] = wall_clock64();
    }

    int32_t cur_hint = 0;  // wave 0: the window's lowest bucket as last seen
    for (;;) {
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
                    ++s_stat[4];
                    uint32_t st = __hip_atomic_fetch_xor(S.tstate + tile, kQ | kR, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
                    if ((st & (kQ | kR)) != kQ) set_flag(S, kFlagWatchdog);
                    s_state = st;
                }
            }
        }
        __syncthreads();
        const int tile = s_tile;
        if (tile < 0) break;
        const uint32_t st = s_state;
        const bool visited = (st & kV) != 0;
        const Prob P = prob_of_tile(A.pt, tile);
        if (tid == 0) {
            const unsigned long long now = wall_clock64();
            s_stat[0] += now - s_stat[8];
            s_stat[8] = now;
        }
        const int tl = tile - P.tile_off;
        const int tx = tl % P.ntx, ty = (tl / P.ntx) % P.nty, tz = tl / (P.ntx * P.nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;

        if (tid < 6) {
            int d = tid >> 1, side = tid & 1;
            int nt[3] = {tx, ty, tz};
            int lim[3] = {P.ntx, P.nty, P.ntz};
            nt[d] += side ? 1 : -1;
            uint32_t w = 0, nid = 0;
            if (nt[d] >= 0 && nt[d] < lim[d]) {
                nid = (uint32_t)(P.tile_off + (nt[2] * P.nty + nt[1]) * P.ntx + nt[0]);
                w = ld_rlx(S.tstate + nid) | 0x40000000u;
            }
            s_nb[tid] = w;
            s_nid[tid] = nid;
            s_face[tid] = kInfBits;
        }
        if (tid == 0) {
            s_done = 0u;
            s_cnt[0] = 0;
            s_cnt[1] = 0;
            s_more[1] = 0;
            s_more[2] = 0;
        }

        // stage own points and the halo: every load goes out before any is used
        constexpr int NXF = 2 * TY * TZ, NYF = 2 * TX * TZ, NZF = C::D3 ? 2 * TX * TY : 0;
        constexpr int NH = NXF + NYF + NZF;
        constexpr int HPT = (NH + NT - 1) / NT;  // halo cells per thread
        // halo cell i: its LDS index, face and global index (-1 outside the grid)
        auto halo_cell = [&](int i, int& L, int& f) -> int64_t {
            int lx, ly, lz;
            if (i < NXF) {
                int side = i / (TY * TZ), r = i % (TY * TZ);
                ly = r % TY; lz = r / TY; lx = side ? TX : -1; f = side;
            } else if (i < NXF + NYF) {
                int k2 = i - NXF, side = k2 / (TX * TZ), r = k2 % (TX * TZ);
                lx = r % TX; lz = r / TX; ly = side ? TY : -1; f = 2 + side;
            } else {
                int k2 = i - NXF - NYF, side = k2 / (TX * TY), r = k2 % (TX * TY);
                lx = r % TX; ly = r / TX; lz = side ? TZ : -1; f = 4 + side;
            }
            L = C::lds(lx, ly, lz);
            const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
            if (x >= 0 && x < P.nx && y >= 0 && y < P.ny && z >= 0 && z < P.nz)
                return P.pt_off + ((int64_t)z * P.ny + y) * P.nx + x;
            return -1;
        };
        bool was_done[NPT];
        uint32_t live = 0;  // bit j: point j is in the grid, not a source, not yet done
        {
            double tv[NPT], gv[NPT], mv[NPT];
            uint8_t pv[NPT];
            double htv[HPT], hmv[HPT];
            uint8_t hpv[HPT];
            uint32_t inb = 0, seed = 0;
#pragma unroll
            for (int j = 0; j < NPT; ++j) {
                const int p = tid + j * NT;
                const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
                const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
                tv[j] = inf64();
                gv[j] = 0.0;
                mv[j] = qnan64();
                pv[j] = 0x80;  // outside points act as done sources
                if (x < P.nx && y < P.ny && z < P.nz) {
                    const int64_t gi = P.pt_off + ((int64_t)z * P.ny + y) * P.nx + x;
                    tv[j] = A.t[gi];
                    pv[j] = A.par[gi];
                    gv[j] = A.g[gi];
                    mv[j] = as_f64(__hip_atomic_load((const uint64_t*)(A.mu + gi), __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT));
                    inb |= 1u << j;
                }
            }
#pragma unroll
            for (int k = 0; k < HPT; ++k) {
                const int i = tid + k * NT;
                htv[k] = inf64();
                hmv[k] = 0.0;
                hpv[k] = 0x80;  // outside cells act as done sources
                if (i < NH) {
                    int L, f;
                    const int64_t gi = halo_cell(i, L, f);
                    if (gi >= 0) {
                        htv[k] = A.t[gi];
                        hpv[k] = A.par[gi];
                        hmv[k] = as_f64(__hip_atomic_load((const uint64_t*)(A.mu + gi), __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT));
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < NPT; ++j) {
                const int p = tid + j * NT;
                const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
                const int L = C::lds(lx, ly, lz);
                double m = 0.0;
                if ((inb >> j) & 1u) m = (pv[j] & 0x80) ? 0.0 : mv[j];
                sT[L] = tv[j];
                sP[L] = pv[j];
                sM[L] = m;
                sG[p] = (inb >> j) & 1u ? gv[j] : 0.0;
                was_done[j] = !(m != m);
                if (((inb >> j) & 1u) && !(pv[j] & 0x80) && !was_done[j]) live |= 1u << j;
                // first run: every point (leaves can sit anywhere); later runs:
                // only boundary points, since nothing inside changed since the
                // last run and readiness can only come from children across a face
                const bool edge = lx == 0 || lx == TX - 1 || ly == 0 || ly == TY - 1 ||
                                  (C::D3 && (lz == 0 || lz == TZ - 1));
                if (!visited || edge) seed |= 1u << (8 * j);
            }
            st_flags<NPT>(sDirty[0] + tid * NPT, seed);
            st_flags<NPT>(sDirty[1] + tid * NPT, 0u);
#pragma unroll
            for (int k = 0; k < HPT; ++k) {
                const int i = tid + k * NT;
                if (i < NH) {
                    int L, f;
                    (void)halo_cell(i, L, f);
                    sT[L] = htv[k];
                    sP[L] = hpv[k];
                    sM[L] = (hpv[k] & 0x80) ? 0.0 : hmv[k];
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            const unsigned long long now = wall_clock64();
            s_stat[1] += now - s_stat[8];
            s_stat[8] = now;
        }

        // Evaluate points whose children are all done, until no point is left
        // to look at (two pass structures with the same result, as in the
        // forward solver: PACK compacts the dirty points first).
        int cb = 0;
        int passes = 0;
        if constexpr (PACK) {
            // Evaluate points whose children are all done, until no point is left
            // to look at.  As in the forward solver, each pass first compacts the
            // points marked dirty into a list (per-point ballots place them, one
            // LDS atomic per wave reserves the wave's segment), so a lane evaluates
            // at most one point per round instead of walking all its own points.
            // A point that becomes done marks its in-tile parents for the next
            // pass; a point that is not ready yet is marked again by the child
            // that completes it.
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
                    const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
                    const int L = C::lds(lx, ly, lz);
                    // every LDS read of the point and its neighbours goes out at once
                    const uint8_t pn = sP[L];
                    const double mself = sM[L];
                    const double tn = sT[L];
                    uint8_t pm[2 * NAX];
                    double mm[2 * NAX], tm[2 * NAX];
    #pragma unroll
                    for (int k = 0; k < NAX; ++k) {
    #pragma unroll
                        for (int side = 0; side < 2; ++side) {
                            const int Lm = side ? L + LSTEP[k] : L - LSTEP[k];
                            pm[2 * k + side] = sP[Lm];
                            mm[2 * k + side] = sM[Lm];
                            tm[2 * k + side] = sT[Lm];
                        }
                    }
                    if (!(mself != mself)) continue;  // already done
                    bool ready = true;
                    double lam = sG[p];
                    // children in neighbour order x-, x+, y-, y+, z-, z+
    #pragma unroll
                    for (int k = 0; k < NAX; ++k) {
    #pragma unroll
                        for (int side = 0; side < 2; ++side) {
                            const uint8_t pmk = pm[2 * k + side];
                            // the minus-side neighbour is a child if its plus-side parent is n
                            const uint32_t want = side ? 1u : 2u;
                            if (!(pmk & 0x80) && ((pmk >> (2 * k)) & 3u) == want) {
                                const double mmk = mm[2 * k + side];
                                if (mmk != mmk) {
                                    ready = false;
                                } else {
                                    double w = tm[2 * k + side] - tn;
                                    lam = lam + mmk * w;
                                }
                            }
                        }
                    }
                    if (!ready) continue;
                    double wk[3] = {0.0, 0.0, 0.0};
    #pragma unroll
                    for (int k = 0; k < NAX; ++k) {
                        const uint32_t code = (pn >> (2 * k)) & 3u;
                        if (code == 1u) wk[k] = tn - tm[2 * k];
                        else if (code == 2u) wk[k] = tn - tm[2 * k + 1];
                    }
                    double W = wk[0] + wk[1];
                    W = W + wk[2];
                    const double mun = lam / W;
                    sM[L] = mun;
                    // parents inside the tile may now be ready
                    uint8_t* nd = sDirty[cb ^ 1];
    #pragma unroll
                    for (int k = 0; k < NAX; ++k) {
                        const uint32_t code = (pn >> (2 * k)) & 3u;
                        const int c = k == 0 ? lx : (k == 1 ? ly : lz);
                        const int lim = k == 0 ? TX : (k == 1 ? TY : TZ);
                        if (code == 1u && c > 0) nd[didx<NT, NPT>(p - PSTEP[k])] = 1;
                        if (code == 2u && c < lim - 1) nd[didx<NT, NPT>(p + PSTEP[k])] = 1;
                    }
                }
                ++passes;
                __syncthreads();
                cb ^= 1;
                if (passes > (1 << 20)) {
                    if (tid == 0) set_flag(S, kFlagWatchdog);
                    break;
                }
            }
        } else {
            static_assert(PACK || NPT == 1, "the direct form has one point per thread");
            // Direct form: each thread owns one point (NT == NP) and keeps its
            // state in registers; only the neighbours come from LDS.  A pass
            // evaluates each dirty point once and marks the in-tile parents of
            // the points it completed in the other flag buffer, so one barrier
            // per pass orders the marks before the next pass's reads.
            {
                const int p = tid;
                const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
                const int L = C::lds(lx, ly, lz);
                const uint8_t pn = sP[L];
                const double tn = sT[L];
                const double gn = sG[p];
                bool done = was_done[0];
                uint32_t dirty = 0;
                {
                    const uint32_t fl = ld_flags<NPT>(sDirty[0] + tid * NPT);
                    dirty = fl & 1u & live;
                    st_flags<NPT>(sDirty[0] + tid * NPT, 0u);
                }
                for (;;) {
                    if (tid == 0) s_more[(passes + 1) % 3] = 0;  // written next pass; last read two barriers ago
                    bool marked = false;
                    uint8_t* nd = sDirty[cb ^ 1];
                    if (dirty && !done) {
                        uint8_t pm[2 * NAX];
                        double mm[2 * NAX], tm[2 * NAX];
    #pragma unroll
                        for (int k = 0; k < NAX; ++k) {
    #pragma unroll
                            for (int side = 0; side < 2; ++side) {
                                const int Lm = side ? L + LSTEP[k] : L - LSTEP[k];
                                pm[2 * k + side] = sP[Lm];
                                mm[2 * k + side] = sM[Lm];
                                tm[2 * k + side] = sT[Lm];
                            }
                        }
                        bool ready = true;
                        double lam = gn;
                        // children in neighbour order x-, x+, y-, y+, z-, z+
    #pragma unroll
                        for (int k = 0; k < NAX; ++k) {
    #pragma unroll
                            for (int side = 0; side < 2; ++side) {
                                const uint8_t pmk = pm[2 * k + side];
                                // the minus-side neighbour is a child if its plus-side parent is n
                                const uint32_t want = side ? 1u : 2u;
                                if (!(pmk & 0x80) && ((pmk >> (2 * k)) & 3u) == want) {
                                    const double mmk = mm[2 * k + side];
                                    if (mmk != mmk) {
                                        ready = false;
                                    } else {
                                        double w = tm[2 * k + side] - tn;
                                        lam = lam + mmk * w;
                                    }
                                }
                            }
                        }
                        if (ready) {
                            double wk[3] = {0.0, 0.0, 0.0};
    #pragma unroll
                            for (int k = 0; k < NAX; ++k) {
                                const uint32_t code = (pn >> (2 * k)) & 3u;
                                if (code == 1u) wk[k] = tn - tm[2 * k];
                                else if (code == 2u) wk[k] = tn - tm[2 * k + 1];
                            }
                            double W = wk[0] + wk[1];
                            W = W + wk[2];
                            const double mun = lam / W;
                            sM[L] = mun;
                            done = true;
                            // parents inside the tile may now be ready
    #pragma unroll
                            for (int k = 0; k < NAX; ++k) {
                                const uint32_t code = (pn >> (2 * k)) & 3u;
                                const int c = k == 0 ? lx : (k == 1 ? ly : lz);
                                const int lim = k == 0 ? TX : (k == 1 ? TY : TZ);
                                if (code == 1u && c > 0) {
                                    nd[didx<NT, NPT>(p - PSTEP[k])] = 1;
                                    marked = true;
                                }
                                if (code == 2u && c < lim - 1) {
                                    nd[didx<NT, NPT>(p + PSTEP[k])] = 1;
                                    marked = true;
                                }
                            }
                        }
                    }
                    if (__ballot(marked) && lane == 0) s_more[passes % 3] = 1;
                    __syncthreads();
                    const bool more = s_more[passes % 3] != 0;
                    ++passes;
                    if (!more) break;
                    cb ^= 1;
                    {
                        uint8_t* df = sDirty[cb] + tid * NPT;
                        const uint32_t fl = ld_flags<NPT>(df);
                        dirty = fl & 1u & live;
                        if (fl) st_flags<NPT>(df, 0u);
                    }
                    if (passes > (1 << 20)) {
                        if (tid == 0) set_flag(S, kFlagWatchdog);
                        break;
                    }
                }
            }
        }

        if (tid == 0) {
            s_stat[6] += (unsigned long long)passes;
            const unsigned long long now = wall_clock64();
            s_stat[2] += now - s_stat[8];
            s_stat[8] = now;
        }
        // write back newly done points (first visit: every point, NaN = not done)
        unsigned int ndone = 0;
        double fkey[6] = {inf64(), inf64(), inf64(), inf64(), inf64(), inf64()};
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int p = tid + j * NT;
            const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
            const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
            if (!(x < P.nx && y < P.ny && z < P.nz)) continue;
            const int L = C::lds(lx, ly, lz);
            const int64_t gi = P.pt_off + ((int64_t)z * P.ny + y) * P.nx + x;
            const double mv = sM[L];
            const bool done_now = !(mv != mv) && !was_done[j];
            const uint8_t pn = sP[L];
            if (done_now || !visited) {
                __hip_atomic_store((uint64_t*)(A.mu + gi), as_u64(mv), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
            if (done_now && !(pn & 0x80)) {
                ++ndone;
                // a face point whose parent lies across that face unblocks the
                // neighbour; the neighbour is keyed by the parent's own time, the
                // earliest bucket in which that parent can be taken (its other
                // children, later in time, are then mostly done as well)
                if (lx == 0 && ((pn >> 0) & 3u) == 1u) fkey[0] = fmin(fkey[0], tref - sT[L - 1]);
                if (lx == TX - 1 && ((pn >> 0) & 3u) == 2u) fkey[1] = fmin(fkey[1], tref - sT[L + 1]);
                if (ly == 0 && ((pn >> 2) & 3u) == 1u) fkey[2] = fmin(fkey[2], tref - sT[L - C::SY]);
                if (ly == TY - 1 && ((pn >> 2) & 3u) == 2u) fkey[3] = fmin(fkey[3], tref - sT[L + C::SY]);
                if (C::D3) {
                    if (lz == 0 && ((pn >> 4) & 3u) == 1u) fkey[4] = fmin(fkey[4], tref - sT[L - C::SZ]);
                    if (lz == TZ - 1 && ((pn >> 4) & 3u) == 2u) fkey[5] = fmin(fkey[5], tref - sT[L + C::SZ]);
                }
            }
        }
        // reduced within each wave, then one LDS atomic per wave
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            if (__ballot(fkey[f] < inf64())) {
                const double m = wave_min(fkey[f]);
                if (lane == 0) atomicMin(&s_face[f], (unsigned long long)as_u64(fmax(m, 0.0)));
            }
        }
        {
            unsigned int cnt = ndone;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
            if (cnt && lane == 0) atomicAdd(&s_done, cnt);
        }
        stores_done();
        __syncthreads();

        if (tid < 64) {
            const int nxt = publish(S, A.tkey, (uint32_t)tile, s_bucket, !visited, s_nb, s_nid, s_face, true);
            if (tid == 0) s_next = nxt;
        }
        if (tid == 0) {
            s_stat[5] += s_done;
            const unsigned long long now = wall_clock64();
            s_stat[3] += now - s_stat[8];
            s_stat[8] = now;
        }
        __syncthreads();
    }
    if (tid == 0) {
        s_stat[0] += wall_clock64() - s_stat[8];
        for (int i = 0; i < 4; ++i)
            __hip_atomic_fetch_add(S.counters + 5 + i, s_stat[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(S.counters + 2, s_stat[6], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(S.counters + 10, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(S.counters + 0, s_stat[4], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(S.counters + 1, s_stat[5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(S.counters + 12, s_stat[7], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace eik

// Wave-per-tile variant of the persistent solver.
//
// Same schedule and hand-off protocol as k_solve, but every wave (64 lanes) of
// a block claims, stages, relaxes and publishes its own tile independently, so
// a block keeps several tiles in flight and no step waits on a block barrier.
// Within a wave the relaxation is wave-synchronous: LDS operations of one wave
// complete in order, so values and work lists written by one lane are seen by
// the others without a barrier.  Each pass works through a dense list of the
// points to evaluate; a lane whose point dropped appends the in-tile
// neighbours to the next pass's list (deduplicated with a per-point pass mark,
// prefix offsets from ballots), so nothing scans the whole tile per pass.
#pragma once

#include "eik_kernels.hpp"

namespace eik {

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int TX, int TY, int TZ, int NW>
__global__ void __launch_bounds__(64 * NW) k_solve_w(SolveArgs A) {
    using C = TileCfg<TX, TY, TZ, 64>;
    constexpr int NP = C::NP;
    constexpr int NPT = C::NPT;
    __shared__ double sT_[NW][C::NLDS];
    __shared__ double sQ_[NW][NP];
    __shared__ uint16_t sList_[NW][2][NP];
    __shared__ uint32_t sMark_[NW][NP];
    __shared__ uint32_t sNb_[NW][6];
    __shared__ uint32_t sNid_[NW][6];
    __shared__ unsigned long long sFace_[NW][6];

    const int w = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    double* sT = sT_[w];
    double* sQ = sQ_[w];
    uint32_t* sMark = sMark_[w];
    const Sched& S = A.s;
    unsigned long long my_visits = 0, my_updates = 0, my_passes = 0;
    unsigned long long ph[4] = {0, 0, 0, 0};
    unsigned long long tm = wall_clock64();

    for (;;) {
        // ---- claim ------------------------------------------------------
        int64_t bucket = 0;
        const int tile = claim(S, &bucket);
        if (tile < 0) break;
        uint32_t st = 0;
        if (lane == 0) {
            st = __hip_atomic_fetch_xor(S.tstate + tile, kQ | kR, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((st & (kQ | kR)) != kQ) set_flag(S, kFlagWatchdog);
            if (S.max_visits > 0) {
                unsigned long long v = __hip_atomic_fetch_add(S.counters + 3, 1ull, __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT);
                if ((long long)v >= S.max_visits) {
                    set_flag(S, kFlagLimit);
                    st |= 0x80000000u;
                }
            }
        }
        st = __shfl(st, 0);
        ++my_visits;
        {
            const unsigned long long now = wall_clock64();
            ph[0] += now - tm;
            tm = now;
        }
        if (st & 0x80000000u) {
            if (lane == 0) drop_run(S, (uint32_t)tile, bucket);
            continue;
        }
        const bool visited = (st & kV) != 0;
        const Prob P = prob_of_tile(A.pt, tile);
        const int tl = tile - P.tile_off;
        const int tx = tl % P.ntx, ty = (tl / P.ntx) % P.nty, tz = tl / (P.ntx * P.nty);
        const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;

        // neighbour states x-, x+, y-, y+, z-, z+ (lanes 0..5)
        uint32_t nbw = 0;
        if (lane < 6) {
            const int d = lane >> 1, side = lane & 1;
            int nt[3] = {tx, ty, tz};
            const int lim[3] = {P.ntx, P.nty, P.ntz};
            nt[d] += side ? 1 : -1;
            uint32_t nid = 0;
            if (nt[d] >= 0 && nt[d] < lim[d]) {
                nid = (uint32_t)(P.tile_off + (nt[2] * P.nty + nt[1]) * P.ntx + nt[0]);
                nbw = ld_rlx(S.tstate + nid) | 0x40000000u;
            }
            sNb_[w][lane] = nbw;
            sNid_[w][lane] = nid;
            sFace_[w][lane] = kInfBits;
        }
        uint32_t nbv[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) nbv[f] = __shfl(nbw, f);

        // ---- stage -------------------------------------------------------
        double t_in[NPT];
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int p = lane + j * 64;
            const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
            const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
            double tv = inf64(), q = 0.0;
            if (x < P.nx && y < P.ny && z < P.nz) {
                const int64_t gi = P.pt_off + ((int64_t)z * P.ny + y) * P.nx + x;
                bool ok;
                q = field_q(A.field[gi], P.h, P.kind, ok);
                if (!ok) {
                    set_flag(S, kFlagDomain);
                    q = 0.0;
                }
                if (visited) {
                    tv = as_f64(__hip_atomic_load((const uint64_t*)(A.t + gi), __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT));
                    if (signbit(tv)) {
                        tv = fabs(tv);
                        q = 0.0;
                    }
                }
            }
            sT[C::lds(lx, ly, lz)] = tv;
            sQ[p] = q;
            sMark[p] = 0u;
            t_in[j] = tv;
        }
        {
            constexpr int NXF = 2 * TY * TZ, NYF = 2 * TX * TZ, NZF = C::D3 ? 2 * TX * TY : 0;
            for (int i = lane; i < NXF + NYF + NZF; i += 64) {
                int lx, ly, lz, f;
                if (i < NXF) {
                    const int side = i / (TY * TZ), r = i % (TY * TZ);
                    ly = r % TY; lz = r / TY; lx = side ? TX : -1; f = side;
                } else if (i < NXF + NYF) {
                    const int k = i - NXF, side = k / (TX * TZ), r = k % (TX * TZ);
                    lx = r % TX; lz = r / TX; ly = side ? TY : -1; f = 2 + side;
                } else {
                    const int k = i - NXF - NYF, side = k / (TX * TY), r = k % (TX * TY);
                    lx = r % TX; ly = r / TX; lz = side ? TZ : -1; f = 4 + side;
                }
                const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
                double v = inf64();
                if ((nbv[f] & kV) && x >= 0 && x < P.nx && y >= 0 && y < P.ny && z >= 0 && z < P.nz)
                    v = hload(A.t + P.pt_off + ((int64_t)z * P.ny + y) * P.nx + x);
                sT[C::lds(lx, ly, lz)] = v;
            }
        }
        // first work list: every point that can change
        int n = 0;
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int p = lane + j * 64;
            const bool d = sQ[p] > 0.0;
            const unsigned long long m = __ballot(d);
            if (d) sList_[w][0][n + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)p;
            n += (int)__popcll(m);
        }
        wave_sync();
        {
            const unsigned long long now = wall_clock64();
            ph[1] += now - tm;
            tm = now;
        }

        // ---- relax until the tile is quiet --------------------------------
        int cb = 0;
        uint32_t pass = 0;
        while (n > 0) {
            ++pass;
            const uint16_t* cur = sList_[w][cb];
            uint16_t* nxt = sList_[w][cb ^ 1];
            int nn = 0;
            for (int base = 0; base < n; base += 64) {
                const int i = base + lane;
                bool ch = false;
                int p = 0;
                if (i < n) {
                    p = cur[i];
                    const double q = sQ[p];
                    const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
                    const int L = C::lds(lx, ly, lz);
                    const double tc = sT[L];
                    const double ax = fmin(sT[L - 1], sT[L + 1]);
                    const double ay = fmin(sT[L - C::SY], sT[L + C::SY]);
                    const double az = C::D3 ? fmin(sT[L - C::SZ], sT[L + C::SZ]) : inf64();
                    const double r = update<C::D3>(ax, ay, az, q, q * q, tc, ch);
                    if (ch) sT[L] = r;
                }
                // append the in-tile neighbours of lowered points, once each
                const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
#pragma unroll
                for (int d = 0; d < (C::D3 ? 6 : 4); ++d) {
                    bool want = false;
                    int m = 0;
                    if (ch) {
                        const int ax = d >> 1, side = d & 1;
                        const int c = ax == 0 ? lx : (ax == 1 ? ly : lz);
                        const int lim = ax == 0 ? TX : (ax == 1 ? TY : TZ);
                        const int step = ax == 0 ? 1 : (ax == 1 ? TX : TX * TY);
                        if (side ? c < lim - 1 : c > 0) {
                            m = side ? p + step : p - step;
                            want = sQ[m] > 0.0 && atomicExch(&sMark[m], pass) != pass;
                        }
                    }
                    const unsigned long long mk = __ballot(want);
                    if (want) nxt[nn + __popcll(mk & ((1ull << lane) - 1ull))] = (uint16_t)m;
                    nn += (int)__popcll(mk);
                }
            }
            wave_sync();
            n = nn;
            cb ^= 1;
            if (pass > (1u << 20)) {
                if (lane == 0) set_flag(S, kFlagWatchdog);
                break;
            }
        }
        {
            const unsigned long long now = wall_clock64();
            ph[2] += now - tm;
            tm = now;
        }

        // ---- write back lowered points, lowered face minima ----------------
        unsigned int nchg = 0;
        double fm[6] = {inf64(), inf64(), inf64(), inf64(), inf64(), inf64()};
#pragma unroll
        for (int j = 0; j < NPT; ++j) {
            const int p = lane + j * 64;
            const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
            const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
            if (x < P.nx && y < P.ny && z < P.nz) {
                const double v = sT[C::lds(lx, ly, lz)];
                const bool lowered = v < t_in[j];
                if (lowered || !visited) tstore(A.t + P.pt_off + ((int64_t)z * P.ny + y) * P.nx + x, v);
                if (lowered) {
                    ++nchg;
                    if (lx == 0) fm[0] = fmin(fm[0], v);
                    if (lx == TX - 1) fm[1] = fmin(fm[1], v);
                    if (ly == 0) fm[2] = fmin(fm[2], v);
                    if (ly == TY - 1) fm[3] = fmin(fm[3], v);
                    if (C::D3) {
                        if (lz == 0) fm[4] = fmin(fm[4], v);
                        if (lz == TZ - 1) fm[5] = fmin(fm[5], v);
                    }
                }
            }
        }
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            const double mf = wave_min(fm[f]);
            if (lane == f && mf < inf64()) sFace_[w][f] = as_u64(mf);
        }
        {
            // wave sum of lowered points
            unsigned int sum = nchg;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
            my_updates += sum;
        }
        my_passes += pass;
        stores_done();
        wave_sync();
        publish(S, A.tkey, (uint32_t)tile, bucket, !visited, sNb_[w], sNid_[w], sFace_[w]);
        {
            const unsigned long long now = wall_clock64();
            ph[3] += now - tm;
            tm = now;
        }
    }
    if (lane == 0) {
        ph[0] += wall_clock64() - tm;
        for (int i = 0; i < 4; ++i)
            __hip_atomic_fetch_add(S.counters + 5 + i, ph[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(S.counters + 0, my_visits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(S.counters + 1, my_updates, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(S.counters + 2, my_passes, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace eik

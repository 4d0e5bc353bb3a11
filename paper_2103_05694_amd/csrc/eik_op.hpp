// Device-side local update operator for the first-order upwind Eikonal scheme.
//
// Definition (paper: Eq. difference_as_root, Algorithm "Eikonal Update
// Operator", and the rounding semantics of section "Achieving Exact Monotonicity
// with Finite Precision Arithmetic", extended to the one-sided case and to three
// axes):
//   a_k      smaller of the two axis-k neighbour times (+inf off the grid),
//   c        fl(q*q) with q = fl(h/v) or fl(h*s),
//   T_k(r)   fl(d*d) with d = fl(r - a_k) when d > 0, else +0,
//   S(r)     T_k summed largest first (ascending a_k): fl(fl(T0 + T1) + T2),
//   result   the smallest binary64 r >= min_k a_k with S(r) >= c.
// S is non-decreasing in r and non-increasing in each a_k even in floating
// point, so the result is monotone and causal (Theorem 1 applies verbatim).
//
// Evaluation: a closed-form guess in the upwind-shifted variables, then the
// predicate on the integer image of positive doubles (which orders them) at the
// guess and its neighbours, with a serial search as fallback.  The guess only
// changes how much work is needed; the returned value is fixed by the predicate.  Compile with -ffp-contract=off: every operation in the predicate
// is a separately rounded binary64 operation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eik {

constexpr uint64_t kInfBits = 0x7FF0000000000000ull;
constexpr uint64_t kSignBit = 0x8000000000000000ull;

__device__ __forceinline__ double as_f64(uint64_t u) { return __longlong_as_double((long long)u); }
__device__ __forceinline__ uint64_t as_u64(double d) { return (uint64_t)__double_as_longlong(d); }
__device__ __forceinline__ double inf64() { return as_f64(kInfBits); }

// S(r) >= c with a0 <= a1 <= a2 (a1, a2 may be +inf).  T_k is computed as
// fl(m * m) with m = max(d, 0): for d > 0 that is fl(d * d), otherwise m is a
// zero of either sign and the square is +0, so the bits are those of the
// definition (d is never NaN: r is finite and every a_k is finite or +inf).
template <bool D3 = true>
__device__ __forceinline__ bool reaches(double r, double a0, double a1, double a2, double c) {
    const double m0 = fmax(r - a0, 0.0);
    const double m1 = fmax(r - a1, 0.0);
    double s = m0 * m0 + m1 * m1;
    if constexpr (D3) {
        const double m2 = fmax(r - a2, 0.0);
        s = s + m2 * m2;
    }
    return s >= c;
}

// Minimum and maximum of two doubles that are never NaN (arrival times and
// the squared terms: non-negative or +inf).  fmin / fmax would first
// canonicalise both operands for NaN semantics, two extra instructions per
// call on the operator's critical path.
__device__ __forceinline__ double nmin(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double nmax(double a, double b) {
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__device__ __forceinline__ void sort3(double& a0, double& a1, double& a2) {
    double lo = nmin(a0, a1), hi = nmax(a0, a1);
    double m = nmin(hi, a2);
    a2 = nmax(hi, a2);
    a0 = nmin(lo, m);
    a1 = nmax(lo, m);
}

// Square root for the estimate below: the hardware reciprocal square root
// refined by one coupled Newton step and one residual correction (about one
// ulp).  Not correctly rounded, and NaN for x == 0: the estimate only steers
// the exact search, which handles any starting point.
__device__ __forceinline__ double est_sqrt(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, hh = 0.5 * y;
    const double e = fma(-g, hh, 0.5);
    g = fma(g, e, g);
    hh = fma(hh, e, hh);
    const double d = fma(-g, g, x);
    return fma(d, hh, g);
}

// Closed-form Godunov estimate from sorted minima (u = r - a0 solves the one-,
// two- or three-term quadratic), without branches; the regime test picks the
// radicand so one square root serves both multi-term cases, and infinities
// select the right candidate (fmax drops NaN).  Accuracy only affects how
// often the exact search below needs its fallback.
template <bool D3 = true>
__device__ __forceinline__ double guess(double a0, double a1, double a2, double q, double c) {
    const double r1 = a0 + q;
    const double b1 = a1 - a0;
    const double b2 = a2 - a0;
    const double e2 = a2 - a1;
    // the answer lies at or below a2 iff S(a2) >= c (always when a2 = +inf):
    // then the two-term root, else the three-term one; one square root
    const bool two = !D3 || !(b2 < inf64()) || b2 * b2 + e2 * e2 >= c;
    const double sb = b1 + b2;
    const double d2 = fmax(c + c - b1 * b1, 0.0);
    const double d3 = fmax(sb * sb - 3.0 * (b1 * b1 + b2 * b2 - c), 0.0);
    const double sq = est_sqrt(two ? d2 : d3);
    const double r = two ? a0 + 0.5 * (b1 + sq) : a0 + (sb + sq) * (1.0 / 3.0);
    return r1 <= a1 ? r1 : r;
}

// Serial search kept for the rare inputs whose guess is more than one ulp off:
// unit steps from G, then bisection (reaches(L) false, reaches(H) true).
__device__ __noinline__ double search_slow(double a0, double a1, double a2, double c, uint64_t A0,
                                           uint64_t G, uint64_t tcb) {
    uint64_t L, H;
    bool ok = false;
    if (reaches(as_f64(G), a0, a1, a2, c)) {
        H = G;
        for (int i = 0; i < 4; ++i) {
            uint64_t P = H - 1;
            if (P == A0 || !reaches(as_f64(P), a0, a1, a2, c)) { ok = true; break; }
            H = P;
        }
        L = A0;
    } else {
        L = G;
        H = tcb - 1;
        for (int i = 0; i < 4; ++i) {
            uint64_t N = L + 1;
            if (reaches(as_f64(N), a0, a1, a2, c)) { H = N; ok = true; break; }
            L = N;
        }
    }
    if (!ok) {
        while (H - L > 1) {
            uint64_t M = L + ((H - L) >> 1);
            if (reaches(as_f64(M), a0, a1, a2, c)) H = M; else L = M;
        }
    }
    return as_f64(H);
}

// The exact operator.  Returns the new value if it is < tcur, else tcur.
// Preconditions: q > 0, c = fl(q*q) in (0, inf), tcur >= 0 (may be +inf).
// `x`, `y`, `z` are the axis minima in any order (+inf where absent).
//
// The predicate is evaluated at G-1, G, G+1 around the guess G as three
// independent chains; the answer is G or G+1 when it is the first of them
// that satisfies it while the one below does not, and comparing it with tcur
// decides whether the point improves (first r < tcur <=> S(prev(tcur)) >= c,
// since S is monotone, which is evaluated only when the window lies wholly
// below the answer).  (Measured over whole solves, the guess is never more than one
// ulp below the answer and never above it, so this window decides every
// case; the serial search covers the rest.)  G is clamped to
// [A0 + 2, prev(tcur)], so G - 1 > A0.
//
// D3 = false (two-dimensional grids, z = +inf) drops the third term: it is +0
// there, and adding +0 to a sum of squares (itself >= +0) changes no bit.
template <bool D3 = true>
__device__ __forceinline__ double update(double x, double y, double z, double q, double c,
                                         double tcur, bool& changed) {
    changed = false;
    double a0, a1, a2;
    if constexpr (D3) {
        a0 = x;
        a1 = y;
        a2 = z;
        sort3(a0, a1, a2);
    } else {
        a0 = nmin(x, y);
        a1 = nmax(x, y);
        a2 = inf64();
    }
    const uint64_t tcb = as_u64(tcur);
    const uint64_t A0 = as_u64(a0);
    uint64_t G = as_u64(guess<D3>(a0, a1, a2, q, c));
    if (!(G >= A0 + 2)) G = A0 + 2;                // also catches a NaN pattern
    if (G > tcb - 1) G = tcb - 1;
    // S is non-decreasing in r, so the three outcomes are false...false
    // true...true and their count locates the answer: 2 -> G, 1 -> G+1;
    // 3 (the answer is below G) or 0 (above G+1) need the search.  The
    // chains are written side by side so that they interleave.
    double r[3], m0[3], m1[3], m2[3], sm[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) r[k] = as_f64(G - 1 + (uint64_t)k);
#pragma unroll
    for (int k = 0; k < 3; ++k) m0[k] = fmax(r[k] - a0, 0.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) m1[k] = fmax(r[k] - a1, 0.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) sm[k] = m0[k] * m0[k] + m1[k] * m1[k];
    if constexpr (D3) {
#pragma unroll
        for (int k = 0; k < 3; ++k) m2[k] = fmax(r[k] - a2, 0.0);
#pragma unroll
        for (int k = 0; k < 3; ++k) sm[k] = sm[k] + m2[k] * m2[k];
    }
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) cnt += sm[k] >= c ? 1 : 0;
    // Nothing lies below tcur when a0 >= tcur (the answer exceeds a0).
    // Otherwise the window decides whether the answer is below tcur: with
    // cnt 1 or 2 it is G + 2 - cnt itself; with 3 it is below G - 1 <= prev(tcur);
    // with 0 it is above G + 1, so below tcur only if G + 1 < prev(tcur) and
    // S(prev(tcur)) >= c -- then the search runs between G and prev(tcur).
    if (!(a0 < tcur)) return tcur;
    if (cnt == 1 || cnt == 2) {
        const uint64_t ans = G + 2 - (uint64_t)cnt;
        changed = ans < tcb;
        return changed ? as_f64(ans) : tcur;
    }
    if (cnt == 0 && !(G + 1 < tcb - 1 && reaches<D3>(as_f64(tcb - 1), a0, a1, a2, c))) return tcur;
    changed = true;
    return search_slow(a0, a1, a2, c, A0, G, tcb);
}

// ---------------------------------------------------------------------------
// rectilinear grids: spacing varying per axis and index
// ---------------------------------------------------------------------------
// Per axis k the two neighbours am, ap and the reciprocal spacings wm, wp to
// them (w = fl(1 / fl(x_i - x_{i-1})) and likewise on the plus side):
//   m_k(r) = max(fl(fl(r - am) * wm), fl(fl(r - ap) * wp)),
//   T_k(r) = fl(m_k * m_k) when m_k > 0, else +0,
//   S(r)   = the T_k summed largest first: fl(fl(T_hi + T_mid) + T_lo),
//   result = the smallest binary64 r >= min_k a_k with S(r) >= c,
// c = fl(s * s) for the slowness s.  Each T_k is monotone in r and
// anti-monotone in its neighbours, and the largest-first sum is symmetric and
// monotone in each term, so the result is monotone and causal (the
// construction of section "Achieving Exact Monotonicity with Finite Precision
// Arithmetic" applied to the irregular-grid scheme).  The order of the
// neighbour values would not do here: with unequal weights it is not the
// order of the terms, and a swap can move the sum the wrong way.  With unit
// spacing the largest term is that of the smallest neighbour and the operator
// is the uniform one bit for bit.

struct RAxis {
    double am, ap, wm, wp;  // the two neighbours and the reciprocal spacings to them
};

__device__ __forceinline__ double rterm(double r, const RAxis& k) {
    const double d1 = (r - k.am) * k.wm;
    const double d2 = (r - k.ap) * k.wp;
    const double m = nmax(d1, d2);
    return m > 0.0 ? m * m : 0.0;
}

// The predicate is symmetric in the axes, so they come in grid order.
template <bool D3>
__device__ __forceinline__ bool reaches_rect(double r, const RAxis& x0, const RAxis& x1, const RAxis& x2, double c) {
    const double t0 = rterm(r, x0), t1 = rterm(r, x1);
    if constexpr (D3) {
        // the terms are >= +0 and never NaN; the smallest goes last
        const double t2 = rterm(r, x2);
        const double lo01 = nmin(t0, t1), hi01 = nmax(t0, t1);
        const double lo = nmin(lo01, t2);
        const double mid = nmax(lo01, t2);
        return (hi01 + mid) + lo >= c;
    } else {
        return t0 + t1 >= c;
    }
}

// Search for the rare inputs whose guess misses the window: steps of doubling
// size from G until the predicate flips, then bisection between the last two
// points (reaches(L) false, reaches(H) true; reaches(A0) is false since
// c > 0, and reaches(tcb - 1) is true when called).
template <bool D3>
__device__ __noinline__ double search_slow_rect(const RAxis x0, const RAxis x1, const RAxis x2, double c,
                                                uint64_t A0, uint64_t G, uint64_t tcb) {
    uint64_t L, H;
    if (reaches_rect<D3>(as_f64(G), x0, x1, x2, c)) {
        H = G;
        L = A0;
        for (uint64_t step = 1; H - A0 > step; step <<= 1) {
            const uint64_t P = H - step;
            if (!reaches_rect<D3>(as_f64(P), x0, x1, x2, c)) { L = P; break; }
            H = P;
        }
    } else {
        L = G;
        H = tcb - 1;
        for (uint64_t step = 1; tcb - 1 - L > step; step <<= 1) {
            const uint64_t N = L + step;
            if (reaches_rect<D3>(as_f64(N), x0, x1, x2, c)) { H = N; break; }
            L = N;
        }
    }
    while (H - L > 1) {
        const uint64_t M = L + ((H - L) >> 1);
        if (reaches_rect<D3>(as_f64(M), x0, x1, x2, c)) H = M; else L = M;
    }
    return as_f64(H);
}

// (a, w) pairs in ascending a: the guess adds axes in that order
__device__ __forceinline__ void pswap(double& a0, double& w0, double& a1, double& w1) {
    const bool s = a1 < a0;
    const double la = s ? a1 : a0, lw = s ? w1 : w0, ha = s ? a0 : a1, hw = s ? w0 : w1;
    a0 = la;
    w0 = lw;
    a1 = ha;
    w1 = hw;
}

// The rectilinear operator; returns the new value if it is < tcur, else tcur.
// n[6] = neighbours x-, x+, y-, y+, z-, z+ (+inf off the grid), w[6] the
// reciprocal spacings to them, c = fl(q * q).  The guess is the real root of
// sum_k w_k^2 (r - a_k)^2 = c over the upwind axes, each with the weight of
// its smaller neighbour, solved for u = r - a0 with b_k = a_k - a0 (the
// unshifted quadratic cancels badly when the a_k are close relative to their
// size); the predicate at G-1, G, G+1 decides as for d-bar.
template <bool D3 = true>
__device__ __forceinline__ double update_rect(const double* n, const double* w, double c, double tcur,
                                              bool& changed) {
    changed = false;
    const RAxis X{n[0], n[1], w[0], w[1]};
    const RAxis Y{n[2], n[3], w[2], w[3]};
    const RAxis Z = D3 ? RAxis{n[4], n[5], w[4], w[5]} : RAxis{inf64(), inf64(), 1.0, 1.0};
    double s0 = nmin(n[0], n[1]), v0 = n[0] <= n[1] ? w[0] : w[1];
    double s1 = nmin(n[2], n[3]), v1 = n[2] <= n[3] ? w[2] : w[3];
    double s2 = inf64(), v2 = 1.0;
    if constexpr (D3) {
        s2 = nmin(n[4], n[5]);
        v2 = n[4] <= n[5] ? w[4] : w[5];
    }
    pswap(s0, v0, s1, v1);
    if constexpr (D3) {
        pswap(s1, v1, s2, v2);
        pswap(s0, v0, s1, v1);
    }
    const double a0 = s0;
    const uint64_t tcb = as_u64(tcur);
    // guess: add axes while the root lies above the next minimum
    double A = 0.0, B = 0.0, C = -c, u = inf64();
    bool go = true;
#pragma unroll
    for (int j = 0; j < (D3 ? 3 : 2); ++j) {
        const double ak = j == 0 ? s0 : (j == 1 ? s1 : s2);
        const double wk = j == 0 ? v0 : (j == 1 ? v1 : v2);
        const double nxt = (j == 0 ? s1 : (j == 1 ? s2 : inf64())) - a0;
        if (go && ak < inf64()) {
            const double b = ak - a0;
            const double w2 = wk * wk;
            A = A + w2;
            B = B + w2 * b;
            C = C + (w2 * b) * b;
            const double disc = B * B - A * C;
            u = (B + __builtin_sqrt(fmax(disc, 0.0))) / A;
            go = u > nxt;
        }
    }
    const double g = a0 + u;
    const uint64_t A0 = as_u64(a0);
    uint64_t G = as_u64(g);
    if (!(G >= A0 + 2)) G = A0 + 2;
    if (G > tcb - 1) G = tcb - 1;
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) cnt += reaches_rect<D3>(as_f64(G - 1 + (uint64_t)k), X, Y, Z, c) ? 1 : 0;
    // as for d-bar: the window decides, prev(tcur) is tested only when the
    // answer lies above the window
    if (!(a0 < tcur)) return tcur;
    if (cnt == 1 || cnt == 2) {
        const uint64_t ans = G + 2 - (uint64_t)cnt;
        changed = ans < tcb;
        return changed ? as_f64(ans) : tcur;
    }
    if (cnt == 0 && !(G + 1 < tcb - 1 && reaches_rect<D3>(as_f64(tcb - 1), X, Y, Z, c))) return tcur;
    changed = true;
    return search_slow_rect<D3>(X, Y, Z, c, A0, G, tcb);
}

// The paper's two explicit two-dimensional formulas (the d-tilde and d-hat
// columns of Tables "tab:prec_1" and "tab:prec_2"), kept for the precision
// ablation: they are not monotone in floating point, so an asynchronous solve
// with them can end in different states for different schedules.  tH, tV are
// the x- and y-axis minima; q = h/v, c = fl(q*q).
//   d-tilde: 1/2 (s + sqrt(s^2 - 2 (tH^2 + tV^2 - c))), s = tH + tV;
//   d-hat:   1/2 ((tH + tV) + sqrt(2c - (tH - tV)^2));
// both fall back to min(tH, tV) + q when |tH - tV| >= q.
__device__ __forceinline__ double op_dtilde(double tH, double tV, double q, double c) {
    if (!(tH < inf64()) && !(tV < inf64())) return inf64();
    if (fabs(tH - tV) >= q) return (tH < tV ? tH : tV) + q;
    const double s = tH + tV;
    const double inner = s * s - 2.0 * ((tH * tH + tV * tV) - c);
    return 0.5 * (s + __builtin_sqrt(inner));
}
__device__ __forceinline__ double op_dhat(double tH, double tV, double q, double c) {
    if (!(tH < inf64()) && !(tV < inf64())) return inf64();
    if (fabs(tH - tV) >= q) return (tH < tV ? tH : tV) + q;
    const double d = tH - tV;
    const double inner = 2.0 * c - d * d;
    return 0.5 * ((tH + tV) + __builtin_sqrt(inner));
}

// The precision section's practical variant: Newton's method on
// alpha(t) = (t - tH)^2 + (t - tV)^2 - c from the d-hat guess, on the
// two-sided branch.  Each step: e0 = t - tH, e1 = t - tV,
// a = fl(fl(e0^2) + fl(e1^2)) - c, da = 2 (e0 + e1), t' = t - a / da, all
// separately rounded; it stops when t' == t, da == 0, or after 8 steps.
__device__ __forceinline__ double op_newton(double tH, double tV, double q, double c) {
    if (!(tH < inf64()) && !(tV < inf64())) return inf64();
    if (fabs(tH - tV) >= q) return (tH < tV ? tH : tV) + q;
    double t = op_dhat(tH, tV, q, c);
    for (int k = 0; k < 8; ++k) {
        const double e0 = t - tH, e1 = t - tV;
        const double a = (e0 * e0 + e1 * e1) - c;
        const double da = 2.0 * (e0 + e1);
        if (da == 0.0) break;
        const double tn = t - a / da;
        if (tn == t) break;
        t = tn;
    }
    return t;
}

// Operator selector: 0 exact monotone d-bar (the solver's operator), 1 d-hat,
// 2 d-tilde, 3 Newton.  Returns the value the operator gives from the axis
// minima.
template <int OP>
__device__ __forceinline__ double apply_op(double ax, double ay, double az, double q) {
    const double c = q * q;
    if constexpr (OP == 1) return op_dhat(ax, ay, q, c);
    else if constexpr (OP == 2) return op_dtilde(ax, ay, q, c);
    else if constexpr (OP == 3) return op_newton(ax, ay, q, c);
    else {
        bool ch;
        return update(ax, ay, az, q, c, inf64(), ch);
    }
}

}  // namespace eik

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
// Evaluation: a closed-form guess in the upwind-shifted variables, then exact
// one-ulp steps of the predicate on the integer image of positive doubles (which
// orders them), with a bisection fallback.  The guess only changes how many
// predicate evaluations are needed; the returned value is fixed by the
// predicate.  Compile with -ffp-contract=off: every operation in the predicate
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

// S(r) >= c with a0 <= a1 <= a2 (a1, a2 may be +inf).
__device__ __forceinline__ bool reaches(double r, double a0, double a1, double a2, double c) {
    double d0 = r - a0;
    double d1 = r - a1;
    double d2 = r - a2;
    double s0 = d0 > 0.0 ? d0 * d0 : 0.0;
    double s1 = d1 > 0.0 ? d1 * d1 : 0.0;
    double s2 = d2 > 0.0 ? d2 * d2 : 0.0;
    double s = s0 + s1;
    s = s + s2;
    return s >= c;
}

__device__ __forceinline__ void sort3(double& a0, double& a1, double& a2) {
    double lo = fmin(a0, a1), hi = fmax(a0, a1);
    double m = fmin(hi, a2);
    a2 = fmax(hi, a2);
    a0 = fmin(lo, m);
    a1 = fmax(lo, m);
}

// Closed-form Godunov estimate from sorted minima (u = r - a0 solves the one-,
// two- or three-term quadratic).  Accuracy only affects the step count below.
__device__ __forceinline__ double guess(double a0, double a1, double a2, double q, double c) {
    double r = a0 + q;
    if (r > a1) {
        double b1 = a1 - a0;
        double disc = fmax(c + c - b1 * b1, 0.0);
        r = a0 + 0.5 * (b1 + __builtin_sqrt(disc));
        if (r > a2) {
            double b2 = a2 - a0;
            double sb = b1 + b2;
            double disc3 = fmax(sb * sb - 3.0 * (b1 * b1 + b2 * b2 - c), 0.0);
            r = a0 + (sb + __builtin_sqrt(disc3)) * (1.0 / 3.0);
        }
    }
    return r;
}

// The exact operator.  Returns the new value if it is < tcur, else tcur.
// Preconditions: q > 0, c = fl(q*q) in (0, inf), tcur >= 0 (may be +inf).
// `x`, `y`, `z` are the axis minima in any order (+inf where absent).
__device__ __forceinline__ double update(double x, double y, double z, double q, double c,
                                         double tcur, bool& changed) {
    changed = false;
    double a0 = x, a1 = y, a2 = z;
    sort3(a0, a1, a2);
    if (!(a0 < tcur)) return tcur;                 // result > a0 >= tcur: nothing to do
    // r < tcur  <=>  S(prev(tcur)) >= c  (S is monotone): one predicate
    // evaluation rejects every non-improving ("empty") update.
    const uint64_t tcb = as_u64(tcur);
    if (!reaches(as_f64(tcb - 1), a0, a1, a2, c)) return tcur;

    const uint64_t A0 = as_u64(a0);                // reaches(a0) is false (all d <= 0)
    double g = guess(a0, a1, a2, q, c);
    uint64_t G = as_u64(g);
    if (!(g > a0)) G = A0 + 1;
    if (G >= tcb) G = tcb - 1;                      // reaches(tcb - 1) holds
    uint64_t L, H;
    bool ok = false;
    if (reaches(as_f64(G), a0, a1, a2, c)) {
        H = G;
        // walk down while the predecessor still satisfies the predicate
#pragma unroll 1
        for (int i = 0; i < 4; ++i) {
            uint64_t P = H - 1;
            if (P == A0 || !reaches(as_f64(P), a0, a1, a2, c)) { ok = true; break; }
            H = P;
        }
        L = A0;
    } else {
        L = G;
        H = tcb - 1;
#pragma unroll 1
        for (int i = 0; i < 4; ++i) {
            uint64_t N = L + 1;
            if (reaches(as_f64(N), a0, a1, a2, c)) { H = N; ok = true; break; }
            L = N;
        }
    }
    if (!ok) {
        // Bisection keeps reaches(L) false and reaches(H) true.
#pragma unroll 1
        while (H - L > 1) {
            uint64_t M = L + ((H - L) >> 1);
            if (reaches(as_f64(M), a0, a1, a2, c)) H = M; else L = M;
        }
    }
    changed = true;
    return as_f64(H);
}

}  // namespace eik

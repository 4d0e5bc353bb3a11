/*
 * CPU oracle for the first-order upwind Eikonal solve and its adjoint.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or call
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg use it.  It shares no code with the HIP path.
 *
 * Everything is plain, sequential binary64 arithmetic.  Build it with
 * `-O2 -ffp-contract=off` and no fast-math: the operator is defined by
 * separately rounded subtract / multiply / add, so no contraction to FMA is
 * allowed anywhere.
 *
 * Grid layout: C-order [nz][ny][nx], x fastest; 2D grids have nz == 1.
 *
 * Operator (the paper's "true monotonicity" rounding, section "Achieving Exact
 * Monotonicity with Finite Precision Arithmetic", extended to the one-sided
 * case and to 3D):
 *   a_k   = min of the two axis-k neighbours of the point (+inf off the grid),
 *   q     = fl(h / v)  (speed field) or fl(h * s) (slowness field),
 *   c     = fl(q * q),
 *   T_k(r)= fl(d * d) with d = fl(r - a_k) when d > 0, else +0,
 *   S(r)  = the T_k summed largest-first, i.e. in ascending order of a_k:
 *           fl(fl(T_(0) + T_(1)) + T_(2)),
 *   dbar  = the smallest binary64 r >= min_k a_k with S(r) >= c.
 * S(r) >= c is the sign test of the paper's root function alpha evaluated in
 * floating point; S is non-decreasing in r and non-increasing in every a_k, so
 * dbar is monotone and causal in floating point (Theorem 1 then gives one fixed
 * point for every schedule).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_SPEED 0
#define ORC_SLOWNESS 1

#define OP_DBAR 0   /* exact monotone rounding */
#define OP_DHAT 1   /* reordered explicit formula (2D only) */
#define OP_DTILDE 2 /* textbook explicit formula (2D only) */
#define OP_NEWTON 3 /* Newton on the root function from the d-hat guess (2D only) */
#define OP_RECT 4   /* exact monotone rounding on a rectilinear grid (see below) */

static uint64_t bits_of(double x) { uint64_t u; memcpy(&u, &x, 8); return u; }
static double double_of(uint64_t u) { double x; memcpy(&x, &u, 8); return x; }

/* ------------------------------------------------------------------------- */
/* the operator                                                               */
/* ------------------------------------------------------------------------- */

static void sort3(double a[3]) {
    double t;
    if (a[1] < a[0]) { t = a[0]; a[0] = a[1]; a[1] = t; }
    if (a[2] < a[1]) { t = a[1]; a[1] = a[2]; a[2] = t; }
    if (a[1] < a[0]) { t = a[0]; a[0] = a[1]; a[1] = t; }
}

/* S(r) >= c for neighbour minima already sorted ascending. */
static int reaches(double r, const double as[3], double c) {
    double T[3];
    for (int k = 0; k < 3; ++k) {
        double d = r - as[k];
        T[k] = (d > 0.0) ? d * d : 0.0;
    }
    double s = T[0] + T[1];
    s = s + T[2];
    return s >= c;
}

/* Any starting point for the search: the exact-arithmetic Godunov solution,
 * trying one, two, then three upwind axes.  Its accuracy affects only how many
 * predicate evaluations the search below needs, never its result. */
static double textbook_guess(const double as[3], double c) {
    double q = sqrt(c);
    double g = as[0] + q;
    if (g <= as[1]) return g;
    double b1 = as[1] - as[0];
    double disc = 2.0 * c - b1 * b1;
    g = as[0] + 0.5 * (b1 + sqrt(disc > 0.0 ? disc : 0.0));
    if (g <= as[2]) return g;
    double b2 = as[2] - as[0];
    double sb = b1 + b2;
    disc = sb * sb - 3.0 * (b1 * b1 + b2 * b2 - c);
    g = as[0] + (sb + sqrt(disc > 0.0 ? disc : 0.0)) / 3.0;
    return g;
}

/* dbar: smallest r >= a_min with S(r) >= c.  Found by an exponential search
 * from a guess on the integer image of positive doubles (which orders them),
 * then bisection; the invariant reaches(L) == 0, reaches(H) == 1 makes the
 * result the smallest such r whatever the guess was. */
double orc_dbar(const double a_in[3], double c) {
    double as[3] = {a_in[0], a_in[1], a_in[2]};
    sort3(as);
    if (!(as[0] < INFINITY)) return INFINITY;
    const uint64_t A0 = bits_of(as[0]);             /* reaches(a_min) == 0 */
    const uint64_t INF = bits_of(INFINITY);         /* reaches(+inf) == 1  */
    double g = textbook_guess(as, c);
    uint64_t G;
    if (!(g > as[0])) G = A0 + 1;
    else if (!(g < INFINITY)) G = INF;
    else G = bits_of(g);
    uint64_t L, H;
    if (reaches(double_of(G), as, c)) {
        H = G;
        uint64_t step = 1;
        for (;;) {
            L = (H - A0 > step) ? G - step : A0;
            if (L == A0 || !reaches(double_of(L), as, c)) break;
            H = L;
            step <<= 1;
        }
    } else {
        L = G;
        uint64_t step = 1;
        for (;;) {
            H = (INF - G > step) ? G + step : INF;
            if (H == INF || reaches(double_of(H), as, c)) break;
            L = H;
            step <<= 1;
        }
    }
    while (H - L > 1) {
        uint64_t M = L + (H - L) / 2;
        if (reaches(double_of(M), as, c)) H = M; else L = M;
    }
    return double_of(H);
}

/* Exported single predicate evaluation, for tests. */
int orc_reaches(double r, const double a_in[3], double c) {
    double as[3] = {a_in[0], a_in[1], a_in[2]};
    sort3(as);
    return reaches(r, as, c);
}

/* ------------------------------------------------------------------------- */
/* the operator on a rectilinear grid                                         */
/* ------------------------------------------------------------------------- */

/* A rectilinear grid has strictly increasing coordinates x_i, y_j, z_k per
 * axis, so the spacing differs between points and between the two sides of a
 * point.  The first-order upwind scheme then compares, per axis, the two
 * one-sided differences (t - t_minus)/h_minus and (t - t_plus)/h_plus and
 * keeps the larger positive one (the Godunov choice); their squares sum to
 * the squared slowness.  Following the construction of the section "Achieving
 * Exact Monotonicity with Finite Precision Arithmetic" -- the result is the
 * smallest float satisfying a predicate that is monotone in floating point --
 * with w = fl(1 / fl(x_i - x_{i-1})) (and likewise on the plus side):
 *   m_k(r) = max(fl(fl(r - am_k) * wm_k), fl(fl(r - ap_k) * wp_k)),
 *   T_k(r) = fl(m_k * m_k) when m_k > 0, else +0,
 *   S(r)   = the T_k summed largest first: fl(fl(T_hi + T_mid) + T_lo),
 *   c      = fl(s * s), s the slowness (fl(1 / v) for a speed field),
 *   result = the smallest binary64 r >= min_k a_k with S(r) >= c.
 * Each T_k is monotone in r and anti-monotone in its neighbour values.  The
 * largest-first sum is a symmetric function of the three terms that is
 * monotone in each of them (within one ordering of the terms it is a chain of
 * rounded additions; where two terms are equal both orderings give the same
 * bits), so S is monotone in r and anti-monotone in every neighbour, and the
 * result is monotone and causal: Theorem 1 applies.  (Ordering the terms by
 * their neighbour values instead, as the uniform operator may, is not
 * monotone here: with unequal weights that order is not the order of the
 * terms, and a one-ulp change of a neighbour that swaps it can move the sum
 * the wrong way.)  With unit spacing, m_k = fl(r - a_k), the largest term is
 * that of the smallest a_k, and the definition is the uniform one with h = 1
 * bit for bit; with any power-of-two spacing it is the uniform one scaled
 * exactly. */

typedef struct {
    const double *wm[3], *wp[3];   /* per axis and index: 1 / spacing to the minus / plus side */
} rect_t;

static const rect_t *g_rect = NULL;  /* set only while a rectilinear entry point runs */

static double rect_term(double r, double am, double ap, double wm, double wp) {
    double d1 = (r - am) * wm;
    double d2 = (r - ap) * wp;
    double m = d1 > d2 ? d1 : d2;
    return m > 0.0 ? m * m : 0.0;
}

/* axes in ascending order of a_k (ties: axis order), for the guess */
static void rect_order(const double a[3], int ord[3]) {
    ord[0] = 0; ord[1] = 1; ord[2] = 2;
    for (int i = 1; i < 3; ++i)
        for (int j = i; j > 0 && a[ord[j]] < a[ord[j - 1]]; --j) {
            int t = ord[j]; ord[j] = ord[j - 1]; ord[j - 1] = t;
        }
}

static int reaches_rect(double r, const double am[3], const double ap[3], const double wm[3],
                        const double wp[3], double c) {
    double T[3];
    for (int k = 0; k < 3; ++k) T[k] = rect_term(r, am[k], ap[k], wm[k], wp[k]);
    /* largest first: put the smallest term last */
    int lo = 0;
    for (int k = 1; k < 3; ++k)
        if (T[k] < T[lo]) lo = k;
    const double p = T[(lo + 1) % 3], q = T[(lo + 2) % 3];
    double s = p + q;
    s = s + T[lo];
    return s >= c;
}

/* The rectilinear d-bar.  Axes absent from the grid have am = ap = +inf.
 * Found like orc_dbar: a guess (the real-arithmetic root with each axis
 * using the weight of its smaller neighbour), exponential search and
 * bisection on the integer image; the invariant reaches(L) == 0,
 * reaches(H) == 1 fixes the result whatever the guess. */
double orc_dbar_rect(const double am[3], const double ap[3], const double wm[3], const double wp[3],
                     double c) {
    double a[3], w[3];
    for (int k = 0; k < 3; ++k) {
        a[k] = am[k] <= ap[k] ? am[k] : ap[k];
        w[k] = am[k] <= ap[k] ? wm[k] : wp[k];
    }
    int ord[3];
    rect_order(a, ord);
    const double amin = a[ord[0]];
    if (!(amin < INFINITY)) return INFINITY;
    double A = 0.0, B = 0.0, C = -c, g = INFINITY;
    for (int j = 0; j < 3; ++j) {
        int k = ord[j];
        if (!(a[k] < INFINITY)) break;
        double w2 = w[k] * w[k];
        A += w2;
        B += w2 * a[k];
        C += w2 * a[k] * a[k];
        double disc = B * B - A * C;
        g = (B + sqrt(disc > 0.0 ? disc : 0.0)) / A;
        if (j == 2 || !(g > a[ord[j + 1]])) break;
    }
    const uint64_t A0 = bits_of(amin);
    const uint64_t INF = bits_of(INFINITY);
    uint64_t G;
    if (!(g > amin)) G = A0 + 1;
    else if (!(g < INFINITY)) G = INF;
    else G = bits_of(g);
    uint64_t L, H;
    if (reaches_rect(double_of(G), am, ap, wm, wp, c)) {
        H = G;
        uint64_t step = 1;
        for (;;) {
            L = (H - A0 > step) ? G - step : A0;
            if (L == A0 || !reaches_rect(double_of(L), am, ap, wm, wp, c)) break;
            H = L;
            step <<= 1;
        }
    } else {
        L = G;
        uint64_t step = 1;
        for (;;) {
            H = (INF - G > step) ? G + step : INF;
            if (H == INF || reaches_rect(double_of(H), am, ap, wm, wp, c)) break;
            L = H;
            step <<= 1;
        }
    }
    while (H - L > 1) {
        uint64_t M = L + (H - L) / 2;
        if (reaches_rect(double_of(M), am, ap, wm, wp, c)) H = M; else L = M;
    }
    return double_of(H);
}

/* Exported single predicate evaluation, for tests. */
int orc_reaches_rect(double r, const double am[3], const double ap[3], const double wm[3],
                     const double wp[3], double c) {
    return reaches_rect(r, am, ap, wm, wp, c);
}

/* The two explicit 2D formulas the paper analyses, with q = fl(h/v), c = fl(q*q).
 * Two-sided branch when |tH - tV| < q, else min(tH, tV) + q. */
double orc_dtilde(double tH, double tV, double c, double q) {
    if (fabs(tH - tV) >= q) return (tH < tV ? tH : tV) + q;
    double s = tH + tV;
    double inner = s * s - 2.0 * ((tH * tH + tV * tV) - c);
    return 0.5 * (s + sqrt(inner));
}

double orc_dhat(double tH, double tV, double c, double q) {
    if (fabs(tH - tV) >= q) return (tH < tV ? tH : tV) + q;
    double d = tH - tV;
    double inner = 2.0 * c - d * d;
    return 0.5 * ((tH + tV) + sqrt(inner));
}

/* ------------------------------------------------------------------------- */
/* grid helpers                                                               */
/* ------------------------------------------------------------------------- */

typedef struct {
    int ndim;
    int64_t nx, ny, nz, n;
    double h;
} grid_t;

static grid_t mkgrid(int ndim, int64_t nx, int64_t ny, int64_t nz, double h) {
    grid_t g = {ndim, nx, ny, nz, nx * ny * nz, h};
    return g;
}

/* Per-point constant q (speed: h/v, slowness: h*s).  Returns -1 when a field
 * value is not a positive finite number or c = q*q is not in (0, inf). */
static int make_q(const grid_t *g, const double *field, int kind, double *q) {
    for (int64_t i = 0; i < g->n; ++i) {
        double f = field[i];
        if (!(f > 0.0) || !(f < INFINITY)) return -1;
        double qq = (kind == ORC_SPEED) ? g->h / f : g->h * f;
        double cc = qq * qq;
        if (!(cc > 0.0) || !(cc < INFINITY)) return -1;
        q[i] = qq;
    }
    return 0;
}

/* a_k for point i: min of the two axis neighbours, +inf off the grid. */
static void neighbour_minima(const grid_t *g, const double *t, int64_t i, double a[3]) {
    int64_t ix = i % g->nx, iy = (i / g->nx) % g->ny, iz = i / (g->nx * g->ny);
    double lo, hi;
    lo = ix > 0 ? t[i - 1] : INFINITY;
    hi = ix < g->nx - 1 ? t[i + 1] : INFINITY;
    a[0] = lo < hi ? lo : hi;
    lo = iy > 0 ? t[i - g->nx] : INFINITY;
    hi = iy < g->ny - 1 ? t[i + g->nx] : INFINITY;
    a[1] = lo < hi ? lo : hi;
    if (g->ndim == 3) {
        int64_t s = g->nx * g->ny;
        lo = iz > 0 ? t[i - s] : INFINITY;
        hi = iz < g->nz - 1 ? t[i + s] : INFINITY;
        a[2] = lo < hi ? lo : hi;
    } else {
        a[2] = INFINITY;
    }
}

/* The Newton variant of the paper's precision section: Newton's method on
 * alpha(t) = (t - tH)^2 + (t - tV)^2 - c, started from d-hat, on the two-sided
 * branch (|tH - tV| < q); the one-sided branch is min(tH, tV) + q as for the
 * explicit formulas.  Each step, in this order:
 *   e0 = fl(t - tH), e1 = fl(t - tV),
 *   a  = fl(fl(fl(e0*e0) + fl(e1*e1)) - c),  da = fl(2 * fl(e0 + e1)),
 *   t' = fl(t - fl(a / da)),
 * stopping when t' == t, da == 0, or after 8 steps (the paper fixes neither
 * the count nor the stopping rule). */
double orc_newton(double tH, double tV, double c, double q) {
    if (fabs(tH - tV) >= q) return (tH < tV ? tH : tV) + q;
    double t = orc_dhat(tH, tV, c, q);
    for (int k = 0; k < 8; ++k) {
        double e0 = t - tH, e1 = t - tV;
        double a = (e0 * e0 + e1 * e1) - c;
        double da = 2.0 * (e0 + e1);
        if (da == 0.0) break;
        double tn = t - a / da;
        if (tn == t) break;
        t = tn;
    }
    return t;
}

/* Apply the chosen operator at point i; returns the candidate value. */
/* Neighbour values on both sides of each axis and the spacing weights at i
 * (rectilinear operator; +inf off the grid and for absent axes). */
static double apply_rect(const grid_t *g, const double *t, const double *q, int64_t i) {
    const int64_t n[3] = {g->nx, g->ny, g->nz};
    const int64_t stride[3] = {1, g->nx, g->nx * g->ny};
    const int64_t coord[3] = {i % g->nx, (i / g->nx) % g->ny, i / (g->nx * g->ny)};
    double am[3] = {INFINITY, INFINITY, INFINITY}, ap[3] = {INFINITY, INFINITY, INFINITY};
    double wm[3] = {1.0, 1.0, 1.0}, wp[3] = {1.0, 1.0, 1.0};
    for (int k = 0; k < g->ndim; ++k) {
        if (coord[k] > 0) am[k] = t[i - stride[k]];
        if (coord[k] < n[k] - 1) ap[k] = t[i + stride[k]];
        wm[k] = g_rect->wm[k][coord[k]];
        wp[k] = g_rect->wp[k][coord[k]];
    }
    double qi = q[i];
    return orc_dbar_rect(am, ap, wm, wp, qi * qi);
}

static double apply_op(const grid_t *g, const double *t, const double *q, int64_t i, int op) {
    if (op == OP_RECT) return apply_rect(g, t, q, i);
    double a[3];
    neighbour_minima(g, t, i, a);
    double qi = q[i];
    double c = qi * qi;
    if (op == OP_DBAR) return orc_dbar(a, c);
    double tH = a[0], tV = a[1];
    if (!(tH < INFINITY) && !(tV < INFINITY)) return INFINITY;
    if (op == OP_DHAT) return orc_dhat(tH, tV, c, qi);
    if (op == OP_NEWTON) return orc_newton(tH, tV, c, qi);
    return orc_dtilde(tH, tV, c, qi);
}

static int nbrs(const grid_t *g, int64_t i, int64_t out[6]) {
    int64_t ix = i % g->nx, iy = (i / g->nx) % g->ny, iz = i / (g->nx * g->ny);
    int k = 0;
    if (ix > 0) out[k++] = i - 1;
    if (ix < g->nx - 1) out[k++] = i + 1;
    if (iy > 0) out[k++] = i - g->nx;
    if (iy < g->ny - 1) out[k++] = i + g->nx;
    if (g->ndim == 3) {
        int64_t s = g->nx * g->ny;
        if (iz > 0) out[k++] = i - s;
        if (iz < g->nz - 1) out[k++] = i + s;
    }
    return k;
}

/* Common set-up: q array, fixed (source) mask, t = +inf with the sources set to
 * their start times (duplicates: the smallest wins). */
static int setup(const grid_t *g, const double *field, int kind, int64_t nsrc,
                 const int64_t *src, const double *t0, double *t, double **q_out,
                 uint8_t **fixed_out) {
    double *q = (double *)malloc(sizeof(double) * (size_t)g->n);
    uint8_t *fixed = (uint8_t *)calloc((size_t)g->n, 1);
    if (!q || !fixed) { free(q); free(fixed); return -2; }
    if (make_q(g, field, kind, q) != 0) { free(q); free(fixed); return -1; }
    for (int64_t i = 0; i < g->n; ++i) t[i] = INFINITY;
    for (int64_t s = 0; s < nsrc; ++s) {
        int64_t i = src[s];
        if (i < 0 || i >= g->n) { free(q); free(fixed); return -3; }
        double v = t0 ? t0[s] : 0.0;
        if (!(v >= 0.0) || !(v < INFINITY) || signbit(v)) { free(q); free(fixed); return -3; }
        if (!fixed[i] || v < t[i]) t[i] = v;
        fixed[i] = 1;
    }
    *q_out = q;
    *fixed_out = fixed;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* binary heap of (t, index) with lazy deletion                               */
/* ------------------------------------------------------------------------- */

typedef struct { double t; int64_t i; } item_t;
typedef struct { item_t *a; int64_t n, cap; } heap_t;

static int item_less(item_t x, item_t y) { return x.t < y.t || (x.t == y.t && x.i < y.i); }

static int heap_push(heap_t *h, double t, int64_t i) {
    if (h->n == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        item_t *na = (item_t *)realloc(h->a, sizeof(item_t) * (size_t)nc);
        if (!na) return -2;
        h->a = na;
        h->cap = nc;
    }
    int64_t k = h->n++;
    item_t it = {t, i};
    while (k > 0) {
        int64_t p = (k - 1) / 2;
        if (!item_less(it, h->a[p])) break;
        h->a[k] = h->a[p];
        k = p;
    }
    h->a[k] = it;
    return 0;
}

static item_t heap_pop(heap_t *h) {
    item_t top = h->a[0];
    item_t last = h->a[--h->n];
    int64_t k = 0;
    for (;;) {
        int64_t l = 2 * k + 1;
        if (l >= h->n) break;
        int64_t m = (l + 1 < h->n && item_less(h->a[l + 1], h->a[l])) ? l + 1 : l;
        if (!item_less(h->a[m], last)) break;
        h->a[k] = h->a[m];
        k = m;
    }
    if (h->n > 0) h->a[k] = last;
    return top;
}

/* ------------------------------------------------------------------------- */
/* schedules                                                                  */
/* ------------------------------------------------------------------------- */

/* stats[0] = pops (non-stale), stats[1] = operator applications,
 * stats[2] = accepted (decreasing) updates. */

/* Fast marching (Algorithm "Fast Marching Method"): pop the smallest entry,
 * apply the operator at every non-source neighbour, push each one that
 * decreased.  Stale heap entries (tagged with an old t) are skipped. */
int orc_fmm(int ndim, int64_t nx, int64_t ny, int64_t nz, double h, const double *field,
            int kind, int64_t nsrc, const int64_t *src, const double *t0, int op,
            double *t, int64_t *stats) {
    grid_t g = mkgrid(ndim, nx, ny, nz, h);
    double *q;
    uint8_t *fixed;
    int rc = setup(&g, field, kind, nsrc, src, t0, t, &q, &fixed);
    if (rc) return rc;
    heap_t hp = {0, 0, 0};
    int64_t pops = 0, applies = 0, accepts = 0;
    for (int64_t s = 0; s < nsrc; ++s)
        if (heap_push(&hp, t[src[s]], src[s])) { rc = -2; goto done; }
    while (hp.n > 0) {
        item_t it = heap_pop(&hp);
        if (it.t != t[it.i]) continue;
        ++pops;
        int64_t nb[6];
        int k = nbrs(&g, it.i, nb);
        for (int j = 0; j < k; ++j) {
            int64_t m = nb[j];
            if (fixed[m]) continue;
            double r = apply_op(&g, t, q, m, op);
            ++applies;
            if (r < t[m]) {
                t[m] = r;
                ++accepts;
                if (heap_push(&hp, r, m)) { rc = -2; goto done; }
            }
        }
    }
done:
    if (stats) { stats[0] = pops; stats[1] = applies; stats[2] = accepts; }
    free(hp.a);
    free(q);
    free(fixed);
    return rc;
}

/* Fast marching resumed from a given state.  On entry t holds, at every point,
 * an upper bound of the solution (>= +0 and not NaN; +inf allowed).  Sources
 * are fixed at their start times again, every other point keeps its value, and
 * every point with a finite value is queued; then the loop of Algorithm "Fast
 * Marching Method" runs as in orc_fmm with the exact monotone operator.  Since
 * that operator is monotone and causal, the state never drops below the
 * solution and every point is re-evaluated after its upwind neighbours last
 * changed, so the result is the one fixed point of Theorem 1 whatever upper
 * bound the loop started from.  With max_pops > 0 the loop stops after that
 * many non-stale pops and returns 1, leaving a state that is still an upper
 * bound (it can be resumed again); otherwise it returns 0 when the heap is
 * empty.  -5: a start value was NaN or negative. */
int orc_fmm_resume(int ndim, int64_t nx, int64_t ny, int64_t nz, double h, const double *field,
                   int kind, int64_t nsrc, const int64_t *src, const double *t0, int64_t max_pops,
                   double *t, int64_t *stats) {
    grid_t g = mkgrid(ndim, nx, ny, nz, h);
    double *start = (double *)malloc(sizeof(double) * (size_t)g.n);
    if (!start) return -2;
    for (int64_t i = 0; i < g.n; ++i) {
        if (t[i] != t[i] || signbit(t[i])) { free(start); return -5; }
        start[i] = t[i];
    }
    double *q;
    uint8_t *fixed;
    int rc = setup(&g, field, kind, nsrc, src, t0, t, &q, &fixed);
    if (rc) { free(start); return rc; }
    for (int64_t i = 0; i < g.n; ++i)
        if (!fixed[i]) t[i] = start[i];
    free(start);
    heap_t hp = {0, 0, 0};
    int64_t pops = 0, applies = 0, accepts = 0;
    for (int64_t i = 0; i < g.n; ++i)
        if (t[i] < INFINITY && heap_push(&hp, t[i], i)) { rc = -2; goto done; }
    while (hp.n > 0) {
        if (max_pops > 0 && pops >= max_pops) { rc = 1; break; }
        item_t it = heap_pop(&hp);
        if (it.t != t[it.i]) continue;
        ++pops;
        int64_t nb[6];
        int k = nbrs(&g, it.i, nb);
        for (int j = 0; j < k; ++j) {
            int64_t m = nb[j];
            if (fixed[m]) continue;
            double r = apply_op(&g, t, q, m, OP_DBAR);
            ++applies;
            if (r < t[m]) {
                t[m] = r;
                ++accepts;
                if (heap_push(&hp, r, m)) { rc = -2; goto done; }
            }
        }
    }
done:
    if (stats) { stats[0] = pops; stats[1] = applies; stats[2] = accepts; }
    free(hp.a);
    free(q);
    free(fixed);
    return rc;
}

/* Topology-driven schedule (Algorithm "topology-driven"): apply the operator at
 * every point, in index order, until a whole round changes nothing. */
int orc_sweep_all(int ndim, int64_t nx, int64_t ny, int64_t nz, double h, const double *field,
                  int kind, int64_t nsrc, const int64_t *src, const double *t0, int op,
                  double *t, int64_t *stats) {
    grid_t g = mkgrid(ndim, nx, ny, nz, h);
    double *q;
    uint8_t *fixed;
    int rc = setup(&g, field, kind, nsrc, src, t0, t, &q, &fixed);
    if (rc) return rc;
    int64_t rounds = 0, accepts = 0;
    int changed = 1;
    while (changed) {
        changed = 0;
        ++rounds;
        for (int64_t i = 0; i < g.n; ++i) {
            if (fixed[i]) continue;
            double r = apply_op(&g, t, q, i, op);
            if (r < t[i]) { t[i] = r; changed = 1; ++accepts; }
        }
    }
    if (stats) { stats[0] = rounds; stats[1] = rounds * g.n; stats[2] = accepts; }
    free(q);
    free(fixed);
    return 0;
}

/* Fast sweeping (Algorithm "Fast Sweeping Method"): Gauss-Seidel sweeps in the
 * 2^ndim alternating axis directions, repeated until a full cycle of sweeps
 * changes nothing. */
int orc_fsm(int ndim, int64_t nx, int64_t ny, int64_t nz, double h, const double *field,
            int kind, int64_t nsrc, const int64_t *src, const double *t0, int op,
            double *t, int64_t *stats) {
    grid_t g = mkgrid(ndim, nx, ny, nz, h);
    double *q;
    uint8_t *fixed;
    int rc = setup(&g, field, kind, nsrc, src, t0, t, &q, &fixed);
    if (rc) return rc;
    int ndir = 1 << ndim;
    int64_t cycles = 0, accepts = 0;
    int changed = 1;
    while (changed) {
        changed = 0;
        ++cycles;
        for (int dir = 0; dir < ndir; ++dir) {
            int fx = !(dir & 1), fy = !(dir & 2), fz = !(dir & 4);
            for (int64_t kz = 0; kz < g.nz; ++kz) {
                int64_t iz = fz ? kz : g.nz - 1 - kz;
                for (int64_t ky = 0; ky < g.ny; ++ky) {
                    int64_t iy = fy ? ky : g.ny - 1 - ky;
                    for (int64_t kx = 0; kx < g.nx; ++kx) {
                        int64_t ix = fx ? kx : g.nx - 1 - kx;
                        int64_t i = (iz * g.ny + iy) * g.nx + ix;
                        if (fixed[i]) continue;
                        double r = apply_op(&g, t, q, i, op);
                        if (r < t[i]) { t[i] = r; changed = 1; ++accepts; }
                    }
                }
            }
        }
    }
    if (stats) { stats[0] = cycles; stats[1] = cycles * ndir * g.n; stats[2] = accepts; }
    free(q);
    free(fixed);
    return 0;
}

/* xorshift64* for the random schedule below */
static uint64_t rng_next(uint64_t *s) {
    uint64_t x = *s;
    x ^= x >> 12;
    x ^= x << 25;
    x ^= x >> 27;
    *s = x;
    return x * 0x2545F4914F6CDD1DULL;
}

/* Unordered data-driven schedule: the worklist is a bag from which a uniformly
 * random item is taken each step (arbitrary priority inversions, the extreme of
 * soft priorities).  A neighbour is pushed whenever it decreased
 * (mode 0) or whenever it changed at all (mode 1, the paper's conservative work
 * tracking; only differs from mode 0 with a non-monotone operator). */
int orc_async_random(int ndim, int64_t nx, int64_t ny, int64_t nz, double h,
                     const double *field, int kind, int64_t nsrc, const int64_t *src,
                     const double *t0, int op, uint64_t seed, int mode, double *t,
                     int64_t *stats) {
    grid_t g = mkgrid(ndim, nx, ny, nz, h);
    double *q;
    uint8_t *fixed;
    int rc = setup(&g, field, kind, nsrc, src, t0, t, &q, &fixed);
    if (rc) return rc;
    int64_t cap = 1024, n = 0;
    int64_t *bag = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    uint64_t st = seed * 0x9E3779B97F4A7C15ULL + 0x632BE59BD9B4E019ULL;
    if (st == 0) st = 1;
    int64_t pops = 0, applies = 0, accepts = 0;
    if (!bag) { rc = -2; goto done; }
    for (int64_t s = 0; s < nsrc; ++s) bag[n++] = src[s];
    while (n > 0) {
        int64_t j = (int64_t)(rng_next(&st) % (uint64_t)n);
        int64_t p = bag[j];
        bag[j] = bag[--n];
        ++pops;
        int64_t nb[6];
        int k = nbrs(&g, p, nb);
        for (int jj = 0; jj < k; ++jj) {
            int64_t m = nb[jj];
            if (fixed[m]) continue;
            double r = apply_op(&g, t, q, m, op);
            ++applies;
            int push = mode ? (r != t[m]) : (r < t[m]);
            if (op == OP_DBAR || mode == 0) {
                if (r < t[m]) { t[m] = r; ++accepts; } else push = 0;
            } else if (push) {
                t[m] = r;
                ++accepts;
            }
            if (push) {
                if (n == cap) {
                    cap *= 2;
                    int64_t *nb2 = (int64_t *)realloc(bag, sizeof(int64_t) * (size_t)cap);
                    if (!nb2) { rc = -2; goto done; }
                    bag = nb2;
                }
                bag[n++] = m;
                if (accepts > 4096 * g.n + 65536) { rc = -4; goto done; }  /* runaway guard */
            }
        }
    }
done:
    if (stats) { stats[0] = pops; stats[1] = applies; stats[2] = accepts; }
    free(bag);
    free(q);
    free(fixed);
    return rc;
}

/* Entry points for rectilinear grids: coordinates per axis (xs: nx values,
 * ys: ny, zs: nz or NULL in 2D), strictly increasing and finite, with
 * finite reciprocal spacings.  They run the schedules above with the
 * rectilinear operator and q = fl(1/v) or s (spacing lives in the weights).
 * -6: bad coordinates. */
int64_t orc_residual(int ndim, int64_t nx, int64_t ny, int64_t nz, double h, const double *field, int kind,
                     int64_t nsrc, const int64_t *src, const double *t, int op, double *maxrel);

typedef int (*rect_body)(int ndim, int64_t nx, int64_t ny, int64_t nz, void *ctx);

static int with_rect(int ndim, int64_t nx, int64_t ny, int64_t nz, const double *xs, const double *ys,
                     const double *zs, rect_body body, void *ctx) {
    const int64_t n[3] = {nx, ny, nz};
    const double *xyz[3] = {xs, ys, zs};
    double *buf = (double *)malloc(sizeof(double) * 2 * (size_t)(nx + ny + nz));
    if (!buf) return -2;
    rect_t r;
    double *p = buf;
    int rc = 0;
    for (int k = 0; k < 3; ++k) {
        double *wm = p, *wp = p + n[k];
        p += 2 * n[k];
        r.wm[k] = wm;
        r.wp[k] = wp;
        for (int64_t i = 0; i < n[k]; ++i) { wm[i] = 1.0; wp[i] = 1.0; }
        if (k >= ndim) continue;
        for (int64_t i = 0; i < n[k]; ++i) {
            if (!(xyz[k][i] > -INFINITY) || !(xyz[k][i] < INFINITY)) { rc = -6; goto done; }
            if (i > 0) {
                double hm = xyz[k][i] - xyz[k][i - 1];
                double w = 1.0 / hm;
                if (!(hm > 0.0) || !(w < INFINITY)) { rc = -6; goto done; }
                wm[i] = w;
                wp[i - 1] = w;
            }
        }
    }
    g_rect = &r;
    rc = body(ndim, nx, ny, nz, ctx);
    g_rect = NULL;
done:
    free(buf);
    return rc;
}

typedef struct {
    const double *field; int kind; int64_t nsrc; const int64_t *src; const double *t0;
    double *t; int64_t *stats; int which; uint64_t seed; double *maxrel; int64_t count;
} rect_ctx;

static int rect_run(int ndim, int64_t nx, int64_t ny, int64_t nz, void *vctx) {
    rect_ctx *c = (rect_ctx *)vctx;
    switch (c->which) {
        case 0: return orc_fmm(ndim, nx, ny, nz, 1.0, c->field, c->kind, c->nsrc, c->src, c->t0, OP_RECT, c->t, c->stats);
        case 1: return orc_sweep_all(ndim, nx, ny, nz, 1.0, c->field, c->kind, c->nsrc, c->src, c->t0, OP_RECT, c->t, c->stats);
        case 2: return orc_fsm(ndim, nx, ny, nz, 1.0, c->field, c->kind, c->nsrc, c->src, c->t0, OP_RECT, c->t, c->stats);
        case 3: return orc_async_random(ndim, nx, ny, nz, 1.0, c->field, c->kind, c->nsrc, c->src, c->t0, OP_RECT,
                                        c->seed, 0, c->t, c->stats);
        default:
            c->count = orc_residual(ndim, nx, ny, nz, 1.0, c->field, c->kind, c->nsrc, c->src, c->t, OP_RECT, c->maxrel);
            return c->count < 0 ? -1 : 0;
    }
}

/* which: 0 fast marching, 1 topology-driven rounds, 2 fast sweeping, 3 random-order worklist. */
int orc_solve_rect(int which, int ndim, int64_t nx, int64_t ny, int64_t nz, const double *xs, const double *ys,
                   const double *zs, const double *field, int kind, int64_t nsrc, const int64_t *src,
                   const double *t0, uint64_t seed, double *t, int64_t *stats) {
    rect_ctx c = {field, kind, nsrc, src, t0, t, stats, which, seed, NULL, 0};
    return with_rect(ndim, nx, ny, nz, xs, ys, zs, rect_run, &c);
}

/* Residual of a state on a rectilinear grid (as orc_residual); < 0 on error. */
int64_t orc_residual_rect(int ndim, int64_t nx, int64_t ny, int64_t nz, const double *xs, const double *ys,
                          const double *zs, const double *field, int kind, int64_t nsrc, const int64_t *src,
                          const double *t, double *maxrel) {
    rect_ctx c = {field, kind, nsrc, src, NULL, (double *)t, NULL, 4, 0, maxrel, 0};
    int rc = with_rect(ndim, nx, ny, nz, xs, ys, zs, rect_run, &c);
    return rc ? rc : c.count;
}

/* Residual metric (Table "tab:error"): re-apply the operator at every non-source
 * point with the final neighbour values; returns the number of points whose
 * value would change and writes the largest |r - t| / t to *maxrel. */
int64_t orc_residual(int ndim, int64_t nx, int64_t ny, int64_t nz, double h,
                     const double *field, int kind, int64_t nsrc, const int64_t *src,
                     const double *t, int op, double *maxrel) {
    grid_t g = mkgrid(ndim, nx, ny, nz, h);
    double *q = (double *)malloc(sizeof(double) * (size_t)g.n);
    uint8_t *fixed = (uint8_t *)calloc((size_t)g.n, 1);
    int64_t bad = 0;
    double worst = 0.0;
    if (!q || !fixed || make_q(&g, field, kind, q) != 0) { bad = -1; goto done; }
    for (int64_t s = 0; s < nsrc; ++s) fixed[src[s]] = 1;
    for (int64_t i = 0; i < g.n; ++i) {
        if (fixed[i]) continue;
        double r = apply_op(&g, t, q, i, op);
        if (r != t[i]) {
            ++bad;
            double rel = fabs(r - t[i]) / fabs(t[i]);
            if (!(rel <= worst)) worst = rel;
        }
    }
done:
    if (maxrel) *maxrel = worst;
    free(q);
    free(fixed);
    return bad;
}

/* ------------------------------------------------------------------------- */
/* parents and adjoint                                                        */
/* ------------------------------------------------------------------------- */

/* Upwind parent record from final times.  Per axis k (bits 2k..2k+1):
 * 0 = axis not upwind (min neighbour >= t), 1 = the minus-side neighbour,
 * 2 = the plus-side neighbour (equal neighbours: minus side).  Bit 7 marks a
 * source point (its other bits are zero). */
void orc_parents(int ndim, int64_t nx, int64_t ny, int64_t nz, const double *t,
                 int64_t nsrc, const int64_t *src, uint8_t *par) {
    grid_t g = mkgrid(ndim, nx, ny, nz, 1.0);
    int64_t stride[3] = {1, g.nx, g.nx * g.ny};
    int64_t dim[3] = {g.nx, g.ny, g.nz};
    for (int64_t i = 0; i < g.n; ++i) {
        int64_t coord[3] = {i % g.nx, (i / g.nx) % g.ny, i / (g.nx * g.ny)};
        uint8_t b = 0;
        for (int k = 0; k < ndim; ++k) {
            double lo = coord[k] > 0 ? t[i - stride[k]] : INFINITY;
            double hi = coord[k] < dim[k] - 1 ? t[i + stride[k]] : INFINITY;
            double m = lo <= hi ? lo : hi;
            if (m < t[i]) b |= (uint8_t)((lo <= hi ? 1 : 2) << (2 * k));
        }
        par[i] = b;
    }
    for (int64_t s = 0; s < nsrc; ++s) par[src[s]] = 0x80;
}

typedef struct { double t; int64_t i; } key_t;
static int key_desc(const void *x, const void *y) {
    const key_t *a = (const key_t *)x, *b = (const key_t *)y;
    if (a->t > b->t) return -1;
    if (a->t < b->t) return 1;
    return (a->i > b->i) - (a->i < b->i);
}

/* Adjoint of the discrete equations sum_k (t_n - t_{p_k})^2 = (h s_n)^2 over the
 * recorded upwind parents p_k (paper silent; implicit differentiation).  With
 * w_{n,k} = fl(t_n - t_{p_k}) and W_n = fl(fl(w_x + w_y) + w_z) (inactive axes
 * +0), processing non-source points in decreasing t:
 *   lambda_n = g_n, then += fl(mu_m * w_{m,k}) for each child m of n, children
 *              taken in the neighbour order x-, x+, y-, y+, z-, z+,
 *   mu_n     = fl(lambda_n / W_n),
 *   grad_n   = fl(fl(mu_n * q_n) * h)   (d loss / d slowness_n),
 * where q_n is the forward constant (h/v or h*s) and sources get mu = grad = 0.
 * mu_out (optional) receives mu. Returns 0, or -1 on a field domain error. */
int orc_adjoint(int ndim, int64_t nx, int64_t ny, int64_t nz, double h, const double *field,
                int kind, const double *t, const uint8_t *par, const double *gin,
                double *grad, double *mu_out) {
    grid_t g = mkgrid(ndim, nx, ny, nz, h);
    int64_t stride[3] = {1, g.nx, g.nx * g.ny};
    int64_t dim[3] = {g.nx, g.ny, g.nz};
    double *mu = (double *)calloc((size_t)g.n, sizeof(double));
    key_t *ord = (key_t *)malloc(sizeof(key_t) * (size_t)g.n);
    int rc = 0;
    if (!mu || !ord) { rc = -2; goto done; }
    int64_t m = 0;
    for (int64_t i = 0; i < g.n; ++i) {
        double f = field[i];
        if (!(f > 0.0) || !(f < INFINITY)) { rc = -1; goto done; }
        grad[i] = 0.0;
        if (!(par[i] & 0x80)) { ord[m].t = t[i]; ord[m].i = i; ++m; }
    }
    qsort(ord, (size_t)m, sizeof(key_t), key_desc);
    for (int64_t j = 0; j < m; ++j) {
        int64_t n = ord[j].i;
        int64_t coord[3] = {n % g.nx, (n / g.nx) % g.ny, n / (g.nx * g.ny)};
        double lam = gin[n];
        for (int k = 0; k < ndim; ++k) {
            /* minus-side neighbour is a child if its plus-side parent is n */
            if (coord[k] > 0) {
                int64_t ch = n - stride[k];
                if (!(par[ch] & 0x80) && ((par[ch] >> (2 * k)) & 3) == 2)
                    lam = lam + mu[ch] * (t[ch] - t[n]);
            }
            if (coord[k] < dim[k] - 1) {
                int64_t ch = n + stride[k];
                if (!(par[ch] & 0x80) && ((par[ch] >> (2 * k)) & 3) == 1)
                    lam = lam + mu[ch] * (t[ch] - t[n]);
            }
        }
        double w[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < ndim; ++k) {
            int code = (par[n] >> (2 * k)) & 3;
            if (code == 1) w[k] = t[n] - t[n - stride[k]];
            else if (code == 2) w[k] = t[n] - t[n + stride[k]];
        }
        double W = (w[0] + w[1]) + w[2];
        double mun = lam / W;
        mu[n] = mun;
        double f = field[n];
        double q = (kind == ORC_SPEED) ? h / f : h * f;
        grad[n] = (mun * q) * h;
    }
    if (mu_out) memcpy(mu_out, mu, sizeof(double) * (size_t)g.n);
done:
    free(mu);
    free(ord);
    return rc;
}

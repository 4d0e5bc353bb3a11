"""Pins of the oracle's local update operator against what the paper and plain
mathematics fix (no GPU).

* the worked examples of Tables tab:prec_1 / tab:prec_2 (explicit formulas,
  digits as printed) -- these pin the constant c = fl(fl(h/v)^2) and the
  formulas' arithmetic;
* the exactly monotone operator dbar (section "Achieving Exact Monotonicity with
  Finite Precision Arithmetic") against the exact real root of the quadratic,
  an exhaustive bisection over all binary64 values, monotonicity and causality
  fuzzing, and one-sided closed forms.
"""
import json
import math
import os
import random
import struct
from decimal import Decimal, getcontext

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
INF = math.inf


def bits(x: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def flt(u: int) -> float:
    return struct.unpack("<d", struct.pack("<Q", u))[0]


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


@pytest.fixture(scope="module")
def tables():
    with open(os.path.join(HERE, "golden", "paper_tables.json")) as f:
        return json.load(f)


# ---------------------------------------------------------------------------
# worked examples (paper tables)
# ---------------------------------------------------------------------------

def test_table_prec_1_dtilde_digits(O, tables):
    T = tables["tab_prec_1"]
    outs = {}
    for k, row in T["rows"].items():
        outs[k] = O.dtilde(T["tH"], row["tV"], T["v"], T["h"])
        assert outs[k] == row["out"], (k, repr(outs[k]))
    # the paper's point: tV decreased from A to B but the value increased
    assert T["rows"]["B"]["tV"] < T["rows"]["A"]["tV"]
    assert outs["B"] > outs["A"]


def test_table_prec_2_dhat_digits(O, tables):
    T = tables["tab_prec_2"]
    outs = {}
    for k, row in T["rows"].items():
        outs[k] = O.dhat(T["tH"], row["tV"], T["v"], T["h"])
        assert outs[k] == row["out"], (k, repr(outs[k]))
    assert T["rows"]["B"]["tV"] < T["rows"]["A"]["tV"]
    assert outs["B"] > outs["A"]


@pytest.mark.parametrize("name", ["tab_prec_1", "tab_prec_2"])
def test_dbar_monotone_where_explicit_formulas_are_not(O, tables, name):
    T = tables[name]
    q = T["h"] / T["v"]
    c = q * q
    rA = O.dbar([T["tH"], T["rows"]["A"]["tV"]], c)
    rB = O.dbar([T["tH"], T["rows"]["B"]["tV"]], c)
    assert rB <= rA
    # and it stays within a few ulps of the exact root of the quadratic
    for k, r in (("A", rA), ("B", rB)):
        R = exact_root([T["tH"], T["rows"][k]["tV"]], c)
        assert abs(Decimal(r) - R) <= 4 * Decimal(math.ulp(r))


def test_constant_order_matters_for_table_prec_2(tables):
    """Only c = fl(fl(h/v)^2) reproduces row B; 2 h^2 / (v v) does not."""
    T = tables["tab_prec_2"]
    tH, tV = T["tH"], T["rows"]["B"]["tV"]
    q = T["h"] / T["v"]
    d = tH - tV
    good = 0.5 * ((tH + tV) + math.sqrt(2.0 * (q * q) - d * d))
    other = 0.5 * ((tH + tV) + math.sqrt(2.0 * T["h"] * T["h"] / (T["v"] * T["v"]) - d * d))
    assert good == T["rows"]["B"]["out"]
    assert other != T["rows"]["B"]["out"]


# ---------------------------------------------------------------------------
# dbar against the exact real root
# ---------------------------------------------------------------------------

def exact_root(a, c):
    """Real root of sum over a_k < R of (R - a_k)^2 = c, computed in 60-digit
    decimal arithmetic from the exact binary values."""
    getcontext().prec = 60
    A = sorted(Decimal(x) for x in a if x != INF)
    C = Decimal(c)
    for m in range(1, len(A) + 1):
        s = sum(A[:m])
        s2 = sum(x * x for x in A[:m])
        disc = s * s - m * (s2 - C)
        if disc < 0:
            continue
        R = (s + disc.sqrt()) / m
        if R >= A[m - 1] and (m == len(A) or R <= A[m]):
            return R
    raise AssertionError("no root")


def rand_case(rng: random.Random):
    scale = 10 ** rng.uniform(-3, 3)
    q = scale * rng.uniform(0.05, 2.0)
    base = scale * rng.uniform(0, 50)
    n = rng.choice([1, 2, 3, 3, 3])
    a = [base + rng.uniform(0, 1.5) * q for _ in range(n)]
    if rng.random() < 0.3 and n >= 2:
        a[1] = a[0]   # ties
    a += [INF] * (3 - n)
    rng.shuffle(a)
    return a, q * q


def test_dbar_matches_exact_root_within_ulps(O):
    rng = random.Random(1)
    for _ in range(3000):
        a, c = rand_case(rng)
        r = O.dbar(a, c)
        R = exact_root(a, c)
        err = abs(Decimal(r) - R)
        assert err <= 6 * Decimal(math.ulp(r)), (a, c, r, R)


def py_reaches(r, a, c):
    """S(r) >= c, written out independently: terms summed largest first."""
    s = sorted(a)
    T = []
    for x in s:
        d = r - x
        T.append(d * d if d > 0 else 0.0)
    return (T[0] + T[1]) + T[2] >= c


def test_dbar_equals_exhaustive_bisection(O):
    """Bisection over every binary64 value in [min a, +inf] (64 steps)."""
    rng = random.Random(2)
    for _ in range(1500):
        a, c = rand_case(rng)
        lo, hi = bits(min(a)), bits(INF)
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if py_reaches(flt(mid), a, c):
                hi = mid
            else:
                lo = mid
        assert O.dbar(a, c) == flt(hi), (a, c)


def test_dbar_predicate_boundary(O):
    rng = random.Random(3)
    for _ in range(1000):
        a, c = rand_case(rng)
        r = O.dbar(a, c)
        assert O.reaches(r, a, c)
        prev = flt(bits(r) - 1)
        assert prev <= min(a) or not O.reaches(prev, a, c)
        assert r > min(a)


# ---------------------------------------------------------------------------
# monotonicity and causality in floating point
# ---------------------------------------------------------------------------

def nudge(x, k):
    return flt(bits(x) + k) if x != INF else x


def test_dbar_monotone_fuzz(O):
    """Lowering any neighbour value never raises the result (ulp-scale windows,
    including around the switch between one- and two-sided updates)."""
    rng = random.Random(4)
    checked = 0
    for _ in range(4000):
        a, c = rand_case(rng)
        q = math.sqrt(c)
        if rng.random() < 0.5 and a.count(INF) <= 1:
            fin = [i for i in range(3) if a[i] != INF]
            i, j = fin[0], fin[1]
            a[j] = a[i] + q * (1 + rng.choice([-1, 1]) * rng.uniform(0, 1e-14))   # branch switch
        k = rng.randrange(3)
        if a[k] == INF:
            continue
        r0 = O.dbar(a, c)
        for step in (-6, -3, -1, 1, 3, 6):
            b = list(a)
            b[k] = nudge(a[k], step)
            if b[k] < 0:
                continue
            r1 = O.dbar(b, c)
            if b[k] < a[k]:
                assert r1 <= r0, (a, b, c)
            else:
                assert r1 >= r0, (a, b, c)
            checked += 1
    assert checked > 10000


def test_dbar_causal_fuzz(O):
    """Neighbours whose value is >= the result do not influence it."""
    rng = random.Random(5)
    for _ in range(3000):
        a, c = rand_case(rng)
        r = O.dbar(a, c)
        for k in range(3):
            if a[k] >= r:
                for newv in (r, nudge(r, 5), r * 2 + 1, INF):
                    b = list(a)
                    b[k] = newv
                    assert O.dbar(b, c) == r, (a, b, c)


def test_dbar_permutation_invariant(O):
    rng = random.Random(6)
    import itertools
    for _ in range(500):
        a, c = rand_case(rng)
        r = O.dbar(a, c)
        for p in itertools.permutations(a):
            assert O.dbar(list(p), c) == r


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------

def test_one_sided_integer_steps(O):
    for k in [0, 1, 2, 7, 1000, 2 ** 20]:
        assert O.dbar([float(k), INF, INF], 1.0) == float(k + 1)


def test_two_and_three_sided_unit_cases(O):
    r2 = O.dbar([1.0, 1.0], 1.0)
    r3 = O.dbar([1.0, 1.0, 1.0], 1.0)
    for r, R in ((r2, 1 + 1 / Decimal(2).sqrt()), (r3, 1 + 1 / Decimal(3).sqrt())):
        assert abs(Decimal(r) - R) <= 2 * Decimal(math.ulp(r))
    # smallest double with fl(2 fl((r-1)^2)) >= 1
    prev = flt(bits(r2) - 1)
    assert ((r2 - 1) ** 2 + (r2 - 1) ** 2) >= 1.0
    assert ((prev - 1) ** 2 + (prev - 1) ** 2) < 1.0


def test_no_finite_neighbour_gives_inf(O):
    assert O.dbar([INF, INF, INF], 1.0) == INF


def test_newton_repairs_the_table_prec_2_pair(O, tables):
    """Newton's method from the d-hat guess (the precision section's practical
    variant) on the pair where d-hat is not monotone: the smaller t_V must not
    give the larger result, and both results sit within one ulp of d-bar."""
    T = tables["tab_prec_2"]
    rows = T["rows"]
    a = O.newton(T["tH"], rows["A"]["tV"], T["v"], T["h"])
    b = O.newton(T["tH"], rows["B"]["tV"], T["v"], T["h"])
    assert rows["B"]["tV"] < rows["A"]["tV"]
    assert b <= a
    q = T["h"] / T["v"]
    for tV, r in ((rows["A"]["tV"], a), (rows["B"]["tV"], b)):
        d = O.dbar([T["tH"], tV, np.inf], q * q)
        assert abs(int(np.float64(r).view(np.int64)) - int(np.float64(d).view(np.int64))) <= 1


def test_newton_converges_to_the_root_of_alpha(O):
    """On the two-sided branch Newton solves the same root problem as d-bar:
    almost always within one ulp of d-bar, never far off; on the one-sided
    branch it is min + q like the explicit formulas."""
    rng = np.random.default_rng(0)
    diffs = []
    for _ in range(4000):
        v = rng.uniform(0.5, 5.0)
        h = rng.uniform(0.1, 10.0)
        q = h / v
        tH = rng.uniform(0.0, 100.0)
        tV = tH + rng.uniform(-0.999, 0.999) * q
        n = O.newton(tH, tV, v, h)
        d = O.dbar([tH, tV, np.inf], q * q)
        assert np.isfinite(n)
        diffs.append(abs(int(np.float64(n).view(np.int64)) - int(np.float64(d).view(np.int64))))
        assert O.newton(tH, tH + 1.5 * q, v, h) == tH + q
    diffs = np.array(diffs)
    assert np.mean(diffs <= 1) > 0.995
    assert diffs.max() <= 16

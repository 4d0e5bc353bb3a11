"""Pins of the oracle's rectilinear-grid operator (no GPU).

The operator applies the construction of the section "Achieving Exact
Monotonicity with Finite Precision Arithmetic" to the first-order upwind
scheme on a grid whose spacing varies per axis and index (the irregular-grid
case the conclusion names).  Pinned by:

* reduction to the uniform operator, bit for bit, with unit and power-of-two
  spacing (the weights are then exact and only scale the predicate), and within
  rounding for any other uniform spacing;
* Theorem 1 on irregular grids: fast marching, topology-driven rounds, fast
  sweeping and random-order worklists reach the same bits, and the residual of
  the result is exactly zero;
* the search against a plain bisection of the predicate over the whole range
  of doubles, and monotonicity / causality of the predicate's root under
  perturbations of each input;
* the order of the sum: S adds the squared terms largest first, a symmetric
  function, so permuting the axes (neighbours and weights together) never
  changes the result, ties included; and one-ulp changes of a neighbour that
  swap two axes near a source never raise the result (ordering the terms by
  their neighbour values instead fails this fuzz);
* closed forms and limits: a stretched 1-D line accumulates h_i / v, and a
  point source on stretched grids converges to r / v at first order.
"""
import math

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def grids(rng):
    out = []
    f = W.random_field((1, 23, 31), rng, 0.5, 4.0, block=3)
    xs, ys = W.jittered_coords(31, 1.0, rng), W.stretched_coords(23, 0.5, 1.08)
    out.append(("2d_jitter_stretch", f, xs, ys, None, np.array([5 * 31 + 7, 400])))
    f = W.random_field((9, 11, 13), rng, 0.5, 4.0, block=2)
    xs, ys, zs = W.jittered_coords(13, 2.0, rng, 0.5), W.jittered_coords(11, 1.0, rng), W.stretched_coords(9, 0.3, 1.2)
    out.append(("3d_jitter", f, xs, ys, zs, np.array([W.flat_index(6, 5, 0, 13, 11)])))
    f = 1.0 / W.random_field((7, 8, 6), rng, 0.5, 4.0)
    xs, ys, zs = W.stretched_coords(6, 1.0, 0.7), W.stretched_coords(8, 0.1, 1.5), W.jittered_coords(7, 3.0, rng)
    out.append(("3d_slowness_strong", f, xs, ys, zs, np.array([0, 200])))
    return out


CASES = grids(np.random.default_rng(91))


@pytest.mark.parametrize("kind", [0, 1])
def test_unit_and_power_of_two_spacing_is_the_uniform_operator(O, kind):
    rng = np.random.default_rng(5)
    # the 3D case is large enough that a different summation order of the
    # squared terms would show (it changes a few in ten thousand results)
    for shape, h in (((1, 40, 33), 1.0), ((30, 40, 40), 1.0), ((1, 25, 30), 4.0), ((5, 7, 9), 0.125)):
        f = W.random_field(shape, rng, 0.5, 4.0, block=3)
        if kind == 1:
            f = 1.0 / f
        nz, ny, nx = shape
        src = rng.choice(f.size, 2, replace=False)
        zs = None if nz == 1 else np.arange(nz) * h
        t = O.solve_rect(f, np.arange(nx) * h, np.arange(ny) * h, zs, src, kind=kind)
        assert np.array_equal(t, O.fmm(f, h, src, kind=kind)), (shape, h)


def test_other_uniform_spacing_agrees_within_rounding(O):
    rng = np.random.default_rng(6)
    f = W.random_field((6, 12, 14), rng, 1500.0, 6000.0, block=3)
    src = np.array([W.flat_index(7, 6, 0, 14, 12)])
    h = 10.0
    t = O.solve_rect(f, np.arange(14) * h, np.arange(12) * h, np.arange(6) * h, src)
    ref = O.fmm(f, h, src)
    m = ref > 0
    assert np.max(np.abs(t[m] - ref[m]) / ref[m]) < 1e-13


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_schedules_agree_bitwise_on_irregular_grids(O, case):
    _, f, xs, ys, zs, src = case
    kind = 1 if "slowness" in case[0] else 0
    ref = O.solve_rect(f, xs, ys, zs, src, kind=kind)
    assert np.all(np.isfinite(ref))
    for sch in ("sweep_all", "fsm"):
        assert np.array_equal(O.solve_rect(f, xs, ys, zs, src, kind=kind, schedule=sch), ref), sch
    for seed in range(5):
        assert np.array_equal(O.solve_rect(f, xs, ys, zs, src, kind=kind, schedule="async_random", seed=seed), ref)
    assert O.residual_rect(ref, f, xs, ys, zs, src, kind=kind) == (0, 0.0)
    # causality: every non-source point lies above its smallest neighbour
    pad = np.pad(ref, 1, constant_values=np.inf)
    mins = np.minimum.reduce([pad[1:-1, 1:-1, :-2], pad[1:-1, 1:-1, 2:], pad[1:-1, :-2, 1:-1],
                              pad[1:-1, 2:, 1:-1], pad[:-2, 1:-1, 1:-1], pad[2:, 1:-1, 1:-1]])
    mask = np.ones(ref.shape, bool)
    mask.reshape(-1)[src] = False
    assert np.all(ref[mask] > mins[mask])


def _bisect(O, am, ap, wm, wp, c):
    """Smallest double above min(a) satisfying the predicate, by plain bisection
    over the integer image of the doubles between min(a) and +inf."""
    lo = np.float64(min(min(am), min(ap))).view(np.uint64).item()
    hi = np.float64(np.inf).view(np.uint64).item()
    while hi - lo > 1:
        mid = lo + (hi - lo) // 2
        if O.reaches_rect(np.uint64(mid).view(np.float64).item(), am, ap, wm, wp, c):
            hi = mid
        else:
            lo = mid
    return np.uint64(hi).view(np.float64).item()


def test_operator_is_the_smallest_root_and_monotone(O):
    rng = np.random.default_rng(12)
    for trial in range(300):
        nax = 3 if trial % 3 else 2
        am = list(rng.uniform(0.0, 5.0, nax))
        ap = list(rng.uniform(0.0, 5.0, nax))
        for k in range(nax):
            if rng.random() < 0.2:
                ap[k] = np.inf
        wm = list(10.0 ** rng.uniform(-2, 2, nax))
        wp = list(10.0 ** rng.uniform(-2, 2, nax))
        c = float(10.0 ** rng.uniform(-2, 2))
        r = O.dbar_rect(am, ap, wm, wp, c)
        assert r == _bisect(O, am, ap, wm, wp, c)
        assert r > min(min(am), min(ap))
        # monotone: raising any neighbour never lowers the result
        for k in range(nax):
            for arr in (am, ap):
                if np.isfinite(arr[k]):
                    up = list(arr)
                    up[k] = np.nextafter(arr[k], np.inf) if rng.random() < 0.5 else arr[k] * 1.01 + 1e-3
                    r2 = O.dbar_rect(up if arr is am else am, up if arr is ap else ap, wm, wp, c)
                    assert r2 >= r
        # causal: a neighbour at or above the result does not matter
        for k in range(nax):
            if am[k] >= r:
                assert O.dbar_rect(am[:k] + [np.inf] + am[k + 1:], ap, wm, wp, c) == r


def test_result_is_invariant_under_axis_permutation(O):
    import itertools
    rng = np.random.default_rng(31)
    for trial in range(400):
        scale = 10.0 ** rng.uniform(-5, 1)
        am = list(rng.uniform(0.0, 1.0, 3) * scale)
        ap = list(rng.uniform(0.0, 1.0, 3) * scale)
        if trial % 2:   # exact ties between axes, with different weights
            am[1] = am[0]
            ap[1] = ap[0] = np.inf
            ap[2] = am[0] if trial % 4 == 1 else ap[2]
        wm = list(10.0 ** rng.uniform(-2, 2, 3))
        wp = list(10.0 ** rng.uniform(-2, 2, 3))
        c = float((scale * rng.uniform(0.2, 3.0)) ** 2 * 10.0 ** rng.uniform(-2, 2))
        ref = O.dbar_rect(am, ap, wm, wp, c)
        for perm in itertools.permutations(range(3)):
            pa = lambda v: [v[k] for k in perm]
            assert O.dbar_rect(pa(am), pa(ap), pa(wm), pa(wp), c) == ref, (trial, perm)


def test_one_ulp_swaps_near_a_source_never_raise_the_result(O):
    """Lower a neighbour by two ulps so that it passes another axis's value:
    the terms change by about as much as one rounding of the sum, which is
    where a sum ordered by neighbour values goes the wrong way."""
    rng = np.random.default_rng(3)
    for trial in range(20000):
        scale = 10.0 ** rng.uniform(-6, 0)
        a = list(rng.uniform(0.0, 1.0, 3) * scale)
        k, j = rng.choice(3, 2, replace=False)
        a[k] = float(np.nextafter(a[j], 2.0))
        wm = list(10.0 ** rng.uniform(-2, 2, 3))
        inf3 = [np.inf] * 3
        c = float((scale * rng.uniform(0.2, 3.0)) ** 2 * 10.0 ** rng.uniform(-2, 2))
        r = O.dbar_rect(a, inf3, wm, [1.0] * 3, c)
        lower = list(a)
        lower[k] = float(np.nextafter(a[j], 0.0))
        assert O.dbar_rect(lower, inf3, wm, [1.0] * 3, c) <= r, trial


def test_stretched_line_accumulates_spacing_over_speed(O):
    """One row: the front crosses cell i in h_i / v, so t(x) = (x - x0) / v up
    to one rounding per step."""
    for ratio in (1.05, 0.97):
        xs = W.stretched_coords(200, 0.25, ratio, x0=3.0)
        f = np.full((1, 1, 200), 3.0)
        t = O.solve_rect(f, xs, np.array([0.0]), None, [0])[0, 0]
        exact = (xs - xs[0]) / 3.0
        rel = np.abs(t[1:] - exact[1:]) / exact[1:]
        assert np.all(rel < 4e-16 * np.arange(1, 200) + 1e-15)


def test_point_source_on_stretched_grids_converges(O):
    """Constant speed, grids stretched geometrically in y and jittered in x:
    the error of t against r / v falls as the grid is refined."""
    errs = []
    for n in (21, 41, 81):
        L = 1.0
        ratio = 1.02 ** (40.0 / (n - 1))
        ys = W.stretched_coords(n, 1.0, ratio)
        ys *= L / ys[-1]
        xs = np.linspace(-L / 2, L / 2, n)
        f = np.full((1, n, n), 2.0)
        c = n // 2
        t = O.solve_rect(f, xs, ys, None, [c])[0]
        X, Y = np.meshgrid(xs - xs[c], ys - ys[0], indexing="xy")
        r = np.hypot(X, Y)
        m = r > 0.2
        errs.append(np.max(np.abs(t[m] - r[m] / 2.0) / (r[m] / 2.0)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.05 and errs[2] < 0.7 * errs[0]


def test_bad_coordinates_rejected(O):
    f = np.ones((1, 4, 5))
    with pytest.raises(O.OracleError):
        O.solve_rect(f, np.array([0.0, 1.0, 1.0, 2.0, 3.0]), np.arange(4.0), None, [0])
    with pytest.raises(O.OracleError):
        O.solve_rect(f, np.array([0.0, 1.0, 0.5, 2.0, 3.0]), np.arange(4.0), None, [0])
    with pytest.raises(O.OracleError):
        O.solve_rect(f, np.array([0.0, 1.0, np.nan, 2.0, 3.0]), np.arange(4.0), None, [0])

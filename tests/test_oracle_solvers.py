"""Pins of the oracle's solve (binary-heap fast marching) against independent
schedules, exact invariants and the continuous problem (no GPU).

* Theorem 1: every schedule of a monotone, causal operator reaches one fixed
  point -> fast marching == topology-driven rounds == fast sweeping ==
  random-order worklists, bitwise;
* the residual metric of Table tab:error is exactly 0 ("true monotonicity");
* exact invariants (symmetry, power-of-two scaling, monotone response to the
  speed, extra sources, causality);
* the continuous limit: point source in a constant medium and the head wave of
  a two-layer medium, with first-order convergence;
* negative control: the explicit formula (Table tab:prec_1's) under random
  order is schedule dependent.
"""
import math

import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def small_cases():
    rng = np.random.default_rng(11)
    out = []
    p = W.point_source_2d(n=21, src=(10, 10))
    out.append(("2d_const", p.field, p.h, p.src, None))
    f = W.blocky_speed(32, 30, rng, block=8)
    src = rng.choice(32 * 30, size=3, replace=False)
    out.append(("2d_blocky_3src", f, 1.0, src, None))
    p = W.layered_3d(12, 10, 8, h=10.0, seed=5, sigma=2.0)
    out.append(("3d_layered", p.field, p.h, p.src, None))
    f = W.random_field((6, 7, 9), rng, 0.5, 5.0)
    src = np.array([3, 200], dtype=np.int64)
    out.append(("3d_random_2src_t0", f, 0.7, src, np.array([0.25, 0.0])))
    f = W.random_field((1, 9, 13), rng, 1.0, 3.0, block=3)
    out.append(("2d_ragged_edge_src", f, 1.0, np.array([0, 9 * 13 - 1]), None))
    return out


CASES = small_cases()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_schedules_agree_bitwise(O, case):
    _, f, h, src, t0 = case
    t_fmm = O.fmm(f, h, src, t0)
    assert np.array_equal(O.sweep_all(f, h, src, t0), t_fmm)
    assert np.array_equal(O.fsm(f, h, src, t0), t_fmm)
    for seed in range(6):
        assert np.array_equal(O.async_random(f, h, src, seed, t0), t_fmm), seed


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_residual_is_exactly_zero(O, case):
    _, f, h, src, t0 = case
    t = O.fmm(f, h, src, t0)
    n, worst = O.residual(t, f, h, src)
    assert n == 0 and worst == 0.0
    assert np.all(np.isfinite(t))


def test_point_source_axis_values_exact(O):
    p = W.point_source_2d()
    t = O.fmm(p.field, p.h, p.src)[0]
    i = np.arange(101)
    assert np.array_equal(t[50, :], np.abs(i - 50).astype(float))
    assert np.array_equal(t[:, 50], np.abs(i - 50).astype(float))
    # D4 symmetry, bitwise
    assert np.array_equal(t, t.T)
    assert np.array_equal(t, t[::-1, :])
    assert np.array_equal(t, t[:, ::-1])
    # first diagonal point: the smallest double above 1 + 1/sqrt(2) meeting the predicate
    assert t[51, 51] == 1.7071067811865477


def test_3d_axis_permutation_symmetry(O):
    rng = np.random.default_rng(3)
    f = W.random_field((7, 7, 7), rng, 0.5, 4.0)
    src = np.array([W.flat_index(2, 3, 5, 7, 7)])
    t = O.fmm(f, 1.0, src)
    # swap x and z (array axes 0 and 2) in the field and the source
    ft = np.ascontiguousarray(f.transpose(2, 1, 0))
    srct = np.array([W.flat_index(5, 3, 2, 7, 7)])
    tt = O.fmm(ft, 1.0, srct)
    assert np.array_equal(tt, t.transpose(2, 1, 0))


def test_power_of_two_scaling_exact(O):
    f, h, src, t0 = CASES[1][1], CASES[1][2], CASES[1][3], None
    t = O.fmm(f, h, src)
    assert np.array_equal(O.fmm(2.0 * f, h, src), t / 2.0)
    assert np.array_equal(O.fmm(f, 2.0 * h, src), t * 2.0)
    # slowness field of the same medium: h * s with s = 1/v is not h / v bitwise,
    # but the slowness path on 1/f == speed path on f when f is a power of two
    f2 = np.full((1, 15, 17), 0.5)
    s = np.array([40])
    assert np.array_equal(O.fmm(f2, 1.0, s), O.fmm(1.0 / f2, 1.0, s, kind=O.SLOWNESS))


def test_slower_medium_never_arrives_earlier(O):
    rng = np.random.default_rng(5)
    f = W.random_field((1, 40, 40), rng, 0.5, 4.0, block=4)
    src = np.array([5 * 40 + 7])
    t = O.fmm(f, 1.0, src)
    slow = f * np.where(rng.random(f.shape) < 0.3, 0.7, 1.0)
    assert np.all(O.fmm(slow, 1.0, src) >= t)


def test_more_sources_never_later_and_joint_below_min(O):
    rng = np.random.default_rng(6)
    f = W.random_field((1, 50, 45), rng, 0.5, 4.0, block=5)
    s1, s2 = 123, 1890
    t1 = O.fmm(f, 1.0, [s1])
    t2 = O.fmm(f, 1.0, [s2])
    tj = O.fmm(f, 1.0, [s1, s2])
    assert np.all(tj <= t1) and np.all(tj <= t2)
    assert np.all(tj <= np.minimum(t1, t2))
    # duplicate source entries: the smaller start time wins
    td = O.fmm(f, 1.0, [s1, s1], t0=[3.0, 0.0])
    assert np.array_equal(td, t1)


def test_causality_invariant(O):
    _, f, h, src, t0 = CASES[3]
    t = O.fmm(f, h, src, t0)
    nz, ny, nx = f.shape
    pad = np.pad(t, 1, constant_values=np.inf)
    mins = np.minimum.reduce([pad[1:-1, 1:-1, :-2], pad[1:-1, 1:-1, 2:], pad[1:-1, :-2, 1:-1],
                              pad[1:-1, 2:, 1:-1], pad[:-2, 1:-1, 1:-1], pad[2:, 1:-1, 1:-1]])
    mask = np.ones(t.shape, bool)
    mask.reshape(-1)[np.asarray(src)] = False
    assert np.all(t[mask] > mins[mask])


def test_continuous_point_source_converges(O):
    """t -> r / v in a constant medium, error O(h log h) for a point source."""
    errs = []
    for n in (41, 81, 161):
        h = 1.0 / (n - 1)
        c = n // 2
        f = np.full((1, n, n), 2.0)
        t = O.fmm(f, h, [c * n + c])[0]
        y, x = np.mgrid[0:n, 0:n]
        r = h * np.hypot(x - c, y - c)
        m = r > 0.2
        errs.append(np.max(np.abs(t[m] - r[m] / 2.0) / (r[m] / 2.0)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.045 and errs[2] < 0.75 * errs[0]


def test_two_layer_head_wave(O):
    """Two flat layers (v1 over v2 > v1, thickness H); beyond the critical
    distance the surface first arrival is the head wave
    x / v2 + 2 H sqrt(1/v1^2 - 1/v2^2)."""
    v1, v2, H, L = 1.0, 3.0, 1.0, 8.0
    errs = []
    for k in (10, 20, 40):
        h = 1.0 / k
        nx, ny = int(L * k) + 1, int(2.5 * k) + 1
        y = np.arange(ny) * h
        f = np.where(y[:, None] < H, v1, v2) * np.ones((ny, nx))
        t = O.fmm(f.reshape(1, ny, nx), h, [0])[0]
        x = np.arange(nx) * h
        far = x > 6.0
        head = x[far] / v2 + 2 * H * math.sqrt(1 / v1 ** 2 - 1 / v2 ** 2)
        errs.append(np.max(np.abs(t[0, far] - head) / head))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.02


def test_explicit_formula_is_schedule_dependent(O):
    """Negative control: with the textbook explicit formula (not monotone in
    floating point) random update orders end in different states, while the
    exactly monotone operator never does."""
    rng = np.random.default_rng(7)
    f = W.blocky_speed(48, 48, rng, block=6, values=(0.5, 0.5860617808911898, 1.0, 2.0, 5.0))
    src = rng.choice(48 * 48, size=3, replace=False)
    base = O.fmm(f, 1.0, src, op=O.OP_DTILDE)
    diffs = 0
    for seed in range(8):
        t = O.async_random(f, 1.0, src, seed, op=O.OP_DTILDE)
        diffs += int(np.count_nonzero(t != base))
    assert diffs > 0
    exact = O.fmm(f, 1.0, src)
    for seed in range(8):
        assert np.array_equal(O.async_random(f, 1.0, src, seed), exact)


def test_resume_from_any_upper_bound_reaches_the_fixed_point(O):
    """Checkpoint / resume (Theorem 1's argument: from any state above the
    fixed point, a maximal sequence of monotone, causal updates ends at it).
    A solve stopped after k pops, resumed (possibly stopped again), equals the
    cold solve bit for bit; so does a resume from the exact solution raised at
    random points, from +inf everywhere, and from a state with holes of +inf."""
    rng = np.random.default_rng(31)
    for _, f, h, src, t0 in CASES:
        ref = O.fmm(f, h, src, t0)
        inf = np.full(f.shape, np.inf)
        t, done = O.fmm_resume(f, h, src, inf, t0)
        assert done and np.array_equal(t, ref)
        for k in (1, 7, f.size // 3):
            part, done = O.fmm_resume(f, h, src, inf, t0, max_pops=k)
            assert not done
            mask = np.ones(f.shape, bool)
            mask.reshape(-1)[np.asarray(src)] = False
            assert np.all(part >= ref) and np.isinf(part[mask]).any()
            part2, _ = O.fmm_resume(f, h, src, part, t0, max_pops=k)
            t, done = O.fmm_resume(f, h, src, part2, t0)
            assert done and np.array_equal(t, ref), k
        up = ref * (1.0 + rng.uniform(0.0, 0.5, f.shape) * (rng.random(f.shape) < 0.3))
        up[rng.random(f.shape) < 0.1] = np.inf
        t, done = O.fmm_resume(f, h, src, up, t0)
        assert done and np.array_equal(t, ref)


def test_resume_rejects_invalid_start(O):
    p = W.point_source_2d(n=9, src=(4, 4))
    bad = np.full(p.field.shape, np.inf)
    bad[0, 0, 0] = np.nan
    with pytest.raises(O.OracleError):
        O.fmm_resume(p.field, p.h, p.src, bad)
    bad[0, 0, 0] = -1.0
    with pytest.raises(O.OracleError):
        O.fmm_resume(p.field, p.h, p.src, bad)

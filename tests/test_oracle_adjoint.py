"""Pins of the oracle's parents record and adjoint (no GPU).

The paper gives no gradient; the adjoint is the implicit derivative of the
discrete equations (Eq. difference_as_root) over the recorded upwind parents.
It is pinned by: a dense linear solve of the same linearised system, central
finite differences of full re-solves, the degree-1 homogeneity identity of
travel times in slowness, and the closed form along a source axis.
"""
import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def tiny_cases():
    rng = np.random.default_rng(21)
    out = []
    f = W.random_field((1, 14, 17), rng, 0.5, 3.0, block=3)
    out.append(("2d", f, 1.0, np.array([3 * 17 + 4]), rng.choice(f.size, 12, replace=False)))
    f = W.random_field((7, 8, 9), rng, 0.8, 2.5, block=2)
    out.append(("3d", f, 0.5, np.array([W.flat_index(4, 4, 0, 9, 8)]), rng.choice(f.size, 20, replace=False)))
    f = W.random_field((1, 12, 12), rng, 1.0, 4.0)
    out.append(("2d_2src", f, 2.0, np.array([0, 143]), rng.choice(f.size, 10, replace=False)))
    return out


CASES = tiny_cases()


def loss_and_g(t, rec, tobs):
    tr = t.reshape(-1)[rec]
    res = tr - tobs
    g = np.zeros(t.size)
    np.add.at(g, rec, res)
    return 0.5 * float(res @ res), g.reshape(t.shape)


def obs_for(O, f, h, src, rec):
    """Observed times from a perturbed medium (the oracle's own solve)."""
    rng = np.random.default_rng(99)
    t = O.fmm(f * (1 + 0.05 * rng.standard_normal(f.shape)).clip(0.5, None), h, src)
    return t.reshape(-1)[rec]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_parents_definition(O, case):
    _, f, h, src, _ = case
    t = O.fmm(f, h, src)
    par = O.parents(t, src)
    nz, ny, nx = t.shape
    ndim = 2 if nz == 1 else 3
    assert np.all(par.reshape(-1)[src] == 0x80)
    for i in range(t.size):
        if i in set(src.tolist()):
            continue
        z, y, x = np.unravel_index(i, t.shape)
        tz = t.reshape(-1)[i]
        b = 0
        for k, (c, n, st) in enumerate(((x, nx, 1), (y, ny, nx), (z, nz, nx * ny))[:ndim]):
            lo = t.reshape(-1)[i - st] if c > 0 else np.inf
            hi = t.reshape(-1)[i + st] if c < n - 1 else np.inf
            if min(lo, hi) < tz:
                b |= (1 if lo <= hi else 2) << (2 * k)
        assert par.reshape(-1)[i] == b
        assert b != 0   # every non-source point has an upwind axis


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_adjoint_matches_dense_solve(O, case):
    _, f, h, src, rec = case
    t = O.fmm(f, h, src)
    par = O.parents(t, src)
    tobs = obs_for(O, f, h, src, rec)
    _, g = loss_and_g(t, rec, tobs)
    grad = O.adjoint(t, par, f, h, g)
    dense = O.dense_adjoint(t, par, f, h, g)
    scale = np.max(np.abs(dense))
    assert scale > 0
    assert np.max(np.abs(grad - dense)) <= 1e-12 * scale
    assert np.all(grad.reshape(-1)[src] == 0.0)


@pytest.mark.parametrize("case", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_adjoint_matches_finite_differences(O, case):
    """Central differences of re-solves with the slowness field; only points
    whose +/- solves keep the same parent record are compared."""
    _, f, h, src, rec = case
    s = 1.0 / f
    t = O.fmm(s, h, src, kind=O.SLOWNESS)
    par = O.parents(t, src)
    tobs = obs_for(O, f, h, src, rec)
    _, g = loss_and_g(t, rec, tobs)
    grad = O.adjoint(t, par, s, h, g, kind=O.SLOWNESS)
    rng = np.random.default_rng(0)
    pts = rng.choice(s.size, 40, replace=False)
    compared = 0
    for i in pts:
        if i in set(src.tolist()):
            continue
        eps = 1e-6 * s.reshape(-1)[i]
        sp, sm = s.copy(), s.copy()
        sp.reshape(-1)[i] += eps
        sm.reshape(-1)[i] -= eps
        tp = O.fmm(sp, h, src, kind=O.SLOWNESS)
        tm = O.fmm(sm, h, src, kind=O.SLOWNESS)
        if not (np.array_equal(O.parents(tp, src), par) and np.array_equal(O.parents(tm, src), par)):
            continue
        Lp, _ = loss_and_g(tp, rec, tobs)
        Lm, _ = loss_and_g(tm, rec, tobs)
        fd = (Lp - Lm) / (2 * eps)
        gi = grad.reshape(-1)[i]
        assert abs(fd - gi) <= 1e-5 * max(abs(gi), 1e-3 * np.max(np.abs(grad))), (i, fd, gi)
        compared += 1
    assert compared >= 10


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_euler_homogeneity_identity(O, case):
    """With zero start times t is homogeneous of degree 1 in slowness, so
    sum_n s_n dL/ds_n = sum_r residual_r * t_r."""
    _, f, h, src, rec = case
    s = 1.0 / f
    t = O.fmm(s, h, src, kind=O.SLOWNESS)
    par = O.parents(t, src)
    tobs = obs_for(O, f, h, src, rec)
    _, g = loss_and_g(t, rec, tobs)
    grad = O.adjoint(t, par, s, h, g, kind=O.SLOWNESS)
    lhs = float(np.sum(s * grad))
    rhs = float(np.sum(g * t))
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


def test_axis_closed_form():
    """Constant unit medium, receiver on the source row: d t_r / d s_k = h on
    every cell of the straight path (source excluded), 0 elsewhere."""
    import oracle as O
    n = 21
    f = np.ones((1, n, n))
    src = np.array([10 * n + 3])
    t = O.fmm(f, 1.0, src)
    par = O.parents(t, src)
    r = 10 * n + 15
    g = np.zeros(f.shape)
    g.reshape(-1)[r] = 1.0
    grad = O.adjoint(t, par, f, 1.0, g).reshape(-1)
    path = np.arange(10 * n + 4, 10 * n + 16)
    assert np.all(grad[path] == 1.0)
    mask = np.ones(grad.size, bool)
    mask[path] = False
    assert np.all(grad[mask] == 0.0)

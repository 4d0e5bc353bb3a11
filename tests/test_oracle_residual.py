"""Pins of the oracle's residual (the error metric of Table "tab:error"), no GPU.

The residual applies the operator once at every non-source point with the
neighbours' values taken from a given state, and reports how many points would
change and the largest relative change |r - t| / |t|.  These tests perturb a
known fixed point in ways whose effect follows from the operator's definition,
so the expected counts and magnitudes are worked out here by hand rather than
by re-running any formula:

* point source in a constant unit medium on a unit grid: the state scaled by
  lambda != 1 moves every non-source point off its operator value; the largest
  relative change sits at the source's axis neighbours, whose operator value is
  exactly 1 (one upwind axis with neighbour 0 and c = 1) while their time is
  lambda, so it is (lambda - 1) / lambda.  A residual that skipped an axis would
  see a different operator value at that axis' source neighbours.
* a point lowered far below its neighbours: the point itself (its operator value
  still comes from the untouched neighbours) and exactly its in-grid neighbours
  (each now has an upwind value far below its own) are counted; nothing else.
  Interior, face, edge and corner points in 3D fix the neighbour count 6/5/4/3,
  so a dropped axis or a wrong boundary test changes the count.
* a raised source value is never counted itself (sources are fixed) but moves
  its axis neighbours.
"""
import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def const_3d(n=9):
    f = np.ones((n, n, n))
    c = n // 2
    src = np.array([W.flat_index(c, c, c, n, n)])
    return f, 1.0, src, c


@pytest.mark.parametrize("lam", [1.0 + 2.0 ** -10, 1.0 - 2.0 ** -7, 1.5])
def test_scaled_state_counts_every_point_2d(O, lam):
    p = W.point_source_2d()
    t = O.fmm(p.field, p.h, p.src)
    assert O.residual(t, p.field, p.h, p.src) == (0, 0.0)
    n, worst = O.residual(t * lam, p.field, p.h, p.src)
    assert n == p.npts - 1
    # at the four axis neighbours of the source: operator value 1, time lam
    assert worst == pytest.approx(abs(lam - 1.0) / lam, rel=1e-14)


@pytest.mark.parametrize("lam", [1.0 + 2.0 ** -10, 1.25])
def test_scaled_state_counts_every_point_3d(O, lam):
    f, h, src, _ = const_3d()
    t = O.fmm(f, h, src)
    assert O.residual(t, f, h, src) == (0, 0.0)
    n, worst = O.residual(t * lam, f, h, src)
    assert n == f.size - 1
    assert worst == pytest.approx(abs(lam - 1.0) / lam, rel=1e-14)


def lowered_count_3d(O, f, h, src, t, x, y, z):
    nz, ny, nx = f.shape
    s = t.copy()
    i = W.flat_index(x, y, z, nx, ny)
    s.reshape(-1)[i] = t.reshape(-1)[i] / 4.0
    return O.residual(s, f, h, src)


@pytest.mark.parametrize("where,expect", [((2, 3, 4), 7), ((0, 3, 4), 6), ((0, 0, 4), 5), ((0, 0, 0), 4)],
                         ids=["interior", "face", "edge", "corner"])
def test_lowered_point_counts_itself_and_its_neighbours_3d(O, where, expect):
    # 8^3 unit grid, source in the far corner so every point below is at least
    # a few cells away: the lowered value t/4 is far below every neighbour
    n = 8
    f = np.ones((n, n, n))
    src = np.array([W.flat_index(n - 1, n - 1, n - 1, n, n)])
    t = O.fmm(f, 1.0, src)
    cnt, worst = lowered_count_3d(O, f, 1.0, src, t, *where)
    assert cnt == expect
    # the lowered point's own relative change: (t - t/4) / (t/4) = 3
    assert worst == pytest.approx(3.0, rel=1e-15)


def test_lowered_point_counts_itself_and_its_neighbours_2d(O):
    p = W.point_source_2d()
    t = O.fmm(p.field, p.h, p.src)[0]
    for (x, y), expect in (((80, 10), 5), ((0, 10), 4), ((0, 0), 3)):
        s = t.copy()
        s[y, x] = t[y, x] / 4.0
        cnt, worst = O.residual(s[None], p.field, p.h, p.src)
        assert cnt == expect, (x, y)
        assert worst == pytest.approx(3.0, rel=1e-15)


def test_raised_source_is_not_counted_but_moves_its_neighbours(O):
    p = W.point_source_2d()
    t = O.fmm(p.field, p.h, p.src)
    s = t.copy()
    s.reshape(-1)[p.src[0]] = 3.0
    cnt, _ = O.residual(s, p.field, p.h, p.src)
    assert cnt == 4
    f, h, src, _ = const_3d()
    t = O.fmm(f, h, src)
    s = t.copy()
    s.reshape(-1)[src[0]] = 3.0
    assert O.residual(s, f, h, src)[0] == 6


def test_symmetric_sources_tie_to_the_minus_side(O):
    """Two sources mirrored about the column x = 20 of a unit medium: the
    solution is mirror-symmetric bit for bit (one fixed point, symmetric
    equations), so every point of that column has equal x neighbours, both
    upwind (each is nearer to one source).  The parent record must mark the x
    axis active with the minus-side neighbour there (the tie rule), and the
    plus side never."""
    ny, nx = 31, 41
    f = np.ones((1, ny, nx))
    src = np.array([15 * nx + 10, 15 * nx + 30])
    t = O.fmm(f, 1.0, src)
    assert np.array_equal(t, t[:, :, ::-1])
    par = O.parents(t, src)[0]
    col = par[:, 20]
    assert np.all(col & 3 == 1)
    # off the mirror line the x parent points towards the nearer source
    assert np.all(par[15, 11:20] & 3 == 1) and np.all(par[15, 21:30] & 3 == 2)

"""GPU parity of the rectilinear-grid solve (eik_solve_rect) against the CPU
oracle, through the C ABI.

The operator is the exactly monotone construction of the section "Achieving
Exact Monotonicity with Finite Precision Arithmetic" applied to the upwind
scheme with spacings that vary per axis and index (the irregular-grid case the
conclusion names).  It is monotone and causal, so Theorem 1 makes every
schedule reach the same bits: the bar is bitwise equality with the oracle's
fast marching on the same coordinates, and with the uniform solve (h = 1) for
unit spacing.
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def gpu_rect(eik, field, xs, ys, zs, src, t0=None, kind="speed", **kw):
    f = torch.from_numpy(np.ascontiguousarray(field)).cuda()
    if zs is None:
        f = f[0]
    t = eik.solve_rect(f, xs, ys, zs, torch.as_tensor(np.asarray(src), dtype=torch.int64),
                       t0=None if t0 is None else np.asarray(t0, dtype=np.float64), kind=kind, **kw)
    torch.cuda.synchronize()
    return t.cpu().numpy().reshape(field.shape)


def assert_bitwise(a, b, what=""):
    if not np.array_equal(a, b):
        bad = np.argwhere(a != b)
        i = tuple(bad[0])
        raise AssertionError(f"{what}: {len(bad)} mismatches, first at {i}: {a[i]!r} vs {b[i]!r}")


def cases():
    rng = np.random.default_rng(2024)
    out = []
    # several tiles in every direction with a ragged tail, two sources with offsets
    f = W.random_field((19, 29, 37), rng, 0.5, 5.0, block=3)
    xs, ys, zs = W.jittered_coords(37, 1.0, rng), W.stretched_coords(29, 0.4, 1.06), W.jittered_coords(19, 2.0, rng, 0.5)
    out.append(("3d_37x29x19_jitter_stretch", f, xs, ys, zs, np.array([W.flat_index(3, 20, 4, 37, 29), 9000]),
                np.array([0.0, 0.75]), 0))
    # strong anisotropy: spacings from 0.05 to several units
    f = 1.0 / W.random_field((13, 17, 45), rng, 0.5, 5.0, block=2)
    xs, ys, zs = W.stretched_coords(45, 0.05, 1.12), W.jittered_coords(17, 3.0, rng), W.stretched_coords(13, 2.0, 0.85)
    out.append(("3d_45x17x13_slowness_anisotropic", f, xs, ys, zs, np.array([0, f.size - 1]), None, 1))
    f = W.random_field((1, 77, 101), rng, 0.5, 5.0, block=4)
    xs, ys = W.jittered_coords(101, 0.5, rng), W.stretched_coords(77, 0.1, 1.04)
    out.append(("2d_101x77", f, xs, ys, None, np.array([3, 5000]), None, 0))
    f = W.random_field((1, 1, 300), rng, 0.5, 2.0)
    out.append(("2d_300x1", f, W.stretched_coords(300, 0.25, 1.01), np.array([7.0]), None, np.array([150]), None, 0))
    f = W.random_field((2, 2, 2), rng, 1.0, 2.0)
    out.append(("3d_2x2x2", f, np.array([0.0, 0.3]), np.array([1.0, 4.0]), np.array([-2.0, -1.5]), np.array([0]),
                None, 0))
    return out


CASES = cases()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_rect_matches_oracle(gpu, O, case):
    name, f, xs, ys, zs, src, t0, kind = case
    ref = O.solve_rect(f, xs, ys, zs, src, t0=t0, kind=kind)
    kname = "slowness" if kind else "speed"
    tiles = [None] + ([(8, 8, 8), (16, 8, 4), (8, 4, 4)] if zs is not None else [(32, 32), (16, 8)])
    for tile in tiles:
        for delta in (0.0, 0.3, 1e6):
            t = gpu_rect(gpu, f, xs, ys, zs, src, t0=t0, kind=kname, tile=tile, delta=delta)
            assert_bitwise(t, ref, f"{name} tile {tile} delta {delta}")


TILES_3D = [(32, 8, 4), (16, 8, 8), (8, 8, 8), (64, 4, 4), (16, 8, 4), (8, 8, 4), (8, 4, 4)]
TILES_2D = [(64, 16), (32, 32), (128, 8), (16, 16), (16, 8)]


def test_every_tile_shape(gpu, O):
    """Every supported tile shape (3D tiles of 1024 points run on 512-thread
    blocks, two points a thread), ragged in every direction, with sources at
    offsets, a slowness field in 2D."""
    rng = np.random.default_rng(31)
    f = W.random_field((11, 21, 70), rng, 0.5, 5.0, block=3)
    xs, ys, zs = W.jittered_coords(70, 1.0, rng), W.stretched_coords(21, 0.6, 1.05), W.jittered_coords(11, 1.5, rng)
    src = np.array([W.flat_index(40, 3, 9, 70, 21), 17])
    t0 = np.array([0.0, 2.5])
    ref = O.solve_rect(f, xs, ys, zs, src, t0=t0)
    for tile in TILES_3D:
        assert_bitwise(gpu_rect(gpu, f, xs, ys, zs, src, t0=t0, tile=tile, delta=0.4), ref, f"3D tile {tile}")
    g = 1.0 / W.random_field((1, 45, 150), rng, 0.5, 5.0, block=5)
    gx, gy = W.stretched_coords(150, 0.2, 1.01), W.jittered_coords(45, 0.5, rng)
    gsrc = np.array([W.flat_index(75, 44, 0, 150, 45)])
    gref = O.solve_rect(g, gx, gy, None, gsrc, kind=1)
    for tile in TILES_2D:
        assert_bitwise(gpu_rect(gpu, g, gx, gy, None, gsrc, kind="slowness", tile=tile, delta=0.3), gref,
                       f"2D tile {tile}")


def test_unit_spacing_is_the_uniform_solve(gpu, O):
    rng = np.random.default_rng(7)
    for shape in ((21, 40, 50), (1, 90, 70)):
        f = W.random_field(shape, rng, 0.5, 5.0, block=3)
        nz, ny, nx = shape
        src = rng.choice(f.size, 3, replace=False)
        zs = None if nz == 1 else np.arange(nz, dtype=np.float64)
        t = gpu_rect(gpu, f, np.arange(nx, dtype=np.float64), np.arange(ny, dtype=np.float64), zs, src)
        fd = torch.from_numpy(f).cuda()
        if nz == 1:
            fd = fd[0]
        u = gpu.solve(fd, 1.0, torch.as_tensor(src)).cpu().numpy().reshape(shape)
        assert_bitwise(t, u, f"unit spacing {shape}")
        assert_bitwise(t, O.fmm(f, 1.0, src), f"unit spacing vs oracle {shape}")


def test_schedule_options_and_warm_start(gpu, O):
    rng = np.random.default_rng(8)
    f = W.random_field((24, 40, 48), rng, 0.5, 5.0, block=4)
    xs, ys, zs = W.jittered_coords(48, 1.0, rng), W.jittered_coords(40, 0.7, rng), W.stretched_coords(24, 0.5, 1.05)
    src = np.array([W.flat_index(10, 30, 12, 48, 40)])
    ref = O.solve_rect(f, xs, ys, zs, src)
    for kw in (dict(horizon=1, delta=0.5), dict(lookahead=3, delta=0.2), dict(grid_blocks=7),
               dict(lookahead=16, delta=0.02, tile=(8, 8, 4))):
        assert_bitwise(gpu_rect(gpu, f, xs, ys, zs, src, **kw), ref, str(kw))
    # warm start from an upper bound (the sources are fixed again whatever the
    # start holds there) and from a solve stopped by the visit cap
    fd = torch.from_numpy(f).cuda()
    sd = torch.as_tensor(src)
    start = torch.from_numpy(ref * 1.5 + 0.25).cuda()
    t = gpu.solve_rect(fd, xs, ys, zs, sd, out=start, warm_start=True)
    assert_bitwise(t.cpu().numpy(), ref, "warm start from a raised solution")
    t = gpu.solve_rect(fd, xs, ys, zs, sd, tile=(8, 8, 8), max_tile_visits=2, check_status=False)
    assert gpu.status(raise_on_error=False).status == -5
    part = t.cpu().numpy()
    assert np.all(part >= ref) and np.isinf(part).any()
    gpu.solve_rect(fd, xs, ys, zs, sd, tile=(16, 8, 4), delta=0.3, out=t, warm_start=True)
    assert_bitwise(t.cpu().numpy(), ref, "resume after the visit cap")


def test_medium_grid_residual_is_zero(gpu, O):
    """96x80x64 stretched grid with many tiles: the oracle re-applies the
    operator at every point of the GPU result and finds nothing to change, and
    the result is the oracle's fast marching bit for bit."""
    rng = np.random.default_rng(9)
    f = W.random_field((64, 80, 96), rng, 1500.0, 6000.0, block=8)
    xs, ys, zs = W.stretched_coords(96, 5.0, 1.01), W.jittered_coords(80, 8.0, rng), W.stretched_coords(64, 2.0, 1.03)
    src = np.array([W.flat_index(48, 40, 0, 96, 80), W.flat_index(5, 70, 63, 96, 80)])
    t = gpu_rect(gpu, f, xs, ys, zs, src, delta=0.002)
    assert np.all(np.isfinite(t))
    assert O.residual_rect(t, f, xs, ys, zs, src) == (0, 0.0)
    assert_bitwise(t, O.solve_rect(f, xs, ys, zs, src), "96x80x64 stretched")


def test_bad_coordinates_raise(gpu):
    f = torch.ones(4, 5, dtype=torch.float64, device="cuda")
    from paper_2103_05694_amd._lib import EikError
    with pytest.raises(EikError):
        gpu.solve_rect(f, [0.0, 1.0, 1.0, 2.0, 3.0], np.arange(4.0), sources=[0])
    with pytest.raises(ValueError):
        gpu.solve_rect(f, np.arange(4.0), np.arange(4.0), sources=[0])


def test_rect_tuner_candidates_agree(gpu):
    """The rectilinear tuner times each (tile, width, lookahead) candidate,
    refines the best width, and refuses any candidate that changes the bits."""
    from paper_2103_05694_amd import autotune
    rng = np.random.default_rng(12)
    f = W.random_field((28, 36, 40), rng, 1500.0, 6000.0, block=4)
    xs, ys, zs = W.jittered_coords(40, 10.0, rng), W.jittered_coords(36, 10.0, rng), W.stretched_coords(28, 5.0, 1.05)
    src = torch.tensor([W.flat_index(20, 18, 0, 40, 36)])
    e = autotune.tune_rect(torch.from_numpy(f).cuda(), xs, ys, zs, src, tiles=[(8, 8, 8), (8, 8, 4)],
                           delta_factors=(0.25, 1.0), lookaheads=(0, 8), reps=1, save=False, log=lambda s: None)
    assert len(e["candidates"]) == 2 * 2 * 2 + 2
    assert tuple(e["tile"]) in ((8, 8, 8), (8, 8, 4)) and e["lookahead"] in (0, 8)
    assert e["ms"] == min(c["ms"] for c in e["candidates"])

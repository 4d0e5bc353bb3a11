"""GPU parity of the forward solve against the CPU oracle, through the C ABI.

Bar: bitwise equality of arrival times (the operator is exactly monotone, so
every schedule reaches the same fixed point, Theorem 1).  At the full
512x512x256 size the oracle's sequential solve is too slow for a test, so the
full-size check is the fixed-point residual: the oracle re-applies the operator
at every point of the GPU result and must find nothing to change.  A state with
zero residual and the given sources is the unique fixed point (same causality
argument as the uniqueness part of Theorem 1), hence equal to the oracle's.
"""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

TILES_3D = [(32, 8, 4), (16, 8, 8), (8, 8, 8), (64, 4, 4), (16, 8, 4), (8, 8, 4), (8, 4, 4)]
TILES_2D = [(64, 16), (32, 32), (128, 8), (16, 16), (16, 8)]


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def gpu_solve(eik, field, h, src, t0=None, kind="speed", **kw):
    f = torch.from_numpy(np.ascontiguousarray(field)).cuda()
    if f.shape[0] == 1 and f.dim() == 3 and kw.pop("as2d", True):
        f = f[0]
    t = eik.solve(f, h, torch.as_tensor(np.asarray(src), dtype=torch.int64),
                  t0=None if t0 is None else torch.as_tensor(np.asarray(t0, dtype=np.float64)),
                  kind=kind, **kw)
    torch.cuda.synchronize()
    return t.cpu().numpy().reshape(field.shape)


def assert_bitwise(a, b, what=""):
    if not np.array_equal(a, b):
        bad = np.argwhere(a != b)
        i = tuple(bad[0])
        rel = np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))
        raise AssertionError(f"{what}: {len(bad)} mismatches, first at {i}: {a[i]!r} vs {b[i]!r}, "
                             f"max rel {rel:.3e}")


def test_point_source_101(gpu, O):
    p = W.point_source_2d()
    ref = O.fmm(p.field, p.h, p.src)
    for tile in TILES_2D:
        t = gpu_solve(gpu, p.field, p.h, p.src, tile=tile)
        assert_bitwise(t, ref, f"101^2 tile {tile}")
    i = np.arange(101)
    assert np.array_equal(t[0, 50], np.abs(i - 50).astype(float))


def ragged_cases():
    rng = np.random.default_rng(123)
    cases = []
    f = W.random_field((11, 29, 37), rng, 0.5, 5.0, block=3)
    cases.append(("3d_37x29x11_3src_t0", f, 0.8, np.array([0, 5000, f.size - 1]), np.array([0.0, 1.5, 0.25])))
    f = W.random_field((1, 77, 101), rng, 0.5, 5.0, block=4)
    cases.append(("2d_101x77_2src", f, 1.0, np.array([3, 7000]), None))
    f = W.random_field((3, 1, 5), rng, 1.0, 2.0)
    cases.append(("3d_5x1x3", f, 1.0, np.array([7]), None))
    f = W.random_field((1, 1, 1), rng, 1.0, 2.0)
    cases.append(("2d_1x1", f, 1.0, np.array([0]), None))
    f = W.random_field((1, 1, 300), rng, 0.5, 2.0)
    cases.append(("2d_300x1", f, 1.0, np.array([150]), None))
    f = W.random_field((2, 2, 2), rng, 1.0, 2.0)
    cases.append(("3d_2x2x2_dup", f, 1.0, np.array([0, 0, 7]), np.array([2.0, 0.5, 0.0])))
    f = W.random_field((9, 33, 65), rng, 0.5, 5.0)
    cases.append(("3d_65x33x9_every_8th_src", f, 1.0, np.arange(0, f.size, 997), None))
    return cases


CASES = ragged_cases()


@pytest.fixture(scope="module")
def layered_small():
    return W.layered_3d(96, 80, 48, h=10.0, seed=2)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_ragged_and_degenerate_shapes(gpu, O, case):
    name, f, h, src, t0 = case
    ref = O.fmm(f, h, src, t0)
    tiles = TILES_2D if f.shape[0] == 1 else TILES_3D
    for tile in tiles:
        for delta, la, hz, pk in ((0.0, 0, 0, False), (0.5, 0, 0, True), (0.25, 3, 0, False), (0.25, 0, 1, True),
                                  (0.5, 2, 2, False), (0.0, 1, 0, True), (0.125, 16, 1, False)):
            t = gpu_solve(gpu, f, h, src, t0, tile=tile, delta=delta, lookahead=la, horizon=hz, packed=pk)
            assert_bitwise(t, ref, f"{name} tile {tile} delta {delta} lookahead {la} horizon {hz} packed {pk}")


def test_slowness_field(gpu, O):
    rng = np.random.default_rng(5)
    s = 1.0 / W.random_field((8, 20, 24), rng, 0.5, 5.0)
    src = np.array([100])
    ref = O.fmm(s, 2.0, src, kind=O.SLOWNESS)
    t = gpu_solve(gpu, s, 2.0, src, kind="slowness")
    assert_bitwise(t, ref, "slowness")


@pytest.mark.parametrize("tile", TILES_3D)
def test_layered_3d_scaled(gpu, O, layered_small, tile):
    p = layered_small
    ref = O.fmm(p.field, p.h, p.src)
    for delta, la, pk in ((0.0, 0, False), (0.02, 0, False), (0.02, 0, True), (0.02, 2, True), (0.2, 1, False),
                          (0.005, 8, True), (0.0025, 16, False)):
        t = gpu_solve(gpu, p.field, p.h, p.src, tile=tile, delta=delta, lookahead=la, packed=pk)
        assert_bitwise(t, ref, f"layered tile {tile} delta {delta} lookahead {la} packed {pk}")


@pytest.mark.parametrize("tile", TILES_2D)
def test_blocky_2d_scaled(gpu, O, tile):
    p = W.blocky_2d(n=512, nsrc=16, seed=3, block=16)
    ref = O.fmm(p.field, p.h, p.src)
    for delta, la, pk in ((0.0, 0, False), (4.0, 0, True), (4.0, 4, False), (64.0, 1, True), (1.0, 16, True)):
        t = gpu_solve(gpu, p.field, p.h, p.src, tile=tile, delta=delta, lookahead=la, packed=pk)
        assert_bitwise(t, ref, f"blocky tile {tile} delta {delta} lookahead {la} packed {pk}")


def test_run_to_run_determinism(gpu, O, layered_small):
    p = layered_small
    ref = O.fmm(p.field, p.h, p.src)
    f = torch.from_numpy(p.field).cuda()
    src = torch.as_tensor(p.src)
    out = torch.empty_like(f)
    for i in range(20):
        gpu.solve(f, p.h, src, delta=0.05, out=out)
        assert_bitwise(out.cpu().numpy(), ref, f"run {i}")


def bench_config(shape, kind="speed"):
    """The launch configuration the benchmark times (the tuning cache), or
    none (library defaults)."""
    from paper_2103_05694_amd import autotune
    cfg = autotune.lookup(shape, kind)
    if not cfg:
        return {}
    return dict(tile=tuple(cfg["tile"]), delta=cfg["delta"], grid_blocks=int(cfg.get("grid_blocks", 0)),
                horizon=int(cfg.get("horizon", 0)), packed=bool(cfg.get("packed", False)),
                lookahead=int(cfg.get("lookahead", 0)))


def test_blocky_full_4096(gpu, O):
    """4096^2 with 16 sources, bitwise against the oracle in the tuned launch
    configuration and in a different schedule."""
    p = W.blocky_2d()
    ref = O.fmm(p.field, p.h, p.src)
    for kw in (bench_config((4096, 4096)), dict(delta=32.0)):
        t = gpu_solve(gpu, p.field, p.h, p.src, **kw)
        assert_bitwise(t, ref, f"4096^2 blocky 16 sources {kw}")


def test_layered_half_size_bitwise(gpu, O):
    p = W.layered_3d(256, 256, 128, h=10.0, seed=2)
    ref = O.fmm(p.field, p.h, p.src)
    t = gpu_solve(gpu, p.field, p.h, p.src, delta=0.05)
    assert_bitwise(t, ref, "256x256x128 layered")


def test_layered_full_size_fixed_point(gpu, O):
    """512x512x256: zero residual at every point (unique fixed point), exact
    source value, determinism over repeated runs."""
    p = W.layered_3d()
    f = torch.from_numpy(p.field).cuda()
    src = torch.as_tensor(p.src)
    # the launch configuration the benchmark times
    cfg = bench_config(p.field.shape)
    t1 = gpu.solve(f, p.h, src, **cfg).cpu().numpy()
    n, worst = O.residual(t1, p.field, p.h, p.src)
    assert n == 0 and worst == 0.0
    # bit for bit the oracle's solution (its stored hash, which the benchmark checks too)
    import hashlib
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "layered_512x512x256_seed2.json")) as fh:
        golden = json.load(fh)
    assert p.sha256() == golden["input_sha256_16"]
    assert hashlib.sha256(np.ascontiguousarray(t1, dtype="<f8").tobytes()).hexdigest() == golden["times_sha256"]
    assert t1.reshape(-1)[p.src[0]] == 0.0
    assert np.all(np.isfinite(t1))
    t2 = gpu.solve(f, p.h, src, **cfg).cpu().numpy()
    assert_bitwise(t2, t1, "repeat full size")
    # another schedule reaches the same bits
    t3 = gpu.solve(f, p.h, src, delta=0.05).cpu().numpy()
    assert_bitwise(t3, t1, "other schedule full size")


def test_parents_match_oracle(gpu, O):
    rng = np.random.default_rng(8)
    for shape, src in (((1, 60, 70), [5, 3000]), ((12, 20, 33), [77])):
        f = W.random_field(shape, rng, 0.5, 4.0, block=2)
        ref_t = O.fmm(f, 1.0, src)
        ref_p = O.parents(ref_t, np.array(src))
        ft = torch.from_numpy(f).cuda()
        if shape[0] == 1:
            ft = ft[0]
        t, par = gpu.solve(ft, 1.0, torch.tensor(src), parents=True)
        assert_bitwise(t.cpu().numpy().reshape(shape), ref_t, "t")
        assert np.array_equal(par.cpu().numpy().reshape(shape), ref_p)
        par2 = gpu.parents_of(t, torch.tensor(src))
        assert np.array_equal(par2.cpu().numpy().reshape(shape), ref_p)


def test_parents_on_exact_ties(gpu, O):
    """Parents where the two neighbours on an axis are equal bit for bit: two
    sources mirrored about a column of a unit medium (2D), and a point source
    in the middle of a constant 3D medium, whose solution has exact mirror
    symmetry on every axis.  The GPU record (in-kernel and eik_parents) equals
    the oracle's, tie rule included."""
    cases = []
    ny, nx = 31, 41
    cases.append((np.ones((1, ny, nx)), np.array([15 * nx + 10, 15 * nx + 30])))
    cases.append((np.ones((1, 101, 101)), np.array([50 * 101 + 50])))
    n = 17
    cases.append((np.full((n, n, n), 2.0), np.array([W.flat_index(8, 8, 8, n, n)])))
    for f, src in cases:
        shape = f.shape
        ref_t = O.fmm(f, 1.0, src)
        ref_p = O.parents(ref_t, src)
        assert np.array_equal(ref_t, ref_t[..., ::-1])
        ft = torch.from_numpy(f).cuda()
        if shape[0] == 1:
            ft = ft[0]
        tiles = [(32, 32), (16, 8)] if shape[0] == 1 else [(8, 8, 8), (16, 8, 4)]
        for tile in tiles:
            t, par = gpu.solve(ft, 1.0, torch.tensor(src), parents=True, tile=tile, delta=1.0)
            assert_bitwise(t.cpu().numpy().reshape(shape), ref_t, f"t {shape} {tile}")
            assert np.array_equal(par.cpu().numpy().reshape(shape), ref_p), f"parents {shape} {tile}"
            par2 = gpu.parents_of(t, torch.tensor(src))
            assert np.array_equal(par2.cpu().numpy().reshape(shape), ref_p), f"eik_parents {shape} {tile}"


def test_domain_error_reported(gpu):
    f = torch.ones(16, 16, dtype=torch.float64, device="cuda")
    f[3, 4] = 0.0
    with pytest.raises(gpu.EikError) as e:
        gpu.solve(f, 1.0, torch.tensor([0]))
    assert e.value.code == -2
    f[3, 4] = float("nan")
    with pytest.raises(gpu.EikError):
        gpu.solve(f, 1.0, torch.tensor([0]))
    # the next good solve on the same stream is unaffected
    f[3, 4] = 1.0
    t = gpu.solve(f, 1.0, torch.tensor([0]))
    assert float(t[15, 15]) > 0


def test_bad_source_reported_from_device(gpu):
    import ctypes
    from paper_2103_05694_amd import _lib
    L = _lib.load()
    f = torch.ones(8, 8, dtype=torch.float64, device="cuda")
    t = torch.empty_like(f)
    src = torch.tensor([5, 64], dtype=torch.int64, device="cuda")   # 64 is out of range
    g = _lib.eik_grid(2, 8, 8, 1, 1.0, 0)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.eik_solve(ctypes.byref(g), f.data_ptr(), 2, src.data_ptr(), None, t.data_ptr(), None,
                       None, stream) == 0
    assert L.eik_status(stream, None) == -7
    t0 = torch.tensor([-1.0], dtype=torch.float64, device="cuda")
    src1 = torch.tensor([5], dtype=torch.int64, device="cuda")
    assert L.eik_solve(ctypes.byref(g), f.data_ptr(), 1, src1.data_ptr(), t0.data_ptr(), t.data_ptr(),
                       None, None, stream) == 0
    assert L.eik_status(stream, None) == -7


def test_visit_cap_gives_upper_bound(gpu, O):
    p = W.layered_3d(64, 64, 32, h=10.0, seed=4)
    ref = O.fmm(p.field, p.h, p.src)
    f = torch.from_numpy(p.field).cuda()
    with pytest.raises(gpu.EikError) as e:
        gpu.solve(f, p.h, torch.as_tensor(p.src), max_tile_visits=5)
    assert e.value.code == -5
    t = gpu.solve(f, p.h, torch.as_tensor(p.src), max_tile_visits=5, check_status=False)
    st = gpu.status(raise_on_error=False)
    assert st.status == -5
    t = t.cpu().numpy()
    assert np.all(t >= ref)
    assert np.isinf(t).any()
    assert t.reshape(-1)[p.src[0]] == 0.0


@pytest.mark.parametrize("horizon", [1, 2, 4])
def test_bucket_horizon(gpu, O, layered_small, horizon):
    """A run that settles only values below (its bucket + k) and requeues the
    tile for the rest reaches the same bits for any k and bucket width."""
    p = layered_small
    ref = O.fmm(p.field, p.h, p.src)
    for tile in ((16, 8, 8), (8, 8, 8)):
        for delta in (0.005, 0.02, 0.1):
            t = gpu_solve(gpu, p.field, p.h, p.src, tile=tile, delta=delta, horizon=horizon)
            assert_bitwise(t, ref, f"horizon {horizon} tile {tile} delta {delta}")
    b = W.blocky_2d(512, nsrc=6, seed=7)
    refb = O.fmm(b.field, b.h, b.src)
    for delta in (1.0, 8.0):
        t = gpu_solve(gpu, b.field, b.h, b.src, tile=(32, 32), delta=delta, horizon=horizon)
        assert_bitwise(t, refb, f"blocky horizon {horizon} delta {delta}")


def test_timeline_records_bucket_advances(gpu, layered_small):
    """EIK_FLAG_TIMELINE: one entry per advance of the lowest open bucket, in
    increasing bucket order and time, all within the launch's span."""
    p = layered_small
    f = torch.from_numpy(p.field).cuda()
    gpu.solve(f, p.h, torch.as_tensor(p.src), tile=(8, 8, 8), delta=0.02, timeline=True)
    st = gpu.status()
    t, b, span = gpu.timeline()
    assert len(t) == st.bucket_advances > 5
    assert np.all(np.diff(b) > 0) and b[0] >= 1
    assert np.all(np.diff(t) >= 0) and 0 < t[-1] <= span
    # no bucket beyond the one holding the largest time is ever opened
    tmax = float(gpu.solve(f, p.h, torch.as_tensor(p.src), tile=(8, 8, 8), delta=0.02).max())
    assert b[-1] <= int(tmax * 50.0) + 1


def test_autotune_candidates_agree(gpu, layered_small):
    """The tuner times each candidate and refuses any that changes the bits."""
    from paper_2103_05694_amd import autotune
    p = W.layered_3d(40, 36, 28, h=10.0, seed=4, sigma=3.0)
    f = torch.from_numpy(p.field).cuda()
    e = autotune.tune(f, p.h, torch.as_tensor(p.src), tiles=[(8, 8, 8), (16, 8, 8)],
                      delta_factors=(0.0, 1.0, 4.0), grid_blocks=(0, 64), horizons=(0, 1), packed=(False, True),
                      lookaheads=(2, 5), lookahead_factors=(0.5,), reps=1, save=False, log=lambda s: None)
    # tiles x (bucket width 0: grid sizes + other widths: horizons x grid sizes) x pass structures
    grid = 2 * (1 * 2 + 2 * 2 * 2) * 2
    # then the best of each tile and pass structure with every (lookahead, width) pair
    window = e["candidates"][grid:grid + 2 * 2 * 2]
    assert [c["lookahead"] for c in window] == [2, 5] * 4
    assert [c["packed"] for c in window] == [False, False, True, True] * 2
    assert all(c["lookahead"] == 0 for c in e["candidates"][:grid])
    # the best bucket width is refined at 2^(+-1/2) of its factor unless it was 0
    extra = e["candidates"][grid + 8:]
    assert len(e["candidates"]) in (grid + 8, grid + 10)
    assert all(c["delta_factor"] not in (0.0, 1.0, 4.0, 0.5) for c in extra)
    assert e["lookahead"] in (0, 2, 5)
    assert tuple(e["tile"]) in ((8, 8, 8), (16, 8, 8))


EXTREME = [((1, 70, 90), 1.0, 0), ((1, 64, 64), 1e-7, 1), ((12, 20, 33), 3.5e5, 0), ((9, 17, 26), 1.0, 1)]


@pytest.mark.parametrize("shape,h,kind", EXTREME, ids=[f"{s[0]}x{s[1]}x{s[2]}_h{h:g}_k{k}" for s, h, k in EXTREME])
def test_extreme_contrast_bitwise(gpu, O, shape, h, kind):
    """Speeds log-uniform over twelve orders of magnitude, point by point, and
    grid steps from 1e-7 to 3.5e5: neighbouring times differ by many orders,
    so the exact operator's closed-form first guess can land far from the
    answer and the search fallback decides.  Bitwise against the oracle for
    both field kinds."""
    rng = np.random.default_rng(41 + shape[1])
    f = 10.0 ** rng.uniform(-6.0, 6.0, size=shape)
    src = rng.choice(f.size, 3, replace=False).astype(np.int64)
    ref = O.fmm(f, h, src, kind=kind)
    assert np.all(np.isfinite(ref))
    kname = "speed" if kind == 0 else "slowness"
    q = h / f if kind == 0 else h * f
    tiles = [(32, 32), (16, 16)] if shape[0] == 1 else [(8, 8, 8), (16, 8, 8), (8, 4, 4)]
    for tile in tiles:
        for delta in (0.0, 4.0 * float(np.median(q))):
            t = gpu_solve(gpu, f, h, src, kind=kname, tile=tile, delta=delta)
            assert_bitwise(t, ref, f"tile {tile} delta {delta:g}")


def test_every_point_a_source(gpu, O):
    """Degenerate case: every point is fixed, so nothing is updated and the
    output is t0 bit for bit (zeros included)."""
    rng = np.random.default_rng(61)
    for shape in ((1, 33, 47), (5, 9, 17)):
        f = W.random_field(shape, rng, 0.5, 2.0)
        src = np.arange(f.size, dtype=np.int64)
        t0 = rng.uniform(0.0, 10.0, f.size)
        t0[::7] = 0.0
        ref = O.fmm(f, 1.0, src, t0)
        assert np.array_equal(ref.reshape(-1), t0)
        tiles = [(32, 32), (16, 16)] if shape[0] == 1 else [(8, 8, 8), (16, 8, 8)]
        for tile in tiles:
            t = gpu_solve(gpu, f, 1.0, src, t0, tile=tile, delta=0.5)
            assert_bitwise(t, ref, f"{shape} tile {tile}")


def test_plane_of_sources_with_mixed_t0(gpu, O):
    """A whole surface plane of sources whose start times span six orders of
    magnitude: the front starts everywhere at once, out of order."""
    rng = np.random.default_rng(62)
    f = W.random_field((20, 24, 40), rng, 0.5, 4.0, block=4)
    iy, ix = np.meshgrid(np.arange(24), np.arange(40), indexing="ij")
    src = W.flat_index(ix.ravel(), iy.ravel(), 0, 40, 24)
    t0 = 10.0 ** rng.uniform(-3.0, 3.0, src.size)
    ref = O.fmm(f, 1.0, src, t0)
    for tile in ((8, 8, 8), (16, 8, 8), (32, 8, 4)):
        for delta in (0.0, 0.5, 20.0):
            t = gpu_solve(gpu, f, 1.0, src, t0, tile=tile, delta=delta)
            assert_bitwise(t, ref, f"tile {tile} delta {delta}")


def test_warm_start_resumes_to_the_same_bits(gpu, O, layered_small):
    """EIK_FLAG_WARM_START (checkpoint / resume, Theorem 1's argument): a solve
    stopped by the visit cap leaves an upper bound; resuming from it, or from
    any other upper bound, gives the cold solve's bits."""
    p = layered_small
    ref = O.fmm(p.field, p.h, p.src)
    f = torch.from_numpy(p.field).cuda()
    src = torch.as_tensor(p.src)
    for tile, delta, la, pk in (((8, 8, 8), 0.02, 0, False), ((16, 8, 8), 0.0, 0, False), ((8, 4, 4), 0.005, 0, False),
                                ((16, 8, 8), 0.004, 16, True)):
        kw = dict(tile=tile, delta=delta, lookahead=la, packed=pk)
        # caps below the tile count (360 tiles of 16x8x8) leave unvisited tiles at +inf
        for cap in ((3, 60, 400) if la == 0 else (3, 60, 150)):
            t = gpu.solve(f, p.h, src, max_tile_visits=cap, check_status=False, **kw)
            assert gpu.status(raise_on_error=False).status == -5
            part = t.cpu().numpy()
            assert np.all(part >= ref) and np.isinf(part).any()
            # stop once more, then finish
            gpu.solve(f, p.h, src, max_tile_visits=cap, out=t, warm_start=True, check_status=False, **kw)
            gpu.status(raise_on_error=False)
            gpu.solve(f, p.h, src, out=t, warm_start=True, **kw)
            assert_bitwise(t.cpu().numpy(), ref, f"resume {kw} cap {cap}")
    # from the oracle's own partial solve, from a raised exact solution, from +inf
    rng = np.random.default_rng(17)
    part, done = O.fmm_resume(p.field, p.h, p.src, np.full(p.field.shape, np.inf), max_pops=p.npts // 4)
    assert not done
    up = ref * (1.0 + rng.uniform(0.0, 0.3, ref.shape) * (rng.random(ref.shape) < 0.2))
    up[rng.random(ref.shape) < 0.05] = np.inf
    for name, start in (("oracle partial", part), ("raised", up), ("inf", np.full(ref.shape, np.inf))):
        t = torch.from_numpy(np.ascontiguousarray(start)).cuda()
        gpu.solve(f, p.h, src, tile=(8, 8, 8), delta=0.02, out=t, warm_start=True)
        assert_bitwise(t.cpu().numpy(), ref, f"warm start from {name}")


def test_warm_start_sources_and_batches(gpu, O):
    """Resume with several sources and start times (the sources are fixed
    again whatever the start state holds there), in 2D and in a batch."""
    name, f, h, src, t0 = CASES[0]
    ref = O.fmm(f, h, src, t0)
    start = ref + 1.0
    start.reshape(-1)[src] = 7.0
    ft = torch.from_numpy(f).cuda()
    out = torch.from_numpy(start).cuda()
    gpu.solve(ft, h, torch.as_tensor(src), t0=torch.as_tensor(t0), tile=(8, 8, 8), delta=0.5, out=out,
              warm_start=True)
    assert_bitwise(out.cpu().numpy(), ref, name)
    q = W.blocky_2d(n=256, nsrc=5, seed=9, block=16)
    refq = O.fmm(q.field, q.h, q.src)
    fq = torch.from_numpy(q.field[0]).cuda()
    tq = gpu.solve(fq, q.h, torch.as_tensor(q.src), tile=(32, 32), delta=4.0, max_tile_visits=20,
                   check_status=False)
    gpu.status(raise_on_error=False)
    gpu.solve(fq, q.h, torch.as_tensor(q.src), tile=(16, 16), delta=1.0, out=tq, warm_start=True)
    assert_bitwise(tq.cpu().numpy()[None], refq, "2D blocky resume")
    rng = np.random.default_rng(4)
    fields = [W.random_field(s, rng, 0.5, 4.0, block=2) for s in ((9, 20, 17), (12, 8, 30), (5, 5, 5))]
    srcs = [np.array([3]), np.array([100, 2000]), np.array([62])]
    b = gpu.pack([torch.from_numpy(x).cuda() for x in fields], 1.0, [torch.as_tensor(s) for s in srcs])
    tb = torch.empty(b.npts, dtype=torch.float64, device="cuda")
    gpu.solve_packed(b, tb, tile=(8, 8, 8), delta=0.5)
    gpu.status()
    tb.mul_(1.5)   # an upper bound of every problem's solution
    from paper_2103_05694_amd import _lib
    import ctypes
    o = gpu.make_opts(0.5, (8, 8, 8), warm_start=True)
    _lib.check(_lib.load().eik_solve_batched(b.nprob, b.grids, b.offsets, b.field.data_ptr(), b.src_off,
                                             b.src.data_ptr(), None, tb.data_ptr(), None, ctypes.byref(o),
                                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    gpu.status()
    for x, s, v in zip(fields, srcs, b.views(tb)):
        assert_bitwise(v.cpu().numpy(), O.fmm(x, 1.0, s), "batched resume")


def test_warm_start_rejects_invalid_start(gpu, O):
    f = torch.ones(20, 30, dtype=torch.float64, device="cuda")
    ref = O.fmm(np.ones((1, 20, 30)), 1.0, np.array([7]))[0]
    for bad in (float("nan"), -1.0, -0.0):
        t = torch.full_like(f, float("inf"))
        t[5, 5] = bad
        gpu.solve(f, 1.0, torch.tensor([7]), out=t, warm_start=True, check_status=False)
        st = gpu.status(raise_on_error=False)
        assert st.status == -1
        # the bad value was replaced by +inf, so the solve itself completed
        assert_bitwise(t.cpu().numpy(), ref, f"start value {bad}")
    with pytest.raises(ValueError):
        gpu.solve(f, 1.0, torch.tensor([7]), warm_start=True)

"""Host checks of the seeded synthetic inputs (the stand-ins for the paper's
workloads) and of the benchmark's bookkeeping: every generator is
deterministic in its seed and produces the structure its recipe states."""
import os

import numpy as np
import pytest

import workloads as W


def test_flat_index_round_trip():
    rng = np.random.default_rng(0)
    nx, ny, nz = 37, 11, 5
    ix, iy, iz = rng.integers(0, nx, 50), rng.integers(0, ny, 50), rng.integers(0, nz, 50)
    idx = W.flat_index(ix, iy, iz, nx, ny)
    assert np.all((idx >= 0) & (idx < nx * ny * nz))
    jx, jy, jz = W.unflatten(idx, nx, ny)
    assert np.array_equal(jx, ix) and np.array_equal(jy, iy) and np.array_equal(jz, iz)


def test_layered_recipe_and_determinism():
    a = W.layered_3d(48, 40, 32, seed=2)
    b = W.layered_3d(48, 40, 32, seed=2)
    c = W.layered_3d(48, 40, 32, seed=3)
    assert np.array_equal(a.field, b.field) and not np.array_equal(a.field, c.field)
    assert a.field.shape == (32, 40, 48) and a.field.dtype == np.float64
    assert np.array_equal(a.src, W.flat_index(24, 20, 0, 48, 40).reshape(1))
    # eight flat layers, 1500 .. 6000 m/s, each times (1 + 0.1 g) with g of unit variance
    z = np.arange(32)
    k = (z * 8) // 32
    vl = 1500.0 + k * 4500.0 / 7
    ratio = a.field / vl[:, None, None]
    assert abs(float(ratio.mean()) - 1.0) < 0.02
    assert 0.05 < float(ratio.std()) < 0.15
    means = a.field.mean(axis=(1, 2))
    layer_means = [means[k == j].mean() for j in range(8)]
    assert all(x < y for x, y in zip(layer_means, layer_means[1:]))


def test_blocky_recipe():
    p = W.blocky_2d(n=256, nsrc=16, seed=3, block=64)
    assert p.field.shape == (1, 256, 256)
    assert set(np.unique(p.field)) <= {0.5, 1.0, 2.0, 5.0}
    blocks = p.field[0].reshape(4, 64, 4, 64)
    assert np.all(blocks == blocks[:, :1, :, :1])  # constant over each 64 x 64 block
    assert len(np.unique(p.src)) == 16 and np.all(np.diff(p.src) > 0)
    q = W.blocky_2d(n=256, nsrc=16, seed=3, block=64)
    assert np.array_equal(p.field, q.field) and np.array_equal(p.src, q.src)


def test_folded_layers_recipe():
    p = W.folded_layers_2d(nx=200, nz=70, up=3)
    assert p.field.shape == (1, 210, 600) and p.h == pytest.approx(1.25 / 3)
    v = p.field[0]
    water = (70 * 9) // 70 * 3
    assert np.all(v[:water] == 1500.0)
    assert np.all(v > 0) and v.max() < 6000.0
    # nearest-neighbour upsampling: constant over every 3 x 3 cell
    cells = v.reshape(70, 3, 200, 3)
    assert np.all(cells == cells[:, :1, :, :1])
    assert np.array_equal(p.src, W.flat_index(300, 0, 0, 600, 210).reshape(1))
    assert np.array_equal(W.folded_layers_2d(nx=200, nz=70, up=3).field, p.field)


def test_batched_shots_structure():
    sizes = ((16, 16, 8), (24, 24, 8), (32, 32, 8))
    shots = W.batched_shots(6, seed=4, sizes=sizes)
    again = W.batched_shots(6, seed=4, sizes=sizes)
    assert len(shots) == 6
    for p, q in zip(shots, again):
        assert (p.nx, p.ny, p.nz) in sizes
        assert np.array_equal(p.field, q.field) and np.array_equal(p.src, q.src)
        assert p.src.size == 1
        ix, iy, iz = W.unflatten(p.src, p.nx, p.ny)
        assert int(iz[0]) == 0  # a surface source
    assert len({p.field.tobytes() for p in shots}) == 6  # independent models


def test_tomography_recipe():
    c = W.tomography(64, 64, 32, nshots=8, nrec_side=8, seed=5, radius=6.0)
    assert c.s0.shape == (32, 64, 64)
    ratio = c.s_true / c.s0
    assert ratio.min() >= 1.0 and ratio.max() <= 1.05 + 1e-12
    cx, cy, cz = c.blob_center
    assert np.unravel_index(np.argmax(ratio), ratio.shape) == (cz, cy, cx)
    _, _, sz = W.unflatten(c.sources, 64, 64)
    rx, ry, rz = W.unflatten(c.receivers, 64, 64)
    assert np.all(sz == 0) and np.all(rz == 0)
    assert len(np.unique(c.receivers)) == 64
    assert set(np.unique(rx)) == set(4 + 8 * np.arange(8))


def test_traffic_is_read_only_for_the_current_kernel(tmp_path, monkeypatch):
    import bench
    h = bench.kernel_source_hash()
    assert h == bench.kernel_source_hash() and len(h) == 16
    f = tmp_path / "pmc.txt"
    f.write_text(f"# header\nhbm_bytes_per_launch=123456\nsource_hash={h}\n")
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(f))
    assert bench.read_traffic(1) == 123456.0
    f.write_text("hbm_bytes_per_launch=123456\nsource_hash=0000000000000000\n")
    assert bench.read_traffic(1) is None
    monkeypatch.setattr(bench, "TRAFFIC_SUMMARY", str(tmp_path / "missing.txt"))
    assert bench.read_traffic(1) is None


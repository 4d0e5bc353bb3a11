"""The C ABI library loads and exports every entry point declared in
include/eik.h; host-side argument checks return their documented codes
without touching a GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2103_05694_amd import build as B
    if B.stale():
        B.build()
    from paper_2103_05694_amd import _lib
    return _lib.load()


def declared_functions():
    with open(os.path.join(ROOT, "include", "eik.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(eik_[a-z_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for n in ("eik_solve", "eik_adjoint", "eik_solve_batched", "eik_adjoint_batched", "eik_status",
              "eik_parents", "eik_release"):
        assert n in names


def test_every_declared_symbol_is_exported(L):
    from paper_2103_05694_amd import _lib
    names = declared_functions()
    assert set(names) == set(_lib.EXPORTED)
    for n in names:
        assert hasattr(L, n), n


def test_version_and_strerror(L):
    assert b"gfx950" in L.eik_version()
    for code in range(0, -9, -1):
        assert len(L.eik_strerror(code)) > 0
    assert L.eik_strerror(-2) == b"field value not positive and finite"


def _grid(ndim=3, nx=8, ny=8, nz=8, h=1.0, kind=0):
    from paper_2103_05694_amd._lib import eik_grid
    return eik_grid(ndim, nx, ny, nz, h, kind)


@pytest.mark.parametrize("kw, code", [
    (dict(ndim=4), -1), (dict(ndim=2, nz=3), -1), (dict(nx=0), -1), (dict(h=0.0), -1),
    (dict(h=float("inf")), -1), (dict(h=float("nan")), -1), (dict(kind=7), -1),
])
def test_solve_rejects_bad_grids(L, kw, code):
    g = _grid(**kw)
    dummy = ctypes.c_void_p(16)
    rc = L.eik_solve(ctypes.byref(g), dummy, 1, dummy, None, dummy, None, None, None)
    assert rc == code
    assert len(L.eik_last_error()) > 0


def test_solve_rejects_bad_counts_and_options(L):
    from paper_2103_05694_amd._lib import eik_opts
    g = _grid()
    dummy = ctypes.c_void_p(16)
    assert L.eik_solve(ctypes.byref(g), dummy, 0, dummy, None, dummy, None, None, None) == -1
    assert L.eik_solve(None, dummy, 1, dummy, None, dummy, None, None, None) == -1
    o = eik_opts()
    o.delta = -1.0
    assert L.eik_solve(ctypes.byref(g), dummy, 1, dummy, None, dummy, None, ctypes.byref(o), None) == -1
    o = eik_opts()
    o.tile[0], o.tile[1], o.tile[2] = 7, 7, 7
    assert L.eik_solve(ctypes.byref(g), dummy, 1, dummy, None, dummy, None, ctypes.byref(o), None) == -6
    o = eik_opts()
    o.tile[0], o.tile[1], o.tile[2] = 32, 32, 1   # a 2D tile for a 3D grid
    assert L.eik_solve(ctypes.byref(g), dummy, 1, dummy, None, dummy, None, ctypes.byref(o), None) == -6
    for bad in (2, 64, 1 << 31):                   # no such flags
        o = eik_opts()
        o.flags = bad
        assert L.eik_solve(ctypes.byref(g), dummy, 1, dummy, None, dummy, None, ctypes.byref(o), None) == -1
    for tiny in (5e-324, 1e-310):                  # 1/delta overflows: no bucket could hold a time
        o = eik_opts()
        o.delta = tiny
        o.horizon = 1
        assert L.eik_solve(ctypes.byref(g), dummy, 1, dummy, None, dummy, None, ctypes.byref(o), None) == -1
        assert b"delta" in L.eik_last_error()
    o = eik_opts()
    o.delta = float("nan")
    assert L.eik_solve(ctypes.byref(g), dummy, 1, dummy, None, dummy, None, ctypes.byref(o), None) == -1
    o = eik_opts()
    o.flags = 8                                    # change tracking needs an ablation operator
    assert L.eik_solve(ctypes.byref(g), dummy, 1, dummy, None, dummy, None, ctypes.byref(o), None) == -1
    o = eik_opts()
    o.horizon = 5
    assert L.eik_solve(ctypes.byref(g), dummy, 1, dummy, None, dummy, None, ctypes.byref(o), None) == -1
    for bad in (-1, 17, 32):                       # the window reads at most 16 buckets past the lowest
        o = eik_opts()
        o.lookahead = bad
        assert L.eik_solve(ctypes.byref(g), dummy, 1, dummy, None, dummy, None, ctypes.byref(o), None) == -1
        assert b"lookahead" in L.eik_last_error()
    o = eik_opts()
    o.op = 3                                       # Newton: 2D only
    assert L.eik_solve(ctypes.byref(g), dummy, 1, dummy, None, dummy, None, ctypes.byref(o), None) == -6
    o = eik_opts()
    o.op = 4                                       # no such operator
    assert L.eik_solve(ctypes.byref(g), dummy, 1, dummy, None, dummy, None, ctypes.byref(o), None) == -1
    o = eik_opts()
    o.op = 1                                       # the explicit formulas are 2D only
    assert L.eik_solve(ctypes.byref(g), dummy, 1, dummy, None, dummy, None, ctypes.byref(o), None) == -6
    o = eik_opts()
    o.op = 2
    o.flags = 16                                   # a warm start needs the monotone operator
    g2 = _grid(ndim=2, nx=64, ny=64, nz=1)
    assert L.eik_solve(ctypes.byref(g2), dummy, 1, dummy, None, dummy, None, ctypes.byref(o), None) == -6


def test_rect_rejects_bad_coordinates_and_options(L):
    from paper_2103_05694_amd._lib import eik_opts
    g = _grid(ndim=2, nx=5, ny=4, nz=1)
    dummy = ctypes.c_void_p(16)

    def arr(v):
        return (ctypes.c_double * len(v))(*v)

    ys = arr([0.0, 1.0, 2.0, 3.0])
    for xs in ([0.0, 1.0, 1.0, 2.0, 3.0], [0.0, 1.0, 0.5, 2.0, 3.0], [0.0, 1.0, float("nan"), 2.0, 3.0],
               [0.0, 1.0, float("inf"), 2.0, 3.0], [0.0, 5e-324, 1.0, 2.0, 3.0]):
        rc = L.eik_solve_rect(ctypes.byref(g), arr(xs), ys, None, dummy, 1, dummy, None, dummy, None, None)
        assert rc == -1, xs
        assert b"coordinates" in L.eik_last_error()
    assert L.eik_solve_rect(ctypes.byref(g), None, ys, None, dummy, 1, dummy, None, dummy, None, None) == -1
    g3 = _grid(ndim=3, nx=5, ny=4, nz=3)
    xs = arr([0.0, 1.0, 2.0, 3.0, 4.0])
    assert L.eik_solve_rect(ctypes.byref(g3), xs, ys, None, dummy, 1, dummy, None, dummy, None, None) == -1
    assert L.eik_solve_rect(ctypes.byref(g), xs, ys, None, dummy, 0, dummy, None, dummy, None, None) == -1
    for op, flags in ((2, 0), (0, 32), (0, 8)):   # ablation operator, packed passes, change tracking
        o = eik_opts()
        o.op, o.flags = op, flags
        rc = L.eik_solve_rect(ctypes.byref(g), xs, ys, None, dummy, 1, dummy, None, dummy, ctypes.byref(o), None)
        assert rc in (-1, -6), (op, flags)


def test_residual_rejects_bad_arguments(L):
    g = _grid()
    dummy = ctypes.c_void_p(16)
    cnt = ctypes.c_int64(0)
    assert L.eik_residual(ctypes.byref(g), dummy, 1, dummy, dummy, 5, ctypes.byref(cnt), None, None) == -1
    assert L.eik_residual(ctypes.byref(g), dummy, 1, dummy, dummy, 1, ctypes.byref(cnt), None, None) == -6
    assert L.eik_residual(ctypes.byref(g), None, 1, dummy, dummy, 0, ctypes.byref(cnt), None, None) == -1
    assert L.eik_residual(ctypes.byref(g), dummy, -1, dummy, dummy, 0, ctypes.byref(cnt), None, None) == -1


def test_batched_rejects_inconsistent_packing(L):
    from paper_2103_05694_amd._lib import eik_grid
    grids = (eik_grid * 2)(_grid(nx=4, ny=4, nz=4), _grid(nx=5, ny=4, nz=4))
    offs = (ctypes.c_int64 * 3)(0, 64, 64 + 79)      # second size is wrong (80)
    soff = (ctypes.c_int64 * 3)(0, 1, 2)
    dummy = ctypes.c_void_p(16)
    assert L.eik_solve_batched(2, grids, offs, dummy, soff, dummy, None, dummy, None, None, None) == -1
    offs = (ctypes.c_int64 * 3)(0, 64, 144)
    soff = (ctypes.c_int64 * 3)(0, 1, 1)              # second problem has no source
    assert L.eik_solve_batched(2, grids, offs, dummy, soff, dummy, None, dummy, None, None, None) == -1
    mixed = (eik_grid * 2)(_grid(nx=4, ny=4, nz=4), _grid(ndim=2, nx=4, ny=4, nz=1))
    offs = (ctypes.c_int64 * 3)(0, 64, 80)
    soff = (ctypes.c_int64 * 3)(0, 1, 2)
    assert L.eik_solve_batched(2, mixed, offs, dummy, soff, dummy, None, dummy, None, None, None) == -1


def test_num_tiles_host_only(L):
    from paper_2103_05694_amd._lib import eik_opts
    g = _grid(nx=512, ny=512, nz=256)
    assert L.eik_num_tiles(ctypes.byref(g), None) == (512 // 16) * (512 // 8) * (256 // 8)  # default 16x8x8
    o = eik_opts()
    o.tile[0], o.tile[1], o.tile[2] = 8, 8, 8
    g2 = _grid(nx=33, ny=9, nz=8)
    assert L.eik_num_tiles(ctypes.byref(g2), ctypes.byref(o)) == 5 * 2 * 1
    g3 = _grid(ndim=2, nx=4096, ny=4096, nz=1)
    assert L.eik_num_tiles(ctypes.byref(g3), None) == (4096 // 32) * (4096 // 32)  # default 32x32
    g4 = _grid(ndim=2, nx=100, ny=33, nz=1)
    assert L.eik_num_tiles(ctypes.byref(g4), None) == 4 * 2


def test_missing_library_fails_loudly(monkeypatch):
    from paper_2103_05694_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", os.path.join(ROOT, "does_not_exist", "libeik.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib.load()


def test_product_package_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2103_05694_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                with open(os.path.join(dirpath, fn)) as f:
                    src = f.read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", src, flags=re.M), fn
                assert "eik_oracle" not in src, fn
                assert "liboracle" not in src, fn


def test_buffer_checks_reject_before_any_launch():
    """The binding validates every caller buffer (dtype, element count,
    device, contiguity) before a raw pointer reaches the library."""
    import torch
    from paper_2103_05694_amd.api import _check_buf
    dev = torch.device("cpu")
    ok = torch.zeros(12, dtype=torch.float64)
    _check_buf(ok, "out", torch.float64, 12, dev)
    with pytest.raises(TypeError):
        _check_buf(ok.float(), "out", torch.float64, 12, dev)
    with pytest.raises(ValueError):
        _check_buf(ok[:11], "out", torch.float64, 12, dev)
    with pytest.raises(ValueError):
        _check_buf(torch.zeros(24, dtype=torch.float64)[::2], "out", torch.float64, 12, dev)
    with pytest.raises(ValueError):
        _check_buf(ok, "out", torch.float64, 12, torch.device("meta"))
    with pytest.raises(TypeError):
        _check_buf(torch.zeros(12, dtype=torch.int64), "parents_out", torch.uint8, 12, dev)

"""The allocation-free entry point (eik_solve_noalloc, workspace in a static
device array) against eik_solve through the C ABI: bit-identical times and
parents on two calls in a row, the second one smaller, plus a resumed solve
and the size limits (rejected before any launch)."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _call(L, name, f, h, src, t_out, par=None, opts=None, kind=0):
    from paper_2103_05694_amd import _lib
    shape = tuple(f.shape)
    if len(shape) == 3:
        g = _lib.eik_grid(3, shape[2], shape[1], shape[0], h, kind)
    else:
        g = _lib.eik_grid(2, shape[1], shape[0], 1, h, kind)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(L, name)(ctypes.byref(g), f.data_ptr(), src.numel(), src.data_ptr(), None, t_out.data_ptr(),
                          par.data_ptr() if par is not None else None,
                          ctypes.byref(opts) if opts is not None else None, stream)
    return rc, stream


def test_noalloc_equals_solve_on_two_calls_the_second_smaller(gpu):
    from paper_2103_05694_amd import _lib
    L = _lib.load()
    cases = [W.layered_3d(96, 80, 48, h=10.0, seed=2), W.layered_3d(40, 36, 28, h=10.0, seed=4, sigma=3.0)]
    for i, p in enumerate(cases):
        print(f"[noalloc] call {i}: {p.nx}x{p.ny}x{p.nz}", flush=True)
        f = torch.from_numpy(p.field).cuda()
        src = torch.as_tensor(p.src).cuda()
        o = gpu.make_opts(0.02, (8, 8, 8))
        t_ref = torch.empty_like(f)
        par_ref = torch.empty(f.shape, dtype=torch.uint8, device="cuda")
        rc, st = _call(L, "eik_solve", f, p.h, src, t_ref, par_ref, o)
        assert rc == 0 and L.eik_status(st, None) == 0
        t = torch.full_like(f, -7.0)
        par = torch.zeros(f.shape, dtype=torch.uint8, device="cuda")
        rc, st = _call(L, "eik_solve_noalloc", f, p.h, src, t, par, o)
        assert rc == 0
        stats = _lib.eik_stats()
        assert L.eik_status(st, ctypes.byref(stats)) == 0
        assert stats.ntiles == L.eik_num_tiles(ctypes.byref(_lib.eik_grid(3, p.nx, p.ny, p.nz, p.h, 0)),
                                               ctypes.byref(o))
        assert stats.tile_visits >= stats.ntiles
        assert torch.equal(t, t_ref), f"times, call {i}"
        assert torch.equal(par, par_ref), f"parents, call {i}"


def test_noalloc_with_window_and_compacted_passes(gpu):
    """The benchmark's kind of launch (16x8x8 tiles, compacted passes, a window
    of 16 buckets) through the allocation-free entry point: the same bits as
    eik_solve with the same options."""
    from paper_2103_05694_amd import _lib
    L = _lib.load()
    p = W.layered_3d(96, 80, 48, h=10.0, seed=2)
    print(f"[noalloc] window 16, compacted: {p.nx}x{p.ny}x{p.nz}", flush=True)
    f = torch.from_numpy(p.field).cuda()
    src = torch.as_tensor(p.src).cuda()
    o = gpu.make_opts(0.005, (16, 8, 8), lookahead=16, packed=True)
    t_ref = torch.empty_like(f)
    rc, st = _call(L, "eik_solve", f, p.h, src, t_ref, None, o)
    assert rc == 0 and L.eik_status(st, None) == 0
    t = torch.full_like(f, -7.0)
    rc, st = _call(L, "eik_solve_noalloc", f, p.h, src, t, None, o)
    assert rc == 0 and L.eik_status(st, None) == 0
    assert torch.equal(t, t_ref)


def test_noalloc_resume_and_2d(gpu):
    from paper_2103_05694_amd import _lib
    L = _lib.load()
    q = W.blocky_2d(n=256, nsrc=5, seed=9, block=16)
    f = torch.from_numpy(q.field[0]).cuda()
    src = torch.as_tensor(q.src).cuda()
    t_ref = torch.empty_like(f)
    rc, st = _call(L, "eik_solve", f, q.h, src, t_ref, None, gpu.make_opts(4.0, (32, 32)))
    assert rc == 0 and L.eik_status(st, None) == 0
    t = torch.empty_like(f)
    o = gpu.make_opts(4.0, (32, 32), max_tile_visits=10)
    rc, st = _call(L, "eik_solve_noalloc", f, q.h, src, t, None, o)
    assert rc == 0 and L.eik_status(st, None) == -5
    rc, st = _call(L, "eik_solve_noalloc", f, q.h, src, t, None, gpu.make_opts(2.0, (16, 16), warm_start=True))
    assert rc == 0 and L.eik_status(st, None) == 0
    assert torch.equal(t, t_ref)


def test_noalloc_limits_rejected_before_launch(gpu):
    from paper_2103_05694_amd import _lib
    L = _lib.load()
    f = torch.ones(256, 512, 512, dtype=torch.float64, device="cuda")   # 131072 tiles of 8x8x8
    t = torch.empty_like(f)
    src = torch.tensor([0], device="cuda")
    rc, _ = _call(L, "eik_solve_noalloc", f, 1.0, src, t, None, gpu.make_opts(0.0, (8, 8, 8)))
    assert rc == -6 and b"65536 tiles" in L.eik_last_error()
    del f, t
    f = torch.ones(300, 300, dtype=torch.float64, device="cuda")
    t = torch.empty_like(f)
    many = torch.arange(70000, device="cuda")
    rc, _ = _call(L, "eik_solve_noalloc", f, 1.0, many, t, None, None)
    assert rc == -6 and b"65536 sources" in L.eik_last_error()
    rc, _ = _call(L, "eik_solve_noalloc", f, 1.0, src, t, None, gpu.make_opts(time_kernels=True))
    assert rc == -6

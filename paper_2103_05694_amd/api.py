"""Python entry points over the C ABI.  PyTorch provides device memory and
streams only; every step of the solve and of the adjoint runs in the HIP
kernels of libeik.so.

Arrays are float64 CUDA (ROCm) tensors laid out [nz][ny][nx] (3D) or [ny][nx]
(2D).  Sources are flat indices (iz*ny + iy)*nx + ix, or an integer tensor of
coordinates with one row (x, y[, z]) per source.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple, Union

import torch

from . import _lib
from ._lib import EikError, check, eik_grid, eik_opts, eik_stats

KINDS = {"speed": _lib.EIK_SPEED, "slowness": _lib.EIK_SLOWNESS}


def _stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _grid_of(shape: Sequence[int], h: float, kind: str) -> eik_grid:
    if kind not in KINDS:
        raise ValueError(f"kind must be one of {sorted(KINDS)}")
    if len(shape) == 2:
        ny, nx = shape
        return eik_grid(2, int(nx), int(ny), 1, float(h), KINDS[kind])
    if len(shape) == 3:
        nz, ny, nx = shape
        return eik_grid(3, int(nx), int(ny), int(nz), float(h), KINDS[kind])
    raise ValueError("field must be 2D [ny, nx] or 3D [nz, ny, nx]")


def make_opts(delta: float = 0.0, tile: Optional[Sequence[int]] = None, grid_blocks: int = 0,
              max_tile_visits: int = 0, time_kernels: bool = False, lookahead: int = 0,
              timeline: bool = False, op: str = "dbar", horizon: int = 0,
              work_ref: Optional[torch.Tensor] = None, track_change: bool = False,
              warm_start: bool = False, packed: bool = False) -> eik_opts:
    o = eik_opts()
    o.delta = float(delta)
    t = tuple(tile) if tile else (0, 0, 0)
    if len(t) == 2:
        t = (t[0], t[1], 1)
    for i in range(3):
        o.tile[i] = int(t[i])
    o.grid_blocks = int(grid_blocks)
    o.max_tile_visits = int(max_tile_visits)
    o.flags = (_lib.EIK_FLAG_TIME_KERNELS if time_kernels else 0) | \
        (_lib.EIK_FLAG_TIMELINE if timeline else 0) | (_lib.EIK_FLAG_TRACK_CHANGE if track_change else 0) | \
        (_lib.EIK_FLAG_WARM_START if warm_start else 0) | (_lib.EIK_FLAG_PACKED if packed else 0)
    o.lookahead = int(lookahead)
    o.horizon = int(horizon)
    o.op = _op_code(op)
    o.work_ref = work_ref.data_ptr() if work_ref is not None else None
    return o


_OPS = {"dbar": _lib.EIK_OP_DBAR, "dhat": _lib.EIK_OP_DHAT, "dtilde": _lib.EIK_OP_DTILDE,
        "newton": _lib.EIK_OP_NEWTON}


def _op_code(op: str) -> int:
    if op not in _OPS:
        raise ValueError(f"op must be one of {sorted(_OPS)}")
    return _OPS[op]


def _check_field(field: torch.Tensor) -> None:
    if not isinstance(field, torch.Tensor) or field.dtype != torch.float64:
        raise TypeError("field must be a float64 tensor")
    if field.device.type != "cuda":
        raise ValueError("field must live on the GPU (there is no CPU path)")
    if not field.is_contiguous():
        raise ValueError("field must be contiguous")


def _check_buf(buf: torch.Tensor, name: str, dtype: torch.dtype, numel: int, device: torch.device) -> None:
    """A caller-supplied buffer the kernels read or write through a raw
    pointer: it must have exactly the dtype, element count and device the call
    assumes, and be contiguous (checked before anything is launched)."""
    if not isinstance(buf, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if buf.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {buf.dtype}")
    if buf.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {buf.numel()}")
    if buf.device != device:
        raise ValueError(f"{name} must be on {device}, got {buf.device}")
    if not buf.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def source_indices(sources, shape: Sequence[int], device) -> torch.Tensor:
    """Flat int64 source indices on `device` from flat indices or coordinates."""
    s = torch.as_tensor(sources)
    if s.dtype not in (torch.int64, torch.int32, torch.int16):
        raise TypeError("sources must be integer")
    s = s.to(torch.int64)
    if s.dim() == 2:
        nd = len(shape)
        if s.shape[1] != nd:
            raise ValueError(f"coordinate sources need {nd} columns (x, y[, z])")
        nx, ny = shape[-1], shape[-2]
        flat = s[:, 0] + nx * s[:, 1]
        if nd == 3:
            flat = flat + nx * ny * s[:, 2]
        s = flat
    s = s.reshape(-1)
    if s.numel() < 1:
        raise ValueError("at least one source is required")
    n = 1
    for d in shape:
        n *= int(d)
    lo, hi = int(s.min()), int(s.max())
    if lo < 0 or hi >= n:
        raise ValueError("source index out of range")
    return s.to(device).contiguous()


def status(stream=None, raise_on_error: bool = True) -> eik_stats:
    """Synchronise the stream and return the device status of its last call."""
    L = _lib.load()
    st = eik_stats()
    rc = L.eik_status(ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(st))
    if raise_on_error and rc != _lib.EIK_OK:
        raise EikError(rc, L.eik_strerror(rc).decode())
    return st


def residual(field: torch.Tensor, h: float, sources, t: torch.Tensor, kind: str = "speed",
             op: str = "dbar", stream=None):
    """(points the operator would still change, largest relative change) for
    the times `t` -- the error metric of the paper's Table "tab:error"."""
    _check_field(field)
    _check_field(t)
    if t.shape != field.shape:
        raise ValueError("t must have the field's shape")
    L = _lib.load()
    g = _grid_of(field.shape, h, kind)
    src = source_indices(sources, field.shape, field.device)
    cnt = ctypes.c_int64(0)
    worst = ctypes.c_double(0.0)
    rc = L.eik_residual(ctypes.byref(g), field.data_ptr(), src.numel(), src.data_ptr(), t.data_ptr(),
                        _op_code(op), ctypes.byref(cnt), ctypes.byref(worst),
                        ctypes.c_void_p(_stream_handle(stream)))
    check(rc)
    return int(cnt.value), float(worst.value)


def timeline(stream=None, cap: int = 1 << 16):
    """Bucket advances of the last launch run with timeline=True: (times in us
    since its reset, bucket moved to, span in us of the whole launch)."""
    import numpy as np
    L = _lib.load()
    t = np.zeros(cap, dtype=np.float64)
    b = np.zeros(cap, dtype=np.int64)
    span = np.zeros(1, dtype=np.float64)
    n = L.eik_timeline(ctypes.c_void_p(_stream_handle(stream)), cap, t.ctypes.data, b.ctypes.data,
                       span.ctypes.data)
    check(n if n < 0 else 0)
    m = min(n, cap)
    return t[:m].copy(), b[:m].copy(), float(span[0])


def solve(field: torch.Tensor, h: float, sources, t0: Optional[torch.Tensor] = None,
          kind: str = "speed", parents: bool = False, delta: float = 0.0,
          tile: Optional[Sequence[int]] = None, grid_blocks: int = 0, max_tile_visits: int = 0,
          out: Optional[torch.Tensor] = None, parents_out: Optional[torch.Tensor] = None,
          check_status: bool = True, stream=None, time_kernels: bool = False, lookahead: int = 0,
          timeline: bool = False, op: str = "dbar", horizon: int = 0,
          work_ref: Optional[torch.Tensor] = None, track_change: bool = False, warm_start: bool = False,
          packed: bool = False):
    """First-arrival times; returns t, or (t, parents) when parents=True.
    `delta` (the priority bucket width), `lookahead` (0..16: how many buckets
    past the lowest open one a claim may take work from), `horizon`, `tile`,
    `grid_blocks` and `packed` (the compacted relaxation passes,
    EIK_FLAG_PACKED) only schedule the work: the result is the same bits for
    every choice (the d-bar operator is monotone and causal).

    With warm_start=True the solve resumes from the times in `out` (required):
    any upper bound of the solution, e.g. the output of a solve stopped by
    max_tile_visits; the result is bit-identical to a cold solve."""
    _check_field(field)
    if warm_start and out is None:
        raise ValueError("warm_start needs the starting times in `out`")
    L = _lib.load()
    g = _grid_of(field.shape, h, kind)
    src = source_indices(sources, field.shape, field.device)
    t0d = None
    if t0 is not None:
        t0d = torch.as_tensor(t0, dtype=torch.float64).reshape(-1).to(field.device).contiguous()
        if t0d.numel() != src.numel():
            raise ValueError("t0 needs one value per source")
    if out is not None:
        _check_buf(out, "out", torch.float64, field.numel(), field.device)
    t = out if out is not None else torch.empty_like(field)
    par = None
    if parents:
        if parents_out is not None:
            _check_buf(parents_out, "parents_out", torch.uint8, field.numel(), field.device)
        par = parents_out if parents_out is not None else torch.empty(field.shape, dtype=torch.uint8,
                                                                       device=field.device)
    if work_ref is not None:
        _check_field(work_ref)
        if work_ref.shape != field.shape:
            raise ValueError("work_ref must have the field's shape")
    o = make_opts(delta, tile, grid_blocks, max_tile_visits, time_kernels, lookahead, timeline, op,
                  horizon, work_ref, track_change, warm_start, packed)
    rc = L.eik_solve(ctypes.byref(g), field.data_ptr(), src.numel(), src.data_ptr(),
                     t0d.data_ptr() if t0d is not None else None, t.data_ptr(),
                     par.data_ptr() if par is not None else None, ctypes.byref(o),
                     ctypes.c_void_p(_stream_handle(stream)))
    check(rc)
    if check_status:
        status(stream)
    return (t, par) if parents else t


def solve_rect(field: torch.Tensor, xs, ys, zs=None, sources=None, t0=None, kind: str = "speed",
               delta: float = 0.0, tile: Optional[Sequence[int]] = None, grid_blocks: int = 0,
               max_tile_visits: int = 0, out: Optional[torch.Tensor] = None, check_status: bool = True,
               stream=None, time_kernels: bool = False, lookahead: int = 0, horizon: int = 0,
               warm_start: bool = False) -> torch.Tensor:
    """First-arrival times on a rectilinear grid: xs, ys[, zs] are the
    coordinates of the points along each axis (host sequences or CPU tensors,
    strictly increasing), so the spacing may vary per axis and index."""
    import numpy as np
    _check_field(field)
    if sources is None:
        raise ValueError("sources are required")
    if warm_start and out is None:
        raise ValueError("warm_start needs the starting times in `out`")
    L = _lib.load()
    g = _grid_of(field.shape, 1.0, kind)
    coords = [np.ascontiguousarray(np.asarray(c, dtype=np.float64).reshape(-1)) for c in (xs, ys)]
    if g.ndim == 3:
        if zs is None:
            raise ValueError("a 3D field needs z coordinates")
        coords.append(np.ascontiguousarray(np.asarray(zs, dtype=np.float64).reshape(-1)))
    for c, n in zip(coords, (g.nx, g.ny, g.nz)):
        if c.size != n:
            raise ValueError("coordinate arrays must match the field's shape")
    src = source_indices(sources, field.shape, field.device)
    t0d = None
    if t0 is not None:
        t0d = torch.as_tensor(t0, dtype=torch.float64).reshape(-1).to(field.device).contiguous()
        if t0d.numel() != src.numel():
            raise ValueError("t0 needs one value per source")
    if out is not None:
        _check_buf(out, "out", torch.float64, field.numel(), field.device)
    t = out if out is not None else torch.empty_like(field)
    o = make_opts(delta, tile, grid_blocks, max_tile_visits, time_kernels, lookahead, horizon=horizon,
                  warm_start=warm_start)
    rc = L.eik_solve_rect(ctypes.byref(g), coords[0].ctypes.data, coords[1].ctypes.data,
                          coords[2].ctypes.data if len(coords) == 3 else None, field.data_ptr(), src.numel(),
                          src.data_ptr(), t0d.data_ptr() if t0d is not None else None, t.data_ptr(),
                          ctypes.byref(o), ctypes.c_void_p(_stream_handle(stream)))
    check(rc)
    if check_status:
        status(stream)
    return t


def parents_of(t: torch.Tensor, sources, stream=None) -> torch.Tensor:
    _check_field(t)
    L = _lib.load()
    g = _grid_of(t.shape, 1.0, "speed")
    src = source_indices(sources, t.shape, t.device)
    par = torch.empty(t.shape, dtype=torch.uint8, device=t.device)
    check(L.eik_parents(ctypes.byref(g), t.data_ptr(), src.numel(), src.data_ptr(), par.data_ptr(),
                        ctypes.c_void_p(_stream_handle(stream))))
    return par


def adjoint(field: torch.Tensor, h: float, t: torch.Tensor, parents: torch.Tensor,
            dL_dt: torch.Tensor, kind: str = "speed", delta: float = 0.0,
            tile: Optional[Sequence[int]] = None, grid_blocks: int = 0,
            out: Optional[torch.Tensor] = None, mu_out: Optional[torch.Tensor] = None,
            check_status: bool = True, stream=None, time_kernels: bool = False,
            lookahead: int = 0, packed: bool = False) -> torch.Tensor:
    """d loss / d slowness from d loss / d t through the recorded upwind parents."""
    for a in (field, t, dL_dt):
        _check_field(a)
    if parents.dtype != torch.uint8 or parents.shape != field.shape:
        raise ValueError("parents must be a uint8 tensor of the field's shape")
    if t.shape != field.shape or dL_dt.shape != field.shape:
        raise ValueError("t and dL_dt must have the field's shape")
    if out is not None:
        _check_buf(out, "out", torch.float64, field.numel(), field.device)
    if mu_out is not None:
        _check_buf(mu_out, "mu_out", torch.float64, field.numel(), field.device)
    for a in (t, parents, dL_dt):
        if a.device != field.device:
            raise ValueError("t, parents and dL_dt must be on the field's device")
    if not parents.is_contiguous():
        raise ValueError("parents must be contiguous")
    L = _lib.load()
    g = _grid_of(field.shape, h, kind)
    grad = out if out is not None else torch.empty_like(field)
    o = make_opts(delta, tile, grid_blocks, 0, time_kernels, lookahead, packed=packed)
    rc = L.eik_adjoint(ctypes.byref(g), field.data_ptr(), t.data_ptr(), parents.data_ptr(),
                       dL_dt.data_ptr(), grad.data_ptr(),
                       mu_out.data_ptr() if mu_out is not None else None, ctypes.byref(o),
                       ctypes.c_void_p(_stream_handle(stream)))
    check(rc)
    if check_status:
        status(stream)
    return grad


class EikonalFn(torch.autograd.Function):
    """t = solve(slowness); backward gives d loss / d slowness (hand-written
    adjoint kernel over the recorded upwind parents)."""

    @staticmethod
    def forward(ctx, slowness: torch.Tensor, h: float, sources, delta: float = 0.0, tile=None):
        t, par = solve(slowness.detach(), h, sources, kind="slowness", parents=True, delta=delta,
                       tile=tile)
        ctx.save_for_backward(slowness.detach(), t, par)
        ctx.h = h
        ctx.delta = delta
        ctx.tile = tile
        return t

    @staticmethod
    def backward(ctx, grad_t: torch.Tensor):
        s, t, par = ctx.saved_tensors
        g = adjoint(s, ctx.h, t, par, grad_t.contiguous().to(torch.float64), kind="slowness",
                    delta=ctx.delta, tile=ctx.tile)
        return g, None, None, None, None


def eikonal(slowness: torch.Tensor, h: float, sources, delta: float = 0.0, tile=None) -> torch.Tensor:
    return EikonalFn.apply(slowness, h, sources, delta, tile)


# ---------------------------------------------------------------------------
# batched problems
# ---------------------------------------------------------------------------

@dataclass
class Batch:
    """Packed description of independent problems solved in one launch."""

    grids: ctypes.Array
    offsets: ctypes.Array
    src_off: ctypes.Array
    nprob: int
    npts: int
    shapes: List[Tuple[int, ...]]
    field: torch.Tensor            # packed
    src: torch.Tensor              # packed local flat indices
    t0: Optional[torch.Tensor]

    def views(self, packed: torch.Tensor) -> List[torch.Tensor]:
        out = []
        off = 0
        for shp in self.shapes:
            n = 1
            for d in shp:
                n *= d
            out.append(packed[off:off + n].view(shp))
            off += n
        return out


def pack(fields: Sequence[torch.Tensor], hs: Union[float, Sequence[float]], sources: Sequence,
         kind: str = "speed", t0s: Optional[Sequence] = None) -> Batch:
    n = len(fields)
    if n < 1:
        raise ValueError("need at least one problem")
    if isinstance(hs, (int, float)):
        hs = [float(hs)] * n
    grids = (eik_grid * n)()
    offsets = (ctypes.c_int64 * (n + 1))()
    src_off = (ctypes.c_int64 * (n + 1))()
    srcs = []
    t0l = []
    off = 0
    soff = 0
    for i, f in enumerate(fields):
        _check_field(f)
        grids[i] = _grid_of(f.shape, hs[i], kind)
        offsets[i] = off
        src_off[i] = soff
        s = source_indices(sources[i], f.shape, f.device)
        srcs.append(s)
        if t0s is not None:
            t0l.append(torch.as_tensor(t0s[i], dtype=torch.float64).reshape(-1).to(f.device))
        off += f.numel()
        soff += s.numel()
    offsets[n] = off
    src_off[n] = soff
    dev = fields[0].device
    field = torch.cat([f.reshape(-1) for f in fields]).contiguous()
    src = torch.cat(srcs).contiguous()
    t0 = torch.cat(t0l).contiguous() if t0s is not None else None
    return Batch(grids, offsets, src_off, n, off, [tuple(f.shape) for f in fields], field, src, t0)


def solve_packed(b: Batch, t_packed: torch.Tensor, par_packed: Optional[torch.Tensor] = None,
                 delta: float = 0.0, tile=None, grid_blocks: int = 0, stream=None,
                 time_kernels: bool = False, lookahead: int = 0, horizon: int = 0,
                 packed: bool = False) -> None:
    """Enqueue one batched forward launch (no host synchronisation)."""
    dev = b.field.device
    _check_buf(t_packed, "t_packed", torch.float64, b.npts, dev)
    if par_packed is not None:
        _check_buf(par_packed, "par_packed", torch.uint8, b.npts, dev)
    L = _lib.load()
    o = make_opts(delta, tile, grid_blocks, 0, time_kernels, lookahead, horizon=horizon, packed=packed)
    check(L.eik_solve_batched(b.nprob, b.grids, b.offsets, b.field.data_ptr(), b.src_off,
                              b.src.data_ptr(), b.t0.data_ptr() if b.t0 is not None else None,
                              t_packed.data_ptr(), par_packed.data_ptr() if par_packed is not None else None,
                              ctypes.byref(o), ctypes.c_void_p(_stream_handle(stream))))


def adjoint_packed(b: Batch, t_packed: torch.Tensor, par_packed: torch.Tensor, g_packed: torch.Tensor,
                   grad_packed: torch.Tensor, mu_packed: Optional[torch.Tensor] = None, delta: float = 0.0,
                   tile=None, grid_blocks: int = 0, stream=None, time_kernels: bool = False,
                   lookahead: int = 0, packed: bool = False) -> None:
    """Enqueue one batched adjoint launch (no host synchronisation)."""
    dev = b.field.device
    _check_buf(t_packed, "t_packed", torch.float64, b.npts, dev)
    _check_buf(par_packed, "par_packed", torch.uint8, b.npts, dev)
    _check_buf(g_packed, "g_packed", torch.float64, b.npts, dev)
    _check_buf(grad_packed, "grad_packed", torch.float64, b.npts, dev)
    if mu_packed is not None:
        _check_buf(mu_packed, "mu_packed", torch.float64, b.npts, dev)
    L = _lib.load()
    o = make_opts(delta, tile, grid_blocks, 0, time_kernels, lookahead, packed=packed)
    check(L.eik_adjoint_batched(b.nprob, b.grids, b.offsets, b.field.data_ptr(), t_packed.data_ptr(),
                                par_packed.data_ptr(), g_packed.data_ptr(), grad_packed.data_ptr(),
                                mu_packed.data_ptr() if mu_packed is not None else None,
                                ctypes.byref(o), ctypes.c_void_p(_stream_handle(stream))))


def solve_batched(fields: Sequence[torch.Tensor], h, sources, kind: str = "speed", parents: bool = False,
                  delta: float = 0.0, tile=None, check_status: bool = True, grid_blocks: int = 0,
                  horizon: int = 0, packed: bool = False, lookahead: int = 0):
    """Solve independent problems (uneven sizes allowed) in one persistent launch."""
    b = pack(fields, h, sources, kind)
    t = torch.empty(b.npts, dtype=torch.float64, device=b.field.device)
    par = torch.empty(b.npts, dtype=torch.uint8, device=b.field.device) if parents else None
    solve_packed(b, t, par, delta, tile, grid_blocks=grid_blocks, horizon=horizon, packed=packed,
                 lookahead=lookahead)
    if check_status:
        status()
    ts = b.views(t)
    if parents:
        return ts, b.views(par)
    return ts


def reserve(ntiles: int, npts: int, stream=None) -> None:
    check(_lib.load().eik_reserve(int(ntiles), int(npts), ctypes.c_void_p(_stream_handle(stream))))


def num_tiles(shape: Sequence[int], tile=None) -> int:
    g = _grid_of(shape, 1.0, "speed")
    o = make_opts(0.0, tile)
    n = _lib.load().eik_num_tiles(ctypes.byref(g), ctypes.byref(o))
    if n < 0:
        raise ValueError("unsupported grid / tile")
    return int(n)


def release() -> None:
    _lib.load().eik_release()

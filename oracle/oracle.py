"""ctypes wrappers over the C oracle, plus the dense adjoint and finite-difference
references written in numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each function cites the passage of the paper it follows:
  * ``dbar``          -- section "Achieving Exact Monotonicity with Finite
                         Precision Arithmetic" (smallest float with alpha >= 0),
                         extended to the one-sided case and to three axes.
  * ``fmm``           -- Algorithm "Fast Marching Method" with the update
                         operator of Algorithm "Eikonal Update Operator".
  * ``fmm_resume``    -- the same loop started from any upper bound of the
                         solution (checkpoint / resume; Theorem 1's argument).
  * ``sweep_all``     -- the topology-driven schedule (rounds over all nodes).
  * ``fsm``           -- Algorithm "Fast Sweeping Method".
  * ``async_random``  -- an unordered worklist with random priority inversions
                         (the extreme case of the soft priorities of Algorithm
                         "Asynchronous Marching Method").
  * ``residual``      -- the error metric of Table "tab:error".
  * ``dtilde``/``dhat`` -- the explicit formulas of Tables "tab:prec_1" and
                         "tab:prec_2".
  * ``newton``        -- Newton's method on the root function from the d-hat
                         guess (the precision section's practical variant).
  * ``dbar_rect``/``solve_rect``/``residual_rect`` -- the same exact-rounding
                         construction on a rectilinear grid (spacing varying
                         per axis and index): the irregular-grid case the
                         conclusion names as the next step.
  * ``parents``/``adjoint`` -- the paper is silent; implicit differentiation of
                         the discrete equations (Eq. "difference_as_root")
                         over the recorded upwind parents.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

from .build import ensure_built

SPEED = 0
SLOWNESS = 1
OP_DBAR = 0
OP_DHAT = 1
OP_DTILDE = 2
OP_NEWTON = 3

_lib = None

_d = ctypes.c_double
_i64 = ctypes.c_int64
_int = ctypes.c_int
_ptr = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        path = ensure_built()
        L = ctypes.CDLL(path)
        L.orc_dbar.restype = _d
        L.orc_dbar.argtypes = [ctypes.POINTER(_d), _d]
        L.orc_reaches.restype = _int
        L.orc_reaches.argtypes = [_d, ctypes.POINTER(_d), _d]
        L.orc_dtilde.restype = _d
        L.orc_dtilde.argtypes = [_d, _d, _d, _d]
        L.orc_dhat.restype = _d
        L.orc_dhat.argtypes = [_d, _d, _d, _d]
        L.orc_newton.restype = _d
        L.orc_newton.argtypes = [_d, _d, _d, _d]
        solve_args = [_int, _i64, _i64, _i64, _d, _ptr, _int, _i64, _ptr, _ptr, _int, _ptr, _ptr]
        for name in ("orc_fmm", "orc_sweep_all", "orc_fsm"):
            f = getattr(L, name)
            f.restype = _int
            f.argtypes = solve_args
        L.orc_async_random.restype = _int
        L.orc_async_random.argtypes = [_int, _i64, _i64, _i64, _d, _ptr, _int, _i64, _ptr, _ptr,
                                       _int, ctypes.c_uint64, _int, _ptr, _ptr]
        L.orc_dbar_rect.restype = _d
        L.orc_dbar_rect.argtypes = [ctypes.POINTER(_d)] * 4 + [_d]
        L.orc_reaches_rect.restype = _int
        L.orc_reaches_rect.argtypes = [_d] + [ctypes.POINTER(_d)] * 4 + [_d]
        L.orc_solve_rect.restype = _int
        L.orc_solve_rect.argtypes = [_int, _int, _i64, _i64, _i64, _ptr, _ptr, _ptr, _ptr, _int, _i64, _ptr, _ptr,
                                     ctypes.c_uint64, _ptr, _ptr]
        L.orc_residual_rect.restype = _i64
        L.orc_residual_rect.argtypes = [_int, _i64, _i64, _i64, _ptr, _ptr, _ptr, _ptr, _int, _i64, _ptr, _ptr,
                                        ctypes.POINTER(_d)]
        L.orc_fmm_resume.restype = _int
        L.orc_fmm_resume.argtypes = [_int, _i64, _i64, _i64, _d, _ptr, _int, _i64, _ptr, _ptr, _i64,
                                     _ptr, _ptr]
        L.orc_residual.restype = _i64
        L.orc_residual.argtypes = [_int, _i64, _i64, _i64, _d, _ptr, _int, _i64, _ptr, _ptr,
                                   _int, ctypes.POINTER(_d)]
        L.orc_parents.restype = None
        L.orc_parents.argtypes = [_int, _i64, _i64, _i64, _ptr, _i64, _ptr, _ptr]
        L.orc_adjoint.restype = _int
        L.orc_adjoint.argtypes = [_int, _i64, _i64, _i64, _d, _ptr, _int, _ptr, _ptr, _ptr,
                                  _ptr, _ptr]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(_ptr)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _prep(field, src, t0):
    field = _f64(field)
    if field.ndim == 2:
        field = field.reshape((1,) + field.shape)
    nz, ny, nx = field.shape
    src = np.ascontiguousarray(np.atleast_1d(src), dtype=np.int64)
    t0 = None if t0 is None else _f64(np.atleast_1d(t0))
    if t0 is not None and t0.shape != src.shape:
        raise ValueError("t0 must have one entry per source")
    return field, nx, ny, nz, src, t0


def _check(rc: int, what: str):
    if rc == -1:
        raise OracleError(f"{what}: field value not positive and finite")
    if rc == -2:
        raise MemoryError(what)
    if rc == -3:
        raise OracleError(f"{what}: bad source index or start time")
    if rc == -4:
        raise OracleError(f"{what}: update count exceeded the runaway guard")
    if rc != 0:
        raise OracleError(f"{what}: error {rc}")


# ---------------------------------------------------------------------------
# operator
# ---------------------------------------------------------------------------

def dbar(a, c: float) -> float:
    """Smallest binary64 r >= min(a) with S(r) >= c (a = up to 3 axis minima)."""
    arr = (_d * 3)(*([float(x) for x in a] + [np.inf] * (3 - len(a))))
    return lib().orc_dbar(arr, float(c))


def reaches(r: float, a, c: float) -> bool:
    arr = (_d * 3)(*([float(x) for x in a] + [np.inf] * (3 - len(a))))
    return bool(lib().orc_reaches(float(r), arr, float(c)))


def dtilde(tH: float, tV: float, v: float, h: float) -> float:
    q = h / v
    return lib().orc_dtilde(tH, tV, q * q, q)


def newton(tH: float, tV: float, v: float, h: float) -> float:
    """The Newton variant (precision section): Newton on alpha = 0 from the
    d-hat guess, two-sided branch; q = fl(h/v), c = fl(q*q)."""
    q = h / v
    return lib().orc_newton(tH, tV, q * q, q)


def dhat(tH: float, tV: float, v: float, h: float) -> float:
    q = h / v
    return lib().orc_dhat(tH, tV, q * q, q)


# ---------------------------------------------------------------------------
# schedules
# ---------------------------------------------------------------------------

def _solve(name: str, field, h, src, t0=None, kind=SPEED, op=OP_DBAR, ndim=None,
           extra=()) -> Tuple[np.ndarray, np.ndarray]:
    field, nx, ny, nz, src, t0 = _prep(field, src, t0)
    if ndim is None:
        ndim = 2 if nz == 1 else 3
    t = np.empty_like(field)
    stats = np.zeros(3, dtype=np.int64)
    f = getattr(lib(), name)
    rc = f(ndim, nx, ny, nz, float(h), _p(field), kind, src.size, _p(src), _p(t0),
           op, *extra, _p(t), _p(stats))
    _check(rc, name)
    return t, stats


def fmm(field, h, src, t0=None, kind=SPEED, op=OP_DBAR, ndim=None, return_stats=False):
    """Binary-heap fast marching; returns t with the field's shape."""
    t, st = _solve("orc_fmm", field, h, src, t0, kind, op, ndim)
    return (t, st) if return_stats else t


def fmm_resume(field, h, src, t_start, t0=None, kind=SPEED, ndim=None, max_pops: int = 0):
    """Fast marching resumed from `t_start` (an upper bound of the solution at
    every point, +inf allowed), sources fixed again.  Returns (t, finished):
    finished is False when max_pops > 0 stopped the loop early, leaving an
    upper bound that can be resumed again."""
    field, nx, ny, nz, src, t0 = _prep(field, src, t0)
    if ndim is None:
        ndim = 2 if nz == 1 else 3
    t = np.array(_f64(t_start).reshape(field.shape), copy=True)
    stats = np.zeros(3, dtype=np.int64)
    rc = lib().orc_fmm_resume(ndim, nx, ny, nz, float(h), _p(field), kind, src.size, _p(src), _p(t0),
                              int(max_pops), _p(t), _p(stats))
    if rc == -5:
        raise OracleError("fmm_resume: a start value is NaN or negative")
    if rc not in (0, 1):
        _check(rc, "fmm_resume")
    return t, rc == 0


def sweep_all(field, h, src, t0=None, kind=SPEED, op=OP_DBAR, ndim=None):
    return _solve("orc_sweep_all", field, h, src, t0, kind, op, ndim)[0]


def fsm(field, h, src, t0=None, kind=SPEED, op=OP_DBAR, ndim=None):
    return _solve("orc_fsm", field, h, src, t0, kind, op, ndim)[0]


def async_random(field, h, src, seed: int, t0=None, kind=SPEED, op=OP_DBAR, ndim=None,
                 push_on_change: bool = False):
    return _solve("orc_async_random", field, h, src, t0, kind, op, ndim,
                  extra=(ctypes.c_uint64(seed), int(push_on_change)))[0]


def residual(t, field, h, src, kind=SPEED, op=OP_DBAR, ndim=None) -> Tuple[int, float]:
    """(number of non-source points the operator would still change, max rel. change)."""
    field, nx, ny, nz, src, _ = _prep(field, src, None)
    if ndim is None:
        ndim = 2 if nz == 1 else 3
    t = _f64(t).reshape(field.shape)
    worst = _d(0.0)
    n = lib().orc_residual(ndim, nx, ny, nz, float(h), _p(field), kind, src.size, _p(src),
                           _p(t), op, ctypes.byref(worst))
    if n < 0:
        raise OracleError("residual: field value not positive and finite")
    return int(n), float(worst.value)


def parents(t, src, ndim=None) -> np.ndarray:
    t = _f64(t)
    if t.ndim == 2:
        t = t.reshape((1,) + t.shape)
    nz, ny, nx = t.shape
    if ndim is None:
        ndim = 2 if nz == 1 else 3
    src = np.ascontiguousarray(np.atleast_1d(src), dtype=np.int64)
    par = np.empty(t.shape, dtype=np.uint8)
    lib().orc_parents(ndim, nx, ny, nz, _p(t), src.size, _p(src), _p(par))
    return par


def adjoint(t, par, field, h, g, kind=SPEED, ndim=None, return_mu=False):
    """d loss / d slowness for d loss / d t = g, by reverse (decreasing t) order."""
    field = _f64(field)
    if field.ndim == 2:
        field = field.reshape((1,) + field.shape)
    nz, ny, nx = field.shape
    if ndim is None:
        ndim = 2 if nz == 1 else 3
    t = _f64(t).reshape(field.shape)
    par = np.ascontiguousarray(par, dtype=np.uint8).reshape(field.shape)
    g = _f64(g).reshape(field.shape)
    grad = np.empty_like(field)
    mu = np.empty_like(field) if return_mu else None
    rc = lib().orc_adjoint(ndim, nx, ny, nz, float(h), _p(field), kind, _p(t), _p(par), _p(g),
                           _p(grad), _p(mu))
    _check(rc, "adjoint")
    return (grad, mu) if return_mu else grad


# ---------------------------------------------------------------------------
# rectilinear grids (per-axis coordinates; the irregular-grid operator)
# ---------------------------------------------------------------------------

def _arr3(v):
    return (_d * 3)(*([float(x) for x in v] + [np.inf] * (3 - len(v))))


def dbar_rect(am, ap, wm, wp, c: float) -> float:
    """Smallest binary64 r >= min(a) with S(r) >= c, S summing per axis the
    square of max(fl(fl(r - am)*wm), fl(fl(r - ap)*wp), 0), largest term first
    (up to three axes; missing axes are +inf with weight 1)."""
    w1 = lambda v: (_d * 3)(*([float(x) for x in v] + [1.0] * (3 - len(v))))
    return lib().orc_dbar_rect(_arr3(am), _arr3(ap), w1(wm), w1(wp), float(c))


def reaches_rect(r: float, am, ap, wm, wp, c: float) -> bool:
    w1 = lambda v: (_d * 3)(*([float(x) for x in v] + [1.0] * (3 - len(v))))
    return bool(lib().orc_reaches_rect(float(r), _arr3(am), _arr3(ap), w1(wm), w1(wp), float(c)))


def _rect_prep(field, xs, ys, zs):
    field = _f64(field)
    if field.ndim == 2:
        field = field.reshape((1,) + field.shape)
    nz, ny, nx = field.shape
    xs = _f64(xs).reshape(-1)
    ys = _f64(ys).reshape(-1)
    ndim = 2 if zs is None else 3
    zs = _f64(zs).reshape(-1) if zs is not None else None
    if xs.size != nx or ys.size != ny or (zs is not None and zs.size != nz) or (zs is None and nz != 1):
        raise ValueError("coordinates must match the field's shape")
    return field, nx, ny, nz, ndim, xs, ys, zs


_RECT_SCHEDULES = {"fmm": 0, "sweep_all": 1, "fsm": 2, "async_random": 3}


def solve_rect(field, xs, ys, zs, src, t0=None, kind=SPEED, schedule: str = "fmm", seed: int = 0):
    """Arrival times on a rectilinear grid (coordinates xs, ys[, zs]; zs None
    for 2D) with the rectilinear exact operator, by the named schedule:
    fast marching, topology-driven rounds, fast sweeping or a random-order
    worklist."""
    field, nx, ny, nz, ndim, xs, ys, zs = _rect_prep(field, xs, ys, zs)
    src = np.ascontiguousarray(np.atleast_1d(src), dtype=np.int64)
    t0 = None if t0 is None else _f64(np.atleast_1d(t0))
    t = np.empty_like(field)
    stats = np.zeros(3, dtype=np.int64)
    rc = lib().orc_solve_rect(_RECT_SCHEDULES[schedule], ndim, nx, ny, nz, _p(xs), _p(ys), _p(zs), _p(field), kind,
                              src.size, _p(src), _p(t0), ctypes.c_uint64(seed), _p(t), _p(stats))
    if rc == -6:
        raise OracleError("solve_rect: coordinates must increase strictly with finite reciprocal spacings")
    _check(rc, "solve_rect")
    return t


def residual_rect(t, field, xs, ys, zs, src, kind=SPEED) -> Tuple[int, float]:
    field, nx, ny, nz, ndim, xs, ys, zs = _rect_prep(field, xs, ys, zs)
    src = np.ascontiguousarray(np.atleast_1d(src), dtype=np.int64)
    t = _f64(t).reshape(field.shape)
    worst = _d(0.0)
    n = lib().orc_residual_rect(ndim, nx, ny, nz, _p(xs), _p(ys), _p(zs), _p(field), kind, src.size, _p(src),
                                _p(t), ctypes.byref(worst))
    if n < 0:
        raise OracleError("residual_rect: bad field or coordinates")
    return int(n), float(worst.value)


# ---------------------------------------------------------------------------
# dense references for tiny grids (numpy)
# ---------------------------------------------------------------------------

def dense_adjoint(t, par, field, h, g, kind=SPEED) -> np.ndarray:
    """Assemble the linearised system dt = J dt + D ds over the upwind parents and
    return D^T (I - J)^{-T} g by a dense solve (tiny grids only)."""
    field = _f64(field)
    if field.ndim == 2:
        field = field.reshape((1,) + field.shape)
    shape = field.shape
    nz, ny, nx = shape
    ndim = 2 if nz == 1 else 3
    n = field.size
    if n > 6000:
        raise ValueError("dense_adjoint is for tiny grids")
    t = _f64(t).ravel()
    par = np.asarray(par, dtype=np.uint8).ravel()
    f = field.ravel()
    q = h / f if kind == SPEED else h * f
    stride = (1, nx, nx * ny)
    J = np.zeros((n, n))
    D = np.zeros(n)
    for i in range(n):
        if par[i] & 0x80:
            continue
        ws = []
        for k in range(ndim):
            code = (par[i] >> (2 * k)) & 3
            if code == 1:
                ws.append((i - stride[k], t[i] - t[i - stride[k]]))
            elif code == 2:
                ws.append((i + stride[k], t[i] - t[i + stride[k]]))
        W = sum(w for _, w in ws)
        for j, w in ws:
            J[i, j] += w / W
        D[i] = h * q[i] / W
    lam = np.linalg.solve((np.eye(n) - J).T, _f64(g).ravel())
    return (D * lam).reshape(shape)

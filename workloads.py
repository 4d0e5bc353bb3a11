"""Seeded synthetic inputs for the Eikonal travel-time workloads.

This module only draws inputs (grids, speed / slowness fields, source and
receiver positions).  It holds none of the solver's arithmetic, so both the CPU
oracle (``oracle/``) and the HIP path may use it without sharing any method code.

Layout everywhere: C-order ``[nz][ny][nx]`` float64, x fastest; a 2D grid has
``nz == 1``.  A grid point (ix, iy, iz) has flat index ``(iz*ny + iy)*nx + ix``.

The paper evaluates on the Marmousi2 model (Materials and Methods section), which
is not available here; the layered, noisy and blocky fields below stand in for
it with the same kind of structure (smooth layering with depth, strong speed
contrasts).
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field as dc_field
from typing import List, Optional, Sequence, Tuple

import numpy as np

SPEED = 0
SLOWNESS = 1


@dataclass
class Problem:
    """One Eikonal solve: grid, field, point sources (t0 = 0 unless given)."""

    ndim: int
    nx: int
    ny: int
    nz: int
    h: float
    field: np.ndarray            # float64, shape (nz, ny, nx)
    kind: int                    # SPEED or SLOWNESS
    src: np.ndarray              # int64 flat indices
    t0: Optional[np.ndarray] = None   # float64 per source, None -> all 0.0
    name: str = ""
    meta: dict = dc_field(default_factory=dict)

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    @property
    def npts(self) -> int:
        return self.nx * self.ny * self.nz

    def sha256(self) -> str:
        m = hashlib.sha256()
        m.update(np.ascontiguousarray(self.field).tobytes())
        m.update(np.ascontiguousarray(self.src, dtype=np.int64).tobytes())
        if self.t0 is not None:
            m.update(np.ascontiguousarray(self.t0, dtype=np.float64).tobytes())
        return m.hexdigest()[:16]


def flat_index(ix, iy, iz, nx: int, ny: int):
    return (np.asarray(iz, dtype=np.int64) * ny + np.asarray(iy, dtype=np.int64)) * nx \
        + np.asarray(ix, dtype=np.int64)


def unflatten(idx, nx: int, ny: int):
    idx = np.asarray(idx, dtype=np.int64)
    ix = idx % nx
    iy = (idx // nx) % ny
    iz = idx // (nx * ny)
    return ix, iy, iz


# ---------------------------------------------------------------------------
# fields
# ---------------------------------------------------------------------------

def smooth_unit_noise(shape: Sequence[int], rng: np.random.Generator,
                      sigma: float = 8.0) -> np.ndarray:
    """Gaussian white noise smoothed by a Gaussian filter of ``sigma`` cells
    (reflecting edges, kernel truncated at 4 sigma), shifted and scaled to zero
    mean and unit population standard deviation."""
    from scipy.ndimage import gaussian_filter

    g = rng.standard_normal(tuple(shape)).astype(np.float32)
    g = gaussian_filter(g, sigma=sigma, mode="reflect", truncate=4.0).astype(np.float64)
    g -= g.mean()
    sd = g.std()
    if sd > 0:
        g /= sd
    return g


def layered_speed(nx: int, ny: int, nz: int, rng: np.random.Generator,
                  vtop: float = 1500.0, vbottom: float = 6000.0, nlayers: int = 8,
                  noise: float = 0.1, sigma: float = 8.0) -> np.ndarray:
    """Flat layers whose speed grows linearly with depth from ``vtop`` to
    ``vbottom`` (layer k of ``nlayers`` covers depths floor(8 z / nz) == k), times
    (1 + noise * g) with g a smoothed unit-variance Gaussian field."""
    z = np.arange(nz)
    k = (z * nlayers) // nz
    vl = vtop + k * (vbottom - vtop) / (nlayers - 1)
    v = np.broadcast_to(vl[:, None, None], (nz, ny, nx)).astype(np.float64)
    if noise != 0.0:
        g = smooth_unit_noise((nz, ny, nx), rng, sigma)
        v = v * (1.0 + noise * g)
    v = np.ascontiguousarray(v)
    if not np.all(v > 0):
        raise ValueError("layered speed produced a non-positive value")
    return v


def blocky_speed(nx: int, ny: int, rng: np.random.Generator, block: int = 64,
                 values: Sequence[float] = (0.5, 1.0, 2.0, 5.0)) -> np.ndarray:
    """2D field made of ``block`` x ``block`` cells, each drawn uniformly from
    ``values`` (a high-contrast, blocky medium)."""
    by = -(-ny // block)
    bx = -(-nx // block)
    choice = rng.integers(0, len(values), size=(by, bx))
    blocks = np.asarray(values, dtype=np.float64)[choice]
    v = np.repeat(np.repeat(blocks, block, axis=0), block, axis=1)[:ny, :nx]
    return np.ascontiguousarray(v.reshape(1, ny, nx))


def blob_perturbation(shape: Tuple[int, int, int], center: Tuple[float, float, float],
                      radius: float = 20.0, amp: float = 0.05) -> np.ndarray:
    """Multiplicative factor 1 + amp * exp(-|x - c|^2 / (2 radius^2)) (cells)."""
    nz, ny, nx = shape
    cx, cy, cz = center
    zz = (np.arange(nz) - cz)[:, None, None] ** 2
    yy = (np.arange(ny) - cy)[None, :, None] ** 2
    xx = (np.arange(nx) - cx)[None, None, :] ** 2
    return 1.0 + amp * np.exp(-(xx + yy + zz) / (2.0 * radius * radius))


# ---------------------------------------------------------------------------
# the five workloads
# ---------------------------------------------------------------------------

def point_source_2d(n: int = 101, h: float = 1.0, v: float = 1.0,
                    src: Tuple[int, int] = (50, 50)) -> Problem:
    """2D n x n grid, constant speed, one point source with t = 0."""
    field = np.full((1, n, n), v, dtype=np.float64)
    s = flat_index(src[0], src[1], 0, n, n).reshape(1)
    return Problem(2, n, n, 1, h, field, SPEED, s, None, name=f"2d_{n}x{n}_const")


def layered_3d(nx: int = 512, ny: int = 512, nz: int = 256, h: float = 10.0,
               seed: int = 2, src: Optional[Tuple[int, int, int]] = None,
               sigma: float = 8.0) -> Problem:
    """3D layered + smoothed-noise speed (1500..6000 m/s, 8 layers), one source
    at the surface centre unless ``src`` is given."""
    rng = np.random.default_rng(seed)
    v = layered_speed(nx, ny, nz, rng, sigma=sigma)
    if src is None:
        src = (nx // 2, ny // 2, 0)
    s = flat_index(*src, nx, ny).reshape(1)
    return Problem(3, nx, ny, nz, h, v, SPEED, s, None,
                   name=f"3d_{nx}x{ny}x{nz}_layered_seed{seed}")


def blocky_2d(n: int = 4096, nsrc: int = 16, seed: int = 3, block: int = 64,
              h: float = 1.0) -> Problem:
    """2D high-contrast blocky speed with ``nsrc`` distinct random point sources
    (all t = 0, solved jointly)."""
    rng = np.random.default_rng(seed)
    v = blocky_speed(n, n, rng, block=block)
    src = rng.choice(n * n, size=nsrc, replace=False).astype(np.int64)
    return Problem(2, n, n, 1, h, v, SPEED, np.sort(src), None,
                   name=f"2d_{n}x{n}_blocky_{nsrc}src_seed{seed}")


def folded_layers_2d(nx: int = 13601, nz: int = 2801, up: int = 4, h: float = 1.25, seed: int = 6,
                     nlayers: int = 14, water_rows: Optional[int] = None, noise: float = 0.05,
                     sigma: float = 8.0) -> Problem:
    """Synthetic stand-in for the paper's upsampled Marmousi grid: a 2D model
    of ``nz`` depth rows by ``nx`` columns (spacing ``h``), then repeated
    ``up`` times along each axis (nearest-neighbour upsampling, spacing
    h / up).  Structure: a water layer of ``water_rows`` rows (default about an
    eighth of the depth) at 1500 m/s over
    ``nlayers`` layers whose speeds rise from 1600 to 4700 m/s with seeded
    jitter, bounded by folded interfaces (sums of three random sinusoids) that a
    steep normal fault offsets in the middle third, times (1 + noise * g) with
    g smoothed unit noise.  One source at the surface centre.  The result is a
    2D Problem with ny = nz * up rows (depth) and nx * up columns."""
    rng = np.random.default_rng(seed)
    if water_rows is None:
        water_rows = max(1, (nz * 9) // 70)
    x = np.arange(nx, dtype=np.float64)
    span = nz - water_rows
    base = water_rows + span * (np.arange(1, nlayers) / nlayers)
    fault_x = nx * (0.4 + 0.2 * rng.random())
    throw = 0.04 * span
    iface = []
    for k in range(nlayers - 1):
        amp = rng.uniform(0.01, 0.05, 3) * span
        wav = rng.uniform(0.5, 4.0, 3) * 2.0 * np.pi / nx
        ph = rng.uniform(0.0, 2.0 * np.pi, 3)
        d = base[k] + (amp[:, None] * np.sin(wav[:, None] * x[None, :] + ph[:, None])).sum(0)
        d = d + np.where(x > fault_x + 0.3 * (d - water_rows), throw, 0.0)
        iface.append(np.clip(d, water_rows + 1, nz - 1))
    speeds = np.concatenate([[1500.0], np.linspace(1600.0, 4700.0, nlayers) *
                             (1.0 + 0.04 * rng.standard_normal(nlayers))])
    z = np.arange(nz, dtype=np.float64)[:, None]
    layer = np.zeros((nz, nx), dtype=np.int16)
    for d in iface:
        layer += (z >= d[None, :]).astype(np.int16)
    layer = np.where(z < water_rows, 0, layer + 1)
    v = speeds[layer]
    if noise != 0.0:
        g = smooth_unit_noise((nz, nx), rng, sigma)
        v = np.where(z < water_rows, v, v * (1.0 + noise * g))
    if up > 1:
        v = np.repeat(np.repeat(v, up, axis=0), up, axis=1)
    v = np.ascontiguousarray(v.reshape(1, nz * up, nx * up))
    if not np.all(v > 0):
        raise ValueError("folded-layer speed produced a non-positive value")
    NX, NY = nx * up, nz * up
    src = flat_index(NX // 2, 0, 0, NX, NY).reshape(1)
    return Problem(2, NX, NY, 1, h / up, v, SPEED, src, None,
                   name=f"2d_{NX}x{NY}_folded_layers_seed{seed}")


BATCH_SIZES = ((128, 128, 128), (192, 192, 128), (256, 256, 128))


def batched_shots(nshots: int = 64, seed: int = 4, h: float = 10.0,
                  sizes: Sequence[Tuple[int, int, int]] = BATCH_SIZES,
                  sigma: float = 8.0) -> List[Problem]:
    """Independent shots on layered + noise models of uneven sizes (drawn from
    ``sizes`` by seed), one random surface source each."""
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(nshots)
    top = np.random.default_rng(ss.spawn(1)[0])
    out = []
    for i in range(nshots):
        nx, ny, nz = sizes[int(top.integers(0, len(sizes)))]
        rng = np.random.default_rng(children[i])
        v = layered_speed(nx, ny, nz, rng, sigma=sigma)
        sx = int(rng.integers(0, nx))
        sy = int(rng.integers(0, ny))
        s = flat_index(sx, sy, 0, nx, ny).reshape(1)
        out.append(Problem(3, nx, ny, nz, h, v, SPEED, s, None,
                           name=f"shot{i}_{nx}x{ny}x{nz}"))
    return out


@dataclass
class TomographyCase:
    """Surface-acquisition travel-time tomography set-up.

    ``s0`` is the background slowness (1/v of a layered + noise model),
    ``s_true`` the same model with a +amp Gaussian slowness blob; the observed
    times are solves on ``s_true`` (computed by whichever solver is tested)."""

    nx: int
    ny: int
    nz: int
    h: float
    s0: np.ndarray
    s_true: np.ndarray
    sources: np.ndarray      # int64 flat indices, one shot each
    receivers: np.ndarray    # int64 flat indices, shared by every shot
    blob_center: Tuple[int, int, int]


def tomography(nx: int = 256, ny: int = 256, nz: int = 128, h: float = 10.0,
               nshots: int = 32, nrec_side: int = 32, seed: int = 5,
               radius: float = 20.0, amp: float = 0.05, sigma: float = 8.0) -> TomographyCase:
    rng = np.random.default_rng(seed)
    v = layered_speed(nx, ny, nz, rng, sigma=sigma)
    s0 = 1.0 / v
    lo = int(min(radius, nx // 4, ny // 4, nz // 4))
    c = (int(rng.integers(lo, nx - lo)), int(rng.integers(lo, ny - lo)),
         int(rng.integers(lo, nz - lo)))
    s_true = s0 * blob_perturbation((nz, ny, nx), c, radius=radius, amp=amp)
    sx = rng.integers(0, nx, size=nshots)
    sy = rng.integers(0, ny, size=nshots)
    sources = flat_index(sx, sy, 0, nx, ny)
    stepx = max(nx // nrec_side, 1)
    stepy = max(ny // nrec_side, 1)
    rx = (stepx // 2 + stepx * np.arange(nrec_side)) % nx
    ry = (stepy // 2 + stepy * np.arange(nrec_side)) % ny
    RX, RY = np.meshgrid(rx, ry, indexing="xy")
    receivers = flat_index(RX.ravel(), RY.ravel(), 0, nx, ny)
    return TomographyCase(nx, ny, nz, h, np.ascontiguousarray(s0),
                          np.ascontiguousarray(s_true), sources.astype(np.int64),
                          receivers.astype(np.int64), c)


def stretched_coords(n: int, h0: float, ratio: float, x0: float = 0.0) -> np.ndarray:
    """n increasing coordinates from x0 whose spacing grows geometrically from
    h0 by `ratio` per cell (ratio 1: uniform spacing h0)."""
    steps = h0 * ratio ** np.arange(n - 1, dtype=np.float64)
    return x0 + np.concatenate([[0.0], np.cumsum(steps)])


def jittered_coords(n: int, h: float, rng: np.random.Generator, jitter: float = 0.3) -> np.ndarray:
    """n increasing coordinates with spacings h * (1 + U(-jitter, jitter))."""
    steps = h * (1.0 + rng.uniform(-jitter, jitter, n - 1))
    return np.concatenate([[0.0], np.cumsum(steps)])


def random_field(shape: Tuple[int, int, int], rng: np.random.Generator,
                 lo: float = 0.5, hi: float = 5.0, block: int = 1) -> np.ndarray:
    """Uniform random speeds in [lo, hi), constant over ``block``-sized cubes."""
    nz, ny, nx = shape
    bz, by, bx = -(-nz // block), -(-ny // block), -(-nx // block)
    f = rng.uniform(lo, hi, size=(bz, by, bx))
    for ax in range(3):
        f = np.repeat(f, block, axis=ax)
    return np.ascontiguousarray(f[:nz, :ny, :nx])


def config(k: int) -> Problem:
    """The single-problem workloads by number (1: 2D 101^2 point source,
    2: 3D 512x512x256 layered, 3: 2D 4096^2 blocky with 16 sources)."""
    if k == 1:
        return point_source_2d()
    if k == 2:
        return layered_3d()
    if k == 3:
        return blocky_2d()
    raise ValueError("config(k) covers the single-problem workloads 1..3")

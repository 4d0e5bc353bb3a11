"""Autotuner for the persistent solver's free parameters: the tile shape, the
priority bucket width delta, the lookahead window of buckets a workgroup may
take work from, the bucket horizon and the pass structure.

The paper leaves the priority scale open and notes that the best trade-off
between priority inversions and contention depends on hardware and input
(section "Deterministic Properties").  Neither parameter can change the
result (Theorem 1), so the tuner times every candidate, checks that all
candidates produce bit-identical times, and stores the fastest in a JSON cache
keyed by (GPU arch, ndim, grid shape, field kind).  Candidate deltas are
multiples of the median per-cell travel time h/v times the tile edge.

    python -m paper_2103_05694_amd.autotune layered512 blocky4096
"""
from __future__ import annotations

import json
import os
import sys
import time
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import torch

from . import api

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned.json")
ARCH = "gfx950"

TILES = {3: [(16, 8, 8), (8, 8, 8), (32, 8, 4)],
         2: [(32, 32), (16, 16), (64, 16)]}
DELTA_FACTORS = (0.0, 0.25, 0.5, 1.0, 2.0, 4.0, 8.0)
GRID_BLOCKS = (0,)       # 0 = as many workgroups as fit on the device
HORIZONS = (0, 1, 2)     # 0 = off; k = settle values below (bucket + k) only
PACKED = (False, True)   # relaxation passes: per-thread points, or compacted lists
LOOKAHEADS = (2, 4, 8, 16)  # second stage: buckets beyond the lowest a claim may take work from
LOOKAHEAD_FACTORS = (0.0625, 0.125, 0.25, 0.5, 1.0)  # bucket widths tried with a lookahead window


def _key(shape: Sequence[int], kind: str) -> str:
    return f"{ARCH}:{len(shape)}d:{'x'.join(str(int(s)) for s in shape)}:{kind}"


def _load() -> Dict[str, dict]:
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def lookup(shape: Sequence[int], kind: str = "speed") -> Optional[dict]:
    """Cached best configuration for this shape (exact), else None."""
    return _load().get(_key(shape, kind))


def _time(fn, reps: int) -> float:
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def tune(field: torch.Tensor, h: float, sources, kind: str = "speed",
         tiles: Optional[Iterable[Tuple[int, ...]]] = None,
         delta_factors: Sequence[float] = DELTA_FACTORS, reps: int = 3,
         grid_blocks: Sequence[int] = GRID_BLOCKS, horizons: Sequence[int] = HORIZONS,
         packed: Sequence[bool] = PACKED, lookaheads: Sequence[int] = LOOKAHEADS,
         lookahead_factors: Sequence[float] = LOOKAHEAD_FACTORS, save: bool = True, log=print) -> dict:
    """Time every (tile, delta, grid size, horizon, pass structure) candidate on
    this problem without a lookahead, then, with the best of them, every
    (lookahead, narrower delta) pair; all candidates must agree bitwise."""
    nd = field.dim()
    tiles = list(tiles) if tiles is not None else TILES[nd]
    f64 = field.to(torch.float64)
    q = (h / f64) if kind == "speed" else (h * f64)
    qmed = float(q.flatten()[:: max(q.numel() // 100000, 1)].median())
    ref = None
    results: List[dict] = []
    out = torch.empty_like(field)

    def run(tile, fac, gb, hz, pk, la=0):
        nonlocal ref
        delta = fac * qmed * min(tile[:nd])
        fn = lambda: api.solve(field, h, sources, kind=kind, delta=delta, tile=tile, out=out,
                               grid_blocks=gb, horizon=hz, packed=pk, lookahead=la, check_status=False)
        fn()
        api.status()
        t = out.clone()
        if ref is None:
            ref = t
        elif not torch.equal(ref, t):
            raise RuntimeError(f"candidate tile={tile} delta={delta} grid={gb} horizon={hz} packed={pk} "
                               f"lookahead={la} changed the result")
        sec = _time(fn, reps)
        api.status()
        results.append({"tile": list(tile), "delta": delta, "delta_factor": fac, "grid_blocks": gb,
                        "horizon": hz, "packed": pk, "lookahead": la, "ms": sec * 1e3})
        log(f"  tile {tile} delta {delta:.4g} ({fac:.3g} x qmed x edge) grid {gb} horizon {hz} packed {pk} "
            f"lookahead {la}: {sec * 1e3:.3f} ms")

    for tile in tiles:
        for fac in delta_factors:
            for hz in (horizons if fac > 0 else (0,)):
                for gb in grid_blocks:
                    for pk in packed:
                        run(tile, fac, gb, hz, pk)
    # a lookahead window with narrower buckets, on the first stage's best for
    # each tile and pass structure (what wins without a window often does not
    # win with it)
    for tile in tiles:
        for pk in packed:
            rows = [r for r in results if tuple(r["tile"]) == tuple(tile) and r["packed"] == pk]
            if not rows:
                continue
            best = min(rows, key=lambda r: r["ms"])
            for la in lookaheads:
                for fac in lookahead_factors:
                    run(tuple(tile), fac, best["grid_blocks"], best["horizon"], pk, la)
    # refine the best bucket width between its neighbours on the doubling grid
    best = min(results, key=lambda r: r["ms"])
    if best["delta_factor"] > 0:
        for step in (2.0 ** -0.5, 2.0 ** 0.5):
            run(tuple(best["tile"]), best["delta_factor"] * step, best["grid_blocks"], best["horizon"],
                best["packed"], best["lookahead"])
    best = min(results, key=lambda r: r["ms"])
    entry = {"tile": best["tile"], "delta": best["delta"], "grid_blocks": best["grid_blocks"],
             "horizon": best["horizon"], "packed": best["packed"], "lookahead": best["lookahead"],
             "ms": best["ms"], "qmed": qmed, "candidates": results}
    if save:
        cache = _load()
        cache[_key(field.shape, kind)] = entry
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return entry


def _batch_key(nshots: int, shape: Sequence[int], kind: str) -> str:
    return f"{ARCH}:batch{int(nshots)}:{len(shape)}d:{'x'.join(str(int(s)) for s in shape)}:{kind}"


def lookup_batch(nshots: int, shape: Sequence[int], kind: str = "slowness") -> Optional[dict]:
    """Cached best configuration for a batch of `nshots` shots of this shape."""
    return _load().get(_batch_key(nshots, shape, kind))


def tune_batch(fields: Sequence[torch.Tensor], h: float, sources, receivers, kind: str = "slowness",
               tiles: Optional[Iterable[Tuple[int, ...]]] = None,
               delta_factors: Sequence[float] = (0.25, 0.5, 1.0, 2.0, 4.0),
               adj_delta_factors: Sequence[float] = (0.0, 0.5, 1.0, 2.0, 4.0, 8.0),
               grid_blocks: Sequence[int] = (0,), packed: Sequence[bool] = PACKED, reps: int = 2,
               lookaheads: Sequence[int] = LOOKAHEADS, lookahead_factors: Sequence[float] = LOOKAHEAD_FACTORS,
               save: bool = True, log=print) -> dict:
    """Tune a batch of shots (forward with parents, then the adjoint) in one
    persistent launch each: a batch has many times the parallel work of one
    shot, so its best trade-off differs, and the readiness-driven adjoint is
    tuned on its own.  All candidates must agree bitwise."""
    nd = fields[0].dim()
    tiles = list(tiles) if tiles is not None else TILES[nd]
    f64 = fields[0].to(torch.float64)
    q = (h / f64) if kind == "speed" else (h * f64)
    qmed = float(q.flatten()[:: max(q.numel() // 100000, 1)].median())
    b = api.pack(fields, [h] * len(fields), sources, kind)
    t = torch.empty(b.npts, dtype=torch.float64, device=b.field.device)
    par = torch.empty(b.npts, dtype=torch.uint8, device=b.field.device)
    g = torch.zeros_like(t)
    offs = [int(b.offsets[i]) for i in range(len(fields))]
    rec = torch.cat([torch.as_tensor(r, device=t.device).reshape(-1) + o for r, o in zip(receivers, offs)])
    g[rec] = 1.0
    grad = torch.empty_like(t)
    fwd: List[dict] = []
    ref = None

    def run_fwd(tile, fac, gb, pk, la=0):
        nonlocal ref
        delta = fac * qmed * min(tile[:nd])
        fn = lambda: api.solve_packed(b, t, par, delta, tile, grid_blocks=gb, packed=pk, lookahead=la)
        fn()
        api.status()
        if ref is None:
            ref = (t.clone(), par.clone())
        elif not (torch.equal(ref[0], t) and torch.equal(ref[1], par)):
            raise RuntimeError(f"batch forward tile={tile} delta={delta} grid={gb} packed={pk} lookahead={la} "
                               "changed the result")
        sec = _time(fn, reps)
        api.status()
        fwd.append({"tile": list(tile), "delta": delta, "delta_factor": fac, "grid_blocks": gb, "packed": pk,
                    "lookahead": la, "ms": sec * 1e3})
        log(f"  batch forward tile {tile} delta {delta:.4g} grid {gb} packed {pk} lookahead {la}: "
            f"{sec * 1e3:.2f} ms")

    for tile in tiles:
        for fac in delta_factors:
            for gb in grid_blocks:
                for pk in packed:
                    run_fwd(tile, fac, gb, pk)
    for tile in tiles:
        for pk in packed:
            rows = [r for r in fwd if tuple(r["tile"]) == tuple(tile) and r["packed"] == pk]
            if not rows:
                continue
            bt = min(rows, key=lambda r: r["ms"])
            for la in lookaheads:
                for fac in lookahead_factors:
                    run_fwd(tuple(tile), fac, bt["grid_blocks"], pk, la)
    bf = min(fwd, key=lambda r: r["ms"])
    if bf["delta_factor"] > 0:
        for step in (2.0 ** -0.5, 2.0 ** 0.5):
            run_fwd(tuple(bf["tile"]), bf["delta_factor"] * step, bf["grid_blocks"], bf["packed"], bf["lookahead"])
    t.copy_(ref[0])
    par.copy_(ref[1])
    adj: List[dict] = []
    gref = None

    def run_adj(tile, fac, gb, pk, la=0):
        nonlocal gref
        delta = fac * qmed * min(tile[:nd])
        fn = lambda: api.adjoint_packed(b, t, par, g, grad, delta=delta, tile=tile, grid_blocks=gb, packed=pk,
                                        lookahead=la)
        fn()
        api.status()
        if gref is None:
            gref = grad.clone()
        elif not torch.equal(gref, grad):
            raise RuntimeError(f"batch adjoint tile={tile} delta={delta} grid={gb} packed={pk} lookahead={la} "
                               "changed the result")
        sec = _time(fn, reps)
        api.status()
        adj.append({"tile": list(tile), "delta": delta, "delta_factor": fac, "grid_blocks": gb, "packed": pk,
                    "lookahead": la, "ms": sec * 1e3})
        log(f"  batch adjoint tile {tile} delta {delta:.4g} grid {gb} packed {pk} lookahead {la}: "
            f"{sec * 1e3:.2f} ms")

    for tile in tiles:
        for fac in adj_delta_factors:
            for gb in grid_blocks:
                for pk in packed:
                    run_adj(tile, fac, gb, pk)
    ba = min(adj, key=lambda r: r["ms"])
    for la in lookaheads:
        for fac in (0.5, 2.0 ** -0.5, 1.0, 2.0 ** 0.5, 2.0):
            run_adj(tuple(ba["tile"]), fac * max(ba["delta_factor"], 0.5), ba["grid_blocks"], ba["packed"], la)
    ba = min(adj, key=lambda r: r["ms"])
    if ba["delta_factor"] > 0:
        for step in (2.0 ** -0.5, 2.0 ** 0.5):
            run_adj(tuple(ba["tile"]), ba["delta_factor"] * step, ba["grid_blocks"], ba["packed"], ba["lookahead"])
    bf = min(fwd, key=lambda r: r["ms"])
    ba = min(adj, key=lambda r: r["ms"])
    entry = {"tile": bf["tile"], "delta": bf["delta"], "grid_blocks": bf["grid_blocks"], "horizon": 0,
             "packed": bf["packed"], "lookahead": bf["lookahead"],
             "adj_tile": ba["tile"], "adj_delta": ba["delta"], "adj_grid_blocks": ba["grid_blocks"],
             "adj_packed": ba["packed"], "adj_lookahead": ba["lookahead"],
             "ms": bf["ms"] + ba["ms"], "forward_ms": bf["ms"], "adjoint_ms": ba["ms"], "qmed": qmed,
             "forward_candidates": fwd, "adjoint_candidates": adj}
    if save:
        cache = _load()
        cache[_batch_key(len(fields), fields[0].shape, kind)] = entry
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return entry


RECT_TILES = {3: [(8, 8, 8), (8, 8, 4), (16, 8, 4), (16, 8, 8)], 2: [(32, 32), (16, 16), (64, 16)]}


def _rect_key(shape: Sequence[int], kind: str) -> str:
    return f"{ARCH}:rect:{len(shape)}d:{'x'.join(str(int(s)) for s in shape)}:{kind}"


def lookup_rect(shape: Sequence[int], kind: str = "speed") -> Optional[dict]:
    """Cached best configuration of the rectilinear solve for this shape."""
    return _load().get(_rect_key(shape, kind))


def tune_rect(field: torch.Tensor, xs, ys, zs, sources, kind: str = "speed",
              tiles: Optional[Iterable[Tuple[int, ...]]] = None,
              delta_factors: Sequence[float] = (0.0625, 0.125, 0.25, 0.5),
              lookaheads: Sequence[int] = (0, 8, 16), reps: int = 3, save: bool = True, log=print) -> dict:
    """Time every (tile, bucket width, lookahead) candidate of the rectilinear
    solve (eik_solve_rect), refine the best width at 2^(+-1/2), and keep the
    fastest; all candidates must agree bitwise.  The width scale is the median
    slowness times the median grid spacing times the tile's shortest edge."""
    import numpy as np
    nd = field.dim()
    tiles = list(tiles) if tiles is not None else RECT_TILES[nd]
    f64 = field.to(torch.float64)
    slow = (1.0 / f64) if kind == "speed" else f64
    gaps = np.concatenate([np.diff(np.asarray(c, dtype=np.float64)) for c in (xs, ys, zs) if c is not None
                           and len(c) > 1])
    qmed = float(slow.median()) * float(np.median(gaps))
    out = torch.empty_like(field)
    ref = None
    results: List[dict] = []

    def run(tile, fac, la):
        nonlocal ref
        delta = fac * qmed * min(tile[:nd])
        fn = lambda: api.solve_rect(field, xs, ys, zs, sources, kind=kind, delta=delta, tile=tile, out=out,
                                    lookahead=la, check_status=False)
        fn()
        api.status()
        if ref is None:
            ref = out.clone()
        elif not torch.equal(ref, out):
            raise RuntimeError(f"rectilinear candidate tile={tile} delta={delta} lookahead={la} changed the result")
        sec = _time(fn, reps)
        api.status()
        results.append({"tile": list(tile), "delta": delta, "delta_factor": fac, "lookahead": la, "ms": sec * 1e3})
        log(f"  rect tile {tile} delta {delta:.4g} ({fac:.3g} x qmed x edge) lookahead {la}: {sec * 1e3:.3f} ms")

    for tile in tiles:
        for fac in delta_factors:
            for la in lookaheads:
                run(tile, fac, la)
    best = min(results, key=lambda r: r["ms"])
    for step in (2.0 ** -0.5, 2.0 ** 0.5):
        run(tuple(best["tile"]), best["delta_factor"] * step, best["lookahead"])
    best = min(results, key=lambda r: r["ms"])
    entry = {"tile": best["tile"], "delta": best["delta"], "lookahead": best["lookahead"], "ms": best["ms"],
             "qmed": qmed, "candidates": results}
    if save:
        cache = _load()
        cache[_rect_key(field.shape, kind)] = entry
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return entry


def _main(argv: List[str]) -> int:
    root = os.path.dirname(HERE)
    sys.path.insert(0, root)
    import workloads as W
    names = argv or ["layered512", "blocky4096"]
    for name in names:
        if name == "layered512":
            p = W.layered_3d()
        elif name == "layered256":
            p = W.layered_3d(256, 256, 128)
        elif name == "paper2d":
            p = W.folded_layers_2d()
            f = torch.from_numpy(p.field[0]).cuda()
            print(f"tuning {p.name}", flush=True)
            e = tune(f, p.h, torch.as_tensor(p.src), tiles=[(32, 32), (16, 16)],
                     delta_factors=(0.5, 1.0, 2.0, 4.0), grid_blocks=(0,), horizons=(0,), reps=2,
                     log=lambda s: print(s, flush=True))
            print(json.dumps({k: v for k, v in e.items() if k != "candidates"}), flush=True)
            continue
        elif name == "rect512":
            import numpy as np
            p = W.layered_3d()
            nz, ny, nx = p.field.shape
            xs, ys = np.arange(nx) * p.h, np.arange(ny) * p.h
            zs = W.stretched_coords(nz, 5.0, 4.0 ** (1.0 / (nz - 2)))
            f = torch.from_numpy(p.field).cuda()
            print("tuning the rectilinear layered model (depth spacing 5 -> 20 m)", flush=True)
            e = tune_rect(f, xs, ys, zs, torch.as_tensor(p.src), log=lambda s: print(s, flush=True))
            print(json.dumps({k: v for k, v in e.items() if k != "candidates"}), flush=True)
            continue
        elif name == "tomo256x32":
            c = W.tomography(256, 256, 128, nshots=32, seed=5)
            f = torch.from_numpy(c.s0).cuda()
            rec = torch.as_tensor(c.receivers).cuda()
            print("tuning the 32-shot tomography batch (forward + adjoint)", flush=True)
            e = tune_batch([f] * 32, c.h, [torch.tensor([int(s)]) for s in c.sources], [rec] * 32,
                           log=lambda s: print(s, flush=True))
            print(json.dumps({k: v for k, v in e.items() if not k.endswith("candidates")}), flush=True)
            continue
        elif name == "tomo256":
            c = W.tomography(256, 256, 128, nshots=1, seed=5)
            f = torch.from_numpy(c.s0).cuda()
            print("tuning tomography slowness model (one shot)", flush=True)
            e = tune(f, c.h, torch.tensor([int(c.sources[0])]), kind="slowness",
                     log=lambda s: print(s, flush=True))
            print(json.dumps({k: v for k, v in e.items() if k != "candidates"}), flush=True)
            continue
        elif name == "blocky4096":
            p = W.blocky_2d()
        else:
            raise SystemExit(f"unknown workload {name}")
        f = torch.from_numpy(p.field).cuda()
        if p.ndim == 2:
            f = f[0]
        print(f"tuning {p.name}", flush=True)
        e = tune(f, p.h, torch.as_tensor(p.src), log=lambda s: print(s, flush=True))
        print(json.dumps({k: v for k, v in e.items() if k != "candidates"}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(_main(sys.argv[1:]))

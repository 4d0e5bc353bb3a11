#!/usr/bin/env python3
"""Benchmark of the Eikonal solver on one MI355X.

Headline (the JSON `value`): grid points solved per second for the 3D
512x512x256 layered + noise model (h = 10 m, 1500..6000 m/s in 8 layers times
(1 + 0.1 g), one source at the surface centre, FP64).  One step = one complete
forward solve through the C ABI: per-solve reset, source placement, the
persistent soft-priority tile kernel and finalisation, with the speed field
already resident in HBM, in the launch configuration of the tuning cache (tile
shape, bucket width, lookahead window, pass structure; the command line can
override all but the pass structure).  After the timed steps the output is checked: the
device status must be clean and the times' SHA-256 must equal the one the
oracle's solve gives (tests/golden/layered_512x512x256_seed2.json).

Also reported on the same JSON line:
  * roofline: the persistent solve kernel's algorithmic bytes (16 B per point:
    read the speed once, write the time once) over its mean duration measured
    with HIP events on its stream during the timed steps, against 8 TB/s;
    `traffic` comes from the committed rocprofv3 counter summary when it was
    taken on the current kernel source, else null.  Beside it, a latency
    estimate: the tile hops from the source tile to the farthest tile (a run
    can pass values on only to its face neighbours) times the busy time of one
    run measured with a single workgroup;
  * cpu_baseline: the oracle, timed in a separate process on the host: one
    sequential binary-heap solve on one core over a bounded sample of the same
    recipe (512x512x128), and the tomography step (forward, parents, adjoint)
    for one shot per host core, all cores in parallel;
  * batched: forward + adjoint shots/s for a tomography batch, one graph replay
    of two persistent launches vs one plain solve + adjoint per shot;
  * the same model on a rectilinear grid (depth spacing stretched 5 -> 20 m),
    the paper's grid shape in 2D, the schedule comparison and the precision
    ablation, as extra entries.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "grid points solved/s & % HBM peak; batched fwd+adjoint shots/s vs plain"
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_solve_layered_512x512x256_pmc.txt")


def kernel_source_hash() -> str:
    csrc = os.path.join(ROOT, "paper_2103_05694_amd", "csrc")
    m = hashlib.sha256()
    for fn in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, fn), "rb") as f:
            m.update(fn.encode())
            m.update(f.read())
    return m.hexdigest()[:16]


def read_traffic(npts: int):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on this kernel source."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    kv = {}
    with open(TRAFFIC_SUMMARY) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_TOMO = None


def _tomo_shot(i: int):
    """One tomography step of shot i on the CPU oracle: forward solve with
    parents, misfit gradient at the receivers, adjoint.  Runs in a worker
    process forked from the baseline process (no GPU there)."""
    import numpy as np
    import oracle
    case, t_obs = _TOMO
    src = np.array([case.sources[i]], dtype=np.int64)
    t = oracle.fmm(case.s0, case.h, src, kind=oracle.SLOWNESS)
    par = oracle.parents(t, src)
    g = np.zeros(t.size)
    np.add.at(g, case.receivers, t.reshape(-1)[case.receivers] - t_obs[i])
    grad = oracle.adjoint(t, par, case.s0, case.h, g.reshape(t.shape), kind=oracle.SLOWNESS)
    return float(np.abs(grad).sum())


def _tomo_obs(i: int):
    import numpy as np
    import oracle
    case = _TOMO[0]
    src = np.array([case.sources[i]], dtype=np.int64)
    return oracle.fmm(case.s_true, case.h, src, kind=oracle.SLOWNESS).reshape(-1)[case.receivers]


def cpu_baseline_worker() -> dict:
    """The oracle timed on the host (this runs in a process of its own that
    never touches the GPU): one sequential solve on one core, and one
    tomography step per core with all cores in parallel."""
    global _TOMO
    import multiprocessing as mp
    import oracle
    import workloads as W
    oracle.lib()
    p = W.layered_3d(512, 512, 128, h=10.0, seed=2)
    t0 = time.perf_counter()
    oracle.fmm(p.field, p.h, p.src)
    dt = time.perf_counter() - t0
    single = {"value": p.npts / dt, "unit": "grid points/s", "cores": 1, "kind": "oracle",
              "sample": "same layered+noise recipe (seed 2, surface-centre source) at 512x512x128 = "
                        f"{p.npts} points, one sequential binary-heap solve, {dt:.1f} s",
              "host_cpu": _host_cpu(), "host_threads": os.cpu_count()}
    # one worker per host core, at most 16 (the host share of one GPU)
    cores = max(1, min(16, os.cpu_count() or 1))
    case = W.tomography(256, 256, 128, nshots=32, seed=5)
    shots = list(range(cores))
    _TOMO = (case, None)
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        t_obs = dict(zip(shots, pool.map(_tomo_obs, shots)))
    _TOMO = (case, t_obs)
    with ctx.Pool(cores) as pool:
        t0 = time.perf_counter()
        pool.map(_tomo_shot, shots)
        wall = time.perf_counter() - t0
    single["batched"] = {
        "value": len(shots) / wall, "unit": "shots/s (forward + parents + adjoint)", "cores": cores,
        "kind": "oracle",
        "sample": f"{len(shots)} of the 32 tomography shots on 256x256x128 (one per core, in parallel worker "
                  f"processes), {wall:.1f} s wall"}
    return single


def cpu_baseline() -> dict:
    """Runs cpu_baseline_worker in a child process (this process has the GPU
    open) and returns its JSON."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-worker"], capture_output=True,
                       text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(f"cpu baseline failed: {r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])


GOLDEN = os.path.join(ROOT, "tests", "golden", "layered_512x512x256_seed2.json")


def times_sha256(t) -> str:
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(t, dtype="<f8").tobytes()).hexdigest()


def latency_estimate(args, torch, eik, W, shape, src_xyz) -> dict:
    """Tile hops from the source's tile to the farthest tile of the headline
    grid (6-connected tile grid: a run passes values only to face
    neighbours), times the busy time of one run (staging, relaxation, write
    and publish) measured with a single workgroup on a 128x128x64 model of
    the same recipe in the same launch configuration."""
    nz, ny, nx = shape
    tx, ty, tz = args.tile
    nt = ((nx + tx - 1) // tx, (ny + ty - 1) // ty, (nz + tz - 1) // tz)
    s = (src_xyz[0] // tx, src_xyz[1] // ty, src_xyz[2] // tz)
    hops = sum(max(s[k], nt[k] - 1 - s[k]) for k in range(3))
    q = W.layered_3d(128, 128, 64, h=10.0, seed=2)
    f = torch.from_numpy(q.field).cuda()
    eik.solve(f, q.h, torch.as_tensor(q.src).cuda(), delta=args.delta, tile=args.tile, grid_blocks=1,
              horizon=args.horizon, packed=args.packed, lookahead=args.lookahead)
    st = eik.status()
    run_us = (st.phase_us[1] + st.phase_us[2] + st.phase_us[3]) / max(st.tile_visits, 1)
    return {"tile_hops": hops, "run_us_one_workgroup": run_us, "latency_bound_ms": hops * run_us * 1e-3}


def bench_single(args, torch, eik, W) -> dict:
    p = W.layered_3d(512, 512, 256, h=10.0, seed=2)
    log(f"input {p.name} sha {p.sha256()}")
    f = torch.from_numpy(p.field).cuda()
    src = torch.as_tensor(p.src).cuda()
    out = torch.empty_like(f)
    kw = dict(delta=args.delta, tile=args.tile, grid_blocks=args.grid_blocks, horizon=args.horizon, out=out,
              packed=args.packed, lookahead=args.lookahead, check_status=False)
    for _ in range(args.warmup):
        eik.solve(f, p.h, src, **kw)
    eik.status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        eik.solve(f, p.h, src, time_kernels=True, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = eik.status()   # raises on any device-side error of the timed solves
    ms = wall * 1e3 / args.steps
    # the timed output is the oracle's solution, bit for bit
    digest = times_sha256(out.cpu().numpy())
    golden = None
    if os.path.exists(GOLDEN):
        with open(GOLDEN) as fh:
            golden = json.load(fh)
    validated = (golden is not None and golden["input_sha256_16"] == p.sha256()
                 and golden["times_sha256"] == digest)
    kernel_ms = st.kernel_ms
    algo_bytes = 16.0 * p.npts
    achieved = algo_bytes / (kernel_ms * 1e-3) / 1e9
    traffic = read_traffic(p.npts)
    res = {
        "npts": p.npts, "ms_per_step": ms, "kernel_ms": kernel_ms,
        "kernel_launches": int(st.kernel_launches),
        "visits_per_tile": st.tile_visits / max(st.ntiles, 1),
        "updates_per_point": st.point_updates / p.npts,
        "passes_per_visit": st.relax_passes / max(st.tile_visits, 1),
        # where the time goes (last solve): the kernel is bound by the latency
        # of each run, not by bandwidth
        "workgroups": int(st.workgroups),
        "us_per_run": {name: st.phase_us[i] / max(st.tile_visits, 1)
                       for i, name in enumerate(("claim_wait", "stage", "relax", "write_publish"))},
        "runs_per_us": st.tile_visits / max(kernel_ms * 1e3, 1e-9),
        "busy_fraction": (st.phase_us[1] + st.phase_us[2] + st.phase_us[3]) /
                         max(st.workgroups * kernel_ms * 1e3, 1e-9),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_solve (persistent soft-priority tile solver)",
                     "algorithmic_bytes_per_launch": algo_bytes},
        "output": {"status": int(st.status), "times_sha256": digest,
                   "oracle_sha256": golden["times_sha256"] if golden else None, "validated": validated},
    }
    if traffic is not None:
        # the counters' HBM bytes over the same mean duration, and their
        # multiple of the algorithmic bytes (re-reads of re-run tiles, halos)
        res["roofline"]["traffic_gbs"] = traffic / (kernel_ms * 1e-3) / 1e9
        res["roofline"]["traffic_frac"] = res["roofline"]["traffic_gbs"] / HBM_PEAK_GBS
        res["roofline"]["traffic_over_algorithmic"] = traffic / algo_bytes
    lat = latency_estimate(args, torch, eik, W, p.shape, (p.nx // 2, p.ny // 2, 0))
    res["roofline"].update(lat)
    res["roofline"]["latency_frac"] = lat["latency_bound_ms"] / kernel_ms
    # with the parent record (adds 9 B/pt)
    if args.parents:
        par = torch.empty(f.shape, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(args.steps // 2, 1)):
            eik.solve(f, p.h, src, parents=True, parents_out=par, **kw)
        torch.cuda.synchronize()
        res["ms_per_step_with_parents"] = (time.perf_counter() - t0) * 1e3 / max(args.steps // 2, 1)
        eik.status()
    return res


def bench_tomography(args, torch, eik, W) -> dict:
    """32 shots on 256x256x128 (h = 10 m), 1024 surface receivers, observed
    times from a +5% slowness blob; batched graph replay vs per-shot plain."""
    from paper_2103_05694_amd.batch import ShotBatch
    case = W.tomography(256, 256, 128, nshots=args.shots, seed=5)
    s0 = torch.from_numpy(case.s0).cuda()
    s_true = torch.from_numpy(case.s_true).cuda()
    srcs = [torch.tensor([int(s)]) for s in case.sources]
    rec = torch.as_tensor(case.receivers).cuda()
    obs = ShotBatch([s_true] * args.shots, case.h, srcs, [rec] * args.shots, kind="slowness",
                    delta=args.tomo_delta, tile=args.tomo_tile, grid_blocks=args.tomo_grid_blocks,
                    horizon=args.tomo_horizon, packed=args.tomo_packed, lookahead=args.tomo_lookahead,
                    **args.adj_cfg)
    obs.step()
    obs.sync()
    eik.status(obs.stream)
    t_obs = [v.reshape(-1).index_select(0, rec) for v in obs.shot_views(obs.t)]
    sb = ShotBatch([s0] * args.shots, case.h, srcs, [rec] * args.shots, t_obs=t_obs, kind="slowness",
                   delta=args.tomo_delta, tile=args.tomo_tile, grid_blocks=args.tomo_grid_blocks,
                   horizon=args.tomo_horizon, packed=args.tomo_packed, lookahead=args.tomo_lookahead,
                   **args.adj_cfg)
    sb.capture()
    reps = max(args.steps // 4, 2)
    for _ in range(2):
        sb.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sb.replay()
    torch.cuda.synchronize()
    batched_s = (time.perf_counter() - t0) / reps
    eik.status(sb.stream)
    t_plain = torch.empty_like(sb.t)
    g_plain = torch.empty_like(sb.grad)
    sb.plain_step(t_plain, g_plain, **args.shot_cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sb.plain_step(t_plain, g_plain, **args.shot_cfg)
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / reps
    eik.status()
    same_t = bool(torch.equal(t_plain, sb.t))
    same_g = bool(torch.equal(g_plain, sb.grad))
    return {"workload": f"tomography {args.shots} shots on 256x256x128, 1024 surface receivers",
            "shots_per_s_batched_graph": args.shots / batched_s,
            "shots_per_s_plain": args.shots / plain_s, "plain_config": "per shot, single-shot tuning",
            "speedup": plain_s / batched_s, "ms_per_batch_graph": batched_s * 1e3,
            "ms_per_batch_plain": plain_s * 1e3, "bitwise_equal_t": same_t,
            "bitwise_equal_grad": same_g, "loss": sb.loss()}


def bench_uneven(args, torch, eik, W) -> dict:
    """64 shots on layered models of uneven sizes (128^3, 192x192x128,
    256x256x128), one random surface source each, misfit at a 32x32 surface
    receiver grid against a +5% blob model; batched graph vs plain."""
    from paper_2103_05694_amd.batch import ShotBatch
    import numpy as np
    shots = W.batched_shots(args.uneven_shots, seed=4)
    fields, fields_true, srcs, recs = [], [], [], []
    rng = np.random.default_rng(44)
    for p in shots:
        s = 1.0 / p.field
        c = (int(rng.integers(20, p.nx - 20)), int(rng.integers(20, p.ny - 20)), int(rng.integers(20, p.nz - 20)))
        fields.append(torch.from_numpy(s).cuda())
        fields_true.append(torch.from_numpy(s * W.blob_perturbation(p.shape, c)).cuda())
        srcs.append(torch.as_tensor(p.src))
        step_x, step_y = p.nx // 32, p.ny // 32
        rx = step_x // 2 + step_x * np.arange(32)
        ry = step_y // 2 + step_y * np.arange(32)
        RX, RY = np.meshgrid(rx, ry, indexing="xy")
        recs.append(torch.as_tensor(W.flat_index(RX.ravel(), RY.ravel(), 0, p.nx, p.ny)).cuda())
    npts = sum(p.npts for p in shots)
    obs = ShotBatch(fields_true, 10.0, srcs, recs, kind="slowness", delta=args.tomo_delta, tile=args.tomo_tile,
                    grid_blocks=args.tomo_grid_blocks, horizon=args.tomo_horizon, packed=args.tomo_packed,
                    lookahead=args.tomo_lookahead, **args.adj_cfg)
    obs.step()
    obs.sync()
    eik.status(obs.stream)
    t_obs = [v.reshape(-1).index_select(0, r) for v, r in zip(obs.shot_views(obs.t), recs)]
    del obs
    sb = ShotBatch(fields, 10.0, srcs, recs, t_obs=t_obs, kind="slowness", delta=args.tomo_delta,
                   tile=args.tomo_tile, grid_blocks=args.tomo_grid_blocks, horizon=args.tomo_horizon,
                   packed=args.tomo_packed, lookahead=args.tomo_lookahead, **args.adj_cfg)
    sb.capture()
    reps = max(args.steps // 8, 2)
    sb.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sb.replay()
    torch.cuda.synchronize()
    batched_s = (time.perf_counter() - t0) / reps
    eik.status(sb.stream)
    t_plain = torch.empty_like(sb.t)
    g_plain = torch.empty_like(sb.grad)
    sb.plain_step(t_plain, g_plain, **args.shot_cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sb.plain_step(t_plain, g_plain, **args.shot_cfg)
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / reps
    eik.status()
    return {"workload": f"{len(shots)} uneven layered shots, {npts} points total",
            "shots_per_s_batched_graph": len(shots) / batched_s,
            "shots_per_s_plain": len(shots) / plain_s, "speedup": plain_s / batched_s,
            "points_per_s_batched_fwd_adj": npts / batched_s,
            "bitwise_equal_t": bool(torch.equal(t_plain, sb.t)),
            "bitwise_equal_grad": bool(torch.equal(g_plain, sb.grad))}


def bench_ablation(args, torch, eik, W) -> dict:
    """Precision ablation in 2D (the paper's Table "tab:error" question on the
    GPU): the exact monotone operator and the two explicit formulas under the
    same asynchronous kernel and five schedules (tile shape, bucket width, grid
    size).  Reports the residual (points the operator would still change) of
    each result and how many points differ from the first schedule's result."""
    p = W.blocky_2d(1024, nsrc=16, seed=3)
    f = torch.from_numpy(p.field[0]).cuda()
    src = torch.as_tensor(p.src).cuda()
    schedules = [dict(tile=(32, 32), delta=0.0), dict(tile=(16, 16), delta=4.0),
                 dict(tile=(64, 16), delta=16.0), dict(tile=(128, 8), delta=0.0, grid_blocks=64),
                 dict(tile=(32, 32), delta=2.0, grid_blocks=16)]
    out = {"workload": "2D 1024x1024 blocky speeds {0.5,1,2,5} in 64-cell blocks, 16 sources, h=1",
           "schedules": [{k: (list(v) if isinstance(v, tuple) else v) for k, v in s.items()} for s in schedules]}
    for name, op, track in (("dtilde", "dtilde", False), ("dhat", "dhat", False),
                            ("dhat+change_tracking", "dhat", True), ("newton", "newton", False),
                            ("dbar", "dbar", False)):
        ts, res, ms = [], [], []
        for sch in schedules:
            t = eik.solve(f, p.h, src, op=op, track_change=track, check_status=False, time_kernels=True, **sch)
            st = eik.status(raise_on_error=False)
            ms.append(st.kernel_ms)
            ts.append(t.clone())
            res.append(eik.residual(f, p.h, src, t, op=op))
        distinct = []
        for t in ts:
            if not any(torch.equal(t, u) for u in distinct):
                distinct.append(t)
        out[name] = {"residual_points": [r[0] for r in res], "residual_max_rel": [r[1] for r in res],
                     "points_differing_from_first": [int((t != ts[0]).sum()) for t in ts],
                     "distinct_results": len(distinct), "kernel_ms": ms}
    return out


def bench_schedules(args, torch, eik, W) -> dict:
    """Schedule comparison in one kernel (the paper's work-efficiency view):
    one bucket (a plain FIFO worklist, the topology-driven extreme), narrow
    buckets (close to fast marching's order) and the tuned width, on the
    headline model.  Every operator evaluation is classified against the final
    times: empty (no change), good (sets the final value), bad (lowers the
    value to something that is lowered again later)."""
    p = W.layered_3d(512, 512, 256, h=10.0, seed=2)
    f = torch.from_numpy(p.field).cuda()
    src = torch.as_tensor(p.src).cuda()
    kw = dict(tile=args.tile, grid_blocks=args.grid_blocks, packed=args.packed, check_status=False)
    ref = eik.solve(f, p.h, src, delta=args.delta, horizon=args.horizon, lookahead=args.lookahead, **kw)
    eik.status()
    out = {"workload": "3D 512x512x256 layered model (the headline solve)", "tile": list(args.tile), "rows": []}
    for name, delta, hz, la in (("one bucket (FIFO)", 0.0, 0, 0), ("narrow buckets", args.delta / 8.0, 0, 0),
                                ("tuned", args.delta, args.horizon, args.lookahead)):
        t = torch.empty_like(f)
        eik.solve(f, p.h, src, delta=delta, horizon=hz, lookahead=la, out=t, **kw)
        eik.status()
        torch.cuda.synchronize()
        eik.solve(f, p.h, src, delta=delta, horizon=hz, lookahead=la, out=t, time_kernels=True, **kw)
        ms = eik.status().kernel_ms
        eik.solve(f, p.h, src, delta=delta, horizon=hz, lookahead=la, out=t, work_ref=ref, **kw)
        st = eik.status()
        ev, imp, good = st.evaluations, st.improving, st.final_updates
        out["rows"].append({"schedule": name, "delta": delta, "horizon": hz, "lookahead": la, "kernel_ms": ms,
                            "visits_per_tile": st.tile_visits / max(st.ntiles, 1),
                            "evaluations_per_point": ev / p.npts, "empty": (ev - imp) / max(ev, 1),
                            "good": good / max(ev, 1), "bad": (imp - good) / max(ev, 1),
                            "bitwise_equal": bool(torch.equal(t, ref))})
    return out


def bench_paper_scale(args, torch, eik, W) -> dict:
    """The paper's grid shape: 2D 11204 x 54404 (609M points), a synthetic
    folded-layer stand-in for its upsampled Marmousi model (spacing 0.3125 m,
    source at the surface centre); one forward solve per step."""
    from paper_2103_05694_amd import autotune
    p = W.folded_layers_2d()
    f = torch.from_numpy(p.field[0]).cuda()
    src = torch.as_tensor(p.src).cuda()
    cfg = autotune.lookup(tuple(f.shape), "speed")
    tile = tuple(cfg["tile"]) if cfg else (32, 32)
    delta = cfg["delta"] if cfg else 32 * p.h / 3000.0
    gb = int(cfg.get("grid_blocks", 0)) if cfg else 0
    hz = int(cfg.get("horizon", 0)) if cfg else 0
    pk = bool(cfg.get("packed", False)) if cfg else False
    la = int(cfg.get("lookahead", 0)) if cfg else 0
    out = torch.empty_like(f)
    kw = dict(tile=tile, delta=delta, grid_blocks=gb, horizon=hz, out=out, packed=pk, lookahead=la,
              check_status=False)
    eik.solve(f, p.h, src, **kw)
    eik.status()
    reps = 3
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        eik.solve(f, p.h, src, time_kernels=True, **kw)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    st = eik.status()
    res = eik.residual(f, p.h, src, out)
    return {"workload": "2D 11204x54404 folded layers (the paper's upsampled grid shape), h=0.3125 m",
            "points": p.npts, "ms_per_solve": ms, "kernel_ms": st.kernel_ms,
            "points_per_s": p.npts / (ms * 1e-3), "tile": list(tile), "delta": delta, "grid_blocks": gb,
            "horizon": hz, "lookahead": la, "visits_per_tile": st.tile_visits / max(st.ntiles, 1),
            "residual_points": res[0]}


def bench_rect(args, torch, eik, W) -> dict:
    """The benchmark's 512x512x256 layered model on a rectilinear grid:
    10 m in x and y, depth spacing stretched geometrically from 5 m to about
    20 m (eik_solve_rect), same source, in the launch configuration of the
    tuning cache (autotune.tune_rect: four tile shapes, four widths, lookahead
    0, 8 or 16); without an entry, 8x8x8 tiles, a 0.0025 s bucket width and a
    lookahead of 16."""
    from paper_2103_05694_amd import autotune
    import numpy as np
    p = W.layered_3d()
    f = torch.from_numpy(p.field).cuda()
    src = torch.as_tensor(p.src).cuda()
    nz, ny, nx = p.field.shape
    xs, ys = np.arange(nx) * p.h, np.arange(ny) * p.h
    zs = W.stretched_coords(nz, 5.0, 4.0 ** (1.0 / (nz - 2)))
    out = torch.empty_like(f)
    cfg = autotune.lookup_rect(tuple(f.shape), "speed") or {"tile": [8, 8, 8], "delta": 0.0025, "lookahead": 16}
    tile, delta, la = tuple(cfg["tile"]), float(cfg["delta"]), int(cfg["lookahead"])
    kw = dict(tile=tile, delta=delta, lookahead=la, out=out, check_status=False)
    eik.solve_rect(f, xs, ys, zs, src, **kw)
    eik.status()
    reps = 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        eik.solve_rect(f, xs, ys, zs, src, **kw)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    st = eik.status()
    return {"workload": "3D 512x512x256 layered speed on a rectilinear grid (dx = dy = 10 m, dz 5 -> 20 m "
                        "geometric), one surface-centre source",
            "points": p.npts, "ms_per_solve": ms, "points_per_s": p.npts / (ms * 1e-3), "tile": list(tile),
            "delta": delta, "lookahead": la, "visits_per_tile": st.tile_visits / max(st.ntiles, 1), "max_time_s": float(out.max())}


def profile_mode(args, torch, eik, W) -> None:
    """A short run for rocprofv3: kernels of known traffic for the counter
    calibration -- a plain 1 GiB device copy (reads and writes 1 GiB), the
    residual kernel over the headline grid (reads its times, speeds and
    source mask: 17 B per point) -- then a few solves of the headline
    workload in the benchmark's launch configuration."""
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    p = W.layered_3d(512, 512, 256, h=10.0, seed=2)
    f = torch.from_numpy(p.field).cuda()
    src = torch.as_tensor(p.src).cuda()
    out = torch.empty_like(f)
    for i in range(args.steps):
        eik.solve(f, p.h, src, delta=args.delta, tile=args.tile, grid_blocks=args.grid_blocks,
                  horizon=args.horizon, packed=args.packed, lookahead=args.lookahead, out=out,
                  check_status=False)
        torch.cuda.synchronize()
        log(f"profile solve {i} done")
    eik.status()
    res = eik.residual(f, p.h, src, out)
    torch.cuda.synchronize()
    print(json.dumps({"profile_mode": True, "copy_bytes_each_way": n * 8, "solves": args.steps,
                      "npts": p.npts, "residual": list(res), "source_hash": kernel_source_hash()}), flush=True)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--delta", type=float, default=None, help="bucket width (s); default from the tuning cache")
    ap.add_argument("--tile", type=str, default=None, help="e.g. 32x8x4; default from the tuning cache")
    ap.add_argument("--grid-blocks", type=int, default=None, help="persistent workgroups; default from the tuning cache")
    ap.add_argument("--horizon", type=int, default=None, help="bucket horizon 0..4; default from the tuning cache")
    ap.add_argument("--lookahead", type=int, default=None,
                    help="buckets a block may take ahead of the lowest open one; default from the tuning cache")
    ap.add_argument("--tomo-delta", type=float, default=None, help="default from the tuning cache")
    ap.add_argument("--tomo-tile", type=str, default=None, help="default from the tuning cache")
    ap.add_argument("--shots", type=int, default=32)
    ap.add_argument("--uneven-shots", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--parents", action="store_true")
    ap.add_argument("--no-ablation", action="store_true")
    ap.add_argument("--no-schedules", action="store_true")
    ap.add_argument("--no-paper-scale", action="store_true")
    ap.add_argument("--no-rect", action="store_true")
    ap.add_argument("--profile-mode", action="store_true")
    ap.add_argument("--cpu-baseline-worker", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.cpu_baseline_worker:
        print(json.dumps(cpu_baseline_worker()), flush=True)
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: there is no multi-GPU path (shots would shard "
              "across GPUs with one all-reduce of the gradient; designed, not implemented).",
              file=sys.stderr)
        return 2

    import torch
    import workloads as W
    import paper_2103_05694_amd as eik
    from paper_2103_05694_amd import autotune
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 2
    if args.tile is not None:
        args.tile = tuple(int(x) for x in args.tile.lower().split("x"))
    cfg = autotune.lookup((256, 512, 512), "speed")
    if args.delta is None:
        args.delta = cfg["delta"] if cfg else 0.04
    if args.tile is None:
        args.tile = tuple(cfg["tile"]) if cfg else (16, 8, 8)
    if args.grid_blocks is None:
        args.grid_blocks = int(cfg.get("grid_blocks", 0)) if cfg else 0
    if args.horizon is None:
        args.horizon = int(cfg.get("horizon", 0)) if cfg else 0
    args.packed = bool(cfg.get("packed", False)) if cfg else False
    if args.lookahead is None:
        args.lookahead = int(cfg.get("lookahead", 0)) if cfg else 0
    tcfg = autotune.lookup_batch(args.shots, (128, 256, 256), "slowness") or \
        autotune.lookup((128, 256, 256), "slowness")
    if args.tomo_tile is not None:
        args.tomo_tile = tuple(int(x) for x in args.tomo_tile.lower().split("x"))
    else:
        args.tomo_tile = tuple(tcfg["tile"]) if tcfg else (16, 8, 8)
    if args.tomo_delta is None:
        args.tomo_delta = tcfg["delta"] if tcfg else 0.02
    args.tomo_grid_blocks = int(tcfg.get("grid_blocks", 0)) if tcfg else 0
    args.tomo_horizon = int(tcfg.get("horizon", 0)) if tcfg else 0
    args.tomo_packed = bool(tcfg.get("packed", False)) if tcfg else False
    args.tomo_lookahead = int(tcfg.get("lookahead", 0)) if tcfg else 0
    args.adj_cfg = {}
    if tcfg and "adj_delta" in tcfg:
        args.adj_cfg = dict(adj_delta=tcfg["adj_delta"], adj_tile=tuple(tcfg["adj_tile"]),
                            adj_grid_blocks=int(tcfg.get("adj_grid_blocks", 0)),
                            adj_packed=bool(tcfg.get("adj_packed", False)),
                            adj_lookahead=int(tcfg.get("adj_lookahead", 0)))
    # the per-shot baseline runs with the single-shot tuning (its best), not the batch's
    scfg = autotune.lookup((128, 256, 256), "slowness")
    args.shot_cfg = (dict(delta=scfg["delta"], tile=tuple(scfg["tile"]), grid_blocks=int(scfg.get("grid_blocks", 0)),
                          horizon=int(scfg.get("horizon", 0)), packed=bool(scfg.get("packed", False)),
                          lookahead=int(scfg.get("lookahead", 0)))
                     if scfg else {})
    args.shot_cfg.update(args.adj_cfg)

    if args.profile_mode:
        profile_mode(args, torch, eik, W)
        return 0

    log(f"single-source 3D solve, delta {args.delta}, tile {args.tile}")
    single = bench_single(args, torch, eik, W)
    log(f"single: {single['ms_per_step']:.3f} ms/step, kernel {single['kernel_ms']:.3f} ms")
    extra = {"single": {k: v for k, v in single.items() if k != "roofline"}}
    if not args.no_batched:
        log("tomography batch")
        extra["tomography_32"] = bench_tomography(args, torch, eik, W)
        log(json.dumps(extra["tomography_32"]))
    if not args.no_uneven:
        log("uneven batch")
        extra["uneven_64"] = bench_uneven(args, torch, eik, W)
        log(json.dumps(extra["uneven_64"]))
    if not args.no_paper_scale:
        log("paper-scale 2D grid")
        extra["paper_scale_2d"] = bench_paper_scale(args, torch, eik, W)
        log(json.dumps(extra["paper_scale_2d"]))
    if not args.no_rect:
        log("rectilinear grid")
        extra["rect_3d"] = bench_rect(args, torch, eik, W)
        log(json.dumps(extra["rect_3d"]))
    if not args.no_schedules:
        log("schedule comparison")
        extra["schedules"] = bench_schedules(args, torch, eik, W)
        log(json.dumps(extra["schedules"]))
    if not args.no_ablation:
        log("precision ablation")
        extra["ablation_2d"] = bench_ablation(args, torch, eik, W)
        log(json.dumps(extra["ablation_2d"]))
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline()
    value = single["npts"] / (single["ms_per_step"] * 1e-3)
    if not single["output"]["validated"]:
        log(f"ERROR: the timed output does not match the oracle's hash: {single['output']}")
    line = {
        "metric": METRIC, "value": value, "unit": "grid points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": single["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "3D 512x512x256 layered+noise speed (h=10 m, 1500-6000 m/s, 8 layers, "
                               "seed 2), one surface-centre source, single forward solve",
                   "delta": args.delta, "tile": list(args.tile), "grid_blocks": args.grid_blocks,
                   "horizon": args.horizon, "packed": args.packed, "lookahead": args.lookahead,
                   "points": single["npts"]},
        "roofline": single["roofline"],
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)
    return 0 if single["output"]["validated"] else 3


if __name__ == "__main__":
    sys.exit(main())

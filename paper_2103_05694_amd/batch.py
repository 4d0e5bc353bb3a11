"""Many-shot forward + adjoint in one graph replay.

Travel-time tomography evaluates, for every shot (source), a forward solve, a
misfit at receivers and the adjoint back to slowness.  `ShotBatch` packs all
shots (grids may differ in size) so that each of the two passes is ONE
persistent kernel launch over every shot's tiles, and captures the whole step
-- reset, source placement, batched solve, parents, misfit gradient, batched
adjoint -- into a HIP graph (torch.cuda.CUDAGraph on ROCm) replayed with a
single launch call.  `plain_step` runs the same work one shot at a time for
comparison; both produce bit-identical results.

The misfit is L = 1/2 sum over shots and receivers of (t - t_obs)^2, so
dL/dt is the residual at receiver points and zero elsewhere.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import torch

from . import api


class ShotBatch:
    def __init__(self, fields: Sequence[torch.Tensor], h, sources: Sequence, receivers: Sequence,
                 t_obs: Optional[Sequence[torch.Tensor]] = None, kind: str = "slowness",
                 delta: float = 0.0, tile=None, stream: Optional[torch.cuda.Stream] = None,
                 grid_blocks: int = 0, horizon: int = 0, adj_delta: Optional[float] = None,
                 adj_tile=None, adj_grid_blocks: Optional[int] = None, packed: bool = False,
                 adj_packed: bool = False, lookahead: int = 0, adj_lookahead: Optional[int] = None):
        self.kind = kind
        self.lookahead = lookahead
        self.adj_lookahead = lookahead if adj_lookahead is None else adj_lookahead
        self.delta = delta
        self.tile = tile
        self.grid_blocks = grid_blocks
        self.horizon = horizon
        self.packed = packed
        self.adj_packed = adj_packed
        # the adjoint is readiness-driven and may prefer other launch parameters
        self.adj_delta = delta if adj_delta is None else adj_delta
        self.adj_tile = tile if adj_tile is None else adj_tile
        self.adj_grid_blocks = grid_blocks if adj_grid_blocks is None else adj_grid_blocks
        self.fields = list(fields)
        self.nshots = len(self.fields)
        self.hs = [float(h)] * self.nshots if isinstance(h, (int, float)) else [float(x) for x in h]
        self.b = api.pack(self.fields, self.hs, sources, kind)
        self.sources = [api.source_indices(s, f.shape, f.device) for s, f in zip(sources, self.fields)]
        dev = self.b.field.device
        n = self.b.npts
        self.t = torch.empty(n, dtype=torch.float64, device=dev)
        self.par = torch.empty(n, dtype=torch.uint8, device=dev)
        self.g = torch.zeros(n, dtype=torch.float64, device=dev)
        self.grad = torch.empty(n, dtype=torch.float64, device=dev)
        self.mu = torch.empty(n, dtype=torch.float64, device=dev)
        # receiver positions in the packed arrays
        offs = [int(self.b.offsets[i]) for i in range(self.nshots)]
        self.rec_local = [torch.as_tensor(r, dtype=torch.int64, device=dev).reshape(-1) for r in receivers]
        self.rec = torch.cat([r + o for r, o in zip(self.rec_local, offs)]).contiguous()
        if t_obs is None:
            self.t_obs = torch.zeros(self.rec.numel(), dtype=torch.float64, device=dev)
        else:
            self.t_obs = torch.cat([torch.as_tensor(x, dtype=torch.float64, device=dev).reshape(-1)
                                    for x in t_obs]).contiguous()
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.graph: Optional[torch.cuda.CUDAGraph] = None

    # -- one batched step: 2 persistent launches for all shots ----------------
    def _enqueue(self) -> None:
        api.solve_packed(self.b, self.t, self.par, self.delta, self.tile, grid_blocks=self.grid_blocks,
                         stream=self.stream, horizon=self.horizon, packed=self.packed, lookahead=self.lookahead)
        self.g.zero_()
        self.g.index_copy_(0, self.rec, self.t.index_select(0, self.rec) - self.t_obs)
        api.adjoint_packed(self.b, self.t, self.par, self.g, self.grad, self.mu, self.adj_delta, self.adj_tile,
                           grid_blocks=self.adj_grid_blocks, stream=self.stream, packed=self.adj_packed,
                           lookahead=self.adj_lookahead)

    def step(self) -> None:
        """Enqueue one batched forward + adjoint (eager launches).  The batch's
        stream first waits for the caller's stream, so work the caller queued
        on its outputs (copies, reads) finishes before they are overwritten."""
        self.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.stream):
            self._enqueue()

    def capture(self) -> None:
        """Warm up on the capture stream (grows the workspace), then record the
        step into a graph."""
        torch.cuda.current_stream().synchronize()
        self.stream.wait_stream(torch.cuda.current_stream())
        self.step()
        self.stream.synchronize()
        api.status(self.stream)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=self.stream):
            self._enqueue()
        self.stream.synchronize()

    def replay(self) -> None:
        """One launch of the captured step, on this batch's stream, after the
        caller's stream (as in step)."""
        if self.graph is None:
            self.capture()
        self.stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(self.stream):
            self.graph.replay()

    def sync(self) -> None:
        self.stream.synchronize()

    def loss(self) -> float:
        r = self.t.index_select(0, self.rec) - self.t_obs
        return 0.5 * float((r * r).sum())

    # -- reference: the same work one shot at a time ---------------------------
    def plain_step(self, t_out: torch.Tensor, grad_out: torch.Tensor, delta: Optional[float] = None,
                   tile=None, grid_blocks: Optional[int] = None, horizon: Optional[int] = None,
                   adj_delta: Optional[float] = None, adj_tile=None,
                   adj_grid_blocks: Optional[int] = None, packed: Optional[bool] = None,
                   adj_packed: Optional[bool] = None, lookahead: Optional[int] = None,
                   adj_lookahead: Optional[int] = None) -> None:
        """Per-shot eik_solve + eik_adjoint launches on the current stream,
        writing into packed outputs.  The launch parameters default to the
        batch's; a single shot may prefer others (it has far less parallel
        work), and none of them changes the results."""
        delta = self.delta if delta is None else delta
        tile = self.tile if tile is None else tile
        grid_blocks = self.grid_blocks if grid_blocks is None else grid_blocks
        horizon = self.horizon if horizon is None else horizon
        packed = self.packed if packed is None else packed
        adj_packed = self.adj_packed if adj_packed is None else adj_packed
        adj_delta = self.adj_delta if adj_delta is None else adj_delta
        adj_tile = self.adj_tile if adj_tile is None else adj_tile
        adj_grid_blocks = self.adj_grid_blocks if adj_grid_blocks is None else adj_grid_blocks
        lookahead = self.lookahead if lookahead is None else lookahead
        adj_lookahead = self.adj_lookahead if adj_lookahead is None else adj_lookahead
        tv = self.b.views(t_out)
        gv = self.b.views(grad_out)
        g = torch.zeros_like(t_out)
        gvv = self.b.views(g)
        rec_off = 0
        for i in range(self.nshots):
            t, par = api.solve(self.fields[i], self.hs[i], self.sources[i], kind=self.kind, parents=True,
                               delta=delta, tile=tile, grid_blocks=grid_blocks, horizon=horizon, out=tv[i],
                               packed=packed, lookahead=lookahead, check_status=False)
            r = self.rec_local[i]
            nr = r.numel()
            gvv[i].view(-1).index_copy_(0, r, t.view(-1).index_select(0, r) - self.t_obs[rec_off:rec_off + nr])
            rec_off += nr
            api.adjoint(self.fields[i], self.hs[i], t, par, gvv[i], kind=self.kind, delta=adj_delta,
                        tile=adj_tile, grid_blocks=adj_grid_blocks, out=gv[i], packed=adj_packed,
                        lookahead=adj_lookahead, check_status=False)

    def shot_views(self, packed: torch.Tensor) -> List[torch.Tensor]:
        return self.b.views(packed)

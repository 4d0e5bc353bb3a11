"""GPU parity of the adjoint (d loss / d slowness) against the oracle's
reverse-order adjoint, through the C ABI; the autograd wrapper; and the
batched forward + adjoint against per-problem oracle solves."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def O(oracle_lib):
    return oracle_lib


def to_gpu(a, squeeze2d=True):
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    if squeeze2d and t.dim() == 3 and t.shape[0] == 1:
        t = t[0]
    return t


def receiver_grad(t, rec, tobs):
    g = np.zeros(t.size)
    np.add.at(g, rec, t.reshape(-1)[rec] - tobs)
    return g.reshape(t.shape)


def assert_close_or_equal(a, b, what):
    if np.array_equal(a, b):
        return
    scale = max(np.max(np.abs(b)), 1e-300)
    err = np.max(np.abs(a - b)) / scale
    n = int(np.count_nonzero(a != b))
    assert err <= 1e-12, f"{what}: {n} differ, max rel {err:.3e}"


CASES = [
    ("2d_blocky", lambda rng: (W.random_field((1, 90, 110), rng, 0.5, 4.0, block=6), 1.0, [1234])),
    ("2d_2src", lambda rng: (W.random_field((1, 64, 64), rng, 1.0, 3.0), 0.5, [0, 4095])),
    ("3d_layered", lambda rng: (W.layered_3d(48, 40, 24, h=10.0, seed=9, sigma=3.0).field, 10.0,
                                [W.flat_index(20, 21, 0, 48, 40)])),
    ("3d_ragged", lambda rng: (W.random_field((13, 17, 35), rng, 0.5, 4.0, block=2), 1.0, [9, 3000])),
    # speeds over six orders of magnitude, point by point
    ("3d_contrast", lambda rng: (10.0 ** rng.uniform(-3.0, 3.0, size=(10, 14, 22)), 2.5, [5, 2000])),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_adjoint_matches_oracle(gpu, O, case):
    name, make = case
    rng = np.random.default_rng(17)
    f, h, src = make(rng)
    src = np.asarray(src, dtype=np.int64)
    t = O.fmm(f, h, src)
    par = O.parents(t, src)
    rec = rng.choice(f.size, 50, replace=False)
    tobs = t.reshape(-1)[rec] * (1 + 0.01 * rng.standard_normal(rec.size))
    g = receiver_grad(t, rec, tobs)
    ref_grad, ref_mu = O.adjoint(t, par, f, h, g, return_mu=True)
    tiles = [(64, 16), (32, 32), (16, 16)] if f.shape[0] == 1 else [(32, 8, 4), (8, 8, 8), (64, 4, 4), (16, 8, 8)]
    for tile in tiles:
        for delta, pk, la in ((0.0, False, 0), (1.0, False, 0), (0.0, True, 0), (1.0, True, 0), (0.25, True, 8),
                              (0.1, False, 16)):
            mu = torch.empty(f.shape, dtype=torch.float64, device="cuda")
            grad = gpu.adjoint(to_gpu(f), h, to_gpu(t), to_gpu(par), to_gpu(g), tile=tile, delta=delta,
                               mu_out=mu.view(to_gpu(f).shape), packed=pk, lookahead=la)
            gr = grad.cpu().numpy().reshape(f.shape)
            assert_close_or_equal(gr, ref_grad, f"{name} grad tile {tile} packed {pk} lookahead {la}")
            m = mu.cpu().numpy()
            assert_close_or_equal(m, ref_mu, f"{name} mu tile {tile} packed {pk} lookahead {la}")


def test_adjoint_end_to_end_from_gpu_forward(gpu, O):
    rng = np.random.default_rng(3)
    f = W.random_field((10, 30, 40), rng, 0.5, 4.0, block=3)
    src = np.array([W.flat_index(20, 15, 0, 40, 30)])
    ft = to_gpu(f)
    t, par = gpu.solve(ft, 1.0, torch.as_tensor(src), parents=True)
    t_ref = O.fmm(f, 1.0, src)
    assert np.array_equal(t.cpu().numpy(), t_ref)
    g = rng.standard_normal(f.shape) * (rng.random(f.shape) < 0.05)
    grad = gpu.adjoint(ft, 1.0, t, par, to_gpu(g))
    ref = O.adjoint(t_ref, O.parents(t_ref, src), f, 1.0, g)
    assert_close_or_equal(grad.cpu().numpy(), ref, "end to end")


def test_autograd_function(gpu, O):
    rng = np.random.default_rng(4)
    f = W.random_field((1, 40, 50), rng, 0.5, 3.0, block=5)
    s = 1.0 / f
    src = [W.flat_index(3, 4, 0, 50, 40)]
    rec = rng.choice(f.size, 30, replace=False)
    st = torch.from_numpy(s[0]).cuda().requires_grad_(True)
    t = gpu.eikonal(st, 2.0, torch.tensor(src))
    tobs = torch.from_numpy(O.fmm(s * 1.02, 2.0, src, kind=O.SLOWNESS).reshape(-1)[rec]).cuda()
    loss = 0.5 * ((t.reshape(-1)[torch.as_tensor(rec).cuda()] - tobs) ** 2).sum()
    loss.backward()
    t_ref = O.fmm(s, 2.0, src, kind=O.SLOWNESS)
    g = receiver_grad(t_ref, rec, tobs.cpu().numpy())
    ref = O.adjoint(t_ref, O.parents(t_ref, np.array(src)), s, 2.0, g, kind=O.SLOWNESS)
    assert_close_or_equal(st.grad.cpu().numpy(), ref[0], "autograd")


def uneven_shots(n, seed):
    rng = np.random.default_rng(seed)
    sizes = [(20, 24, 16), (33, 17, 9), (16, 16, 16), (40, 12, 10)]
    out = []
    for i in range(n):
        nx, ny, nz = sizes[i % len(sizes)]
        f = W.random_field((nz, ny, nx), rng, 0.5, 4.0, block=2)
        src = np.array([int(rng.integers(0, nx)) + nx * int(rng.integers(0, ny))])
        out.append((f, src))
    return out


def test_batched_forward_equals_per_problem(gpu, O):
    shots = uneven_shots(9, 1)
    fields = [to_gpu(f) for f, _ in shots]
    srcs = [torch.as_tensor(s) for _, s in shots]
    for kw in (dict(delta=0.5), dict(delta=0.1, tile=(16, 8, 8), packed=True, lookahead=16)):
        ts, pars = gpu.solve_batched(fields, 1.0, srcs, parents=True, **kw)
        for (f, s), t, p in zip(shots, ts, pars):
            ref = O.fmm(f, 1.0, s)
            assert np.array_equal(t.cpu().numpy(), ref), kw
            assert np.array_equal(p.cpu().numpy(), O.parents(ref, s)), kw


def test_batched_adjoint_equals_per_problem(gpu, O):
    shots = uneven_shots(6, 2)
    rng = np.random.default_rng(5)
    fields = [to_gpu(f) for f, _ in shots]
    srcs = [torch.as_tensor(s) for _, s in shots]
    b = gpu.pack(fields, 1.0, srcs)
    t = torch.empty(b.npts, dtype=torch.float64, device="cuda")
    par = torch.empty(b.npts, dtype=torch.uint8, device="cuda")
    gpu.solve_packed(b, t, par)
    gpu.status()
    gs = [rng.standard_normal(f.shape) * (rng.random(f.shape) < 0.1) for f, _ in shots]
    gp = torch.cat([to_gpu(g).reshape(-1) for g in gs])
    grad = torch.empty_like(t)
    gpu.adjoint_packed(b, t, par, gp, grad)
    gpu.status()
    grad2 = torch.empty_like(t)
    gpu.adjoint_packed(b, t, par, gp, grad2, packed=True, tile=(8, 8, 8), delta=0.3)
    gpu.status()
    assert torch.equal(grad, grad2)
    gpu.adjoint_packed(b, t, par, gp, grad2, packed=True, tile=(16, 8, 8), delta=0.05, lookahead=16)
    gpu.status()
    assert torch.equal(grad, grad2)
    for (f, s), g, gr in zip(shots, gs, b.views(grad)):
        tr = O.fmm(f, 1.0, s)
        ref = O.adjoint(tr, O.parents(tr, s), f, 1.0, g)
        assert_close_or_equal(gr.cpu().numpy(), ref, "batched adjoint")


def test_adjoint_degenerate_gradients(gpu, O):
    """dL/dt = 0 gives a zero gradient everywhere; dL/dt only at the sources
    also gives zero (a source has no parents to pass it on to); both agree with
    the oracle bit for bit."""
    rng = np.random.default_rng(71)
    f = W.random_field((9, 14, 21), rng, 0.5, 3.0, block=3)
    src = np.array([5, 1000, 2500], dtype=np.int64)
    t = O.fmm(f, 1.0, src)
    par = O.parents(t, src)
    for name, g in (("zero", np.zeros(f.shape)), ("sources", np.zeros(f.shape))):
        if name == "sources":
            g.reshape(-1)[src] = rng.standard_normal(src.size)
        ref = O.adjoint(t, par, f, 1.0, g)
        assert not np.any(ref)
        for tile, pk in (((8, 8, 8), False), ((16, 8, 8), True), ((16, 8, 8), False)):
            grad = gpu.adjoint(to_gpu(f), 1.0, to_gpu(t), to_gpu(par), to_gpu(g), tile=tile, packed=pk)
            got = grad.cpu().numpy().reshape(f.shape)
            assert np.array_equal(got, ref), (name, tile)


def test_graph_capture_with_different_forward_and_adjoint_tiles(gpu, O):
    """A batch whose forward and adjoint run with different tile shapes (two
    device problem tables): warm-up uploads both, the captured graph replays
    without any upload, and every replay equals the per-shot plain launches
    bit for bit."""
    from paper_2103_05694_amd.batch import ShotBatch
    shots = uneven_shots(5, 3)
    fields = [to_gpu(1.0 / f) for f, _ in shots]
    srcs = [torch.as_tensor(s) for _, s in shots]
    recs = [torch.arange(0, f.size, 7, device="cuda") for f, _ in shots]
    sb = ShotBatch(fields, 1.0, srcs, recs, kind="slowness", delta=0.1, tile=(16, 8, 8), packed=True,
                   adj_delta=0.6, adj_tile=(8, 8, 8), lookahead=8, adj_lookahead=4)
    sb.capture()
    t_plain = torch.empty_like(sb.t)
    g_plain = torch.empty_like(sb.grad)
    sb.plain_step(t_plain, g_plain)
    torch.cuda.synchronize()
    gpu.status()
    for rep in range(3):
        sb.replay()
        sb.sync()
        gpu.status(sb.stream)
        assert torch.equal(sb.t, t_plain), f"replay {rep} times"
        assert torch.equal(sb.grad, g_plain), f"replay {rep} gradient"
        torch.cuda.synchronize()
    for i, (f, s) in enumerate(shots):
        ref = O.fmm(1.0 / f, 1.0, s, kind=O.SLOWNESS)
        assert np.array_equal(sb.shot_views(sb.t)[i].cpu().numpy(), ref)


def test_bad_buffers_raise_before_launch(gpu):
    f = torch.ones(8, 9, 10, dtype=torch.float64, device="cuda")
    src = torch.tensor([0])
    with pytest.raises(TypeError):
        gpu.solve(f, 1.0, src, out=torch.empty(8, 9, 10, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        gpu.solve(f, 1.0, src, out=torch.empty(719, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        gpu.solve(f, 1.0, src, out=torch.empty(720, dtype=torch.float64))
    with pytest.raises(TypeError):
        gpu.solve(f, 1.0, src, parents=True, parents_out=torch.empty(720, dtype=torch.int32, device="cuda"))
    t, par = gpu.solve(f, 1.0, src, parents=True)
    g = torch.zeros_like(f)
    with pytest.raises(ValueError):
        gpu.adjoint(f, 1.0, t, par, g, mu_out=torch.empty(10, dtype=torch.float64, device="cuda"))
    b = gpu.pack([f, f], 1.0, [src, src])
    with pytest.raises(ValueError):
        gpu.solve_packed(b, torch.empty(b.npts - 1, dtype=torch.float64, device="cuda"))
    tt = torch.empty(b.npts, dtype=torch.float64, device="cuda")
    pp = torch.empty(b.npts, dtype=torch.uint8, device="cuda")
    with pytest.raises(TypeError):
        gpu.adjoint_packed(b, tt, pp, torch.zeros(b.npts, dtype=torch.float32, device="cuda"), tt.clone())

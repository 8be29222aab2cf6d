"""Degenerate and limit cases at the boundary: an empty free set, the
smallest grid, the largest axis, sizes beyond the limits, empty network
batches."""
import numpy as np
import pytest
import torch

from oracle.core import KIND_FREE, Oracle
from paper_2407_14675_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dpo():
    from paper_2407_14675_amd import dpo as mod
    mod.load()
    return mod


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def sweep_tol(V, Vref):
    """1e-5*max(1,|V|) plus 1e-6 of the largest |V| a foot's cell can hold
    (float32 lerps round at the magnitude of the corners)."""
    from scipy.ndimage import maximum_filter
    corner = maximum_filter(np.abs(np.asarray(V, dtype=np.float64)), size=7, mode="nearest")
    return 1e-5 * np.maximum(1.0, np.abs(Vref)) + 1e-6 * corner


def one_sweep_parity(dpo, p, seed):
    """One Bellman sweep from a random value field against the oracle, both
    kernel paths where they apply."""
    o = Oracle(p)
    V = inputs.random_value(p, seed=seed, frac_M=0.1).astype(np.float32)
    Vo, _, _, margin = o.bellman_sweep(V.astype(np.float64))
    free = o.kind == KIND_FREE
    ctx = dpo.Context(p)
    paths = [1, 2] if ctx.kernel_path() == 2 else [1]
    for path in paths:
        ctx.set_kernel_path(path)
        Vin = torch.from_numpy(V).cuda()
        Vout = Vin.clone()
        ang, thr = ctx.empty_policy()
        ctx.bellman_sweep(Vin, Vout, ang, thr)
        err = np.abs(host(Vout) - Vo)
        # the minimum of an exhaustive table is unique; the continuous search
        # is compared away from ties between basins
        sel = free if p["search"]["mode"] == "table" else free & (margin >= 1e-4 * np.maximum(1.0, np.abs(Vo)))
        if sel.any():
            ok = err[sel] <= sweep_tol(V, Vo)[sel]
            assert ok.mean() >= 0.999, (path, ok.mean())
        np.testing.assert_array_equal(host(Vout)[~free], V[~free])
    return int(free.sum())


def test_empty_free_set(dpo):
    """A reduced grid with no active node: sweeps are no-ops, residuals are
    zero and both solvers stop at their first check."""
    print("empty free set", flush=True)
    p = inputs.with_grid(inputs.PI48, (6, 6, 6, 6))
    mask = torch.zeros((6, 6, 6, 6), dtype=torch.uint8, device="cuda")
    ctx = dpo.Context(p, mask=mask)
    assert ctx.n_free == 0
    V = ctx.init_value()
    W = V.clone()
    ang, thr = ctx.empty_policy()
    resid = torch.full((5,), 7.0, dtype=torch.float64, device="cuda")
    ctx.bellman_sweep(V, W, ang, thr, resid)
    np.testing.assert_array_equal(host(resid), np.zeros(5))
    np.testing.assert_array_equal(host(W), host(V))
    rc, st = ctx.solve_vi(V, ang, thr, tol_rel=1e-6, max_sweeps=10, check_every=1)
    assert rc == dpo.DPO_OK and st["sweeps"] == 1
    rc, st = ctx.solve_pi(V, ang, thr, tol_rel=1e-6, eval_sweeps=20, max_outer=10)
    assert rc == dpo.DPO_OK and st["sweeps"] == 1
    net = dpo.Mlp(inputs.mlp_params32())
    seed = net.propose(ctx)
    assert float(host(seed).max()) == 0.0
    assert ctx.feasible_nodes(V, 1e30).numel() == 0


@pytest.mark.parametrize("search", ["table", "scan_golden"])
def test_two_nodes_per_axis(dpo, search):
    print("2^4 grid", search, flush=True)
    base = inputs.VI12 if search == "table" else inputs.PI48
    n = one_sweep_parity(dpo, inputs.with_grid(base, (2, 2, 2, 2)), seed=61)
    assert n > 0


def test_largest_axis(dpo):
    """256 nodes along r (the packed-coordinate limit) with short other axes."""
    print("256 x 3 x 3 x 2", flush=True)
    n = one_sweep_parity(dpo, inputs.with_grid(inputs.PI48, (256, 3, 3, 2)), seed=62)
    assert n > 0


def test_sizes_beyond_the_limits(dpo):
    for n in [(257, 2, 2, 2), (2, 2, 2, 300), (256, 256, 256, 64)]:
        with pytest.raises(dpo.DpoError) as e:
            dpo.Context(inputs.with_grid(inputs.VI12, n))
        assert e.value.code == dpo.DPO_EINVAL


def test_network_empty_and_single_batches(dpo):
    net = dpo.Mlp(inputs.mlp_params32())
    x = torch.zeros((0, 4), dtype=torch.float32, device="cuda")
    assert net.forward(x).shape == (0, 3)
    with pytest.raises(dpo.DpoError):
        net.grad(x, x)
    xs, ts = inputs.mlp_random_samples(5, seed=9)
    hist = net.train_epoch(torch.from_numpy(xs).cuda(), torch.from_numpy(ts).cuda(), batch=4096)
    assert hist.numel() == 1 and np.isfinite(host(hist)).all() and net.steps() == 1


def test_ceiling_probes(dpo):
    """The machine-ceiling probes: the copy copies, the read and the FMA loop
    run, and bad sizes are refused."""
    print("ceiling probes", flush=True)
    src = torch.arange(1 << 20, dtype=torch.float32, device="cuda")
    dst = torch.zeros_like(src)
    sink = torch.zeros(1, dtype=torch.float32, device="cuda")
    dpo.probe_copy(src, dst)
    dpo.probe_read(src, sink)
    dpo.probe_fma(8, 16, sink)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    assert float(sink[0]) == 0.0
    with pytest.raises(dpo.DpoError):
        dpo.probe_copy(src[:6], dst[:6])
    with pytest.raises(dpo.DpoError):
        dpo.probe_fma(0, 16, sink)


def test_binding_refuses_mis_sized_and_mis_typed_arrays(dpo):
    """Arrays are checked before any launch: a node array of the wrong size
    or type (which a kernel would index past its end, or read as other
    values) is refused, and so is a residual buffer that is too short."""
    print("binding argument checks", flush=True)
    p = inputs.with_grid(inputs.PI48, (8, 7, 6, 5))
    ctx = dpo.Context(p)
    V = ctx.init_value()
    W = V.clone()
    a, t = ctx.empty_policy()
    bad = [
        dict(V_in=V[:-1].contiguous() if V.dim() == 1 else V.reshape(-1)[:-1]),
        dict(V_in=V.double()),
        dict(V_out=W.reshape(-1)[::2]),
        dict(pol_ang=a.half()),
        dict(pol_thr=t.int()),
        dict(resid=torch.zeros(4, dtype=torch.float64, device="cuda")),
        dict(resid=torch.zeros(5, dtype=torch.float32, device="cuda")),
        dict(V_in=V.cpu()),
    ]
    for kw in bad:
        args = dict(V_in=V, V_out=W, pol_ang=a, pol_thr=t, resid=None)
        args.update(kw)
        with pytest.raises(dpo.DpoError):
            ctx.bellman_sweep(args["V_in"], args["V_out"], args["pol_ang"], args["pol_thr"], args["resid"])
    with pytest.raises(dpo.DpoError):
        ctx.solve_pi(V.reshape(-1)[:10], a, t, max_outer=1)
    with pytest.raises(dpo.DpoError):
        ctx.value_at(V.double(), inputs.X0)
    # the right arrays in any node-count shape are accepted
    ctx.bellman_sweep(V.reshape(-1), W.reshape(-1), a.reshape(-1), t.reshape(-1),
                      torch.zeros(5, dtype=torch.float64, device="cuda"))
    b = dpo.Batch([inputs.with_grid(inputs.VI12, (6, 6, 6, 6)), inputs.with_grid(inputs.VI12, (7, 6, 6, 6))])
    Vs = b.init_values()
    with pytest.raises(dpo.DpoError):
        b.solve_vi(Vs[:1], max_sweeps=2)
    with pytest.raises(dpo.DpoError):
        b.solve_vi([Vs[1], Vs[0]], max_sweeps=2)

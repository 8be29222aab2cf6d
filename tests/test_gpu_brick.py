"""The frozen-policy sweeps with LDS value bricks (eq:p_eval applied once,
workgroups walking columns of nodes through the mass planes) against the
kernels that gather from global memory and against the oracle, through the
C ABI: the form driven by the greedy step's foot descriptors (policy
iteration's evaluation sweeps) and the form that takes the policy arrays.

Each brick kernel forms the same cell and lerps as its global-memory
counterpart, so their values agree bit for bit at every node; the
residual's maxima and counts agree exactly, its sum up to summation order.
Cases: grids whose r side is and is not a multiple of 4 (16-byte and 4-byte
brick loads), ragged tiles, a reduced grid with inactive nodes, two thrust
levels, the 96 x 96 x 96 x 64 grid in full, and the no-allocation entry
point on the brick path."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle.core import KIND_FREE, Oracle
from paper_2407_14675_amd import inputs

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dpo():
    from paper_2407_14675_amd import dpo as mod
    mod.load()
    return mod


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dtype).contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def random_policy(p, seed):
    """Throttle 0/1 and angles: uniform, plus exact scan-table angles (the
    table's own sin/cos) on a quarter of the nodes."""
    n = p["n"]
    shape = (n[3], n[2], n[1], n[0])
    rng = np.random.default_rng(seed)
    thr = rng.integers(0, 2, size=shape).astype(np.uint8)
    ang = rng.uniform(-math.pi, math.pi, size=shape).astype(np.float32)
    K = p["search"].get("n_scan", p["search"].get("n_angles", 16))
    table = np.array([-math.pi + 2 * math.pi * k / K for k in range(K)], dtype=np.float64).astype(np.float32)
    pick = rng.random(shape) < 0.25
    ang[pick] = table[rng.integers(0, K, size=int(pick.sum()))]
    return ang, thr


def both_paths(ctx, V, ang, thr):
    outs, res = [], []
    for path in (1, 2):
        ctx.set_eval_path(path)
        W = torch.full_like(V, -5.0)
        r = torch.zeros(5, dtype=torch.float64, device="cuda")
        ctx.policy_eval_sweep(V, W, ang, thr, r)
        outs.append(host(W))
        res.append(host(r))
    ctx.set_eval_path(0)
    return outs, res


CASES = {
    "pi48_16x10x9x7": (inputs.with_grid(inputs.PI48, (16, 10, 9, 7)), None),
    "pi48_9x10x11x6_scalar": (inputs.with_grid(inputs.PI48, (9, 10, 11, 6)), None),
    "large_a1e-3_20x24x13x16": (inputs.with_grid(inputs.large_problem(accel=1e-3), (20, 24, 13, 16)), None),
    "large_a5e-4_24x24x24x16": (inputs.with_grid(inputs.large_problem(accel=5e-4), (24, 24, 24, 16)), None),
    "pi48_12x12x12x12_masked": (inputs.with_grid(inputs.PI48, (12, 12, 12, 12)), 0.7),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_brick_matches_free_list_and_oracle(dpo, case):
    p, keep = CASES[case]
    _say("brick sweep", case)
    mask = None
    if keep is not None:
        n = p["n"]
        mask = (np.random.default_rng(5).random((n[3], n[2], n[1], n[0])) < keep).astype(np.uint8)
    ctx = dpo.Context(p, mask=None if mask is None else dev(mask, torch.uint8))
    o = Oracle(p, mask=mask)
    V = inputs.random_value(p, seed=11, frac_M=0.1).astype(np.float32)
    ang, thr = random_policy(p, 12)
    Vd = dev(V)
    (w1, w2), (r1, r2) = both_paths(ctx, Vd, dev(ang), dev(thr, torch.uint8))
    free = o.kind == KIND_FREE
    np.testing.assert_array_equal(w1, w2)
    assert np.all(w2[~free] == -5.0)  # fixed nodes are not written
    assert r1[0] == r2[0] and r1[2] == r2[2] and r1[3] == r2[3]
    assert r2[1] == pytest.approx(r1[1], rel=1e-12)
    want = o.policy_eval_sweep(V.astype(np.float64), ang.astype(np.float64), thr)
    from scipy.ndimage import maximum_filter
    corner = maximum_filter(np.abs(V.astype(np.float64)), size=7, mode="nearest")
    tol = 1e-5 * np.maximum(1.0, np.abs(want)) + 1e-6 * corner
    assert np.all(np.abs(w2 - want)[free] <= tol[free])
    _say("  free", int(free.sum()), "of", o.N)


@pytest.mark.parametrize("case", ["pi48_16x10x9x7", "pi48_9x10x11x6_scalar", "large_a1e-3_20x24x13x16",
                                  "pi48_12x12x12x12_masked"])
def test_descriptor_brick_matches_global_gathers_and_oracle(dpo, case):
    """Policy iteration's evaluation sweep: the descriptors of one greedy
    sweep drive the brick kernel and the global-gather kernel to the same
    values bit for bit, and to the oracle's Q of the greedy policy."""
    p, keep = CASES[case]
    _say("descriptor brick sweep", case)
    mask = None
    if keep is not None:
        n = p["n"]
        mask = (np.random.default_rng(5).random((n[3], n[2], n[1], n[0])) < keep).astype(np.uint8)
    ctx = dpo.Context(p, mask=None if mask is None else dev(mask, torch.uint8))
    o = Oracle(p, mask=mask)
    V = inputs.random_value(p, seed=13, frac_M=0.1).astype(np.float32)
    Vd = dev(V)
    W = Vd.clone()
    ang, thr = ctx.empty_policy()
    ctx.bellman_sweep(Vd, W, ang, thr)
    assert ctx.eval_path() == 2
    outs = []
    for path in (1, 2):
        ctx.set_eval_path(path)
        E = torch.full_like(Vd, -5.0)
        ctx.policy_eval_sweep_last(Vd, E)
        outs.append(host(E))
    ctx.set_eval_path(0)
    free = o.kind == KIND_FREE
    np.testing.assert_array_equal(outs[0], outs[1])
    assert np.all(outs[1][~free] == -5.0)
    nodes = np.flatnonzero(free.reshape(-1))
    q = o.q_many(V.astype(np.float64), nodes, host(thr).reshape(-1)[nodes],
                 host(ang).reshape(-1)[nodes].astype(np.float64))
    from scipy.ndimage import maximum_filter
    corner = maximum_filter(np.abs(V.astype(np.float64)), size=7, mode="nearest").reshape(-1)[nodes]
    ve = outs[1].reshape(-1)[nodes].astype(np.float64)
    assert np.all(np.abs(ve - q) <= 1e-5 * np.maximum(1.0, np.abs(q)) + 1e-6 * corner)


@pytest.mark.parametrize("n_m", [64, 60, 32, 9])
def test_brick_full_size_96x96x96x64(dpo, n_m):
    """The 96^3 x 64 grid (runs of 8 mass planes per workgroup), 96^3 x 60
    (seven runs of 8 and a last run of 4), 96^3 x 32 (runs of 4) and
    96^3 x 9 (one GPU's slab of an 8-way split: runs of 2 and a last run of
    1), the greedy policy of a partly converged value: each brick sweep
    equals its global-gather counterpart at every node (descriptor form and
    policy-array form), and the no-allocation entry point on the brick path
    equals both policy-array sweeps."""
    p = inputs.large_problem(accel=1e-3)
    if n_m != 64:
        p = inputs.with_grid(p, (96, 96, 96, n_m))
    _say("brick sweep 96^3 x", n_m)
    ctx = dpo.Context(p)
    assert ctx.eval_path() == 2
    V = ctx.init_value()
    ang, thr = ctx.empty_policy()
    ctx.solve_vi(V, ang, thr, tol_rel=0.0, max_sweeps=64, check_every=64)
    W = torch.empty_like(V)
    ctx.bellman_sweep(V, W, ang, thr)
    desc = []
    for path in (1, 2):
        ctx.set_eval_path(path)
        E = torch.full_like(V, -5.0)
        ctx.policy_eval_sweep_last(W, E)
        torch.cuda.synchronize()
        desc.append(E)
    assert torch.equal(desc[0], desc[1])
    del desc
    outs = []
    for path in (1, 2):
        ctx.set_eval_path(path)
        E = torch.full_like(V, -5.0)
        ctx.policy_eval_sweep(W, E, ang, thr)
        torch.cuda.synchronize()
        outs.append(E)
    assert torch.equal(outs[0], outs[1])
    S = torch.full_like(V, -5.0)
    r = torch.zeros(5, dtype=torch.float64, device="cuda")
    ctx.set_eval_path(2)
    ctx.policy_eval_sweep_static(W, S, ang, thr, r)
    torch.cuda.synchronize()
    assert torch.equal(S, outs[1])
    assert np.isfinite(host(r)).all()
    del outs, S, W, V, ang, thr
    ctx.close()
    torch.cuda.empty_cache()


def test_packed_descriptors_reproduce_the_greedy_q(dpo):
    """On a grid stored per node the descriptors keep the two cell
    coordinates to 2^-24 of a cell: the evaluation sweep of the greedy
    policy then reproduces the greedy step's own Q to within float32
    rounding of the corner values (the coordinates' rounding moves an
    interpolant by at most 2^-25 of each of the two corner differences it
    spans, under three units in the last place of the corners here)."""
    p = inputs.with_grid(inputs.PI48, (11, 10, 9, 8))
    _say("packed descriptors")
    ctx = dpo.Context(p)
    o = Oracle(p)
    free = o.kind == KIND_FREE
    nf = int(free.sum())
    assert ctx.eval_sweep_bytes() == 16 * nf + 8 * (o.N - nf)  # the packed per-node form
    V = inputs.random_value(p, seed=91, low=0, high=40).astype(np.float32)
    Vd = dev(V)
    W = Vd.clone()
    ang, thr = ctx.empty_policy()
    ctx.bellman_sweep(Vd, W, ang, thr)
    for path in (1, 2):
        ctx.set_eval_path(path)
        E = Vd.clone()
        ctx.policy_eval_sweep_last(Vd, E)
        from scipy.ndimage import maximum_filter
        corner = maximum_filter(np.abs(V), size=7, mode="nearest")
        ulp = np.spacing(corner.astype(np.float32)).astype(np.float64)
        d = np.abs(host(E).astype(np.float64) - host(W).astype(np.float64))
        _say("  path", path, "largest difference in corner ulps", float((d / ulp)[free].max()))
        assert np.all(d[free] <= 4 * ulp[free])  # measured: 2
        np.testing.assert_array_equal(host(E)[~free], V[~free])
    ctx.set_eval_path(0)

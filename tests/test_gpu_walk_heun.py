"""Parity of the table walk and of the Heun (second-order Runge-Kutta) foot
point on the device, through the C ABI, with the CPU oracle.

Tolerances are those of the other sweep tests: one sweep within
1e-5*max(1,|V|) plus the float32 rounding of the corners a foot touches;
controls compared on nodes whose oracle tie margin is at least
1e-4*max(1,|V|); converged values within 1e-4*max(1,|V|).
"""
import math
import sys

import numpy as np
import pytest
import torch

from feedback_parity import check_feedback
from oracle.core import KIND_FREE, Oracle
from paper_2407_14675_amd import inputs

pytestmark = pytest.mark.gpu

K_WALK = 16


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


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(1.0, np.abs(b))


def sweep_tol(V, Vref):
    from scipy.ndimage import maximum_filter
    corner = maximum_filter(np.abs(np.asarray(V, dtype=np.float64)), size=7, mode="nearest")
    return 1e-5 * np.maximum(1.0, np.abs(Vref)) + 1e-6 * corner


def heun(p):
    q = dict(p)
    q["integrator"] = "heun"
    return q


def walk_problem(p=inputs.VI12):
    q = dict(p)
    q["search"] = dict(mode="table_walk", n_angles=K_WALK)
    return q


def table_angles(K):
    return np.array([-math.pi + 2 * math.pi * k / K for k in range(K)])


# ------------------------------------------------------------------ walk
@pytest.mark.parametrize("path", [1, 2])
def test_walk_sweep_parity(dpo, path):
    """One walk sweep from random table start angles: values, throttles and
    table angles equal the oracle's walk away from ties; the walk's thrust
    evaluation count (resid[4]) is that of the oracle's walk."""
    p = walk_problem()
    _say("walk sweep, path", path)
    o = Oracle(p)
    V32 = inputs.random_value(p, seed=81, frac_M=0.1).astype(np.float32)
    rng = np.random.default_rng(82)
    start = table_angles(K_WALK)[rng.integers(0, K_WALK, size=o.shape)]
    Vo, ao, to, margin, evals_o = o.bellman_sweep_walk(V32.astype(np.float64), start.astype(np.float32))
    ctx = dpo.Context(p)
    ctx.set_kernel_path(path)
    Vin = dev(V32)
    Vout = Vin.clone()
    ang = dev(start)
    thr = torch.zeros(o.shape, dtype=torch.uint8, device="cuda")
    resid = torch.zeros(5, dtype=torch.float64, device="cuda")
    ctx.bellman_sweep(Vin, Vout, ang, thr, resid)
    Vg, ag, tg, res = host(Vout), host(ang), host(thr), host(resid)
    free = o.kind == KIND_FREE
    tol = sweep_tol(V32, Vo)
    clear = free & (margin >= 1e-4 * np.maximum(1.0, np.abs(Vo)))
    ok = np.abs(Vg - Vo)[clear] <= tol[clear]
    assert ok.mean() >= 0.999, ok.mean()
    same = (tg[clear] == to[clear]) & (np.abs(ag[clear] - ao[clear]) < 1e-6)
    assert same.mean() >= 0.999, same.mean()
    _say("  non-tie", int(clear.sum()), "of", int(free.sum()), "evals", res[4], evals_o)
    # a different path at a tie node changes the count by a few evaluations
    assert abs(res[4] - evals_o) <= 0.002 * evals_o
    np.testing.assert_array_equal(Vg[~free], V32[~free])


@pytest.mark.parametrize("path", [1, 2])
def test_walk_from_the_table_optimum(dpo, path):
    """Started at the exhaustive table's own choice for the same V, the walk
    stays put: the same values, controls and three thrust evaluations per
    free node."""
    p = walk_problem()
    _say("walk from the table optimum, path", path)
    V32 = inputs.random_value(p, seed=83, frac_M=0.1).astype(np.float32)
    ct = dpo.Context(dict(p, search=dict(mode="table", n_angles=K_WALK)))
    ct.set_kernel_path(path)
    Vin = dev(V32)
    Vt = Vin.clone()
    at, tt = ct.empty_policy()
    ct.bellman_sweep(Vin, Vt, at, tt)
    cw = dpo.Context(p)
    cw.set_kernel_path(path)
    Vw = Vin.clone()
    aw = at.clone()
    tw = torch.zeros_like(tt)
    resid = torch.zeros(5, dtype=torch.float64, device="cuda")
    cw.bellman_sweep(Vin, Vw, aw, tw, resid)
    np.testing.assert_array_equal(host(Vw), host(Vt))
    np.testing.assert_array_equal(host(tw), host(tt))
    np.testing.assert_array_equal(host(aw), host(at))
    assert host(resid)[4] == 3 * cw.n_free


def test_walk_solvers(dpo):
    """Value and policy iteration with the walk on the 12^4 problem: both
    converge, both end nowhere below the exhaustive table's fixed point (a
    walk value is a table value), and close to the oracle's walk solution;
    the evaluation counts are those of one full table sweep plus at least
    three thrust evaluations and one coast per node and walk sweep."""
    p = walk_problem()
    _say("walk VI / PI")
    o = Oracle(p)
    free = o.kind == KIND_FREE
    ref = np.load("tests/golden/vi12_table16.npz")["V"]
    ctx = dpo.Context(p)
    n = ctx.n_free
    V1 = ctx.init_value()
    a1, t1 = ctx.empty_policy()
    rc, st = ctx.solve_vi(V1, a1, t1, tol_rel=1e-7, max_sweeps=20000, check_every=8)
    _say("  VI sweeps", st["sweeps"], "evals", st["evals"], "converged", st["converged"])
    assert st["converged"] or st["stalled"]
    k = st["sweeps"]
    assert n * (1 + K_WALK) + (k - 1) * n * 4 <= st["evals"] <= n * (1 + K_WALK) + (k - 1) * n * (K_WALK + 4)
    V2 = ctx.init_value()
    a2, t2 = ctx.empty_policy()
    rc, st2 = ctx.solve_pi(V2, a2, t2, tol_rel=1e-6, eval_sweeps=20, max_outer=5000)
    _say("  PI steps", st2["sweeps"], "evals", st2["evals"])
    assert rc == dpo.DPO_OK
    Vv, Vp = host(V1), host(V2)
    for Vg in (Vv, Vp):
        assert np.all((Vg - ref)[free] >= -1e-4 * np.maximum(1.0, np.abs(ref[free])))
    wo = np.load("tests/golden/vi12_walk16.npz")["V"]
    close = rel_err(Vv, wo)[free] <= 1e-4
    _say("  VI walk within 1e-4 of the oracle's walk:", close.mean())
    assert close.mean() >= 0.99


# ------------------------------------------------------------------ Heun
def test_heun_probe_foot_matches_oracle(dpo):
    """Foot displacement of the Heun step at random (node, control) pairs:
    the device's float correction against the oracle's FP64 step."""
    p = heun(inputs.VI12)
    _say("Heun probe_foot")
    o = Oracle(p)
    nodes = inputs.random_nodes(p, 3000, seed=84)
    rng = np.random.default_rng(85)
    thr = rng.integers(0, 2, size=nodes.size).astype(np.uint8)
    ang = rng.uniform(-math.pi, math.pi, size=nodes.size).astype(np.float32)
    ctx = dpo.Context(p)
    assert ctx.kernel_path() == 1
    off = host(ctx.probe_foot(nodes, thr, ang))
    lo = np.array(p["lo"])
    h = (np.array(p["hi"]) - lo) / (np.array(p["n"]) - 1)
    euler = Oracle(inputs.VI12)
    moved = 0
    for c in range(nodes.size):
        x = o.node_coords(int(nodes[c]))
        want = (o.step(x, int(thr[c]), float(ang[c])) - x) / h
        np.testing.assert_allclose(off[c], want, atol=2e-6, rtol=0)
        ze = (euler.step(x, int(thr[c]), float(ang[c])) - x) / h
        moved += np.max(np.abs(want - ze)) > 1e-4
    assert moved > nodes.size // 2  # the correction is not negligible on this grid


@pytest.mark.parametrize("search", ["table", "scan_golden"])
def test_heun_sweep_parity(dpo, search):
    """One Bellman sweep with the Heun foot (direct path) against the oracle."""
    base = inputs.VI12 if search == "table" else inputs.with_grid(inputs.PI48, (10, 10, 10, 10))
    p = heun(base)
    _say("Heun sweep", search)
    o = Oracle(p)
    if search == "table":
        V32 = inputs.random_value(p, seed=86, frac_M=0.1).astype(np.float32)
    else:
        ax = [np.linspace(p["lo"][k], p["hi"][k], p["n"][k]) for k in range(4)]
        R, VR, VT, MM = np.meshgrid(*ax, indexing="ij")
        V = (400 * (R - 1.05) ** 2 + 900 * VR ** 2 + 2000 * (VT - 0.976) ** 2 + 50 * (1 - MM)).transpose(3, 2, 1, 0)
        V32 = V.astype(np.float32)
    ctx = dpo.Context(p)
    assert ctx.kernel_path() == 1
    with pytest.raises(dpo.DpoError):
        ctx.set_kernel_path(2)
    Vin = dev(V32)
    Vout = Vin.clone()
    ang, thr = ctx.empty_policy()
    ctx.bellman_sweep(Vin, Vout, ang, thr)
    Vo, ao, to, margin = o.bellman_sweep(V32.astype(np.float64))
    Vg, tg = host(Vout), host(thr)
    free = o.kind == KIND_FREE
    tol = sweep_tol(V32, Vo)
    clear = free & (margin >= 1e-4 * np.maximum(1.0, np.abs(Vo)))
    ok = np.abs(Vg - Vo)[clear] <= tol[clear]
    assert ok.mean() >= 0.999, ok.mean()
    assert (tg[clear] == to[clear]).mean() >= 0.999
    # the Euler sweep of the same V differs beyond the tolerance at most nodes
    Ve, _, _, _ = Oracle(base).bellman_sweep(V32.astype(np.float64))
    assert (np.abs(Ve - Vo) > tol)[free].mean() > 0.5
    # the frozen-policy sweep of the greedy policy (eq:p_eval after eq:p_impr)
    # applies the greedy step's own operator: where the controls are table
    # entries the same sin/cos, foot and lerps, equal up to the compiler's
    # different contraction of the same expressions in the two kernels (a few
    # ulps); golden-section angles get sincosf where the search rotated,
    # within one evaluation
    E = Vin.clone()
    ctx.policy_eval_sweep(Vin, E, ang, thr)
    Eg = host(E).astype(np.float64)
    if search == "table":
        assert np.all(np.abs(Eg - Vg)[free] <= 1e-6 * np.maximum(1.0, np.abs(Vg))[free])
    else:
        assert np.all(np.abs(Eg - Vg)[free] <= tol[free])


def test_heun_policy_eval_and_pi(dpo):
    """Frozen-policy sweep with the Heun foot against the oracle; modified
    policy iteration with Heun (evaluation sweeps recompute the foot from the
    stored angle) against the oracle's value iteration (stored solution)."""
    p = heun(inputs.VI12)
    _say("Heun policy eval / PI")
    o = Oracle(p)
    V32 = inputs.random_value(p, seed=87, frac_M=0.1).astype(np.float32)
    rng = np.random.default_rng(88)
    thr = rng.integers(0, 2, size=o.shape).astype(np.uint8)
    ang = rng.uniform(-math.pi, math.pi, size=o.shape).astype(np.float32)
    ctx = dpo.Context(p)
    Vin = dev(V32)
    Vout = Vin.clone()
    ctx.policy_eval_sweep(Vin, Vout, dev(ang), dev(thr, torch.uint8))
    Vo = o.policy_eval_sweep(V32.astype(np.float64), ang.astype(np.float64), thr)
    free = o.kind == KIND_FREE
    assert np.all(np.abs(host(Vout) - Vo)[free] <= sweep_tol(V32, Vo)[free])
    with pytest.raises(dpo.DpoError):
        ctx.policy_eval_sweep_last(Vin, Vout)
    ref = np.load("tests/golden/vi12_table16_heun.npz")["V"]
    V = ctx.init_value()
    a, t = ctx.empty_policy()
    rc, st = ctx.solve_pi(V, a, t, tol_rel=1e-6, eval_sweeps=20, max_outer=5000)
    _say("  PI steps", st["sweeps"], "V(x0)", ctx.value_at(V, inputs.X0), o.value_at(ref, inputs.X0))
    assert rc == dpo.DPO_OK
    assert rel_err(host(V), ref)[free].max() <= 1e-4
    assert ctx.value_at(V, inputs.X0) == pytest.approx(o.value_at(ref, inputs.X0), rel=1e-4)


def test_heun_feedback_parity(dpo):
    p = heun(inputs.VI12)
    _say("Heun feedback")
    gold = np.load("tests/golden/vi12_table16_heun.npz")
    o = Oracle(p)
    ctx = dpo.Context(p)
    V32 = gold["V"].astype(np.float32)
    states = inputs.random_states(p, 4000, seed=89)  # ~57 of them clear of ties
    ang, thr, q = ctx.feedback(dev(V32), states)
    n, n_clear, n_thr = check_feedback(o, V32.astype(np.float64), states, host(ang), host(thr), host(q),
                                       n_table=p["search"]["n_angles"], min_clear=40)
    _say("  states", n, "clear of ties", n_clear, "thrust compared", n_thr)


def test_heun_and_walk_refused_where_they_do_not_apply(dpo):
    """The batched solver needs the factorised Euler sweep; a walk sweep
    needs its start angles."""
    p = heun(inputs.VI12)
    with pytest.raises(dpo.DpoError):
        dpo.Batch([p, p])
    ctx = dpo.Context(walk_problem())
    V = ctx.init_value()
    with pytest.raises(dpo.DpoError):
        ctx.bellman_sweep(V, V.clone())

"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Tolerances (derived from float32 arithmetic on the device against the FP64
oracle):
  * one Q evaluation or one sweep: |d| <= 1e-5 * max(1, |V|)
  * converged value function: |d| <= 1e-4 * max(1, |V_oracle|)
  * policy, on nodes whose oracle tie margin is at least 1e-4 * max(1, |V|):
    tabulated search: same control index on >= 99.9 %; continuous search:
    same throttle on >= 99.9 %, the device angle reaches the oracle's minimal
    Q within 1e-5 * max(1, |V|), and the angle agrees to 1.2e-3 rad (twice
    the final golden width) wherever Q is sharp enough to determine it
    (see check_thrust_angles).
"""
import math
import sys

import numpy as np
import pytest
import torch

from feedback_parity import check_feedback
from oracle.core import KIND_FREE, Oracle, mask_from_coarse
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


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(1.0, np.abs(b))


def wrapped(du):
    return np.abs((np.asarray(du) + np.pi) % (2 * np.pi) - np.pi)


ANGLE_TOL = 1.2e-3   # twice the final golden-section width
ANGLE_ROUND = 1e-4   # angle equivalent of float32 foot rounding (1e-7 cell / g ~ 2e-5 rad), x5


def check_thrust_angles(o, V, free_clear, thr_g, ang_g, thr_o, ang_o):
    """Thrust angles of the continuous search.

    What is unique is the minimal Q: at every node where both choose thrust,
    the device angle must reach the oracle's minimum within the per-evaluation
    tolerance (Q is evaluated by the oracle in FP64 at both angles).  The angle
    itself is compared only where Q rises by at least 1e-5*max(1,|V|) within
    ANGLE_TOL on both sides of the oracle's angle; elsewhere Q is flatter than
    float32 resolves and every angle in the flat band is a correct answer.
    """
    both = free_clear & (thr_g == 1) & (thr_o == 1)
    nodes = np.flatnonzero(both.reshape(-1))
    if nodes.size == 0:
        return 0, 0
    one = np.ones(nodes.size, dtype=np.uint8)
    uo = ang_o.reshape(-1)[nodes]
    ug = ang_g.reshape(-1)[nodes].astype(np.float64)
    q_o = o.q_many(V, nodes, one, uo)
    q_g = o.q_many(V, nodes, one, ug)
    scale = np.maximum(1.0, np.abs(q_o))
    assert np.all(q_g - q_o <= 1e-5 * scale), np.max((q_g - q_o) / scale)
    q_lo = o.q_many(V, nodes, one, uo - ANGLE_TOL)
    q_hi = o.q_many(V, nodes, one, uo + ANGLE_TOL)
    sharp = (np.minimum(q_lo, q_hi) - q_o) >= 1e-5 * scale
    if sharp.sum():
        assert (wrapped(ug[sharp] - uo[sharp]) <= ANGLE_TOL).mean() >= 0.999
    return int(nodes.size), int(sharp.sum())


def sweep_tol(V, Vref):
    """Per-node tolerance of one float32 sweep against FP64: 1e-5*max(1,|V|)
    plus 1e-6 (about 8 float32 ulps) of the largest |V| among the nodes a foot
    can touch (3 cells around the node): the lerps round at the magnitude of
    the corners, which can exceed the result by far (M = 1e3 next to V ~ 1)."""
    from scipy.ndimage import maximum_filter
    corner = maximum_filter(np.abs(np.asarray(V, dtype=np.float64)), size=7, mode="nearest")
    return 1e-5 * np.maximum(1.0, np.abs(Vref)) + 1e-6 * corner


def check_search_values(o, V, free, Vg, tg, ag, Vo, margin, n_scan=64):
    """Values of the continuous search (scan + golden section).

    The golden section follows its comparisons, so on a multimodal Q(u) a
    comparison that float32 and FP64 decide differently leads to another, equally
    valid, search result.  What is checked, with the tolerance of sweep_tol:
      * on nodes whose oracle tie margin is >= 1e-4*max(1,|V|), the values agree
        on >= 99.9 % of them;
      * on every free node the device value either equals the oracle value or
        is the Q of the device's own control (evaluated by the oracle in FP64),
        and it is no worse than the best of the coast and the n_scan tabulated
        thrust angles.
    """
    tol = sweep_tol(V, Vo)
    scale = np.maximum(1.0, np.abs(Vo))
    clear = free & (margin >= 1e-4 * scale)
    ok = np.abs(Vg[clear] - Vo[clear]) <= tol[clear]
    assert ok.mean() >= 0.999, (ok.mean(), np.max(rel_err(Vg[clear], Vo[clear])))
    nodes = np.flatnonzero(free.reshape(-1))
    thr = tg.reshape(-1)[nodes]
    ang = ag.reshape(-1)[nodes].astype(np.float64)
    vg = Vg.reshape(-1)[nodes].astype(np.float64)
    tl = tol.reshape(-1)[nodes]
    # The device value is the Q of its own control.  Where the optimum sits on
    # the jump to M at a domain face, float32 and FP64 feet (~1e-7 cell apart)
    # fall on different sides, so the angle is allowed ANGLE_ROUND of slack.
    attained = np.abs(vg - Vo.reshape(-1)[nodes]) <= tl
    for du in (0.0, -ANGLE_ROUND, ANGLE_ROUND):
        q = o.q_many(V, nodes, thr, ang + du)
        attained |= np.abs(vg - q) <= tl
    if not attained.all():
        bad = np.flatnonzero(~attained)[:6]
        info = []
        for b in bad:
            qs = [o.q_many(V, nodes[b:b + 1], thr[b:b + 1], ang[b:b + 1] + du)[0]
                  for du in (0.0, -ANGLE_ROUND, ANGLE_ROUND)]
            qc = o.q_many(V, nodes[b:b + 1], np.zeros(1, np.uint8), np.zeros(1))[0]
            info.append((int(nodes[b]), float(vg[b]), int(thr[b]), float(ang[b]), qs, float(qc),
                         float(Vo.reshape(-1)[nodes[b]])))
        raise AssertionError(f"device value not attained at its own control: {info}")
    best = o.q_many(V, nodes, np.zeros(nodes.size, np.uint8), np.zeros(nodes.size))
    one = np.ones(nodes.size, np.uint8)
    for s in range(n_scan):
        u = -math.pi + 2 * math.pi * s / n_scan
        best = np.minimum(best, o.q_many(V, nodes, one, np.full(nodes.size, u)))
    assert np.all(vg <= best + tl)
    return int(clear.sum())


# ------------------------------------------------------------- a1 kinds
@pytest.mark.parametrize("n", [(12, 12, 12, 12), (7, 9, 5, 6)])
def test_classification_and_compaction(dpo, n):
    p = inputs.with_grid(inputs.VI12, n)
    _say("classify", n)
    rng = np.random.default_rng(5)
    mask = (rng.random(tuple(reversed(n))) < 0.6).astype(np.uint8)
    o = Oracle(p, mask=mask)
    ctx = dpo.Context(p, mask=dev(mask, torch.uint8))
    k = host(ctx.kind())
    np.testing.assert_array_equal(k, o.kind)
    assert ctx.n_free == int((o.kind == KIND_FREE).sum())


# ----------------------------------------------------- a2..a4 probes
def test_probe_interp_multilinear(dpo):
    p = inputs.orbit_problem((5, 6, 7, 4))
    _say("probe_interp")
    o = Oracle(p)
    rng = np.random.default_rng(11)
    V = rng.uniform(-3, 3, size=(4, 7, 6, 5))
    n = np.array(p["n"])
    pts = rng.random((5000, 4)) * (n - 1)
    pts[:50] = np.floor(pts[:50])          # nodes
    pts[50:60, 0] = n[0] - 1               # top faces
    pts[60:70, 3] = 0.0                    # bottom faces
    ctx = dpo.Context(p)
    got = host(ctx.probe_interp(dev(V), pts))
    Vf = V.astype(np.float32).astype(np.float64)
    want = np.array([o.interp(Vf, s.astype(np.float32).astype(np.float64)) for s in pts])
    assert np.max(np.abs(got - want)) < 2e-6 * 3
    out = np.array([[-1e-3, 1, 1, 1], [1, 1, 1, n[3] - 1 + 1e-3]], dtype=np.float32)
    assert np.all(host(ctx.probe_interp(dev(V), out)) == p["M"])


def test_probe_foot_matches_oracle(dpo):
    p = inputs.VI12
    _say("probe_foot")
    o = Oracle(p)
    nodes = inputs.random_nodes(p, 3000, seed=7)
    rng = np.random.default_rng(8)
    thr = rng.integers(0, 2, size=nodes.size).astype(np.uint8)
    ang = rng.uniform(-math.pi, math.pi, size=nodes.size).astype(np.float32)
    ctx = dpo.Context(p)
    off = host(ctx.probe_foot(nodes, thr, ang))
    lo = np.array(p["lo"])
    h = (np.array(p["hi"]) - lo) / (np.array(p["n"]) - 1)
    for c in range(nodes.size):
        x = o.node_coords(int(nodes[c]))
        z = o.step(x, int(thr[c]), float(ang[c]))
        want = (z - x) / h
        np.testing.assert_allclose(off[c], want, atol=2e-6, rtol=0)


def test_feet_on_faces_match_oracle(dpo):
    """Odd grids have a node with v_r exactly 0; there the v_t displacement of
    the coast is exactly 0, so on the v_t faces the coast foot lies on the face
    (inside).  Device and oracle must agree on every coast foot and Q."""
    p = inputs.orbit_problem((7, 7, 7, 7), target_radius=1.068, accel=1.04e-3)
    _say("feet on faces")
    o = Oracle(p)
    ctx = dpo.Context(p)
    nodes = np.arange(o.N, dtype=np.int64)
    thr = np.zeros(o.N, dtype=np.uint8)
    off = host(ctx.probe_foot(nodes, thr, np.zeros(o.N, np.float32)))
    n = np.array(p["n"])
    i = np.stack([nodes % n[0], (nodes // n[0]) % n[1], (nodes // (n[0] * n[1])) % n[2],
                  nodes // (n[0] * n[1] * n[2])], axis=1)
    s = i + off
    inside = np.all((s >= 0) & (s <= n - 1), axis=1)
    V = inputs.random_value(p, seed=5, low=0, high=30)
    q_or = o.q_many(V, nodes, thr, np.zeros(o.N))
    inside_or = q_or < p["M"]  # outside gives dt + M
    np.testing.assert_array_equal(inside, inside_or)
    q = host(ctx.probe_q(dev(V), nodes, thr, np.zeros(o.N, np.float32)))
    assert np.max(rel_err(q, q_or)) < 1e-5


def test_probe_q_matches_oracle(dpo):
    p = inputs.VI12
    _say("probe_q")
    o = Oracle(p)
    V = inputs.random_value(p, seed=3, frac_M=0.05).astype(np.float32)
    nodes = inputs.random_nodes(p, 4000, seed=9)
    rng = np.random.default_rng(10)
    thr = rng.integers(0, 2, size=nodes.size).astype(np.uint8)
    ang = rng.uniform(-math.pi, math.pi, size=nodes.size).astype(np.float32)
    ctx = dpo.Context(p)
    q = host(ctx.probe_q(dev(V), nodes, thr, ang))
    want = np.array([o.q(V.astype(np.float64), int(j), int(t), float(a)) for j, t, a in zip(nodes, thr, ang)])
    assert np.max(rel_err(q, want)) < 1e-5


# ------------------------------------------------------- a5..a8 sweeps
def _sweep_both(dpo, p, V, mask=None, search=None, path=0):
    o = Oracle(p, mask=mask)
    ctx = dpo.Context(p, mask=None if mask is None else dev(mask, torch.uint8))
    if search is not None:
        ctx.set_search(search)
    ctx.set_kernel_path(path)
    Vin = dev(V)
    Vout = Vin.clone()
    ang, thr = ctx.empty_policy()
    resid = torch.zeros(5, dtype=torch.float64, device="cuda")
    ctx.bellman_sweep(Vin, Vout, ang, thr, resid)
    Vo, ango, thro, margin = o.bellman_sweep(V.astype(np.float32).astype(np.float64), search=search)
    return o, ctx, host(Vout), host(ang), host(thr), host(resid), Vo, ango, thro, margin


@pytest.mark.parametrize("path", [1, 2])
@pytest.mark.parametrize("which", ["random", "converged"])
def test_table_sweep_parity(dpo, which, path):
    p = inputs.VI12
    _say("table sweep", which, "path", path)
    if which == "random":
        V = inputs.random_value(p, seed=21, frac_M=0.1)
    else:
        V = np.load("tests/golden/vi12_table16.npz")["V"]
    V32 = V.astype(np.float32)
    o, ctx, Vg, ag, tg, res, Vo, ao, to, margin = _sweep_both(dpo, p, V32, path=path)
    free = o.kind == KIND_FREE
    assert np.max(rel_err(Vg[free], Vo[free])) < 1e-5
    clear = free & (margin >= 1e-4 * np.maximum(1.0, np.abs(Vo)))
    agree = (tg[clear] == to[clear]) & ((to[clear] == 0) | (wrapped(ag[clear] - ao[clear]) < 1e-6))
    # coast or not, the best thrust angle is the same table entry where no tie
    assert agree.mean() >= 0.999
    # FP64 residual of the same float arrays
    want = o.residual(V32.astype(np.float64), Vg.astype(np.float64))
    assert res[0] == want["max_rel"] and res[2] == want["max_abs"]
    assert res[1] == pytest.approx(want["sum_abs"], rel=1e-12)
    assert res[3] == 0


@pytest.mark.parametrize("path", [1, 2])
def test_scan_golden_sweep_parity(dpo, path):
    p = inputs.with_grid(inputs.PI48, (10, 10, 10, 10))
    _say("scan-golden sweep, path", path)
    V = inputs.random_value(p, seed=23, low=0, high=30)
    # smooth it so that Q(u) is unimodal enough for the search to be meaningful
    ax = [np.linspace(p["lo"][k], p["hi"][k], p["n"][k]) for k in range(4)]
    R, VR, VT, MM = np.meshgrid(*ax, indexing="ij")
    V = (400 * (R - 1.05) ** 2 + 900 * VR ** 2 + 2000 * (VT - 0.976) ** 2 + 50 * (1 - MM)).transpose(3, 2, 1, 0)
    V32 = V.astype(np.float32)
    o, ctx, Vg, ag, tg, res, Vo, ao, to, margin = _sweep_both(dpo, p, V32, path=path)
    free = o.kind == KIND_FREE
    check_search_values(o, V32.astype(np.float64), free, Vg, tg, ag, Vo, margin)
    clear = free & (margin >= 1e-4 * np.maximum(1.0, np.abs(Vo)))
    same_thr = tg[clear] == to[clear]
    assert same_thr.mean() >= 0.999
    n_thr, n_sharp = check_thrust_angles(o, V32.astype(np.float64), clear, tg, ag, to, ao)
    _say("  thrust nodes", n_thr, "sharp", n_sharp)


@pytest.mark.parametrize("path", [1, 2])
def test_scan_golden_random_masked_ragged(dpo, path):
    """Random values with M patches, a random reduced grid and a ragged grid
    whose node count is not a multiple of the workgroup size: values only
    (random fields make Q(u) multimodal, so the argmin is not unique)."""
    p = inputs.with_grid(inputs.PI48, (13, 9, 11, 7))
    _say("scan-golden random masked, path", path)
    rng = np.random.default_rng(29)
    mask = (rng.random((7, 11, 9, 13)) < 0.7).astype(np.uint8)
    V32 = inputs.random_value(p, seed=28, frac_M=0.15).astype(np.float32)
    o, ctx, Vg, ag, tg, res, Vo, ao, to, margin = _sweep_both(dpo, p, V32, mask=mask, path=path)
    free = o.kind == KIND_FREE
    n_clear = check_search_values(o, V32.astype(np.float64), free, Vg, tg, ag, Vo, margin)
    _say("  non-tie nodes", n_clear, "of", int(free.sum()))
    # fixed nodes are not written
    np.testing.assert_array_equal(Vg[~free], V32[~free])


def test_policy_eval_parity(dpo):
    p = inputs.VI12
    _say("policy eval")
    o = Oracle(p)
    V = inputs.random_value(p, seed=31, frac_M=0.1).astype(np.float32)
    rng = np.random.default_rng(32)
    thr = rng.integers(0, 2, size=o.shape).astype(np.uint8)
    ang = rng.uniform(-math.pi, math.pi, size=o.shape).astype(np.float32)
    ctx = dpo.Context(p)
    Vin = dev(V)
    Vout = Vin.clone()
    resid = torch.zeros(5, dtype=torch.float64, device="cuda")
    ctx.policy_eval_sweep(Vin, Vout, dev(ang), dev(thr, torch.uint8), resid)
    Vo = o.policy_eval_sweep(V.astype(np.float64), ang.astype(np.float64), thr)
    free = o.kind == KIND_FREE
    assert np.max(rel_err(host(Vout)[free], Vo[free])) < 1e-5


@pytest.mark.parametrize("path", [1, 2])
def test_policy_eval_of_last_sweep(dpo, path):
    """The descriptor-driven evaluation sweep equals the oracle's frozen-policy
    sweep for the policy the Bellman sweep just chose."""
    p = inputs.with_grid(inputs.PI48, (10, 10, 10, 10))
    _say("policy eval of last sweep, path", path)
    V32 = inputs.random_value(p, seed=33, low=0, high=40).astype(np.float32)
    o = Oracle(p)
    ctx = dpo.Context(p)
    ctx.set_kernel_path(path)
    Vin = dev(V32)
    Vg = Vin.clone()
    ang, thr = ctx.empty_policy()
    ctx.bellman_sweep(Vin, Vg, ang, thr)
    W = Vin.clone()
    ctx.policy_eval_sweep_last(Vg, W)
    # the oracle evaluates the device's chosen policy on the device's T V
    Vg_h = host(Vg).astype(np.float64)
    want = o.policy_eval_sweep(Vg_h, host(ang).astype(np.float64), host(thr))
    free = o.kind == KIND_FREE
    tol = sweep_tol(Vg_h, want)
    assert np.all(np.abs(host(W) - want)[free] <= tol[free])
    np.testing.assert_array_equal(host(W)[~free], V32[~free])


# ------------------------------------------------------------- solvers
def test_vi12_value_iteration_parity(dpo):
    """12^4, 16 angles + coast, VI to convergence vs the stored oracle solution."""
    p = inputs.VI12
    _say("12^4 VI")
    gold = np.load("tests/golden/vi12_table16.npz")
    o = Oracle(p)
    ctx = dpo.Context(p)
    V = ctx.init_value()
    ang, thr = ctx.empty_policy()
    rc, st = ctx.solve_vi(V, ang, thr, tol_rel=1e-7, max_sweeps=20000, check_every=8)
    _say("  sweeps", st["sweeps"], "resid", st["resid_max_rel"], "seconds", st["seconds"])
    assert st["converged"] or st["stalled"]
    Vg = host(V)
    free = o.kind == KIND_FREE
    err = rel_err(Vg, gold["V"])
    assert err[free].max() <= 1e-4, err.max()
    # policy agreement away from ties (margin from one oracle sweep at the fixed point)
    _, _, _, margin = o.bellman_sweep(gold["V"])
    clear = free & (margin >= 1e-4 * np.maximum(1.0, np.abs(gold["V"])))
    tg, ag = host(thr), host(ang)
    agree = (tg[clear] == gold["thr"][clear]) & (wrapped(ag[clear] - gold["angle"][clear]) < 1e-6)
    assert agree.mean() >= 0.999
    assert ctx.value_at(V, inputs.X0) == pytest.approx(o.value_at(gold["V"], inputs.X0), rel=1e-4)


def test_pi_matches_vi_on_device(dpo):
    """Value and policy iteration on the device reach the same fixed point."""
    p = inputs.VI12
    _say("12^4 PI vs VI")
    ctx = dpo.Context(p)
    V1 = ctx.init_value()
    a1, t1 = ctx.empty_policy()
    ctx.solve_vi(V1, a1, t1, tol_rel=1e-7, max_sweeps=20000, check_every=8)
    V2 = ctx.init_value()
    a2, t2 = ctx.empty_policy()
    rc, st = ctx.solve_pi(V2, a2, t2, tol_rel=1e-6, eval_sweeps=20, max_outer=5000)
    assert rc == dpo.DPO_OK
    _say("  PI outer", st["sweeps"], "evals", st["evals"])
    assert np.max(rel_err(host(V2), host(V1))) <= 1e-4


def test_pi_edge_cases(dpo):
    """Policy iteration with no evaluation sweeps is value iteration with the
    incumbent rule and reaches the same fixed point; a solve cut by max_outer
    reports its steps and sweeps."""
    p = inputs.VI12
    _say("PI edge cases")
    ctx = dpo.Context(p)
    V1 = ctx.init_value()
    a1, t1 = ctx.empty_policy()
    rc, st = ctx.solve_vi(V1, a1, t1, tol_rel=1e-6, max_sweeps=20000, check_every=1)
    assert rc == dpo.DPO_OK
    V2 = ctx.init_value()
    a2, t2 = ctx.empty_policy()
    rc, st = ctx.solve_pi(V2, a2, t2, tol_rel=1e-6, eval_sweeps=0, max_outer=20000)
    assert rc == dpo.DPO_OK and st["eval_sweeps"] == 0
    assert np.max(rel_err(host(V2), host(V1))) <= 1e-4
    # a solve cut by max_outer: every greedy step counted, each followed by
    # its evaluation sweeps, and the result finite and no larger than V0
    V3 = ctx.init_value()
    a3, t3 = ctx.empty_policy()
    rc, st = ctx.solve_pi(V3, a3, t3, tol_rel=0.0, eval_sweeps=5, max_outer=3)
    assert rc == dpo.DPO_ENOCONV and st["sweeps"] == 3 and st["eval_sweeps"] == 15
    # the device times of the greedy and evaluation sweeps, within the wall time
    assert 0 < st["greedy_seconds"] < st["seconds"] and 0 < st["eval_seconds"] < st["seconds"]
    v3 = host(V3)
    assert np.isfinite(v3).all() and np.all(v3 <= host(ctx.init_value()) + 3 * 6 * p["dt"])


@pytest.fixture(scope="module")
def small_pi_ref():
    p = inputs.with_grid(inputs.PI48, (10, 10, 10, 10))
    o = Oracle(p)
    ref = o.solve_pi(tol_abs=1e-8, eval_sweeps=20)
    assert ref["converged"]
    return p, o, ref


@pytest.mark.parametrize("path", [1, 2])
def test_small_pi_scan_golden_parity(dpo, small_pi_ref, path):
    """Modified PI (scan 64 + golden 12, 20 evaluation sweeps) on 10^4 against the oracle."""
    p, o, ref = small_pi_ref
    _say("small PI scan-golden, path", path)
    ctx = dpo.Context(p)
    ctx.set_kernel_path(path)
    V = ctx.init_value()
    ang, thr = ctx.empty_policy()
    rc, st = ctx.solve_pi(V, ang, thr, tol_rel=1e-6, eval_sweeps=20, max_outer=5000)
    assert rc == dpo.DPO_OK
    _say("  outer", st["sweeps"], "oracle outer", ref["outer"])
    free = o.kind == KIND_FREE
    Vg = host(V)
    assert rel_err(Vg, ref["V"])[free].max() <= 1e-4
    _, _, _, margin = o.bellman_sweep(ref["V"])
    clear = free & (margin >= 1e-4 * np.maximum(1.0, np.abs(ref["V"])))
    tg, ag = host(thr), host(ang)
    assert (tg[clear] == ref["thr"][clear]).mean() >= 0.999
    n_thr, n_sharp = check_thrust_angles(o, ref["V"], clear, tg, ag, ref["thr"], ref["angle"])
    _say("  thrust nodes", n_thr, "sharp", n_sharp)


def test_eikonal_on_device(dpo):
    """2-D minimum time: exact |x|/s on the axis nodes (float32 rounding)."""
    p = inputs.eikonal_problem(17)
    _say("eikonal")
    ctx = dpo.Context(p)
    V = ctx.init_value()
    ang, thr = ctx.empty_policy()
    rc, st = ctx.solve_vi(V, ang, thr, tol_rel=0.0, max_sweeps=400, check_every=8)
    Vg = host(V)
    h = 2.0 / 16
    for i in range(-8, 9):
        assert Vg[0, 8 + i, 8, 0] == pytest.approx(abs(i) * h, abs=2e-6)
        assert Vg[0, 8, 8 + i, 0] == pytest.approx(abs(i) * h, abs=2e-6)


# ---------------------------------------------------- a9 read-out, feedback
def test_value_at_and_feedback_parity(dpo):
    p = inputs.VI12
    _say("value_at / feedback")
    gold = np.load("tests/golden/vi12_table16.npz")
    o = Oracle(p)
    ctx = dpo.Context(p)
    Vd = dev(gold["V"])
    V32 = gold["V"].astype(np.float32).astype(np.float64)
    # most states of this coarse grid are ties (Q is dominated by the exit
    # value there): 4000 states leave ~60 clear of ties
    states = inputs.random_states(p, 4000, seed=41)
    for x in states[:50]:
        assert ctx.value_at(Vd, x) == pytest.approx(o.value_at(V32, x), rel=1e-12, abs=1e-9)
    ang, thr, q = ctx.feedback(Vd, states)
    n, n_clear, n_thr = check_feedback(o, V32, states, host(ang), host(thr), host(q), n_table=p["search"]["n_angles"],
                                       min_clear=40)
    _say("  states", n, "clear of ties", n_clear, "thrust compared", n_thr)


def test_feedback_parity_scan_golden(dpo):
    """eq:feed with the continuous search (scan 64 + golden 12) at random
    states of the 10^4 policy-iteration problem, on its converged value."""
    p = inputs.with_grid(inputs.PI48, (10, 10, 10, 10))
    _say("feedback scan-golden")
    o = Oracle(p)
    ref = o.solve_pi(tol_abs=1e-8, eval_sweeps=20)
    V32 = ref["V"].astype(np.float32).astype(np.float64)
    ctx = dpo.Context(p)
    states = inputs.random_states(p, 500, seed=43)
    ang, thr, q = ctx.feedback(dev(V32), states)
    n, n_clear, n_thr = check_feedback(o, V32, states, host(ang), host(thr), host(q), min_clear=100)
    _say("  states", n, "clear of ties", n_clear, "thrust compared", n_thr)


# ----------------------------------------------------------- a1 mask
def test_mask_from_coarse_parity(dpo):
    _say("mask")
    gold = np.load("tests/golden/vi12_table16.npz")
    Vc32 = gold["V"].astype(np.float32)
    fine = inputs.with_grid(inputs.PI48, (24, 24, 24, 24))
    thresh = inputs.MASK_THRESHOLD_FRAC * inputs.VI12["M"]
    want = mask_from_coarse(inputs.VI12, Vc32.astype(np.float64), fine, inputs.MASK_DILATE, thresh)
    ctx = dpo.Context(inputs.VI12)
    got = host(ctx.mask_from_coarse(dev(Vc32), fine, thresh, inputs.MASK_DILATE))
    np.testing.assert_array_equal(got, want)


# ------------------------------------------------------------ ABI errors
def test_abi_error_paths(dpo):
    _say("abi errors")
    import copy
    p = copy.deepcopy(inputs.VI12)
    bad = inputs.with_grid(p, (1, 12, 12, 12))
    with pytest.raises(dpo.DpoError) as e:
        dpo.Context(bad)
    assert e.value.code == dpo.DPO_EINVAL
    p2 = copy.deepcopy(p)
    p2["search"] = dict(mode="scan_golden", n_scan=4, n_golden=12)
    with pytest.raises(dpo.DpoError):
        dpo.Context(p2)
    ctx = dpo.Context(p)
    V = ctx.init_value()
    with pytest.raises(dpo.DpoError) as e:
        ctx.bellman_sweep(V, V)
    assert e.value.code == dpo.DPO_EINVAL
    with pytest.raises(dpo.DpoError):
        ctx.probe_q(V, np.array([ctx.N + 5]), np.array([1]), np.array([0.0]))
    # non-finite values are reported, not hidden
    Vn = V.clone()
    Vn.view(-1)[int(np.flatnonzero(host(ctx.kind()).reshape(-1) == 0)[0])] = float("nan")
    ang, thr = ctx.empty_policy()
    with pytest.raises(dpo.DpoError) as e:
        ctx.solve_vi(Vn, ang, thr, tol_rel=1e-7, max_sweeps=16, check_every=1)
    assert e.value.code == dpo.DPO_ENUMERIC
    # max_sweeps exhausted -> ENOCONV with valid output
    V = ctx.init_value()
    rc, st = ctx.solve_vi(V, ang, thr, tol_rel=1e-12, max_sweeps=5, check_every=1)
    assert rc == dpo.DPO_ENOCONV and st["sweeps"] == 5


# ------------------------------------------------------- seeded greedy step
def check_seeded_sweep(o, V, free, Vg, tg, ag, Vo, margin, fb, sr):
    """Values of the seeded search against the oracle's.

    Where the oracle kept its local result clearly (|Q - V_in| below half the
    fallback threshold) and has no tie, the device ran the same local search
    from the same seed: its value agrees within sweep_tol on >= 99.9 % of
    those nodes.  Everywhere the device value is the Q of its own control."""
    tol = sweep_tol(V, Vo)
    vin = np.asarray(V, dtype=np.float64)
    thresh = sr["fallback_tol"] * np.maximum(1.0, np.abs(vin))
    scale = np.maximum(1.0, np.abs(Vo))
    keep = free & (fb == 0) & (np.abs(Vo - vin) < 0.5 * thresh) & (margin >= 1e-4 * scale)
    ok = np.abs(Vg[keep] - Vo[keep]) <= tol[keep]
    assert ok.mean() >= 0.999, ok.mean()
    nodes = np.flatnonzero(free.reshape(-1))
    thr = tg.reshape(-1)[nodes]
    ang = ag.reshape(-1)[nodes].astype(np.float64)
    vg = Vg.reshape(-1)[nodes].astype(np.float64)
    tl = tol.reshape(-1)[nodes]
    attained = np.abs(vg - Vo.reshape(-1)[nodes]) <= tl
    for du in (0.0, -ANGLE_ROUND, ANGLE_ROUND):
        attained |= np.abs(vg - o.q_many(V, nodes, thr, ang + du)) <= tl
    assert attained.all()
    return int(keep.sum())


@pytest.mark.parametrize("path,near_frac", [(1, 2 / 3), (2, 2 / 3), (2, 0.97)])
def test_seeded_sweep_parity(dpo, small_pi_ref, path, near_frac):
    """Seeded greedy step at the converged 10^4 value function: seeds near the
    optimal angles on a fraction of the nodes, random elsewhere (those fall
    back to the full search).  With 3 % random seeds most waves have only a
    few falling-back lanes, which the factorised path defers to its second
    pass; with a third, most waves do the full search in place."""
    p, o, ref = small_pi_ref
    _say("seeded sweep, path", path, "near", near_frac)
    sr = inputs.SEEDED
    V32 = ref["V"].astype(np.float32)
    rng = np.random.default_rng(31)
    near = rng.random(o.shape) < near_frac
    seed = np.where(near, ref["angle"] + rng.normal(0.0, 0.02, o.shape),
                    rng.uniform(-math.pi, math.pi, o.shape)).astype(np.float32)
    ctx = dpo.Context(p)
    ctx.set_kernel_path(path)
    ctx.set_search(sr)
    Vin = dev(V32)
    Vout = Vin.clone()
    ang, thr = ctx.empty_policy()
    resid = torch.zeros(5, dtype=torch.float64, device="cuda")
    ctx.bellman_sweep_seeded(Vin, Vout, ang, thr, dev(seed), resid)
    Vo, ao, to, margin, fb = o.bellman_sweep_seeded(V32.astype(np.float64), seed.astype(np.float64), search=sr)
    free = o.kind == KIND_FREE
    n_keep = check_seeded_sweep(o, V32.astype(np.float64), free, host(Vout), host(thr), host(ang), Vo, margin, fb,
                                sr)
    n_fb_dev, n_fb_or = int(host(resid)[4]), int(fb[free].sum())
    _say("  kept-local nodes compared", n_keep, "fallbacks device", n_fb_dev, "oracle", n_fb_or, "of",
         int(free.sum()))
    # fallback decisions are float32 vs FP64 comparisons against a threshold
    assert abs(n_fb_dev - n_fb_or) <= 0.01 * free.sum() + 2


def test_walk_seeded_pi_matches_plain(dpo, small_pi_ref):
    """Seeds taken from the previous greedy step's own angles (seed aliasing
    the policy array): the warm-started minimisation of the paper reaches the
    plain PI fixed point within 1e-4."""
    p, o, ref = small_pi_ref
    _say("walk-seeded PI")
    ctx = dpo.Context(p)
    ctx.set_search(inputs.SEEDED)
    V = ctx.init_value()
    ang, thr = ctx.empty_policy()
    rc, st = ctx.solve_pi(V, ang, thr, tol_rel=1e-6, eval_sweeps=20, max_outer=5000, seed=ang)
    assert rc == dpo.DPO_OK
    free = o.kind == KIND_FREE
    _say("  outer", st["sweeps"], "fallback nodes", st["fallback_nodes"], "evals", st["evals"])
    assert rel_err(host(V), ref["V"])[free].max() <= 1e-4


@pytest.mark.parametrize("path", [1, 2])
def test_seeded_pi_is_certified_by_the_full_search(dpo, small_pi_ref, path):
    """A seeded solve stops only on a full-search greedy step, which runs the
    scan + golden search of the context's SEEDED parameters (here a coarse
    8-angle scan, so that the scan alone is far from the golden-refined
    minimum): at its result no node's scan + golden value lies below its
    value by more than the stop tolerance, as at the result of an unseeded
    solve.  The seeds are fixed random angles, so the local searches settle
    in wrong basins that only the full search can leave."""
    p, o, ref = small_pi_ref
    _say("seeded PI certified by scan + golden, path", path)
    sr = dict(inputs.SEEDED, n_scan=8)
    tol = 1e-6
    ctx = dpo.Context(p)
    ctx.set_kernel_path(path)
    ctx.set_search(sr)
    V = ctx.init_value()
    ang, thr = ctx.empty_policy()
    seed = dev(np.random.default_rng(32).uniform(-math.pi, math.pi, o.shape).astype(np.float32))
    # the solve's first greedy step is a full step with no incumbent yet: from
    # V0 it is one scan + golden sweep, bit for bit
    sg = dict(mode="scan_golden", n_scan=8, n_golden=12)
    V1 = ctx.init_value()
    a1, t1 = ctx.empty_policy()
    rc, _ = ctx.solve_pi(V1, a1, t1, tol_rel=0.0, eval_sweeps=0, max_outer=1, seed=seed)
    assert rc == dpo.DPO_ENOCONV
    ctx.set_search(sg)
    V0 = ctx.init_value()
    G = V0.clone()
    a0, t0 = ctx.empty_policy()
    ctx.bellman_sweep(V0, G, a0, t0)
    np.testing.assert_array_equal(host(V1), host(G))
    np.testing.assert_array_equal(host(t1), host(t0))
    np.testing.assert_array_equal(host(a1), host(a0))
    ctx.set_search(sr)
    rc, st = ctx.solve_pi(V, ang, thr, tol_rel=tol, eval_sweeps=20, max_outer=5000, seed=seed)
    assert rc == dpo.DPO_OK and st["verify_steps"] >= 1
    ctx.set_search(sg)
    W = V.clone()
    a2, t2 = ctx.empty_policy()
    ctx.bellman_sweep(V, W, a2, t2)
    free = o.kind == KIND_FREE
    Vh, Wh = host(V).astype(np.float64), host(W).astype(np.float64)
    gain = ((Vh - Wh) / np.maximum(1.0, np.abs(Vh)))[free]
    _say("  outer", st["sweeps"], "full-search steps", st["verify_steps"], "largest full-search gain", gain.max())
    assert gain.max() <= 2 * tol, gain.max()


# ----------------------------------------------- foot-descriptor formats
@pytest.mark.parametrize("case", ["per_node", "per_free_node", "flat_code"])
def test_descriptor_formats(dpo, case):
    """The evaluation sweep from descriptors in each storage form equals the
    oracle's Q of the greedy step's policy: codes stored per node (most nodes
    free), per free node (a sparse reduced grid), and 32-bit flat codes (feet
    farther than the compact code reaches: dt = 2 on a 12^4 grid, the direct
    kernel path)."""
    _say("descriptor format", case)
    mask = None
    if case == "flat_code":
        p = dict(inputs.with_grid(inputs.PI48, (12, 12, 12, 12)), dt=2.0)
    else:
        p = inputs.with_grid(inputs.PI48, (11, 10, 9, 8))
        if case == "per_free_node":
            rng = np.random.default_rng(71)
            mask = (rng.random((8, 9, 10, 11)) < 0.35).astype(np.uint8)
    o = Oracle(p, mask=mask)
    ctx = dpo.Context(p, mask=None if mask is None else dev(mask, torch.uint8))
    free = o.kind == KIND_FREE
    nf = int(free.sum())
    want = {"per_node": 16 * nf + 8 * (o.N - nf), "per_free_node": 22 * nf, "flat_code": 24 * nf}[case]
    assert ctx.eval_sweep_bytes() == want
    V = inputs.random_value(p, seed=73, frac_M=0.1).astype(np.float32)
    Vin = dev(V)
    W = Vin.clone()
    ang, thr = ctx.empty_policy()
    ctx.bellman_sweep(Vin, W, ang, thr)
    E = Vin.clone()
    ctx.policy_eval_sweep_last(Vin, E)
    nodes = np.flatnonzero(free.reshape(-1))
    from scipy.ndimage import maximum_filter
    corner = maximum_filter(np.abs(V.astype(np.float64)), size=7, mode="nearest").reshape(-1)[nodes]
    ve = host(E).reshape(-1)[nodes].astype(np.float64)
    # the sweep reproduces the greedy step's own Q of the chosen control
    vg = host(W).reshape(-1)[nodes].astype(np.float64)
    assert np.all(np.abs(ve - vg) <= 1e-5 * np.maximum(1.0, np.abs(vg)) + 1e-6 * corner)
    np.testing.assert_array_equal(host(E)[~free], V[~free])
    # and the oracle's Q of the same control
    tg = host(thr).reshape(-1)[nodes]
    ag = host(ang).reshape(-1)[nodes].astype(np.float64)
    q = o.q_many(V.astype(np.float64), nodes, tg, ag)
    ok = np.abs(ve - q) <= 1e-5 * np.maximum(1.0, np.abs(q)) + 1e-6 * corner
    if case == "flat_code":
        # Feet 35 cells away: the float32 foot is ~1e-5 cell from the FP64 one,
        # so where the oracle's foot lies that close to a domain face the two
        # can fall on different sides of the jump to M (a quarter of the nodes
        # here: the best angle often puts the foot just inside a face).
        # Compared exactly at every node whose FP64 foot is farther than 1e-3
        # cell from every face; at the others the value must be the oracle's Q
        # within ANGLE_ROUND of the device's angle.
        n = p["n"]
        h = [(p["hi"][k] - p["lo"][k]) / (n[k] - 1) for k in range(4)]
        near = np.zeros(nodes.size, dtype=bool)
        for c, j in enumerate(nodes):
            z = o.step(o.node_coords(int(j)), int(tg[c]), float(ag[c]))
            s = [(z[k] - p["lo"][k]) / h[k] for k in range(4)]
            near[c] = any(min(abs(s[k]), abs(s[k] - (n[k] - 1))) < 1e-3 for k in range(4))
        _say("  flat codes: nodes compared with the oracle", int((~near).sum()), "of", nodes.size)
        assert (~near).sum() >= 0.6 * nodes.size
        tol = 1e-5 * np.maximum(1.0, np.abs(q)) + 1e-6 * corner
        for du in (-ANGLE_ROUND, ANGLE_ROUND):
            qd = o.q_many(V.astype(np.float64), nodes, tg, ag + du)
            ok |= near & (np.abs(ve - qd) <= tol)
    assert np.all(ok)

"""Exact policy evaluation on the device (eq:p_eval solved by GMRES with the
frozen-policy sweep as the operator) against the oracle's direct sparse
solve of the same system, and policy iteration with exact evaluation against
the oracle's converged value.

The device stops on the node-wise relative residual max_j |b - A v|_j /
max(1, |v_j|).  Checked: that residual, recomputed in FP64 by the oracle's
own frozen-policy sweep, is within a few times the tolerance (float32
rounding of v adds ~1e-7 |v|), and the max-norm error against the direct
solve is within the max-norm residual divided by 1 - exp(-lambda dt) (the
inverse of I - exp(-lambda dt) P has that max-norm for a substochastic P).
"""
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


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(1.0, np.abs(b))


@pytest.mark.parametrize("integrator,n", [("euler", (8, 6, 6, 8)), ("heun", (8, 6, 6, 8)),
                                          ("heun", (16, 10, 10, 12))])
def test_exact_evaluation_parity(dpo, integrator, n):
    """Against the oracle's direct sparse solve: 2,304 nodes with either foot,
    and 19,200 nodes (several GMRES restarts over a basis of 8)."""
    p = inputs.crown_problem(n, integrator=integrator)
    _say("exact evaluation", integrator, n)
    o = Oracle(p)
    rng = np.random.default_rng(141)
    ang = rng.uniform(-math.pi, math.pi, size=o.shape).astype(np.float32)
    thr = rng.integers(0, 2, size=o.shape).astype(np.uint8)
    want = o.policy_evaluate_exact(o.init_value(), ang.astype(np.float64), thr)
    ctx = dpo.Context(p)
    V = ctx.init_value()
    # float32 floor of the node-wise residual: ~3e-7 (values next to the exit faces carry M = 1e6)
    rc, mv, rel = ctx.policy_evaluate(V, dev(ang), dev(thr, torch.uint8), tol_rel=1e-6, max_iter=2000)
    _say("  operator applications", mv, "relative residual", rel)
    assert rc == dpo.DPO_OK and rel <= 1e-6
    v = host(V).astype(np.float64)
    free = o.kind == KIND_FREE
    r = (o.policy_eval_sweep(v, ang.astype(np.float64), thr) - v)[free]
    rel64 = np.max(np.abs(r) / np.maximum(1.0, np.abs(v[free])))
    gamma = math.exp(-p["lam"] * p["dt"])
    err = np.max(np.abs(v - want)[free])
    _say(f"  FP64 node-wise residual {rel64:.2e}, max error {err:.3e} (bound {np.max(np.abs(r)) / (1 - gamma):.3e}),"
         f" max relative error {rel_err(v, want).max():.2e}")
    assert rel64 <= 3e-6
    assert err <= 1.01 * np.max(np.abs(r)) / (1 - gamma)
    assert rel_err(v, want).max() <= 1e-4


def test_exact_evaluation_full_size_a_posteriori(dpo):
    """The paper's Example 1 grid (110 x 30 x 30 x 30, 2.97M unknowns, Heun
    foot) under a random policy, solved by GMRES to a node-wise relative
    residual of 1e-6: at 100,000 sampled nodes the oracle's FP64 frozen-policy
    step (its Q of the node's control at the device's solution) moves the
    solution by no more than a few times the tolerance, which bounds the
    error by the residual over 1 - exp(-lambda dt)."""
    p = inputs.EX1
    _say("exact evaluation, Example 1 grid")
    ctx = dpo.Context(p)
    o = Oracle(p)
    rng = np.random.default_rng(143)
    ang = rng.uniform(-math.pi, math.pi, size=o.shape).astype(np.float32)
    thr = rng.integers(0, 2, size=o.shape).astype(np.uint8)
    V = ctx.init_value()
    rc, mv, rel = ctx.policy_evaluate(V, dev(ang), dev(thr, torch.uint8), tol_rel=1e-6, max_iter=5000)
    _say("  operator applications", mv, "relative residual", rel)
    assert rc == dpo.DPO_OK and rel <= 1e-6
    v = host(V).astype(np.float64)
    nodes = np.sort(rng.choice(o.N, size=100000, replace=False)).astype(np.int64)
    q = o.q_many(v, nodes, thr.reshape(-1)[nodes], ang.reshape(-1)[nodes].astype(np.float64))
    vn = v.reshape(-1)[nodes]
    r = np.abs(q - vn) / np.maximum(1.0, np.abs(vn))
    _say(f"  FP64 node-wise residual at the sampled nodes: max {r.max():.2e}, 99.9 % {np.quantile(r, 0.999):.2e}")
    assert r.max() <= 3e-6


def test_policy_iteration_with_exact_evaluation(dpo):
    p = inputs.crown_problem((8, 6, 6, 8))
    _say("PI with exact evaluation")
    gold = np.load("tests/golden/crown8_table72.npz")
    ctx = dpo.Context(p)
    V = ctx.init_value()
    a, t = ctx.empty_policy()
    rc, st = ctx.solve_pi(V, a, t, tol_rel=1e-6, eval_sweeps=-1, max_outer=200)
    _say("  greedy steps", st["sweeps"], "operator applications", st["eval_sweeps"])
    assert st["converged"] or st["stalled"]
    assert rel_err(host(V), gold["V"]).max() <= 1e-4
    V2 = ctx.init_value()
    a2, t2 = ctx.empty_policy()
    rc2, st2 = ctx.solve_pi(V2, a2, t2, tol_rel=1e-6, eval_sweeps=20, max_outer=2000)
    _say("  modified PI: greedy steps", st2["sweeps"], "evaluation sweeps", st2["eval_sweeps"])
    assert st["sweeps"] < st2["sweeps"]


def test_exact_evaluation_refusals(dpo):
    ctx = dpo.Context(inputs.VI12)  # lambda = 0
    V = ctx.init_value()
    a, t = ctx.empty_policy()
    with pytest.raises(dpo.DpoError):
        ctx.policy_evaluate(V, a, t)
    with pytest.raises(dpo.DpoError):
        ctx.solve_pi(V, a, t, eval_sweeps=-1, max_outer=3)

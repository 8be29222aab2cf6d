"""Pins of the oracle's Heun (second-order Runge-Kutta) foot point and of the
table walk from the previous optimum, against facts that do not come from
the oracle itself: the local error of an accurate ODE integration, exact
special cases, and brute-force enumeration of the whole control table."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle.core import KIND_FREE, Oracle
from paper_2407_14675_amd import inputs


def heun(problem):
    p = dict(problem)
    p["integrator"] = "heun"
    return p


def exact_flow(p, x, thr, u, tau):
    """The planar orbit dynamics with the control held fixed, integrated to
    1e-13 by an eighth-order Runge-Kutta method."""
    mu, a, c = p["mu"], p["accel"], p["mdot"]

    def f(_t, y):
        r, vr, vt, m = y
        acc = a / m if thr else 0.0
        return [vr, vt * vt / r - mu / (r * r) + acc * math.sin(u), -vr * vt / r + acc * math.cos(u),
                -c * thr]

    sol = solve_ivp(f, (0.0, tau), list(x), method="DOP853", rtol=1e-13, atol=1e-15)
    return sol.y[:, -1]


@pytest.mark.parametrize("thr", [0, 1])
def test_heun_step_has_third_order_local_error(thr):
    """One Heun step from x differs from the exact flow by O(tau^3): halving
    tau divides the error by ~8.  One Euler step (second-order local error)
    divides it by ~4.  A Heun step that dropped its corrector, used the
    predictor's slope only, or evaluated the second slope at the wrong point
    falls back to the Euler ratio."""
    base = dict(inputs.VI12)
    base["accel"] = 0.05  # thrust comparable to the orbit's curvature terms
    rng = np.random.default_rng(71)
    ratios = {"euler": [], "heun": []}
    for x in inputs.random_states(base, 40, seed=72):
        u = rng.uniform(-math.pi, math.pi)
        for name in ("euler", "heun"):
            p = dict(base, integrator=name)
            o = Oracle(p)
            errs = []
            for tau in (0.2, 0.1):
                z = o.step(x, thr, u, tau=tau)
                errs.append(np.linalg.norm(z - exact_flow(p, x, thr, u, tau)))
            ratios[name].append(errs[0] / errs[1])
    assert 7.5 < min(ratios["heun"]) and max(ratios["heun"]) < 8.5, ratios["heun"]
    assert 3.8 < min(ratios["euler"]) and max(ratios["euler"]) < 4.2, ratios["euler"]


def test_heun_special_cases():
    """Mass falls by exactly c*tau under thrust whatever the integrator (its
    rate is constant); the eikonal field does not depend on the state, so
    Heun and Euler give the same point; a state on a circular orbit is a
    zero of the coast field, so both steps leave it in place."""
    p = inputs.VI12
    oe, oh = Oracle(p), Oracle(heun(p))
    for x in inputs.random_states(p, 50, seed=73):
        zh = oh.step(x, 1, 0.3)
        assert zh[3] == pytest.approx(x[3] - p["mdot"] * p["dt"], abs=1e-15)
    pe = inputs.eikonal_problem(9)
    e1, e2 = Oracle(pe), Oracle(heun(pe))
    for u in np.linspace(-3, 3, 7):
        np.testing.assert_array_equal(e1.step([0, 0.1, -0.2, 0], 1, u), e2.step([0, 0.1, -0.2, 0], 1, u))
    x = np.array([1.03, 0.0, 1.03 ** -0.5, 1.0])
    for o in (oe, oh):
        np.testing.assert_allclose(o.step(x, 0, 0.0, tau=0.05), x, rtol=0, atol=1e-14)


def test_heun_foot_at_nodes_matches_the_step():
    """The node Q uses the foot in grid coordinates; it must be the same
    point as the physical step mapped onto the grid."""
    p = heun(inputs.with_grid(inputs.VI12, (7, 7, 7, 7)))
    o = Oracle(p)
    V = inputs.random_value(p, seed=74)
    h = [(p["hi"][k] - p["lo"][k]) / (p["n"][k] - 1) for k in range(4)]
    rng = np.random.default_rng(75)
    for j in rng.choice(np.flatnonzero(o.kind.reshape(-1) == KIND_FREE), 60, replace=False):
        u = rng.uniform(-math.pi, math.pi)
        x = o.node_coords(int(j))
        z = o.step(x, 1, u)
        s = [(z[k] - p["lo"][k]) / h[k] for k in range(4)]
        want = p["dt"] * (p["w_time"] + p["w_fuel"]) + o.interp(V, s)
        assert o.q(V, int(j), 1, u) == pytest.approx(want, rel=1e-12, abs=1e-12)


# ------------------------------------------------------------------- walk
def _table(K):
    return np.array([-math.pi + 2 * math.pi * k / K for k in range(K)])


def test_walk_ends_on_a_local_minimiser_reached_downhill():
    """From any start, the walk's angle k* is a local minimiser of the cyclic
    table of thrust Q values (enumerated in full), reached from the start by
    a run of strictly decreasing Q in one direction that begins at the lower
    neighbour; where the table has a single local minimum the walk finds the
    exhaustive table's answer."""
    K = 16
    p = inputs.with_grid(inputs.VI12, (5, 5, 5, 5))
    p["search"] = dict(mode="table_walk", n_angles=K)
    o = Oracle(p)
    V = inputs.random_value(p, seed=76, frac_M=0.2)
    rng = np.random.default_rng(77)
    free = np.flatnonzero(o.kind.reshape(-1) == KIND_FREE)
    start = rng.integers(0, K, size=o.N)
    prev = _table(K)[start].reshape(o.shape)
    Vw, aw, tw, mw, evals = o.bellman_sweep_walk(V, prev)
    Vt, at, tt, mt = o.bellman_sweep(V, dict(mode="table", n_angles=K))
    tab = _table(K)
    unimodal = 0
    for j in free[:300]:
        q = np.array([o.q(V, j, 1, u) for u in tab])
        qc = o.q(V, j, 0, 0.0)
        k0 = int(start[j])
        ks = int(np.argmin(np.abs(np.angle(np.exp(1j * (tab - aw.reshape(-1)[j]))))))
        assert q[ks] <= q[(ks - 1) % K] and q[ks] <= q[(ks + 1) % K]
        assert Vw.reshape(-1)[j] == min(qc, q[ks]) and tw.reshape(-1)[j] == (1 if q[ks] < qc else 0)
        if ks != k0:
            lo, hi = q[(k0 - 1) % K], q[(k0 + 1) % K]
            d = -1 if (lo < q[k0] and lo <= hi) else 1
            path = [(k0 + d * s) % K for s in range((ks - k0) * d % K + 1)]
            assert path[-1] == ks
            assert np.all(np.diff(q[path]) < 0)
        n_min = sum(q[k] <= q[(k - 1) % K] and q[k] <= q[(k + 1) % K] for k in range(K))
        if n_min == 1:
            unimodal += 1
            assert Vw.reshape(-1)[j] == Vt.reshape(-1)[j]
    assert unimodal > 20
    assert evals >= 3 * free.size


def test_walk_from_the_optimum_costs_three_evaluations():
    """Started on the exhaustive table's angle, the walk stays there: the
    same values and controls, three thrust evaluations per node."""
    K = 16
    p = inputs.with_grid(inputs.VI12, (6, 6, 6, 6))
    o = Oracle(p)
    V = inputs.random_value(p, seed=78, frac_M=0.2)
    Vt, at, tt, mt = o.bellman_sweep(V, dict(mode="table", n_angles=K))
    Vw, aw, tw, mw, evals = o.bellman_sweep_walk(V, at, dict(mode="table_walk", n_angles=K))
    np.testing.assert_array_equal(Vw, Vt)
    np.testing.assert_array_equal(tw, tt)
    assert evals == 3 * int((o.kind == KIND_FREE).sum())


def test_walk_fixed_point_never_below_the_table_fixed_point():
    """A walk value is one of the table's values, so the walk operator is >=
    the exhaustive one pointwise; both are monotone, so value iteration with
    the walk (full table on the first sweep) converges to a fixed point that
    is nowhere below the exhaustive table's, and policy iteration with the
    walk reaches the same values as value iteration with it.  (How often the
    two fixed points agree is measured, not pinned: on this coarse grid the
    walk stops on the plateaus where every foot of a range of angles leaves
    the domain and Q is exactly dt + M.)"""
    p = inputs.with_grid(inputs.VI12, (8, 8, 8, 8))
    o = Oracle(p)
    walk_search = dict(mode="table_walk", n_angles=16)
    ref = o.solve_vi(tol_abs=1e-10, max_sweeps=20000)
    walk = o.solve_vi(tol_abs=1e-10, max_sweeps=20000, search=walk_search)
    wpi = o.solve_pi(tol_abs=1e-10, eval_sweeps=20, max_outer=5000, search=walk_search)
    assert ref["converged"] and walk["converged"] and wpi["converged"]
    free = o.kind == KIND_FREE
    d = walk["V"][free] - ref["V"][free]
    assert d.min() > -1e-8
    np.testing.assert_allclose(wpi["V"][free], walk["V"][free], rtol=0, atol=1e-6)

"""Pins of the oracle's closed loop (feedback eq:feed applied to the model
integrated by the classical fourth-order Runge-Kutta method): the local
error order of the integrator against an accurate integration, a circular
orbit's exact motion, the eikonal problem's straight path home, and the
work and torque of Example 2's drag."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle.core import Oracle
from paper_2407_14675_amd import inputs


def test_rk4_local_error_is_fifth_order():
    """One RK4 step differs from the exact flow by O(h^5): halving h divides
    the error by ~32, on the orbit model and on the crown model."""
    rng = np.random.default_rng(111)
    cases = [(dict(inputs.VI12, accel=0.05), 0.4, inputs.VI12, 1.0, 0.0),
             (dict(inputs.crown_problem((8, 6, 6, 8)), accel=2e-3), 400.0, inputs.EX1, 1e-3, 0.0),
             (dict(inputs.VI12, accel=0.05), 0.4, inputs.VI12, 1.0, 0.05),
             (dict(inputs.crown_problem((8, 6, 6, 8)), accel=2e-3), 400.0, inputs.EX1, 1e-3, 5e-6)]
    for p, h0, box, vscale, drag in cases:
        o = Oracle(p)
        ratios = []
        for x in inputs.random_states(box, 15, seed=112):
            u = rng.uniform(-math.pi, math.pi)

            def f(_t, y):
                r, vr, vt, z = y
                acc = p["accel"] / (z if p["model"] == "orbit" else 1.0)
                last = -p["mdot"] if p["model"] == "orbit" else vt / r
                dv = drag * math.hypot(vr, vt)
                return [vr, vt * vt / r - p["mu"] / (r * r) + acc * math.sin(u) - dv * vr,
                        -vr * vt / r + acc * math.cos(u) - dv * vt, last]

            errs = []
            for h in (h0, h0 / 2):
                ref = solve_ivp(f, (0, h), list(x), method="DOP853", rtol=3e-14, atol=1e-14 * vscale).y[:, -1]
                d = (o.rk4_step(x, 1, u, h, drag) - ref) / np.array([1.0, vscale, vscale, vscale])
                errs.append(np.linalg.norm(d))
            ratios.append(errs[0] / errs[1])
        # ~32 (a lower-order step gives 16 or less); the steps are not quite asymptotic
        assert 24 < min(ratios) and max(ratios) < 40, ratios
        assert 29 < np.median(ratios) < 35, ratios


def test_circular_orbit_coasts_exactly():
    """A circular orbit is a rest point of (r, v_r, v_t) and theta grows at
    the constant rate v_t/r: every RK4 stage sees zero there, so the closed
    loop's coast leaves r, v_r, v_t unchanged and theta(t) = theta0 + t v_t/r."""
    p = inputs.crown_problem((8, 6, 6, 8))
    o = Oracle(p)
    r = 7000.0
    x = np.array([r, 0.0, math.sqrt(p["mu"] / r), 0.3])
    y = x.copy()
    for _ in range(500):
        y = o.rk4_step(y, 0, 0.0, 10.0)
    np.testing.assert_allclose(y[:3], x[:3], rtol=1e-13, atol=1e-15)
    assert y[3] == pytest.approx(0.3 + 5000.0 * x[2] / r, rel=1e-12)


def test_eikonal_closed_loop_goes_straight_home():
    """Minimum time to the origin at speed s: from an axis node the feedback
    points straight at the origin (angles of the 16-entry table include the
    four axis directions) and constant velocity is integrated exactly, so
    after k steps of tau = h/s the state is k cells closer, and it stops at
    the origin's cell."""
    p = inputs.eikonal_problem(17)
    o = Oracle(p)
    res = o.solve_vi(tol_abs=1e-13, max_sweeps=2000)
    h = 2.0 / 16
    tau = h / p["speed"]
    starts = np.array([[0.0, 0.0, 6 * h, 0.0], [0.0, -5 * h, 0.0, 0.0], [0.0, 7 * h, 0.0, 0.0]])
    final, traj, thr, ang = o.simulate(res["V"], starts, tau, steps=4)
    for c, x0 in enumerate(starts):
        direction = -np.sign(x0) * (np.abs(x0) > 0)
        for k in range(5):
            np.testing.assert_allclose(traj[k, c], x0 + k * h * direction, atol=1e-12)
        assert np.all(thr[:, c] == 1)
    np.testing.assert_array_equal(final, traj[-1])


@pytest.mark.parametrize("model", ["orbit", "crown"])
def test_drag_work_and_torque(model):
    """Example 2's drag a_D = -C |v| v (per unit mass) does work a_D . v =
    -C |v|^3 and exerts the torque r x a_D = -C |v| (r x v): on a coast the
    model alone keeps the energy v^2/2 - mu/r and the angular momentum r v_t,
    so over a short step the drag alone changes them by -C |v|^3 h and
    -C |v| r v_t h (to first order in h).  A wrong sign, a missing speed
    factor or a drag on the wrong component fails one of the two."""
    if model == "orbit":
        p, r, C, h = dict(inputs.VI12), 1.03, 0.05, 1e-3
    else:
        p, r, C, h = inputs.crown_problem((8, 6, 6, 8)), 7000.0, 1e-6, 1.0
    o = Oracle(p)
    mu = p["mu"]
    rng = np.random.default_rng(113)
    for _ in range(5):
        vt = math.sqrt(mu / r) * rng.uniform(0.98, 1.02)
        # a radial speed of 10-20 % of the speed, so that drag on one component
        # only would miss the work by 1-4 %
        vr = math.sqrt(mu / r) * rng.uniform(0.1, 0.2) * rng.choice([-1.0, 1.0])
        x = np.array([r, vr, vt, 1.0 if model == "orbit" else 0.4])
        speed = math.hypot(vr, vt)

        def energy(y):
            return 0.5 * (y[1] ** 2 + y[2] ** 2) - mu / y[0]

        y0 = o.rk4_step(x, 0, 0.0, h, 0.0)
        y1 = o.rk4_step(x, 0, 0.0, h, C)
        dE = (energy(y1) - energy(y0)) / h
        dH = (y1[0] * y1[2] - y0[0] * y0[2]) / h
        assert dE == pytest.approx(-C * speed ** 3, rel=2e-3)
        assert dH == pytest.approx(-C * speed * r * vt, rel=2e-3)
    # a long coast with drag loses energy at every step
    y = np.array([r, 0.0, math.sqrt(mu / r), 1.0 if model == "orbit" else 0.4])
    e_prev = 0.5 * y[2] ** 2 - mu / y[0]
    for _ in range(200):
        y = o.rk4_step(y, 0, 0.0, h * 10, C)
        e = 0.5 * (y[1] ** 2 + y[2] ** 2) - mu / y[0]
        assert e < e_prev
        e_prev = e


def test_drag_off_is_the_model():
    """drag = 0 gives the model's own closed loop bit for bit; the simulated
    trajectory with drag differs."""
    p = inputs.crown_problem((8, 6, 6, 8))
    o = Oracle(p)
    V = 1e3 + 1e-3 * np.arange(np.prod(o.shape), dtype=np.float64).reshape(o.shape)
    starts = inputs.random_states(p, 4, seed=114, margin=0.1)
    a = o.simulate(V, starts, p["dt"], 20)
    b = o.simulate(V, starts, p["dt"], 20, drag=0.0)
    c = o.simulate(V, starts, p["dt"], 20, drag=1e-9)
    np.testing.assert_array_equal(a[1], b[1])
    assert np.any(a[1][-1] != c[1][-1])

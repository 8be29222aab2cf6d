"""Pins of the oracle's crown problem (the paper's Example 1: polar state on a
circular crown, theta periodic, orbital-element running cost, discount)
against facts that do not come from the oracle: the Cartesian eccentricity
vector and vis-viva, points of the target orbit, periodic multilinear
functions, the exact polar step of theta, the local error of the Heun step,
and the discounted operator's contraction."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle.core import KIND_FREE, Oracle
from paper_2407_14675_amd import inputs

MU = inputs.EX1_MU


def small(n=(9, 6, 6, 8), **kw):
    return inputs.crown_problem(n, **kw)


def cartesian_elements(x):
    """Semi-major axis (vis-viva) and eccentricity vector from the Cartesian
    position and velocity of the polar state (r, v_r, v_t, theta)."""
    r, vr, vt, th = x
    c, s = math.cos(th), math.sin(th)
    R = np.array([r * c, r * s])
    V = np.array([vr * c - vt * s, vr * s + vt * c])
    v2 = V @ V
    a = 1.0 / (2.0 / r - v2 / MU)
    e = ((v2 - MU / r) * R - (R @ V) * V) / MU
    return a, e


def test_elements_match_the_cartesian_eccentricity_vector():
    o = Oracle(small())
    rng = np.random.default_rng(91)
    for x in inputs.random_states(inputs.EX1, 300, seed=92):
        x = x.copy()
        x[3] = rng.uniform(-4, 10)  # any angle, also outside [0, 2 pi)
        a, e, = cartesian_elements(x)
        el = o.elements(x)
        assert el[0] == pytest.approx(a, rel=1e-10)
        np.testing.assert_allclose(el[1:], e, atol=1e-11, rtol=0)


def test_running_cost_vanishes_on_the_target_orbit():
    """Every point of the target ellipse (a = 7000 km, e = 0.001, perigee at
    theta = 0), periapsis and apoapsis included, has zero element cost; the
    fuel term is alpha * u_bar under thrust."""
    p = small()
    o = Oracle(p)
    a, e, w = p["el_a"], p["el_e"], p["el_omega"]
    pp = a * (1 - e * e)
    for nu in np.linspace(-math.pi, math.pi, 37):
        r = pp / (1 + e * math.cos(nu))
        x = [r, math.sqrt(MU / pp) * e * math.sin(nu), math.sqrt(MU / pp) * (1 + e * math.cos(nu)), w + nu]
        assert o.running_cost(x, 0) == pytest.approx(0.0, abs=1e-12)
        assert o.running_cost(x, 1) == pytest.approx(p["w_fuel"], rel=1e-9, abs=1e-20)
    # the two readings of the fuel weight's units: alpha times the thrust
    # acceleration (5e-7 km/s^2), or alpha per second of thrust
    q = small(fuel_reading="throttle")
    assert p["w_fuel"] == pytest.approx(2.04e-8 * 5e-7, rel=1e-12)
    assert q["w_fuel"] == pytest.approx(2.04e-8, rel=1e-12)
    assert Oracle(q).running_cost(x, 1) - Oracle(q).running_cost(x, 0) == pytest.approx(2.04e-8, rel=1e-9)
    with pytest.raises(ValueError):
        small(fuel_reading="kg")
    # a circular orbit 22 km below: cost beta*22^2 + gamma*e_bar^2
    r = 6978.0
    want = p["el_beta"] * (r - a) ** 2 + p["el_gamma"] * e * e
    assert o.running_cost([r, 0.0, math.sqrt(MU / r), 1.0], 0) == pytest.approx(want, rel=1e-9)


def test_periodic_interpolation():
    """Along theta the interpolant wraps: between the last node and node 0 it
    is the linear blend of those two nodes' values, and shifting the foot by
    n cells leaves it unchanged; the other axes keep the closed-box rule."""
    p = small((5, 4, 4, 6))
    o = Oracle(p)
    n = p["n"]
    rng = np.random.default_rng(93)
    g = rng.uniform(0, 10, size=n[3])
    lin = rng.uniform(-1, 1, size=3)
    i = [np.arange(n[k]) for k in range(3)]
    L = lin[0] * i[0][None, None, :] + lin[1] * i[1][None, :, None] + lin[2] * i[2][:, None, None]
    V = g[:, None, None, None] * (1.0 + 0.1 * L[None])
    for _ in range(200):
        s = [rng.uniform(0, n[0] - 1), rng.uniform(0, n[1] - 1), rng.uniform(0, n[2] - 1),
             rng.uniform(-2 * n[3], 3 * n[3])]
        w = s[3] % n[3]
        b = int(math.floor(w))
        t = w - b
        gb = (1 - t) * g[b] + t * g[(b + 1) % n[3]]
        want = gb * (1.0 + 0.1 * (lin[0] * s[0] + lin[1] * s[1] + lin[2] * s[2]))
        assert o.interp(V, s) == pytest.approx(want, rel=1e-12, abs=1e-12)
        assert o.interp(V, [s[0], s[1], s[2], s[3] + n[3]]) == pytest.approx(want, rel=1e-12, abs=1e-12)
    assert o.interp(V, [n[0] - 1 + 1e-9, 0, 0, 0]) == p["M"]


def test_theta_moves_by_the_angular_rate_and_the_heun_step_is_third_order():
    """Euler moves theta by dt*v_t/r exactly; one Heun step of the polar
    system differs from an accurate integration by O(dt^3)."""
    p = small(integrator="euler")
    o = Oracle(p)
    for x in inputs.random_states(inputs.EX1, 20, seed=94):
        z = o.step(x, 1, 0.4)
        assert z[3] == pytest.approx(x[3] + p["dt"] * x[2] / x[0], rel=1e-15, abs=1e-15)
    q = dict(small(integrator="heun"), accel=2e-3)
    oh = Oracle(q)
    rng = np.random.default_rng(95)
    ratios = []
    for x in inputs.random_states(inputs.EX1, 20, seed=96):
        u = rng.uniform(-math.pi, math.pi)

        def f(_t, y):
            r, vr, vt, th = y
            return [vr, vt * vt / r - MU / (r * r) + q["accel"] * math.sin(u),
                    -vr * vt / r + q["accel"] * math.cos(u), vt / r]

        errs = []
        for tau in (200.0, 100.0):
            ref = solve_ivp(f, (0, tau), list(x), method="DOP853", rtol=1e-13, atol=1e-12).y[:, -1]
            errs.append(np.linalg.norm((oh.step(x, 1, u, tau=tau) - ref) / np.array([1, 1e-3, 1e-3, 1e-3])))
        ratios.append(errs[0] / errs[1])
    assert 7.5 < min(ratios) and max(ratios) < 8.5, ratios


def test_discounted_operator_is_a_monotone_contraction():
    """With lambda > 0 the Bellman operator contracts sup-norm distances by
    exp(-lambda dt) and preserves order."""
    p = small()
    o = Oracle(p)
    free = o.kind == KIND_FREE
    assert free.all()  # no target set and no mask
    rng = np.random.default_rng(97)
    V = rng.uniform(0, 1e4, size=o.shape)
    W = V + rng.uniform(0, 50, size=o.shape)
    TV, _, _, _ = o.bellman_sweep(V)
    TW, _, _, _ = o.bellman_sweep(W)
    assert np.all(TW >= TV - 1e-9)
    gamma = math.exp(-p["lam"] * p["dt"])
    assert np.max(np.abs(TW - TV)) <= gamma * np.max(np.abs(W - V)) * (1 + 1e-12)


def test_velocity_faces_clamp_and_circular_faces_exit():
    """The crown problem's state constraint (Section 3, the polar grid): the
    exit value M applies on the two circular faces rho = rho_min, rho_max
    only; a foot beyond a velocity face (v_rho or v_theta) is put onto that
    face.  Checked on the whole Q of every node of a small grid for several
    controls, with everything recomputed here: the Euler foot of the polar
    system in physical units, mapped to grid coordinates and clamped by hand,
    and a value field whose Q1 interpolant is known in closed form (a
    periodic blend along theta times an affine function of the other three
    grid coordinates).  Zero element weights make the running cost vanish, so
    Q = exp(-lambda dt) * I[V](foot)."""
    p = dict(small((9, 6, 5, 8), integrator="euler"), el_beta=0.0, el_gamma=0.0, w_fuel=0.0)
    # a thrust strong enough to carry feet across both velocity faces
    p["accel"] = 4e-3
    o = Oracle(p)
    n = p["n"]
    lo, hi = p["lo"], p["hi"]
    h = [(hi[k] - lo[k]) / (n[k] - 1) for k in range(3)] + [2 * math.pi / n[3]]
    rng = np.random.default_rng(98)
    g = rng.uniform(1, 10, size=n[3])
    c = rng.uniform(-1, 1, size=3)
    i0, i1, i2 = np.arange(n[0]), np.arange(n[1]), np.arange(n[2])
    aff = 1.0 + 0.1 * (c[0] * i0[None, None, :] + c[1] * i1[None, :, None] + c[2] * i2[:, None, None])
    V = g[:, None, None, None] * aff[None]
    gamma = math.exp(-p["lam"] * p["dt"])

    def expected(x, thr, u):
        r, vr, vt, th = x
        acc = p["accel"] if thr else 0.0
        b = [vr, vt * vt / r - MU / (r * r) + acc * math.sin(u), -vr * vt / r + acc * math.cos(u), vt / r]
        s = [(x[k] + p["dt"] * b[k] - lo[k]) / h[k] for k in range(4)]
        if s[0] < 0 or s[0] > n[0] - 1:
            return gamma * p["M"], "rho"  # I = M outside, discounted like any foot value
        face = None
        for k in (1, 2):
            if s[k] < 0 or s[k] > n[k] - 1:
                face = "v"
                s[k] = min(max(s[k], 0.0), n[k] - 1.0)
        w = s[3] % n[3]
        b3 = int(math.floor(w))
        t3 = w - b3
        gb = (1 - t3) * g[b3] + t3 * g[(b3 + 1) % n[3]]
        return gamma * gb * (1.0 + 0.1 * (c[0] * s[0] + c[1] * s[1] + c[2] * s[2])), face

    seen = {"rho": 0, "v": 0, None: 0}
    for j in range(o.N):
        x = o.node_coords(j)
        for thr, u in ((0, 0.0), (1, math.pi / 2), (1, -math.pi / 2), (1, 0.0), (1, math.pi),
                       (1, rng.uniform(-math.pi, math.pi))):
            want, why = expected(x, thr, u)
            seen[why] += 1
            got = o.q(V, j, thr, u)
            assert got == pytest.approx(want, rel=1e-12, abs=1e-12), (j, thr, u, why)
    # the grid and controls reach every case: interior feet, velocity faces, circular faces
    assert min(seen.values()) > 20, seen

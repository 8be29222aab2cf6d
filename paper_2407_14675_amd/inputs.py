"""Workload definitions and seeded input generators.

This module is shared by the device path and by the CPU oracle, so it holds
numbers and random draws only: grid extents, physical constants, search sizes
and seeded fields.  It contains none of the method's arithmetic (no dynamics,
no interpolation, no target snapping, no Bellman operator).

The benchmark workloads are the nondimensional planar orbit-transfer
problem (mu = 1, r0 = 1) in the state (r, v_r, v_t, m).  The paper's own
Example 1 (Section 4) is the crown problem below, in kilometres and seconds,
state (rho, v_rho, v_theta, theta) with theta periodic.
"""
from __future__ import annotations

import copy
import math

import numpy as np

INF = float("inf")

# Axis order of every state tuple and of every grid: (r, v_r, v_t, m).
AXES = ("r", "v_r", "v_t", "m")

# Domain of the orbit-transfer workloads.
ORBIT_LO = (0.98, -0.05, 0.93, 0.90)
ORBIT_HI = (1.08, 0.05, 1.02, 1.00)

# Target box half-widths in (r, v_r, v_t); mass is unconstrained.
TARGET_HALF_WIDTH = (0.005, 0.003, 0.003, INF)

# Read-out point: circular orbit at r0 = 1 with full mass.
X0 = (1.0, 0.0, 1.0, 1.0)


def orbit_problem(n, *, target_radius=1.05, accel=1e-3, mdot=1e-3, dt=0.05,
                  w_fuel=0.0, M=1e3, lam=0.0, search=None, name="orbit"):
    """Planar orbit-transfer problem on a closed uniform grid with n[k] nodes per axis."""
    if search is None:
        search = dict(mode="table", n_angles=16)
    return dict(
        name=name,
        model="orbit",
        n=tuple(int(v) for v in n),
        lo=ORBIT_LO,
        hi=ORBIT_HI,
        mu=1.0,
        accel=float(accel),
        mdot=float(mdot),
        dt=float(dt),
        lam=float(lam),
        w_time=1.0,
        w_fuel=float(w_fuel),
        M=float(M),
        speed=0.0,
        tgt_c=(float(target_radius), 0.0, float(target_radius) ** -0.5, 0.0),
        tgt_w=TARGET_HALF_WIDTH,
        search=dict(search),
    )


def eikonal_problem(n_side=17, *, half=1.0, speed=1.0, n_angles=16, M=1e3, lam=0.0):
    """2-D minimum-time problem x' = speed*(sin u, cos u) embedded in axes (v_r, v_t).

    Axes r and m are dummy axes with two nodes and no motion.  With
    dt*speed equal to the grid step, moves along the axes land on nodes.
    """
    h = 2.0 * half / (n_side - 1)
    return dict(
        name=f"eikonal_{n_side}",
        model="eikonal",
        n=(2, n_side, n_side, 2),
        lo=(0.0, -half, -half, 0.0),
        hi=(1.0, half, half, 1.0),
        mu=0.0,
        accel=0.0,
        mdot=0.0,
        dt=h / speed,
        lam=float(lam),
        w_time=1.0,
        w_fuel=0.0,
        M=float(M),
        speed=float(speed),
        tgt_c=(0.0, 0.0, 0.0, 0.0),
        tgt_w=(INF, 0.0, 0.0, INF),
        search=dict(mode="table", n_angles=n_angles),
    )


SCAN_GOLDEN = dict(mode="scan_golden", n_scan=64, n_golden=12)

# Plain value iteration, discrete table of 16 angles plus coast, 12^4 grid.
VI12 = orbit_problem((12, 12, 12, 12), name="vi_12^4")
VI12_TOL_ABS = 1e-8

# Modified policy iteration on 48^4 with the reachability-masked active set.
PI48 = orbit_problem((48, 48, 48, 48), search=SCAN_GOLDEN, name="pi_48^4_masked")
EVAL_SWEEPS = 20
# Reduced grid of the 48^4 workload: a fine node is active where the 12^4
# value, interpolated at the node, is below MASK_THRESHOLD_FRAC * M (the
# target is reached with positive weight), dilated by MASK_DILATE cells.
MASK_THRESHOLD_FRAC = 0.98
MASK_DILATE = (1, 1, 1, 1)

# Large single problem, 96 x 96 x 96 x 64, dt = 0.02, cost 1 + 0.1*throttle.
def large_problem(accel=1e-3, n=(96, 96, 96, 64)):
    return orbit_problem(n, accel=accel, dt=0.02, w_fuel=0.1, search=SCAN_GOLDEN,
                         name=f"orbit_{'x'.join(map(str, n))}_a{accel:g}")


def batch_draws(n_prob=16, seed=3):
    """Sixteen transfer problems: target radius, thrust level and grid side.

    Problem 0 is forced to the smallest side (24) and the last to the largest (64).
    """
    rng = np.random.default_rng(seed)
    radius = rng.uniform(1.02, 1.08, size=n_prob)
    accel = rng.uniform(3e-4, 2e-3, size=n_prob)
    side = rng.integers(24, 65, size=n_prob)
    side[0] = 24
    side[-1] = 64
    return [dict(target_radius=float(radius[i]), accel=float(accel[i]), side=int(side[i]))
            for i in range(n_prob)]


def batch_problems(n_prob=16, seed=3, side_scale=1.0):
    out = []
    for i, d in enumerate(batch_draws(n_prob, seed)):
        side = max(4, int(round(d["side"] * side_scale)))
        out.append(orbit_problem((side,) * 4, target_radius=d["target_radius"],
                                 accel=d["accel"], name=f"batch_p{i}_{side}^4"))
    return out


# ---------------------------------------------------------------- Example 1
# The paper's Example 1 (Section 4): target orbit a = 7000 km, e = 0.001,
# argument of perigee 0; thrust acceleration 5e-7 km/s^2 (no mass change);
# cost weights alpha = 2.04e-8 (on the thrust acceleration), beta = 2.31e-2,
# gamma = 1.5; discount 1e-3 1/s; dt = 10 s; 73 controls (72 angles at 5
# degrees and coast); rho in [6930, 7070] km, theta in [0, 2 pi), v_rho in
# [-0.01, 0.01] km/s, v_theta in [7.526, 7.566] km/s on 110 x 30 x 30 x 30
# nodes.  Axes here: (rho, v_rho, v_theta, theta), theta periodic (axis 3).
# M, the value of a foot beyond the circular faces rho = 6930 and 7070 km
# (the state constraint; feet beyond a velocity face are put on it), is 1e6:
# above the largest running cost on the domain (~750) divided by the
# discount rate.
EX1_MU = 398600.4
EX1_ACCEL = 5e-7
EX1_ALPHA = 2.04e-8


def crown_problem(n=(110, 30, 30, 30), *, integrator="heun", n_angles=72, M=1e6, name="example1_crown",
                  fuel_reading="accel"):
    """The paper's Example 1.  fuel_reading: how the fuel term alpha*u_bar of
    the running cost is read, the units of the weights not being stated:
    "accel" takes u_bar as the thrust acceleration in km/s^2 (alpha*u_bar =
    1.02e-14 per second of thrust), "throttle" takes u_bar as 1 while the
    thruster fires (alpha = 2.04e-8 per second of thrust)."""
    if fuel_reading not in ("accel", "throttle"):
        raise ValueError(fuel_reading)
    return dict(
        name=name,
        model="crown",
        n=tuple(int(v) for v in n),
        lo=(6930.0, -0.01, 7.526, 0.0),
        hi=(7070.0, 0.01, 7.566, 2.0 * math.pi),
        mu=EX1_MU,
        accel=EX1_ACCEL,
        mdot=0.0,
        dt=10.0,
        lam=1e-3,
        w_time=0.0,
        w_fuel=EX1_ALPHA * (EX1_ACCEL if fuel_reading == "accel" else 1.0),
        M=float(M),
        speed=0.0,
        tgt_c=(0.0, 0.0, 0.0, 0.0),
        tgt_w=(-1.0, -1.0, -1.0, -1.0),  # no target set: the cost steers towards the orbit
        integrator=integrator,
        el_beta=2.31e-2,
        el_gamma=1.5,
        el_a=7000.0,
        el_e=0.001,
        el_omega=0.0,
        search=dict(mode="table", n_angles=int(n_angles)),
    )


EX1 = crown_problem()
# Start of the paper's closed-loop orbit raise: circular orbit at 6978 km.
EX1_START_RADIUS = 6978.0

# Example 2's drag on the simulated system (Section 4): acceleration
# C |v|^2 against the velocity with C = C_D S rho_D / (2 m); C_D = 2.2,
# S = 2.25 m^2, rho_D = 8.09e-14 kg/m^3, m = 350 kg give C in 1/m, times 1000
# for the crown grid's km (a = C v^2 with v in km/s then comes out in km/s^2).
EX2_DRAG = 2.2 * 2.25 * 8.09e-14 / (2.0 * 350.0) * 1000.0


def with_grid(problem, n):
    """Same physics on another grid."""
    p = copy.deepcopy(problem)
    p["n"] = tuple(int(v) for v in n)
    p["name"] = problem["name"] + "@" + "x".join(map(str, n))
    return p


def n_nodes(problem):
    n = problem["n"]
    return int(n[0]) * int(n[1]) * int(n[2]) * int(n[3])


# ---------------------------------------------------------------- random draws
def random_value(problem, seed, low=0.0, high=50.0, frac_M=0.0):
    """Random value field in C order [m][v_t][v_r][r] (float64)."""
    rng = np.random.default_rng(seed)
    n = problem["n"]
    V = rng.uniform(low, high, size=(n[3], n[2], n[1], n[0]))
    if frac_M > 0:
        V[rng.random(V.shape) < frac_M] = problem["M"]
    return V


def random_states(problem, count, seed, margin=0.0):
    """Uniform random states inside the domain box (count x 4, float64)."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(problem["lo"], dtype=np.float64)
    hi = np.asarray(problem["hi"], dtype=np.float64)
    span = hi - lo
    return lo + margin * span + rng.random((count, 4)) * span * (1.0 - 2.0 * margin)


def random_multilinear_coeffs(seed=11):
    """Sixteen coefficients, one per subset S of the four axes (bit k = axis k)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=16)


def random_nodes(problem, count, seed):
    """Distinct random flat node indices."""
    rng = np.random.default_rng(seed)
    total = n_nodes(problem)
    count = min(count, total)
    return np.sort(rng.choice(total, size=count, replace=False)).astype(np.int64)


def mlp_init(seed=4, widths=(4, 128, 128, 3)):
    """Initial MLP parameters (uniform fan-in init), float64, as a list of (W, b)."""
    rng = np.random.default_rng(seed)
    params = []
    for fan_in, fan_out in zip(widths[:-1], widths[1:]):
        bound = 1.0 / math.sqrt(fan_in)
        W = rng.uniform(-bound, bound, size=(fan_out, fan_in))
        b = rng.uniform(-bound, bound, size=(fan_out,))
        params.append((W, b))
    return params


def mlp_params32(seed=4):
    """mlp_init flattened in the library's parameter order (W1, b1, W2, b2,
    W3, b3), float32."""
    return np.concatenate([a.reshape(-1) for W, b in mlp_init(seed) for a in (W, b)]).astype(np.float32)


# Learned control proposal: training pairs come from the converged solution
# at nodes whose value is not the exit penalty (V < 0.98 M, the mask's
# threshold; on these grids the numerical diffusion of the penalty leaves
# almost no value below M/2), sampled without replacement in random order,
# seed 4; batch 16384 (one 64-sample tile per CU), 10 epochs, Adam with step
# size 2e-3, each epoch in its own random order of batch-sized windows of the
# shuffled pairs.
MLP_PAIRS = 2_000_000
MLP_BATCH = 16384
MLP_EPOCHS = 10
MLP_LR = 2e-3
MLP_SEED = 4
MLP_FEASIBLE_FRAC = 0.98

# Seeded greedy step: 8 thrust evaluations on [seed - w, seed + w], full
# scan + golden search where the result moves the node's value by more than
# 1e-5 relative.
SEEDED = dict(mode="seeded", n_scan=64, n_golden=12, n_local=8, local_half_width=0.1, fallback_tol=1e-5)


def mlp_pair_selection(n_feasible, n_pairs=MLP_PAIRS, seed=MLP_SEED):
    """Indices of the training pairs among the feasible nodes, in random
    order (int32)."""
    rng = np.random.default_rng(seed)
    k = min(int(n_pairs), int(n_feasible))
    return rng.choice(int(n_feasible), size=k, replace=False).astype(np.int32)


def mlp_epoch_orders(n, epochs=MLP_EPOCHS, seed=MLP_SEED, batch=MLP_BATCH):
    """The sample order of each epoch (int32, a permutation of range(n)),
    drawn lazily: the pairs, already in random order, cut into windows of
    `batch` consecutive samples starting at a random offset (cyclically), and
    the windows taken in random order.  Drawing one takes a few milliseconds
    for 2M pairs (a full random permutation of 2M takes tens), so the next
    epoch's order is ready while the device trains on the current one."""
    rng = np.random.default_rng(seed + 1000)
    n = int(n)
    nb = (n + batch - 1) // batch
    within = np.arange(batch, dtype=np.int32)
    for _ in range(epochs):
        shift = int(rng.integers(n))
        idx = (rng.permutation(nb).astype(np.int32)[:, None] * np.int32(batch) + within[None, :]).reshape(-1)
        if n % batch:
            idx = idx[idx < n]
        idx += np.int32(shift)
        np.subtract(idx, np.int32(n), out=idx, where=idx >= n)
        yield idx


def mlp_random_samples(n, seed, thrust_frac=0.6):
    """Synthetic network samples: inputs uniform in [-1, 1]^4; targets
    (cos u, sin u, throttle, 0) with u uniform and throttle Bernoulli."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, size=(n, 4))
    u = rng.uniform(-math.pi, math.pi, size=n)
    t = (rng.random(n) < thrust_frac).astype(np.float64)
    tgt = np.stack([np.cos(u), np.sin(u), t, np.zeros(n)], axis=1)
    return x.astype(np.float32), tgt.astype(np.float32)

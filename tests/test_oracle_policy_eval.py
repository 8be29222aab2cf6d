"""Pins of the oracle's exact policy evaluation (eq:p_eval as the sparse
linear system of Section 3, solved by a direct factorisation): it equals the
limit of repeated frozen-policy sweeps, a separate code path (the sweep
interpolates, the system is assembled from the corner weights), and on the
eikonal problem it reproduces the closed form |x|/s under the optimal
policy."""
import math

import numpy as np
import pytest

from oracle.core import KIND_FREE, Oracle
from paper_2407_14675_amd import inputs


def test_exact_evaluation_is_the_limit_of_frozen_policy_sweeps():
    p = inputs.crown_problem((8, 6, 6, 8))
    o = Oracle(p)
    rng = np.random.default_rng(131)
    ang = rng.uniform(-math.pi, math.pi, size=o.shape)
    thr = rng.integers(0, 2, size=o.shape).astype(np.uint8)
    V0 = o.init_value()
    v = o.policy_evaluate_exact(V0, ang, thr)
    W = V0.copy()
    for _ in range(6000):  # contraction exp(-lambda dt) = 0.990 per sweep
        W = o.policy_eval_sweep(W, ang, thr)
    np.testing.assert_allclose(v, W, rtol=1e-9, atol=1e-6)
    # the evaluated policy's value is a fixed point of its own sweep
    np.testing.assert_allclose(o.policy_eval_sweep(v, ang, thr), v, rtol=1e-11, atol=1e-8)


def test_exact_evaluation_of_the_optimal_eikonal_policy():
    """Minimum time to the origin: evaluating the converged policy gives the
    converged value (i h / s on the axes); the target's nodes stay 0."""
    p = inputs.eikonal_problem(17)
    o = Oracle(p)
    res = o.solve_vi(tol_abs=1e-13, max_sweeps=2000)
    v = o.policy_evaluate_exact(o.init_value(), res["angle"], res["thr"])
    free = o.kind == KIND_FREE
    np.testing.assert_allclose(v[free], res["V"][free], rtol=0, atol=1e-10)
    h = 2.0 / 16
    for i in range(-8, 9):
        assert v[0, 8 + i, 8, 0] == pytest.approx(abs(i) * h / p["speed"], abs=1e-10)

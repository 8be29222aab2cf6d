"""Pins of the FP64 network reference: closed forms and finite differences."""
import math

import numpy as np

from oracle import mlp
from paper_2407_14675_amd import inputs


def test_gelu_closed_forms():
    """GELU(z) = z*Phi(z): 0 at 0, z for large z, 0 for very negative z;
    derivative Phi(z) + z*phi(z) is 1/2 at 0."""
    z = np.array([0.0, 8.0, -8.0, 1.0])
    g = mlp.gelu(z)
    assert g[0] == 0.0 and abs(g[1] - 8.0) < 1e-12 and abs(g[2]) < 1e-12
    assert abs(g[3] - 0.8413447460685429) < 1e-12  # Phi(1) = 0.841344746...
    assert abs(mlp.gelu_grad(np.array([0.0]))[0] - 0.5) < 1e-15
    h = 1e-6
    for zz in (-2.3, -0.4, 0.7, 3.1):
        fd = (mlp.gelu(np.array([zz + h])) - mlp.gelu(np.array([zz - h])))[0] / (2 * h)
        assert abs(fd - mlp.gelu_grad(np.array([zz]))[0]) < 1e-8


def test_parameter_count():
    assert mlp.N_PARAMS == 17539  # 4*128+128 + 128*128+128 + 3*128+3


def test_loss_special_cases():
    """Coasting targets (thr = 0) contribute the BCE term only; BCE(0, t) = log 2."""
    y = np.array([[0.3, -0.2, 0.0], [0.9, 0.1, 0.0]])
    t = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    assert abs(mlp.loss(y, t) - math.log(2.0)) < 1e-15
    t2 = np.array([[0.3, -0.2, 1.0], [0.9, 0.1, 1.0]])
    assert abs(mlp.loss(y, t2) - math.log(2.0)) < 1e-15


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(7)
    theta = mlp.from_init(inputs.mlp_init(seed=4))
    x = rng.uniform(-1, 1, size=(6, 4))
    ang = rng.uniform(-math.pi, math.pi, size=6)
    t = np.stack([np.cos(ang), np.sin(ang), (rng.random(6) < 0.6).astype(float)], axis=1)
    L, g = mlp.loss_grad(theta, x, t)
    idx = rng.choice(mlp.N_PARAMS, size=200, replace=False)
    idx = np.concatenate([idx, [0, 511, 512, 639, 640, 16000, 16767, 16768, 17151, 17152, 17535, 17538]])
    h = 1e-6
    for k in idx:
        e = np.zeros_like(theta)
        e[k] = h
        fd = (mlp.loss(mlp.forward(theta + e, x)[0], t) - mlp.loss(mlp.forward(theta - e, x)[0], t)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_adam_first_step_is_sign_step():
    """With zero moments, the first bias-corrected Adam step moves each
    parameter by lr * g / (|g| + eps), i.e. about lr against the gradient."""
    theta = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, 1e-3, -1e-4])
    new, m, v = mlp.adam_step(theta, g, np.zeros(5), np.zeros(5), 1, lr=1e-3)
    np.testing.assert_allclose(new, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_bf16_rounding_ties_to_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9])
    r = mlp.bf16(x)
    np.testing.assert_array_equal(r, [1.0, 1.0, 1.0 + 2 ** -6, 1.0])

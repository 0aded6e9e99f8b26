"""Pins of the FP64 warm-start reference (oracle/mlp_ref.py): finite differences,
a least-squares closed form, GELU special values and the first AdamW step."""
import math

import numpy as np

from oracle import mlp_ref as M
from paper_2403_04578_amd import workloads as W


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    sizes = [6, 5, 5, 4]
    p = rng.normal(0, 0.7, M.num_params(sizes))
    x = rng.normal(0, 1, (7, 6))
    t = rng.normal(0, 1, (7, 4))
    _, g = M.loss_and_grad(p, sizes, x, t)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (M.loss_and_grad(p + e, sizes, x, t)[0] - M.loss_and_grad(p - e, sizes, x, t)[0]) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())


def test_linear_model_gradient_vanishes_at_least_squares():
    rng = np.random.default_rng(1)
    sizes = [5, 3]  # no hidden layer: y = x W^T + b
    x = rng.normal(0, 1, (40, 5))
    t = rng.normal(0, 1, (40, 3))
    X1 = np.concatenate([x, np.ones((40, 1))], axis=1)
    sol, *_ = np.linalg.lstsq(X1, t, rcond=None)
    p = np.concatenate([sol[:5].T.ravel(), sol[5]])
    loss, g = M.loss_and_grad(p, sizes, x, t)
    assert np.abs(g).max() < 1e-12
    assert abs(loss - np.mean((X1 @ sol - t) ** 2)) < 1e-14


def test_gelu_special_values():
    assert M.gelu(np.array(0.0)) == 0.0
    assert abs(M.gelu_grad(np.array(0.0)) - 0.5) < 1e-15
    assert abs(M.gelu(np.array(10.0)) - 10.0) < 1e-12
    assert abs(M.gelu(np.array(-10.0))) < 1e-12
    z = np.linspace(-4, 4, 81)
    fd = (M.gelu(z + 1e-6) - M.gelu(z - 1e-6)) / 2e-6
    assert np.abs(fd - M.gelu_grad(z)).max() < 1e-8
    # Phi(1) = 0.841344746...
    assert abs(M.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15


def test_first_adamw_step_is_sign_step():
    rng = np.random.default_rng(2)
    p = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = M.adamw_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3, wd=0.0)
    assert np.allclose(p1 - p, -1e-3 * g / (np.abs(g) + 1e-8), atol=1e-15)
    p2, _, _ = M.adamw_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-3, wd=0.1)
    assert np.allclose(p2 - p1, -1e-3 * 0.1 * p, atol=1e-15)


def test_features_and_targets_layout():
    S = np.array([[0.01 + 0.002j, 0.02 + 0.004j]])
    x = M.features(S, np.array([360]))
    assert np.allclose(x[0, :4], [0.5, 1.0, 0.1, 0.2])
    assert np.allclose(x[0, 4:], [1.0, 0.0, 0.0, 1.0], atol=1e-15)  # 6 h: quarter day; day 0
    x2 = M.features(S, np.array([1440 * 365 + 720]))
    assert np.allclose(x2[0, 4:], [0.0, -1.0, 0.0, 1.0], atol=1e-12)  # noon, day 365 == day 0
    V = np.array([[0.98 - 0.01j, 0.97 - 0.02j]])
    y = M.targets(V)
    assert np.allclose(y, [[-0.4, -0.6, -0.2, -0.4]])
    assert np.allclose(M.to_voltage(y), V)


def test_parameter_count_of_the_warm_start_network():
    sizes = W.mlp_sizes(99)
    assert sizes == [202, 256, 256, 256, 198]
    assert M.num_params(sizes) == 234_438
    p = W.mlp_init_params(sizes)
    assert p.dtype == np.float32 and p.size == 234_438

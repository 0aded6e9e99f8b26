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


def test_adamw_constant_gradient_gives_unit_steps():
    """With a constant gradient and no weight decay the bias-corrected moments are
    exactly g and g^2 at every step (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so
    every step moves each parameter by -lr g / (|g| + eps).  Dropping the moment
    memory or using a wrong bias-correction exponent breaks this from step 2 on."""
    rng = np.random.default_rng(3)
    p0 = rng.normal(size=40)
    g = rng.normal(size=40) * np.logspace(-3, 1, 40)
    p, m, v = p0.copy(), np.zeros(40), np.zeros(40)
    for t in range(1, 8):
        p, m, v = M.adamw_step(p, g, m, v, t, lr=1e-3, wd=0.0)
        assert np.allclose(m, (1 - 0.9 ** t) * g, rtol=1e-14, atol=0)
        assert np.allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-13, atol=0)
        assert np.allclose(p - p0, -t * 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-16)


def test_adamw_three_varying_steps_written_out():
    """Three steps with different gradients, the moments expanded by hand:
    m_3 = 0.081 g1 + 0.09 g2 + 0.1 g3, v_3 = 0.000998001 g1^2 + 0.000999 g2^2 + 0.001 g3^2,
    each step's update -lr (m_t/(1-0.9^t)) / (sqrt(v_t/(1-0.999^t)) + eps) - lr wd p_{t-1}."""
    g1, g2, g3 = 0.5, -2.0, 0.25
    p0, lr, wd, eps = 1.5, 1e-2, 0.1, 1e-8
    p = np.array([p0])
    m = v = np.zeros(1)
    out = []
    for t, gg in enumerate((g1, g2, g3), start=1):
        p, m, v = M.adamw_step(p, np.array([gg]), m, v, t, lr=lr, wd=wd)
        out.append((float(p[0]), float(m[0]), float(v[0])))
    m1, v1 = 0.1 * g1, 0.001 * g1 ** 2
    m2, v2 = 0.09 * g1 + 0.1 * g2, 0.000999 * g1 ** 2 + 0.001 * g2 ** 2
    m3 = 0.081 * g1 + 0.09 * g2 + 0.1 * g3
    v3 = 0.000998001 * g1 ** 2 + 0.000999 * g2 ** 2 + 0.001 * g3 ** 2
    q = p0
    for (pm, mm, vm), (mt, vt, t) in zip(out, ((m1, v1, 1), (m2, v2, 2), (m3, v3, 3))):
        assert abs(mm - mt) < 1e-15 and abs(vm - vt) < 1e-17
        q = q - lr * ((mt / (1 - 0.9 ** t)) / (math.sqrt(vt / (1 - 0.999 ** t)) + eps) + wd * q)
        assert abs(pm - q) < 1e-14, (t, pm, q)


def test_adamw_is_invariant_to_gradient_scale():
    """Adam's update is homogeneous of degree zero in g (up to eps): scaling every
    gradient of a run by 1000 leaves the trajectory unchanged."""
    rng = np.random.default_rng(4)
    p0 = rng.normal(size=30)
    gs = rng.normal(size=(5, 30))
    runs = []
    for c in (1.0, 1000.0):
        p, m, v = p0.copy(), np.zeros(30), np.zeros(30)
        for t in range(5):
            p, m, v = M.adamw_step(p, c * gs[t], m, v, t + 1, lr=1e-3, wd=0.01, eps=0.0)
        runs.append(p)
    assert np.allclose(runs[0], runs[1], rtol=0, atol=1e-15)

"""Pins of the FP64 MLP cost-model reference: finite differences, closed forms, Adam's first step."""
import numpy as np

import workloads
from oracle import mlp


def _params(seed=0, f=12, h=64):
    return {k: v.astype(np.float64) for k, v in workloads.mlp_init(seed, f, h).items()}


def test_gradients_match_central_differences():
    g = np.random.default_rng(0)
    p = _params(1, f=5, h=7)
    x = g.standard_normal((9, 5))
    t = g.standard_normal(9)
    y, cache = mlp.forward(p, x)
    grads = mlp.backward(p, cache, y, t)
    for name in mlp.NAMES:
        num = np.zeros_like(p[name])
        it = np.nditer(p[name], flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            h = 1e-6 * max(1.0, abs(p[name][idx]))
            pp = {k: v.copy() for k, v in p.items()}
            pm = {k: v.copy() for k, v in p.items()}
            pp[name][idx] += h
            pm[name][idx] -= h
            num[idx] = (mlp.loss(mlp.forward(pp, x)[0], t) - mlp.loss(mlp.forward(pm, x)[0], t)) / (2 * h)
        err = np.linalg.norm(num - grads[name]) / max(1e-12, np.linalg.norm(num))
        assert err < 1e-6, (name, err)


def test_zero_network_outputs_bias_and_blocks_gradients():
    p = {k: np.zeros_like(v) for k, v in _params(2, f=4, h=6).items()}
    p["b3"] = np.array([0.75])
    x = np.random.default_rng(1).standard_normal((5, 4))
    t = np.arange(5.0)
    y, cache = mlp.forward(p, x)
    np.testing.assert_array_equal(y, np.full(5, 0.75))
    gr = mlp.backward(p, cache, y, t)
    for k in ("W1", "b1", "W2", "b2", "W3"):
        assert not gr[k].any(), k
    np.testing.assert_allclose(gr["b3"], [np.mean(2 * (0.75 - t))])


def test_one_unit_network_closed_form_gradient():
    # f = 1, hidden = 1, all pre-activations positive: y = w3 (w2 (w1 x + b1) + b2) + b3,
    # L = (y - t)^2 for one sample, dL/dw1 = 2 (y - t) w3 w2 x.
    p = {"W1": np.array([[0.5]]), "b1": np.array([0.25]), "W2": np.array([[2.0]]),
         "b2": np.array([0.5]), "W3": np.array([[3.0]]), "b3": np.array([-1.0])}
    x, t = np.array([[2.0]]), np.array([4.0])
    y, cache = mlp.forward(p, x)
    assert y[0] == 3.0 * (2.0 * (0.5 * 2.0 + 0.25) + 0.5) - 1.0     # 8.5
    gr = mlp.backward(p, cache, y, t)
    r = 2 * (y[0] - t[0])
    assert gr["W1"][0, 0] == r * 3.0 * 2.0 * 2.0
    assert gr["b1"][0] == r * 3.0 * 2.0
    assert gr["W2"][0, 0] == r * 3.0 * 1.25
    assert gr["W3"][0, 0] == r * 3.0
    assert gr["b3"][0] == r


def test_adam_first_step_is_signed_learning_rate():
    p = _params(3, f=3, h=4)
    g = {k: np.random.default_rng(4).standard_normal(v.shape) for k, v in p.items()}
    newp, m, v = mlp.adam_step(p, g, mlp.zeros_like(p), mlp.zeros_like(p), 1, lr=1e-2)
    for k in mlp.NAMES:
        # m_hat = g, v_hat = g^2 at step 1
        np.testing.assert_allclose(newp[k], p[k] - 1e-2 * g[k] / (np.abs(g[k]) + 1e-8),
                                   rtol=1e-12, atol=1e-15)


def test_training_reduces_loss():
    g = np.random.default_rng(5)
    x = g.standard_normal((256, 6))
    t = np.sin(x[:, 0]) + 0.5 * x[:, 1] ** 2
    p = _params(6, f=6, h=32)
    m, v = mlp.zeros_like(p), mlp.zeros_like(p)
    l0 = mlp.loss(mlp.forward(p, x)[0], t)
    for step in range(1, 301):
        y, c = mlp.forward(p, x)
        p, m, v = mlp.adam_step(p, mlp.backward(p, c, y, t), m, v, step, lr=1e-2)
    assert mlp.loss(mlp.forward(p, x)[0], t) < 0.2 * l0


def test_adam_two_steps_closed_form():
    """Two Adam steps on one scalar parameter, worked by hand (Kingma and Ba, 2015, Algorithm 1).
    beta1 = 1/2, beta2 = 3/4, lr = 0.1, eps = 0, gradients g1 = 2 then g2 = 1:
      step 1: m1 = (1/2) 2 = 1, v1 = (1/4) 4 = 1, m^ = 1 / (1 - 1/2) = 2, v^ = 1 / (1 - 3/4) = 4,
              theta1 = theta0 - 0.1 * 2 / 2 = theta0 - 0.1;
      step 2: m2 = (1/2) 1 + (1/2) 1 = 1, v2 = (3/4) 1 + (1/4) 1 = 1,
              m^ = 1 / (1 - 1/4) = 4/3, v^ = 1 / (1 - 9/16) = 16/7,
              theta2 = theta1 - 0.1 * (4/3) / (4 / sqrt 7) = theta1 - 0.1 sqrt(7) / 3.
    A bias correction left at beta^1 on step 2 would give m^ = 2, v^ = 4 and theta2 = theta1 - 0.1;
    moments without their (1 - beta) weights, or v from g instead of g^2, change step 1 already."""
    p0 = {k: np.full(s, 0.5) for k, s in (("W1", (1, 1)), ("b1", (1,)), ("W2", (1, 1)), ("b2", (1,)),
                                          ("W3", (1, 1)), ("b3", (1,)))}
    g1 = {k: np.full_like(v, 2.0) for k, v in p0.items()}
    g2 = {k: np.full_like(v, 1.0) for k, v in p0.items()}
    kw = dict(lr=0.1, beta1=0.5, beta2=0.75, eps=0.0)
    p1, m1, v1 = mlp.adam_step(p0, g1, mlp.zeros_like(p0), mlp.zeros_like(p0), 1, **kw)
    p2, m2, v2 = mlp.adam_step(p1, g2, m1, v1, 2, **kw)
    for k in mlp.NAMES:
        assert m1[k].item() == 1.0 and v1[k].item() == 1.0
        assert p1[k].item() == 0.5 - 0.1
        assert m2[k].item() == 1.0 and v2[k].item() == 1.0
        np.testing.assert_allclose(p2[k].item(), 0.4 - 0.1 * np.sqrt(7.0) / 3.0, rtol=1e-15)
    # default hyper-parameters, equal gradients: both bias-corrected moments equal g and g^2 at
    # every step, so each step moves by lr * g / (|g| + eps)
    q1, a1, b1 = mlp.adam_step(p0, g2, mlp.zeros_like(p0), mlp.zeros_like(p0), 1, lr=1e-3)
    q2, _, _ = mlp.adam_step(q1, g2, a1, b1, 2, lr=1e-3)
    for k in mlp.NAMES:
        np.testing.assert_allclose(q2[k].item(), 0.5 - 2e-3 / (1.0 + 1e-8), rtol=1e-14)

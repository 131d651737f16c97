"""Pins of the FP64 reference MLP: central finite differences and an Adam closed form."""

import numpy as np

from oracle import mlp


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    sizes = [6, 5, 4, 3]
    params = mlp.init_params(sizes, seed=1)
    params = [p + 0.1 * rng.standard_normal(p.shape) for p in params]   # nonzero biases
    x = rng.standard_normal((7, sizes[0]))
    t = rng.standard_normal((7, sizes[-1]))
    _, grads = mlp.loss_and_grads(params, x, t)
    h = 1e-6
    for pi, p in enumerate(params):
        for idx in [tuple(rng.integers(0, s) for s in p.shape) for _ in range(4)]:
            pp = [q.copy() for q in params]
            pm = [q.copy() for q in params]
            pp[pi][idx] += h
            pm[pi][idx] -= h
            fd = (mlp.loss_and_grads(pp, x, t)[0] - mlp.loss_and_grads(pm, x, t)[0]) / (2 * h)
            assert abs(fd - grads[pi][idx]) <= 1e-7 * max(1.0, abs(fd)), (pi, idx)


def test_silu_derivative():
    z = np.linspace(-6, 6, 41)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.dsilu(z), fd, rtol=1e-8, atol=1e-10)


def test_adam_first_step_is_sign_times_lr():
    # after one step with zero moments, m_hat = g and v_hat = g^2: p -= lr g / (|g| + eps)
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -4.0, 1e-3])]
    opt = mlp.Adam(p, lr=0.01, eps=1e-12)
    out = opt.step(p, g)[0]
    np.testing.assert_allclose(out, p[0] - 0.01 * np.sign(g[0]), rtol=0, atol=1e-9)

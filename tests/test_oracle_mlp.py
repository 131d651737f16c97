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


def test_features_of_a_maxwellian_match_its_fourier_transform():
    # the coefficients of a Gaussian sampled on a wide, fine grid are its continuous
    # Fourier transform: fhat_k / fhat_0 = exp(-i xi.u - T |xi|^2 / 2); the sampling
    # (Poisson summation) error is ~2 exp(-2 pi^2 T / dv^2) = 1e-31 at dv = 0.5, T = 0.9
    import fks_inputs
    n, L, m = 32, 8.0, 8
    rho, u, T = 1.3, np.array([0.4, -0.7, 0.2]), 0.9
    f = fks_inputs.maxwellian_on_grid(n, L, [rho], [u], [T])[0]
    x, r = mlp.features(f, L, m)
    k = np.arange(-m // 2, m // 2)
    KX, KY, KZ = np.meshgrid(k, k, k, indexing="ij")
    xi = np.pi / L * np.stack([KX, KY, KZ], -1)
    expect = np.exp(-1j * (xi @ u) - 0.5 * T * np.sum(xi ** 2, -1)).ravel()
    assert abs(r - rho) <= 1e-12
    np.testing.assert_allclose(x[0::2], expect.real, atol=1e-12)
    np.testing.assert_allclose(x[1::2], expect.imag, atol=1e-12)


def test_moment_indicator_special_cases():
    from oracle.conserve import project
    from oracle.grid import make_grid
    n, L = 8, 4.0
    rng = np.random.default_rng(3)
    q = rng.standard_normal((n, n, n))
    # a constant has mass only: |sum q| = sum |q|
    assert abs(mlp.moment_indicator(np.ones((n, n, n)), L) - 1.0) <= 1e-15
    # after the conservation projection every invariant moment vanishes
    qp = project(q, make_grid(n, L))
    assert mlp.moment_indicator(qp, L) <= 1e-13
    # the indicator is scale invariant
    assert abs(mlp.moment_indicator(3.7 * q, L) - mlp.moment_indicator(q, L)) <= 1e-15


def test_spectral_shift_moves_a_maxwellian():
    # shifting the samples of M(u0) by delta gives the samples of M(u0 - delta) to
    # spectral accuracy; the shift preserves mass exactly and shifting back restores the
    # input.  Error budget at n = 32, L = 8, T = 1.1, centres within 0.5 of the origin:
    # the dropped Nyquist coefficient is exp(-T (2 pi)^2 / 2) = 2e-10 of the mean and the
    # periodic images at distance 15 contribute exp(-7.5^2 / 2.2) = 8e-12
    import fks_inputs
    n, L = 32, 8.0
    u0, delta, T = np.array([0.3, -0.2, 0.1]), np.array([0.37, -0.21, 0.43]), 1.1
    f = fks_inputs.maxwellian_on_grid(n, L, [1.2], [u0], [T])[0]
    g = mlp.spectral_shift(f, delta, L)
    expect = fks_inputs.maxwellian_on_grid(n, L, [1.2], [u0 - delta], [T])[0]
    assert np.max(np.abs(g - expect)) <= 2e-9 * np.max(expect)
    assert abs(g.sum() - f.sum()) <= 1e-13 * f.sum()
    back = mlp.spectral_shift(g, -delta, L)           # = f with its Nyquist modes dropped
    assert np.max(np.abs(back - mlp.spectral_shift(f, np.zeros(3), L))) <= 1e-14 * np.max(f)
    # the mean velocity of the shifted samples moves by -delta
    np.testing.assert_allclose(mlp.mean_velocity(g, L), u0 - delta, atol=1e-12)


def test_centred_features_of_a_maxwellian_are_real():
    # in its own mean-velocity frame a Maxwellian's coefficients are exp(-T |xi|^2 / 2)
    import fks_inputs
    n, L, m = 32, 8.0, 8
    f = fks_inputs.maxwellian_on_grid(n, L, [0.9], [[0.7, -0.4, 1.3]], [0.8])[0]
    x, _ = mlp.features(f, L, m, center=True)
    k = np.arange(-m // 2, m // 2)
    KX, KY, KZ = np.meshgrid(k, k, k, indexing="ij")
    xi2 = (np.pi / L) ** 2 * (KX ** 2 + KY ** 2 + KZ ** 2)
    np.testing.assert_allclose(x[0::2], np.exp(-0.4 * xi2).ravel(), atol=1e-12)
    np.testing.assert_allclose(x[1::2], 0.0, atol=1e-12)

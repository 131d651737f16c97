"""Oracle pins of the normalised non-equilibrium residual (deviatoric stress and heat flux of
f against their Maxwellian values, the moments of Section 3 one order further): zero for a
Maxwellian, the closed forms of two-Maxwellian mixtures, invariances."""

import numpy as np

import fks_inputs
from oracle.bgk import noneq_residual
from oracle.grid import make_grid

N, L = 32, 8.0


def mixture(parts):
    """sum of rho M(u, T) on the grid and its exact stress and heat flux (central moments):
    P = sum rho_k (T_k I + d_k d_k^T), q = 1/2 sum rho_k (|d_k|^2 + 5 T_k) d_k, d_k = u_k - u."""
    rhos = [p[0] for p in parts]
    us = [np.asarray(p[1], dtype=np.float64) for p in parts]
    Ts = [p[2] for p in parts]
    f = fks_inputs.maxwellian_on_grid(N, L, rhos, us, Ts).sum(axis=0)
    rho = sum(rhos)
    u = sum(r * v for r, v in zip(rhos, us)) / rho
    P = sum(r * (T * np.eye(3) + np.outer(v - u, v - u)) for r, v, T in zip(rhos, us, Ts))
    q = 0.5 * sum(r * (np.dot(v - u, v - u) + 5.0 * T) * (v - u) for r, v, T in zip(rhos, us, Ts))
    T = np.trace(P) / (3.0 * rho)
    r_exact = np.linalg.norm(P - rho * T * np.eye(3)) / (rho * T) + np.linalg.norm(q) / (rho * T ** 1.5)
    return np.asarray(f).reshape(N, N, N), r_exact


def test_maxwellian_has_zero_residual():
    g = make_grid(N, L)
    for rho, u, T in ((1.0, (0.0, 0.0, 0.0), 1.0), (0.4, (0.3, -0.2, 0.1), 0.9)):
        f, r_exact = mixture([(rho, u, T)])
        assert r_exact < 1e-15
        assert noneq_residual(f, g) < 1e-10


def test_two_beam_closed_form():
    # symmetric beams along x: u = 0, sigma = rho a^2 diag(2, -1, -1)/3, q = 0
    g = make_grid(N, L)
    a, T = 1.0, 1.0
    f, r_exact = mixture([(0.5, (a, 0, 0), T), (0.5, (-a, 0, 0), T)])
    assert abs(r_exact - (a * a * np.sqrt(6) / 3) / (T + a * a / 3)) < 1e-14
    assert abs(noneq_residual(f, g) - r_exact) < 1e-9


def test_random_mixtures_against_closed_form():
    # asymmetric mixtures carry a heat flux: (|d|^2 + 5T) d / 2 per component
    g = make_grid(N, L)
    rng = np.random.default_rng(5)
    for _ in range(4):
        # |u| <= 1.5 and T <= 1.2 keep the tails 5.9 standard deviations inside the box
        parts = [(rng.uniform(0.3, 1.0), rng.uniform(-0.85, 0.85, 3), rng.uniform(0.6, 1.2)) for _ in range(2)]
        f, r_exact = mixture(parts)
        assert r_exact > 0.05
        assert abs(noneq_residual(f, g) - r_exact) < 1e-7 * r_exact


def test_invariances():
    g = make_grid(N, L)
    f, _ = mixture([(0.6, (0.5, 0.1, -0.2), 1.1), (0.3, (-0.8, 0.4, 0.3), 0.7)])
    r0 = noneq_residual(f, g)
    assert abs(noneq_residual(3.7 * f, g) - r0) < 1e-12
    # a velocity shift of every component is a change of frame (Galilean invariance)
    s = np.array([0.3, -0.45, 0.2])
    f2, _ = mixture([(0.6, np.array((0.5, 0.1, -0.2)) + s, 1.1), (0.3, np.array((-0.8, 0.4, 0.3)) + s, 0.7)])
    assert abs(noneq_residual(f2, g) - r0) < 1e-8 * r0

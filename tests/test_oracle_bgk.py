"""Pins of the oracle's macroscopic variables, BGK relaxation, eq. DM_update and the
stiff (exponential) collision step, against closed forms and invariants."""

import numpy as np

import fks_inputs
from oracle import bgk, make_grid, make_plan, transport
from oracle.collide import collide_fast
from oracle.conserve import moments
from oracle.integrators import euler, exp_dt, exp_euler, fks_step_bgk


def mixture_primitive(parts):
    """Closed form of (rho, u, T) of a sum of Maxwellians (moments are linear in f)."""
    rho = sum(r for r, _, _ in parts)
    mom = sum(r * np.asarray(u) for r, u, _ in parts)
    E = sum(1.5 * r * T + 0.5 * r * np.dot(u, u) for r, u, T in parts)
    u = mom / rho
    T = (E - 0.5 * rho * np.dot(u, u)) / (1.5 * rho)
    return np.array([rho, u[0], u[1], u[2], T])


def test_to_primitive_of_maxwellian_moments():
    # well-resolved Maxwellians (dv^2 / T small, tails far inside [-L, L)): the discrete
    # moments reproduce (rho, u, T) to rounding
    n, L = 32, 8.0
    g = make_grid(n, L)
    for rho, u, T in [(1.0, (0.0, 0.0, 0.0), 1.0), (0.7, (0.4, -0.3, 0.2), 0.8), (1.4, (-0.5, 0.1, 0.3), 0.6)]:
        M = fks_inputs.maxwellian_on_grid(n, L, [rho], [u], [T])[0]
        W = bgk.primitive(moments(M, g, exact=True))
        np.testing.assert_allclose(W, [rho, *u, T], rtol=0, atol=1e-12)
        np.testing.assert_allclose(bgk.maxwellian(W, g), M, rtol=0, atol=1e-12 * M.max())


def test_to_primitive_of_a_mixture_matches_closed_form():
    n, L = 32, 8.0
    g = make_grid(n, L)
    parts = [(0.6, (0.3, 0.0, -0.2), 0.7), (0.5, (-0.4, 0.2, 0.1), 0.9)]
    f = sum(fks_inputs.maxwellian_on_grid(n, L, [r], [u], [T])[0] for r, u, T in parts)
    W = bgk.primitive(moments(f, g, exact=True))
    np.testing.assert_allclose(W, mixture_primitive(parts), rtol=0, atol=1e-12)
    # ToConservative inverts ToPrimitive
    U = moments(f, g, exact=True)
    np.testing.assert_allclose(bgk.conservative(W), U, rtol=1e-14, atol=1e-15)


def test_bgk_vanishes_at_equilibrium_and_conserves():
    n, L, nu = 32, 8.0, 3.0
    g = make_grid(n, L)
    M = fks_inputs.maxwellian_on_grid(n, L, [1.1], [(0.2, -0.1, 0.3)], [0.9])[0]
    assert np.abs(bgk.bgk_operator(M, moments(M, g), nu, g)).max() <= 1e-12 * M.max()
    parts = [(0.6, (0.3, 0.0, -0.2), 0.7), (0.5, (-0.4, 0.2, 0.1), 0.9)]
    f = sum(fks_inputs.maxwellian_on_grid(n, L, [r], [u], [T])[0] for r, u, T in parts)
    Q = bgk.bgk_operator(f, moments(f, g), nu, g)
    scale = nu * np.abs(f).sum() * g.dv ** 3
    assert np.abs(moments(Q, g)).max() <= 1e-13 * scale
    assert np.abs(Q).max() > 1e-2 * nu * f.max()        # f is far from equilibrium


def test_conservative_maxwellian_restores_the_moments():
    # a coarse grid with a hot, drifting state: the sampled Maxwellian misses U by about
    # 5e-5 (tails beyond the box); the corrected E has U's moments exactly and differs from
    # M by a small affine factor in the invariants
    n, L = 16, 8.0
    g = make_grid(n, L)
    f = fks_inputs.maxwellian_on_grid(n, L, [1.0], [(1.5, -1.0, 0.5)], [2.5])[0]
    f += fks_inputs.maxwellian_on_grid(n, L, [0.5], [(-0.5, 0.5, 0.0)], [0.6])[0]
    U = moments(f, g)
    M = bgk.maxwellian(bgk.primitive(U), g)
    assert np.abs(moments(M, g) - U).max() >= 1e-5 * np.abs(U).max()
    E = bgk.conservative_maxwellian(U, g)
    np.testing.assert_allclose(moments(E, g), U, rtol=0, atol=1e-13 * np.abs(U).max())
    assert np.abs(E - M).max() <= 0.1 * M.max()
    # fine, well-resolved grid: the correction vanishes
    g2 = make_grid(32, 8.0)
    M2 = fks_inputs.maxwellian_on_grid(32, 8.0, [1.0], [(0.2, 0.0, -0.1)], [0.8])[0]
    np.testing.assert_allclose(bgk.conservative_maxwellian(moments(M2, g2), g2), M2, rtol=0, atol=1e-13 * M2.max())


def test_exact_relaxation_properties():
    rng = np.random.default_rng(3)
    f = rng.random(64)
    E = rng.random(64)
    nu = 2.5
    # semigroup: two steps equal one step of the summed length (exact ODE flow)
    a = bgk.relax_exact(bgk.relax_exact(f, E, nu, 0.3), E, nu, 0.45)
    np.testing.assert_allclose(a, bgk.relax_exact(f, E, nu, 0.75), rtol=1e-14, atol=1e-15)
    # small dt: the slope is nu (E - f); Euler agrees to second order
    dt = 1e-5
    np.testing.assert_allclose((bgk.relax_exact(f, E, nu, dt) - f) / dt, nu * (E - f), rtol=0,
                               atol=nu * nu * dt * np.abs(E - f).max())
    np.testing.assert_allclose(bgk.relax_exact(f, E, nu, dt), bgk.relax_euler(f, E, nu, dt), rtol=0,
                               atol=(nu * dt) ** 2 * np.abs(E - f).max())
    # stiff limit: the state is the Maxwellian; positivity for every nu dt
    np.testing.assert_allclose(bgk.relax_exact(f, E, nu, 40.0), E, rtol=1e-15, atol=1e-40)
    for ndt in (0.5, 2.0, 7.0):
        assert np.all(bgk.relax_exact(f, E, 1.0, ndt) >= 0)
        assert ndt <= 1.0 or np.any(bgk.relax_euler(f, E, 1.0, ndt) < 0)


def test_dm_update_equals_direct_moments_over_many_steps():
    # eq. DM_update accumulated over transport steps equals the moments of the
    # transported masses recomputed directly; the box total mass is unchanged
    n, L = 4, 8.0
    shape = (5, 4, 3)
    dx, dt = 1.0, 0.37
    g = make_grid(n, L)
    rng = np.random.default_rng(11)
    ncells = int(np.prod(shape))
    f = rng.random((ncells, n ** 3))
    vel = transport.velocity_table(n, L)
    phi = transport.invariants_table(n, L)
    U = f @ phi * g.dv ** 3
    mass0 = U[:, 0].sum()
    s = np.zeros_like(vel)
    moved_any = 0
    for _ in range(12):
        delta, s = transport.advance(s, vel, dt, dx)
        moved_any += int(np.any(delta != 0))
        U = transport.dm_update(U, f, delta, shape, phi, g.dv)
        f = transport.shift(f, delta, shape)
        direct = f @ phi * g.dv ** 3
        np.testing.assert_allclose(U, direct, rtol=0, atol=1e-12 * np.abs(direct).max())
    assert moved_any >= 6
    assert abs(U[:, 0].sum() - mass0) <= 1e-13 * mass0
    # no particle moves: U is unchanged exactly
    U2 = transport.dm_update(U, f, np.zeros((n ** 3, 3), dtype=np.int64), shape, phi, g.dv)
    assert np.array_equal(U2, U)


def test_dm_update_counts_only_the_moved_particles():
    # one moved velocity, one cell of nonzero mass: the closed form of the update
    n, L = 4, 8.0
    shape = (3, 1, 1)
    g = make_grid(n, L)
    phi = transport.invariants_table(n, L)
    f = np.zeros((3, n ** 3))
    k = 5
    f[0, k] = 2.0
    delta = np.zeros((n ** 3, 3), dtype=np.int64)
    delta[k] = (1, 0, 0)
    U = transport.dm_update(np.zeros((3, 5)), f, delta, shape, phi, g.dv)
    w = g.dv ** 3
    np.testing.assert_array_equal(U[0], -2.0 * phi[k] * w)   # the particle left cell 0
    np.testing.assert_array_equal(U[1], 2.0 * phi[k] * w)    # its sister entered cell 1
    np.testing.assert_array_equal(U[2], np.zeros(5))


def test_fks_bgk_step_conserves_and_relaxes():
    n, L = 16, 8.0
    g = make_grid(n, L)
    shape = (4, 2, 2)
    dx, dt = 1.0 / 16, 0.004375
    f = fks_inputs.maxwellian_mixture(n, L, int(np.prod(shape)), seed=21)
    U = moments(f, g)
    tot0 = U.sum(axis=0)
    s = np.zeros((n ** 3, 3))
    f1, U1, s, delta, fstar = fks_step_bgk(f, U, s, g, shape, dx, dt, nu=5.0)
    # the macroscopic variables after transport are those of f*; the relaxation keeps them
    np.testing.assert_allclose(U1, moments(fstar, g), rtol=0, atol=1e-12 * np.abs(U1).max())
    np.testing.assert_allclose(moments(f1, g), U1, rtol=0, atol=1e-13 * np.abs(U1).max())
    np.testing.assert_allclose(U1.sum(axis=0), tot0, rtol=1e-13, atol=1e-13 * np.abs(tot0).max())
    # stiff limit: every cell becomes its (moment-preserving) Maxwellian
    f2, U2, _, _, _ = fks_step_bgk(f1, U1, s, g, shape, dx, dt, nu=1e5)
    W2 = bgk.primitive(U2)
    for c in range(f2.shape[0]):
        np.testing.assert_allclose(f2[c], bgk.conservative_maxwellian(U2[c], g), rtol=0, atol=1e-14 * f2[c].max())
        np.testing.assert_allclose(f2[c], bgk.maxwellian(W2[c], g), rtol=0, atol=1e-3 * f2[c].max())
    # the collision frequency does not enter the transported conservative variables
    f3, U3, _, _, _ = fks_step_bgk(f, U, np.zeros((n ** 3, 3)), g, shape, dx, dt, nu=5.0, nu_density=True)
    np.testing.assert_allclose(U3, U1, rtol=0, atol=1e-15 * np.abs(U1).max())


def test_exponential_step_limits_and_stability():
    n, L = 16, 8.0
    plan = make_plan(n, L, 6.0, a1=4, a2=4, C=0.25)
    f = fks_inputs.maxwellian_mixture(n, L, 1, seed=7)[0]
    Q = collide_fast(f, plan)
    mu = 60.0
    # small mu dt: Euler, with the Taylor remainder mu dt^2 |Q| / 2
    dt = 1e-4
    d = np.abs(exp_euler(f, Q, mu, dt) - euler(f, Q, dt)).max()
    assert d <= 0.5 * mu * dt * dt * np.abs(Q).max() * 1.01
    assert abs(exp_dt(mu, dt) - dt) <= 0.5 * mu * dt * dt * 1.01
    np.testing.assert_allclose(exp_euler(f, Q, mu, dt), f + exp_dt(mu, dt) * Q, rtol=0, atol=1e-15 * f.max())
    # large mu dt: f + Q / mu exactly
    np.testing.assert_allclose(exp_euler(f, Q, mu, 50.0), f + Q / mu, rtol=0, atol=1e-15 * f.max())
    # mass is conserved exactly by both (sum Q = 0); the exponential step stays bounded
    # by |f| + |Q| / mu for every dt while Euler grows with dt
    for dt in (0.1, 1.0, 10.0):
        fx = exp_euler(f, Q, mu, dt)
        assert abs(fx.sum() - f.sum()) <= 1e-13 * np.abs(f).sum()
        assert np.abs(fx).max() <= np.abs(f).max() + np.abs(Q).max() / mu
        assert np.abs(euler(f, Q, dt)).max() >= 0.5 * dt * np.abs(Q).max()

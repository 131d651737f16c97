"""Exact-shift transport: a permutation per velocity, mass exact, free streaming exact."""

import numpy as np

from oracle import transport
from oracle.integrators import fks_step


def test_shift_is_a_permutation_per_velocity():
    rng = np.random.default_rng(0)
    shape = (4, 3, 5)
    nv = 27
    f = rng.random((np.prod(shape), nv))
    delta = rng.integers(-1, 2, size=(nv, 3))
    g = transport.shift(f, delta, shape)
    for k in range(nv):
        assert np.array_equal(np.sort(f[:, k]), np.sort(g[:, k]))
        F = f[:, k].reshape(shape)
        G = g[:, k].reshape(shape)
        j = (1, 2, 3)
        src = tuple((j[a] - delta[k, a]) % shape[a] for a in range(3))
        assert G[j] == F[src]
    assert np.array_equal(g.sum(axis=0), f.sum(axis=0)) or np.allclose(g.sum(axis=0), f.sum(axis=0), rtol=1e-15)


def test_offsets_stay_in_cell_and_track_free_streaming():
    n, L = 8, 8.0
    vel = transport.velocity_table(n, L)
    dx, dt = 1.0 / 16, 0.004375
    s = np.zeros_like(vel)
    total = np.zeros_like(vel, dtype=np.int64)
    for step in range(40):
        d, s = transport.advance(s, vel, dt, dx)
        total += d
        assert np.all(s >= -0.5 * dx) and np.all(s < 0.5 * dx)
    # cumulative integer shift + offset = exact displacement v * t
    disp = total * dx + s
    assert np.abs(disp - vel * dt * 40).max() <= 1e-12


def test_free_streaming_of_a_profile_is_exact():
    # with Q = 0 a step is a pure permutation: a cell profile moves by whole cells
    n, L = 4, 8.0
    vel = transport.velocity_table(n, L)
    shape = (8, 4, 4)
    rng = np.random.default_rng(1)
    f = rng.random((np.prod(shape), n, n, n))
    s = np.zeros_like(vel)
    dx, dt = 1.0, 0.3
    g = f.copy()
    tot = np.zeros_like(vel, dtype=np.int64)
    for _ in range(5):
        g, s, d = fks_step(g, s, vel, shape, dx, dt, collide=lambda c: np.zeros_like(c))
        tot += d
    ref = transport.shift(f.reshape(len(f), -1), tot, shape).reshape(f.shape)
    assert np.array_equal(g, ref)
    assert np.isclose(g.sum(), f.sum(), rtol=1e-15)

"""Exact-shift transport of the Fast Kinetic Scheme (FP64 offsets).

Test infrastructure only (see the package header).

Section 2.1 (transport step): the piecewise-constant profile of every velocity
is shifted exactly by v_k dt.  Section 3 (particle interpretation): all cells
share one generic cell; its particle k sits at the sub-cell offset s_k.  When
s_k leaves the half-open cell [-dx/2, dx/2) the particle is relabelled to the
neighbouring cell: the integer shift delta_k is the number of cell faces
crossed, s_k drops by delta_k dx, and every cell receives the mass of the
particle that was delta_k cells behind it.  On a periodic box this is the
permutation f_new[j, k] = f_old[(j - delta_k) mod shape, k].

The floating-point order of operations below is part of the definition (the
integer shift is decided by floor in FP64):
    t     = s + v*dt            (product rounded, then sum rounded)
    delta = floor((t + dx/2) / dx)
    s'    = t - delta*dx

dm_update follows eq. DM_update: the conservative variables of a cell after the
transport step, from their previous values plus the masses of the particles that
left the cell and of their sisters that entered it.
"""

import numpy as np


def advance(s: np.ndarray, vel: np.ndarray, dt: float, dx: float):
    """s, vel: (nv, 3) FP64.  Returns (delta int64 (nv, 3), s_new)."""
    prod = vel * dt
    t = s + prod
    u = (t + 0.5 * dx) / dx
    delta = np.floor(u)
    s_new = t - delta * dx
    return delta.astype(np.int64), s_new


def shift(f: np.ndarray, delta: np.ndarray, shape) -> np.ndarray:
    """f: (ncells, nv) with cells in C order of `shape`; delta: (nv, 3)."""
    nx, ny, nz = shape
    out = np.empty_like(f)
    F = f.reshape(nx, ny, nz, -1)
    O = out.reshape(nx, ny, nz, -1)
    keys, inverse = np.unique(delta, axis=0, return_inverse=True)
    inverse = inverse.reshape(-1)
    for gi, d in enumerate(keys):
        cols = np.nonzero(inverse == gi)[0]
        O[..., cols] = np.roll(F[..., cols], shift=(int(d[0]), int(d[1]), int(d[2])),
                               axis=(0, 1, 2))
    return out


def velocity_table(n: int, L: float) -> np.ndarray:
    """(n^3, 3) velocity of every grid point in C order, v = -L + j * (2L/n)."""
    dv = 2.0 * L / n
    v1 = -L + np.arange(n) * dv
    X, Y, Z = np.meshgrid(v1, v1, v1, indexing="ij")
    return np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1)


def dm_update(U, f_old, delta, shape, phi, dv):
    """Eq. DM_update (Section 3): the conservative variables after one transport step.

    U: (ncells, 5) FP64 values at t^n; f_old: (ncells, nv) masses at t^n (cells in C
    order of `shape`); delta: (nv, 3) integer shifts of this step; phi: (nv, 5) the
    collision invariants (1, v, |v|^2/2) of every velocity.  A particle k that left its
    cell (delta_k != 0) is replaced in cell j by its sister from cell j - delta_k, so
        U_j^{n+1} = U_j^n + sum_{k moved} (m_{j - delta_k, k} - m_{j, k}) phi(v_k) dv^3.
    Velocities that stay put contribute nothing.
    """
    nx, ny, nz = shape
    out = np.array(U, dtype=np.float64, copy=True)
    F = f_old.reshape(nx, ny, nz, -1)
    moved = np.nonzero(np.any(delta != 0, axis=1))[0]
    w = dv ** 3
    for k in moved:
        d = delta[k]
        sister = np.roll(F[..., k], shift=(int(d[0]), int(d[1]), int(d[2])), axis=(0, 1, 2))
        diff = (sister - F[..., k]).reshape(-1)
        out += np.outer(diff, phi[k]) * w
    return out


def invariants_table(n: int, L: float) -> np.ndarray:
    """(n^3, 5) collision invariants (1, v_x, v_y, v_z, |v|^2/2) of every velocity in C order."""
    v = velocity_table(n, L)
    return np.concatenate([np.ones((v.shape[0], 1)), v, 0.5 * np.sum(v * v, axis=1, keepdims=True)], axis=1)

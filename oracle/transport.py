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

"""Time integrators of the collision stage (FP64).

Test infrastructure only (see the package header).

euler: the explicit Euler step of eq. disc_relax, f^{n+1} = f* + dt Q(f*).
heun:  the two-stage Heun / SSP-RK2 step (the paper allows other integrators in
       place of Euler; it is used for the space-homogeneous BKW run):
       f1 = f + dt Q(f);  f^{n+1} = (f + f1 + dt Q(f1)) / 2.
fks_step: one split step of Section 2.1 on a periodic box of cells: exact
       transport (transport.advance/shift), then the Euler collision stage in
       every cell.
"""

import numpy as np

from . import transport


def euler(f, Q, dt):
    return f + dt * Q


def heun(f, collide, dt):
    f1 = f + dt * collide(f)
    return 0.5 * (f + f1 + dt * collide(f1))


def fks_step(f_cells, s, vel, shape, dx, dt, collide):
    """f_cells: (ncells, n, n, n); s: (nv, 3) offsets.  Returns (f_new, s_new, delta)."""
    ncells = f_cells.shape[0]
    nv = f_cells[0].size
    delta, s_new = transport.advance(s, vel, dt, dx)
    fstar = transport.shift(f_cells.reshape(ncells, nv), delta, shape).reshape(f_cells.shape)
    fnew = np.stack([euler(fstar[c], collide(fstar[c]), dt) for c in range(ncells)])
    return fnew, s_new, delta

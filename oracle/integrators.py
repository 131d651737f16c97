"""Time integrators of the collision stage (FP64).

Test infrastructure only (see the package header).

euler: the explicit Euler step of eq. disc_relax, f^{n+1} = f* + dt Q(f*).
heun:  the two-stage Heun / SSP-RK2 step (the paper allows other integrators in
       place of Euler; it is used for the space-homogeneous BKW run):
       f1 = f + dt Q(f);  f^{n+1} = (f + f1 + dt Q(f1)) / 2.
exp_euler: a stiff-capable first-order step (Section 2.1 asks for special care in
       the stiff limit).  With a penalty mu > 0 the equation df/dt = Q(f) is split as
       df/dt = -mu f + (Q(f) + mu f); the linear part is integrated exactly and the
       rest is frozen at f*:
           f^{n+1} = e^{-mu dt} f* + (1 - e^{-mu dt}) (f* + Q(f*) / mu)
                   = f* + dt_eff Q(f*),   dt_eff = (1 - e^{-mu dt}) / mu.
       It is a convex combination of f* and f* + Q/mu, so if mu bounds the
       collision frequency (Q = G - nu f with G >= 0, nu <= mu) the step keeps f >= 0
       for every dt, where explicit Euler needs nu dt <= 1.  It conserves whatever Q
       conserves and tends to Euler as mu dt -> 0.
fks_step: one split step of Section 2.1 on a periodic box of cells: exact
       transport (transport.advance/shift), then the Euler collision stage in
       every cell.
fks_step_bgk: the sequential FKS algorithm of Section 4.1 with the BGK operator:
       transport, conservative variables by eq. DM_update, relaxation towards the
       cells' moment-preserving Maxwellians (Section 2.2.1; bgk.conservative_maxwellian).
"""

import numpy as np

from . import bgk, transport


def euler(f, Q, dt):
    return f + dt * Q


def heun(f, collide, dt):
    f1 = f + dt * collide(f)
    return 0.5 * (f + f1 + dt * collide(f1))


def exp_dt(mu, dt):
    """Effective step (1 - e^{-mu dt}) / mu of exp_euler (dt itself for mu = 0)."""
    if mu == 0.0:
        return dt
    return -np.expm1(-mu * dt) / mu


def exp_euler(f, Q, mu, dt):
    """e^{-mu dt} f + (1 - e^{-mu dt}) (f + Q / mu)."""
    a = np.exp(-mu * dt)
    return a * f + (1.0 - a) * (f + Q / mu)


def fks_step(f_cells, s, vel, shape, dx, dt, collide):
    """f_cells: (ncells, n, n, n); s: (nv, 3) offsets.  Returns (f_new, s_new, delta)."""
    ncells = f_cells.shape[0]
    nv = f_cells[0].size
    delta, s_new = transport.advance(s, vel, dt, dx)
    fstar = transport.shift(f_cells.reshape(ncells, nv), delta, shape).reshape(f_cells.shape)
    fnew = np.stack([euler(fstar[c], collide(fstar[c]), dt) for c in range(ncells)])
    return fnew, s_new, delta


def fks_step_bgk(f_cells, U, s, grid, shape, dx, dt, nu, nu_density=False, exact=True):
    """One FKS step with the BGK operator; U (ncells, 5) are the conservative variables
    of f_cells at t^n.  Returns (f_new, U_new, s_new, delta, fstar)."""
    ncells = f_cells.shape[0]
    n = grid.n
    nv = n ** 3
    vel = transport.velocity_table(n, grid.L)
    phi = transport.invariants_table(n, grid.L)
    delta, s_new = transport.advance(s, vel, dt, dx)
    flat = f_cells.reshape(ncells, nv)
    U_new = transport.dm_update(U, flat, delta, shape, phi, grid.dv)
    fstar = transport.shift(flat, delta, shape).reshape(f_cells.shape)
    fnew = np.empty_like(fstar)
    for c in range(ncells):
        E = bgk.conservative_maxwellian(U_new[c], grid)
        nuc = nu * U_new[c, 0] if nu_density else nu
        fnew[c] = bgk.relax_exact(fstar[c], E, nuc, dt) if exact else bgk.relax_euler(fstar[c], E, nuc, dt)
    return fnew, U_new, s_new, delta, fstar

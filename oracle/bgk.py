"""Macroscopic variables and the BGK relaxation operator (FP64).

Test infrastructure only (see the package header).

Section 2 of the paper: the conservative variables are U = (rho, rho u, E), the
moments of f against phi(v) = (1, v, |v|^2/2); the temperature follows from
(3/2) rho T = E - (1/2) rho |u|^2; the local equilibrium is the Maxwellian
M[f](v) = rho (2 pi T)^{-3/2} exp(-|v - u|^2 / (2T)); the BGK operator is
Q_BGK(f) = nu (M[f] - f) with the collision frequency nu.

Section 2.2.1: in the FKS the BGK collision term of velocity v_k in cell j is
nu (E_jk - f_jk), E_jk the Maxwellian of the cell's macroscopic variables
evaluated at v_k.  The macroscopic variables are collision invariants, so they
do not change during the relaxation and E is fixed over the collision step.

The sampled Maxwellian M[W](v_k) does not have exactly the discrete moments U on the
truncated grid (the tails beyond the box and the rectangle rule), so a relaxation
towards it would change U, which the FKS keeps by eq. DM_update assuming collisions
conserve.  The "suitable approximation" E used here is the sampled Maxwellian times
the affine correction in the invariants that restores the moments exactly:
    E = M (1 + lambda . phi),  G lambda = U - dv^3 sum_k M phi,  G = dv^3 sum_k M phi phi^T.
For a well-resolved Maxwellian lambda is at rounding level and E = M.

Relaxation of one step dt at frozen E (the collision stage of eq. disc_relax):
  euler: f + dt nu (E - f)             (eq. disc_relax)
  exact: E + (f - E) exp(-nu dt)        (the ODE df/dt = nu (E - f) solved exactly;
                                         stable and positivity preserving for any
                                         nu dt, the stiff limit named in Section 2.1)
"""

import numpy as np

from .grid import Grid, velocity_vectors


def primitive(U):
    """ToPrimitive: U (..., 5) = (rho, rho u_x, rho u_y, rho u_z, E) -> (rho, u_x, u_y, u_z, T)."""
    U = np.asarray(U, dtype=np.float64)
    rho = U[..., 0]
    u = U[..., 1:4] / rho[..., None]
    T = (2.0 / 3.0) * (U[..., 4] / rho - 0.5 * np.sum(u * u, axis=-1))
    return np.concatenate([rho[..., None], u, T[..., None]], axis=-1)


def conservative(W):
    """ToConservative: (rho, u, T) -> (rho, rho u, E) with E = (3/2) rho T + (1/2) rho |u|^2."""
    W = np.asarray(W, dtype=np.float64)
    rho = W[..., 0]
    u = W[..., 1:4]
    T = W[..., 4]
    E = 1.5 * rho * T + 0.5 * rho * np.sum(u * u, axis=-1)
    return np.concatenate([rho[..., None], rho[..., None] * u, E[..., None]], axis=-1)


def maxwellian(W, g: Grid):
    """M(v_k) = rho (2 pi T)^{-3/2} exp(-|v_k - u|^2 / (2T)) on the grid, for one cell W (5,)."""
    rho, u, T = W[0], np.asarray(W[1:4]), W[4]
    V = velocity_vectors(g)
    w2 = np.sum((V - u) ** 2, axis=-1)
    return rho * (2.0 * np.pi * T) ** -1.5 * np.exp(-w2 / (2.0 * T))


def conservative_maxwellian(U, g: Grid):
    """E = M (1 + lambda . phi) with the discrete moments of E equal to U (one cell, U (5,))."""
    U = np.asarray(U, dtype=np.float64)
    M = maxwellian(primitive(U), g).reshape(-1)
    V = velocity_vectors(g).reshape(-1, 3)
    phi = np.stack([np.ones(len(V)), V[:, 0], V[:, 1], V[:, 2], 0.5 * np.sum(V * V, axis=1)])
    w = g.dv ** 3
    G = (phi * M) @ phi.T * w
    m = phi @ M * w
    lam = np.linalg.solve(G, U - m)
    return (M * (1.0 + lam @ phi)).reshape(g.n, g.n, g.n)


def bgk_operator(f, U, nu, g: Grid):
    """Q_BGK = nu (E[U] - f) for one cell with conservative variables U."""
    return nu * (conservative_maxwellian(U, g) - f)


def relax_euler(f, E, nu, dt):
    return f + dt * nu * (E - f)


def relax_exact(f, E, nu, dt):
    return E + (f - E) * np.exp(-nu * dt)


def noneq_residual(f, g: Grid):
    """Normalised non-equilibrium residual of one cell's f (FP64), from its central moments:
    with rho, u, T of f and c = v - u, the deviatoric stress
    sigma = dv^3 sum f c c^T - rho T I and the heat flux q = dv^3 sum f |c|^2 c / 2 vanish for a
    Maxwellian; r = |sigma|_F / (rho T) + |q| / (rho T^{3/2})."""
    f = np.asarray(f, dtype=np.float64).reshape(-1)
    V = velocity_vectors(g).reshape(-1, 3)
    w = g.dv ** 3
    rho = w * f.sum()
    u = w * (f @ V) / rho
    c = V - u
    P = w * (c * f[:, None]).T @ c
    T = np.trace(P) / (3.0 * rho)
    sigma = P - rho * T * np.eye(3)
    q = 0.5 * w * ((np.sum(c * c, axis=1) * f) @ c)
    return float(np.linalg.norm(sigma) / (rho * T) + np.linalg.norm(q) / (rho * T ** 1.5))

"""Macroscopic moments and the FP64 conservation projection.

Test infrastructure only (see the package header).

moments: U_j = dv^3 sum_k phi(v_k) f_{j,k}, phi = (1, v_x, v_y, v_z, |v|^2/2)
(Section 2 collision invariants; Section 3 macroscopic variables of the particle
interpretation).

project: the spectral Q conserves mass exactly but momentum and energy only to
spectral accuracy.  The correction is the least-squares (minimum L2 norm)
change of Q that makes its discrete invariant moments vanish:
    Q_c = Q - Phi^T (Phi Phi^T)^{-1} Phi Q,
rows of Phi = phi_i(v_k).  This step is not part of the paper; it is the
standard constrained-optimisation correction of spectral methods, applied in
FP64.
"""

import math

import numpy as np

from .grid import Grid, velocity_vectors


def invariants(g: Grid) -> np.ndarray:
    """Phi, shape (5, n^3): 1, v_x, v_y, v_z, |v|^2/2 at every grid point."""
    V = velocity_vectors(g).reshape(-1, 3)
    return np.stack([np.ones(V.shape[0]), V[:, 0], V[:, 1], V[:, 2],
                     0.5 * (V * V).sum(axis=1)])


def moments(f: np.ndarray, g: Grid, exact=False) -> np.ndarray:
    """U for one cell (f shape (n,n,n)) or a batch (..., n, n, n) -> (..., 5)."""
    Phi = invariants(g)
    flat = f.reshape(f.shape[:-3] + (-1,))
    w = g.dv ** 3
    if exact:
        if flat.ndim != 1:
            raise ValueError("exact summation is for one cell")
        return np.array([math.fsum(Phi[i] * flat) * w for i in range(5)])
    return flat @ Phi.T * w


def project(Q: np.ndarray, g: Grid) -> np.ndarray:
    """Q - Phi^T (Phi Phi^T)^{-1} Phi Q for one cell or a batch."""
    Phi = invariants(g)
    flat = Q.reshape(Q.shape[:-3] + (-1,))
    m = flat @ Phi.T
    lam = np.linalg.solve(Phi @ Phi.T, m.T).T
    return (flat - lam @ Phi).reshape(Q.shape)

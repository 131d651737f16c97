"""Closed-form Bobylev-Krook-Wu (BKW) solution for Maxwell molecules (FP64).

Test infrastructure only (see the package header).

Space-homogeneous Boltzmann equation with the constant kernel B = 1/(4 pi)
(alpha = 0 in eq. J9hb, C = 1/(4 pi)), density 1, zero mean velocity and
temperature 1, in three dimensions:
    f(t, v) = exp(-|v|^2 / (2K)) / (2 (2 pi K)^{3/2})
              * [ (5K - 3)/K + (1 - K) |v|^2 / K^2 ],   K(t) = 1 - exp(-t/6).
The formula is not in the paper; it is a classical exact solution.  Its time
scale and normalisation are pinned in the tests against a brute-force
quadrature of the sigma-form collision integral (oracle.sigma_form).  f >= 0
requires K >= 3/5.
"""

import numpy as np


def K_of_t(t):
    return 1.0 - np.exp(-t / 6.0)


def f_bkw(t, v):
    """v: (..., 3)."""
    K = K_of_t(t)
    r2 = np.sum(np.asarray(v) ** 2, axis=-1)
    c = 0.5 * (2.0 * np.pi * K) ** -1.5
    return c * np.exp(-r2 / (2.0 * K)) * ((5.0 * K - 3.0) / K + (1.0 - K) * r2 / K ** 2)


def dfdt_bkw(t, v):
    """Analytic time derivative (chain rule through K)."""
    K = K_of_t(t)
    dK = (1.0 - K) / 6.0
    r2 = np.sum(np.asarray(v) ** 2, axis=-1)
    c = 0.5 * (2.0 * np.pi * K) ** -1.5
    e = np.exp(-r2 / (2.0 * K))
    a = 5.0 - 3.0 / K
    b = 1.0 / K ** 2 - 1.0 / K
    da = 3.0 / K ** 2
    db = -2.0 / K ** 3 + 1.0 / K ** 2
    dfdK = c * e * ((-1.5 / K + r2 / (2.0 * K ** 2)) * (a + b * r2) + da + db * r2)
    return dfdK * dK

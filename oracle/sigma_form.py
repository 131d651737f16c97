"""Brute-force quadrature of the Boltzmann collision integral in sigma form.

Test infrastructure only (see the package header).

Section 2.2, eq. boltzmann:
    Q(v) = int_{R^3} int_{S^2} B(|g|) [f(v') f(v'_*) - f(v) f(v_*)] d omega d v_*,
    v' = (v + v_* + |g| omega)/2,  v'_* = (v + v_* - |g| omega)/2,  g = v - v_*,
with the variable-hard-sphere kernel B = |g| sigma, sigma = C |g|^(alpha - 1)
(eq. J9hb with b_alpha = C), i.e. B = C |g|^alpha.

Used only as an independent check of the whole spectral chain on analytic f
(no periodisation, no truncation, no Fourier modes).  The relative velocity is
written in spherical coordinates around v (g = r ghat, dv_* = r^2 dr dghat);
r uses Gauss-Legendre on [0, r_max], both unit-vector integrals use
Gauss-Legendre in cos(theta) times the trapezoidal rule in the azimuth.
"""

import numpy as np


def _sphere_rule(n_theta, n_phi):
    x, w = np.polynomial.legendre.leggauss(n_theta)
    ph = np.arange(n_phi) * (2.0 * np.pi / n_phi)
    ct = np.repeat(x, n_phi)
    st = np.sqrt(1.0 - ct * ct)
    pp = np.tile(ph, n_theta)
    dirs = np.stack([st * np.cos(pp), st * np.sin(pp), ct], axis=1)
    wts = np.repeat(w, n_phi) * (2.0 * np.pi / n_phi)
    return dirs, wts


def collision_integral(fun, v, C, alpha, r_max=12.0, n_r=48, n_g=(16, 32), n_w=(16, 32)):
    """Q(v) for a vectorised callable fun(points (...,3)) -> values; v shape (3,)."""
    v = np.asarray(v, dtype=np.float64)
    xr, wr = np.polynomial.legendre.leggauss(n_r)
    r = 0.5 * r_max * (xr + 1.0)
    wr = 0.5 * r_max * wr
    gh, wg = _sphere_rule(*n_g)
    om, wo = _sphere_rule(*n_w)
    fv = fun(v[None, :])[0]
    total = 0.0
    for i in range(n_r):
        B = C * r[i] ** alpha
        g = r[i] * gh                                  # (Ng, 3) relative velocities v - v_*
        vstar = v[None, :] - g                         # (Ng, 3)
        loss = fv * fun(vstar)                         # (Ng,)
        mid = 0.5 * (v[None, :] + vstar)               # (Ng, 3)
        half = 0.5 * r[i] * om                         # (No, 3)
        vp = mid[:, None, :] + half[None, :, :]
        vps = mid[:, None, :] - half[None, :, :]
        gain = (fun(vp) * fun(vps)) @ wo               # (Ng,)
        inner = ((gain - loss * wo.sum()) * wg).sum()
        total += wr[i] * r[i] ** 2 * B * inner
    return total


def maxwellian(rho, u, T):
    u = np.asarray(u, dtype=np.float64)

    def fun(p):
        d = p - u
        return rho * (2.0 * np.pi * T) ** -1.5 * np.exp(-np.sum(d * d, axis=-1) / (2.0 * T))
    return fun


def mixture(components):
    funs = [maxwellian(*c) for c in components]

    def fun(p):
        return sum(f(p) for f in funs)
    return fun

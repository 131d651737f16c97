"""Kernel tables of the separable fast spectral method, FP64.

Test infrastructure only (see the package header).

Follows Appendix A of the paper:
  * Carleman form of Q with the kernel B~(x, y) and the truncated weights
    B_F(l, m) = int_{B_R} int_{B_R} B~ delta(x.y) e^{i(xi_l.x + xi_m.y)} dx dy;
  * power-law kernel B~ = 4 C (|x|^2+|y|^2)^{-(1-alpha)/2} (eq. Btilde_pl), which
    is the constant 4C for hard spheres (alpha = 1);
  * the separable quadrature B_F(l, m) ~ sum_t alpha_t(l) alpha'_t(m) over
    discrete directions e_t = e(theta_p, phi_q).

Readings taken where the printed formulas are garbled (each is pinned by tests):
  * phi_R(s) = int_{-R}^{R} |rho| e^{i rho s} d rho
             = 2 [R sin(Rs)/s + (cos(Rs) - 1)/s^2]    (polar Jacobian |rho|);
  * psi_R(s) = Fourier transform of the radius-R disc in the plane normal to e
             = int_0^pi phi_R(s cos t) dt = 2 pi R J1(Rs)/s;
  * directions: theta_p = (p + 1/2) pi / A1 (p < A1), phi_q = q pi / A2 (q < A2),
    weight pi^2 sin(theta_p) / (A1 A2)  (midpoint rule on the half sphere with
    its spherical Jacobian);
  * the loss weight B_F(m, m) uses the same quadrature as the gain:
    lambda(m) = sum_t alpha_t(m) alpha'_t(m);
  * B~ = 4 sigma(|u|), |u|^2 = |x|^2 + |y|^2, i.e. 4 C |u|^(alpha - 1).
For alpha < 1 (non-separable B~, e.g. Maxwell molecules alpha = 0) the radial
integral over |x| is done by Gauss-Legendre on [0, R] and the disc integral in
the plane normal to e by a fixed high-order Gauss-Legendre rule in |y|; each
radial node is then one more separable term.
"""

from dataclasses import dataclass
from math import factorial

import numpy as np
from scipy import special

from .grid import Grid, make_grid, mode_vectors

HARD_SPHERES = "hard_spheres"
VHS = "vhs"


def phi_R(s, R):
    """phi_R(s) = int_{-R}^{R} |rho| e^{i rho s} d rho (real and even in s)."""
    s = np.asarray(s, dtype=np.float64)
    x = R * np.abs(s)
    out = np.empty_like(x)
    small = x < 0.5
    xs = x[small]
    # 2 sum_j (-1)^j (2j+1) x^{2j} / (2j+2)!  (Taylor series of the closed form)
    acc = np.zeros_like(xs)
    for j in range(12):
        acc += (-1) ** j * (2 * j + 1) * xs ** (2 * j) / factorial(2 * j + 2)
    out[small] = 2.0 * R * R * acc
    xb = x[~small]
    sb = np.abs(s[~small])
    out[~small] = 2.0 * (R * np.sin(xb) / sb + (np.cos(xb) - 1.0) / (sb * sb))
    return out


def psi_R(s, R):
    """psi_R(s) = int over the radius-R disc of e^{i eta.y}, |eta| = s: 2 pi R J1(Rs)/s."""
    s = np.abs(np.asarray(s, dtype=np.float64))
    x = R * s
    out = np.empty_like(x)
    small = x < 1e-3
    xs = x[small]
    out[small] = 2.0 * np.pi * R * R * (0.5 - xs * xs / 16.0 + xs ** 4 / 384.0)
    out[~small] = 2.0 * np.pi * R * special.j1(x[~small]) / s[~small]
    return out


def directions(a1: int, a2: int):
    """Unit vectors e_t and weights w_t of the half-sphere midpoint rule."""
    th = (np.arange(a1) + 0.5) * np.pi / a1
    ph = np.arange(a2) * np.pi / a2
    T, P = np.meshgrid(th, ph, indexing="ij")
    e = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], axis=-1)
    w = (np.pi ** 2 / (a1 * a2)) * np.sin(T)
    return e.reshape(-1, 3), w.reshape(-1)


def radial_g(s, rho_r, R, alpha, C, n_gl=256):
    """g_r(s) = 2 pi int_0^R rho' B~(rho_r, rho') J0(rho' s) d rho' for the power-law B~.

    rho_r may be a scalar or an array of radial nodes; the result has shape
    s.shape + rho_r.shape.  The integrand is smooth for rho_r > 0; a fixed
    n_gl-point Gauss-Legendre rule on [0, R] is used (pinned against adaptive
    quadrature by the tests).
    """
    x, wx = np.polynomial.legendre.leggauss(n_gl)
    rp = 0.5 * R * (x + 1.0)
    wr = 0.5 * R * wx
    rr = np.atleast_1d(np.asarray(rho_r, dtype=np.float64))
    bt = 4.0 * C * (rr[None, :] ** 2 + rp[:, None] ** 2) ** (0.5 * (alpha - 1.0))  # (n_gl, nr)
    W = 2.0 * np.pi * (wr * rp)[:, None] * bt
    s = np.asarray(s, dtype=np.float64)
    flat = s.reshape(-1)
    out = np.empty((flat.size, rr.size))
    chunk = 8192
    for i in range(0, flat.size, chunk):
        out[i:i + chunk] = special.j0(np.outer(flat[i:i + chunk], rp)) @ W
    out = out.reshape(s.shape + rr.shape)
    return out[..., 0] if np.ndim(rho_r) == 0 else out


@dataclass
class Plan:
    grid: Grid
    R: float
    kernel: str
    alpha: float
    C: float
    a1: int
    a2: int
    n_radial: int
    P: int
    A: np.ndarray      # (T, K, K, K) first separable factor alpha_t(l)
    Ap: np.ndarray     # (T, K, K, K) second separable factor alpha'_t(m)
    lam: np.ndarray    # (K, K, K) loss weight, quadrature of B_F(m, m)

    @property
    def n_terms(self) -> int:
        return self.A.shape[0]


def make_plan(n, L, R, kernel=HARD_SPHERES, C=0.25, a1=4, a2=4, n_radial=8,
              alpha=None, P=None) -> Plan:
    """Build the FP64 tables for grid size n on [-L, L)^3 with Carleman cut-off R."""
    g = make_grid(n, L)
    if P is None:
        P = 3 * n // 2
    xi = mode_vectors(g)                       # (K, K, K, 3)
    e, w = directions(a1, a2)
    A_list, Ap_list = [], []
    if kernel == HARD_SPHERES:
        alpha = 1.0
        for t in range(e.shape[0]):
            proj = xi @ e[t]                               # xi_l . e_t
            perp = np.linalg.norm(xi - proj[..., None] * e[t], axis=-1)
            A_list.append(phi_R(proj, R))
            Ap_list.append(w[t] * 4.0 * C * psi_R(perp, R))
    elif kernel == VHS:
        if alpha is None:
            alpha = 0.0
        xr, wr = np.polynomial.legendre.leggauss(n_radial)
        rho = 0.5 * R * (xr + 1.0)
        wrho = 0.5 * R * wr
        for t in range(e.shape[0]):
            proj = xi @ e[t]
            perp = np.linalg.norm(xi - proj[..., None] * e[t], axis=-1)
            gr = radial_g(perp, rho, R, alpha, C)              # (K, K, K, n_radial)
            for r in range(n_radial):
                # 2 int_0^R rho cos(rho xi.e) g(rho, .) d rho by Gauss-Legendre in rho
                A_list.append(2.0 * wrho[r] * rho[r] * np.cos(rho[r] * proj))
                Ap_list.append(w[t] * gr[..., r])
    else:
        raise ValueError(kernel)
    A = np.stack(A_list)
    Ap = np.stack(Ap_list)
    lam = (A * Ap).sum(axis=0)
    return Plan(grid=g, R=float(R), kernel=kernel, alpha=float(alpha), C=float(C),
                a1=a1, a2=a2, n_radial=n_radial if kernel == VHS else 0, P=int(P),
                A=A, Ap=Ap, lam=lam)


def bhat_F_quadrature(plan: Plan, xi_l, xi_m):
    """Quadrature value of B_F(l, m) for explicit wave vectors (used by pins)."""
    e, w = directions(plan.a1, plan.a2)
    xi_l = np.asarray(xi_l, dtype=np.float64)
    xi_m = np.asarray(xi_m, dtype=np.float64)
    if plan.kernel != HARD_SPHERES:
        raise NotImplementedError
    pl = e @ xi_l
    pm = e @ xi_m
    perp = np.sqrt(np.maximum(xi_m @ xi_m - pm * pm, 0.0))
    return float(np.sum(phi_R(pl, plan.R) * w * 4.0 * plan.C * psi_R(perp, plan.R)))

"""Pins of the oracle's kernel tables against definitions and closed forms.

phi_R, psi_R and the angular rule are the garbled part of Appendix A; each
reading is checked against the integral it must equal.
"""

import numpy as np
import pytest
from scipy import integrate, special

from oracle.tables import (HARD_SPHERES, VHS, bhat_F_quadrature, directions,
                           make_plan, phi_R, psi_R, radial_g)

R = 6.0


@pytest.mark.parametrize("s", [0.0, 1e-4, 0.01, 0.05, 0.0833, 0.3, 1.7, 4.1, 9.9])
def test_phi_R_is_the_radial_line_integral(s):
    # phi_R(s) = int_{-R}^{R} |rho| e^{i rho s} d rho  (App. A, polar Jacobian reading)
    ref = 2.0 * integrate.quad(lambda r: r * np.cos(r * s), 0.0, R, epsabs=1e-14, epsrel=1e-14,
                               limit=400)[0]
    assert abs(phi_R(np.array([s]), R)[0] - ref) <= 1e-13 * max(1.0, abs(ref))


def test_phi_R_series_branch_is_continuous():
    # both sides of the series / closed-form switch at R|s| = 0.5 match the integral
    for s in (0.5 / R * (1 - 1e-9), 0.5 / R * (1 + 1e-9)):
        ref = 2.0 * integrate.quad(lambda r: r * np.cos(r * s), 0.0, R, epsabs=1e-14,
                                   epsrel=1e-14)[0]
        assert abs(phi_R(np.array([s]), R)[0] - ref) <= 1e-13 * R * R
    assert phi_R(np.array([0.0]), R)[0] == R * R
    s = np.linspace(-3, 3, 101)
    assert np.array_equal(phi_R(s, R), phi_R(-s, R))          # real and even


@pytest.mark.parametrize("s", [0.0, 5e-5, 0.3, 1.7, 4.1, 9.9])
def test_psi_R_is_the_disc_transform(s):
    # psi_R(s) = Fourier transform of the radius-R disc = int_0^pi phi_R(s cos t) dt
    x, w = np.polynomial.legendre.leggauss(200)
    t = 0.5 * np.pi * (x + 1.0)
    via_phi = 0.5 * np.pi * np.sum(w * phi_R(s * np.cos(t), R))
    # direct 2-D disc quadrature in polar coordinates: int_0^R r 2 pi J0(r s) dr
    disc = integrate.quad(lambda r: 2 * np.pi * r * special.j0(r * s), 0.0, R, epsabs=1e-13,
                          limit=400)[0]
    val = psi_R(np.array([s]), R)[0]
    assert abs(val - via_phi) <= 1e-12 * max(1.0, abs(val))
    assert abs(val - disc) <= 1e-11 * max(1.0, abs(val))


def test_direction_rule_weights():
    e, w = directions(4, 4)
    assert e.shape == (16, 3)
    np.testing.assert_allclose(np.linalg.norm(e, axis=1), 1.0, rtol=0, atol=1e-15)
    # half-sphere area 2 pi to O(A1^-2) (midpoint rule with sin(theta) Jacobian)
    for a in (4, 16, 64):
        _, w = directions(a, a)
        assert abs(w.sum() - 2 * np.pi) <= 2 * np.pi * 1.0 / a ** 2


def test_bhat_F_closed_forms():
    # B_F(0,0) = 2 pi^2 R^4 and B_F(l,0) = B_F(0,l) = 4 pi^2 R^2 (1 - cos(R|xi|))/|xi|^2
    # (exact integrals of the truncated Carleman weight, hard spheres B~ = 1).
    plan = make_plan(8, 8.0, R, a1=64, a2=64, C=0.25)
    b00 = bhat_F_quadrature(plan, [0, 0, 0], [0, 0, 0])
    assert abs(b00 / (2 * np.pi ** 2 * R ** 4) - 1) < 2e-4
    rng = np.random.default_rng(0)
    for _ in range(4):
        xi = rng.normal(size=3) * 0.7
        r = np.linalg.norm(xi)
        exact = 4 * np.pi ** 2 * R ** 2 * (1 - np.cos(R * r)) / r ** 2
        assert abs(bhat_F_quadrature(plan, xi, [0, 0, 0]) - exact) <= 2e-3 * 2 * np.pi ** 2 * R ** 4
        assert abs(bhat_F_quadrature(plan, [0, 0, 0], xi) - exact) <= 2e-3 * 2 * np.pi ** 2 * R ** 4


def test_angular_rule_converges_second_order():
    errs = []
    for a in (4, 8, 16):
        plan = make_plan(8, 8.0, R, a1=a, a2=a, C=0.25)
        errs.append(abs(bhat_F_quadrature(plan, [0, 0, 0], [0, 0, 0]) / (2 * np.pi ** 2 * R ** 4) - 1))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5


@pytest.mark.parametrize("alpha", [0.0, 0.5])
@pytest.mark.parametrize("s", [0.0, 0.7, 3.3, 9.0])
@pytest.mark.parametrize("rr", [0.055, 0.12, 3.0])
def test_radial_g_against_adaptive_quadrature(s, rr, alpha):
    # eq. Btilde_pl: B~ = 4C (|x|^2 + |y|^2)^{(alpha - 1)/2}
    C = 1.0 / (4 * np.pi)
    ref = integrate.quad(lambda r: 2 * np.pi * r * 4 * C * (rr ** 2 + r ** 2) ** (0.5 * (alpha - 1.0))
                         * special.j0(r * s), 0.0, R, epsabs=1e-14, limit=400)[0]
    assert abs(radial_g(np.array([s]), rr, R, alpha, C)[0] - ref) <= 1e-11 * max(1.0, abs(ref))


def test_vhs_radial_quadrature_at_alpha_one_is_hard_spheres():
    # at alpha = 1 the power-law kernel is the constant 4C: the radial Gauss-Legendre
    # terms must rebuild the closed-form hard-sphere tables (phi_R, psi_R), so the two
    # operators agree to rounding; this pins the alpha dependence of the VHS path
    import fks_inputs
    from oracle.collide import collide_fast
    n, L = 16, 8.0
    f = fks_inputs.maxwellian_mixture(n, L, 1, seed=3)[0]
    qh = collide_fast(f, make_plan(n, L, R, a1=3, a2=4, C=0.25))
    qv = collide_fast(f, make_plan(n, L, R, kernel=VHS, alpha=1.0, a1=3, a2=4, n_radial=16, C=0.25))
    assert np.linalg.norm(qv - qh) / np.linalg.norm(qh) <= 1e-11


def test_tables_are_even_in_k():
    # alpha_t(-k) = alpha_t(k): the reality of A_t, B_t relies on it
    for kern in (HARD_SPHERES, VHS):
        plan = make_plan(8, 8.0, R, kernel=kern, a1=2, a2=3, n_radial=3, C=0.25)
        np.testing.assert_array_equal(plan.A, plan.A[:, ::-1, ::-1, ::-1])
        np.testing.assert_allclose(plan.Ap, plan.Ap[:, ::-1, ::-1, ::-1], rtol=1e-14, atol=0)

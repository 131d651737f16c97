"""O-direct (plain eq. CF1 sum) against O-fast (padded FFTs), and exact invariants."""

import json
import os

import numpy as np
import pytest

import fks_inputs
from oracle import make_plan
from oracle.collide import collide_direct, collide_fast
from oracle.conserve import moments, project
from oracle.tables import VHS

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _case(n, L=8.0, R=6.0, seed=3, **kw):
    plan = make_plan(n, L, R, **kw)
    f = fks_inputs.maxwellian_mixture(n, L, 1, seed=seed)[0]
    return plan, f


@pytest.mark.parametrize("n", [8, 12])
def test_direct_equals_fast(n):
    # Linear convolution through the padded FFT (P >= 3N/2) reproduces the
    # truncated double sum of eq. CF1 exactly, up to rounding; so does P = 2N.
    plan, f = _case(n, a1=3, a2=4)
    Qd, imd = collide_direct(f, plan, return_imag=True)
    scale = np.linalg.norm(Qd)
    for P in (3 * n // 2, 2 * n):
        Qf, imf = collide_fast(f, plan, P=P, return_imag=True)
        assert np.linalg.norm(Qf - Qd) <= 1e-11 * scale
        assert imf <= 1e-14 * np.abs(Qf).max() * 10
    assert imd <= 1e-13 * np.abs(Qd).max()


def test_direct_equals_fast_vhs():
    plan, f = _case(8, L=6.0, R=4.0, kernel=VHS, alpha=0.0, C=1 / (4 * np.pi), a1=2, a2=3, n_radial=3)
    Qd = collide_direct(f, plan)
    Qf = collide_fast(f, plan)
    assert np.linalg.norm(Qf - Qd) <= 1e-11 * np.linalg.norm(Qd)


def test_cyclic_padding_differs():
    # P = N is the aliased cyclic convolution: it must NOT equal the Galerkin sum
    plan, f = _case(8, a1=3, a2=4)
    Qd = collide_direct(f, plan)
    Qa = collide_fast(f, plan, P=8)
    assert np.linalg.norm(Qa - Qd) > 1e-6 * np.linalg.norm(Qd)


def test_packed_equals_unpacked():
    plan, f = _case(16, a1=4, a2=4)
    Qp = collide_fast(f, plan, packed=True)
    Qu = collide_fast(f, plan, packed=False)
    # rounding of the gain - loss cancellation: G and L are ~5x |Q| here
    assert np.linalg.norm(Qp - Qu) <= 1e-11 * np.linalg.norm(Qu)


@pytest.mark.parametrize("n", [8, 16])
def test_mass_is_exact(n):
    # beta(-m, m) = 0 with the loss taken by the gain's quadrature: Qhat_0 = 0
    plan, f = _case(n, a1=4, a2=4)
    Q = collide_fast(f, plan)
    # exact up to rounding of the gain - loss difference (a mismatched loss quadrature gives ~1e-2)
    assert abs(Q.sum()) <= 1e-12 * np.abs(Q).sum()


def test_bilinearity_reflection_translation_swap():
    # exact symmetries hold to rounding (~1e-12 of |Q| after the gain - loss
    # cancellation); a broken direction rule or transposed index gives ~1e-1
    plan, f = _case(16, a1=4, a2=4, seed=5)
    Q = collide_fast(f, plan)
    s = np.linalg.norm(Q)
    # Q(c f) = c^2 Q(f)
    assert np.linalg.norm(collide_fast(2.5 * f, plan) - 6.25 * Q) <= 5e-12 * 6.25 * s
    # reflection v -> -v maps grid index j -> (n - j) mod n
    ref = lambda a: np.roll(a[::-1, ::-1, ::-1], 1, axis=(0, 1, 2))
    assert np.linalg.norm(collide_fast(ref(f), plan) - ref(Q)) <= 5e-12 * s
    # translation by whole grid steps commutes with Q (periodic grid)
    tr = lambda a: np.roll(a, (1, -2, 3), axis=(0, 1, 2))
    assert np.linalg.norm(collide_fast(tr(f), plan) - tr(Q)) <= 5e-12 * s
    # swapping v_x and v_y maps the direction set e(theta_p, phi_q) onto itself (A2 = 4)
    sw = lambda a: a.transpose(1, 0, 2)
    assert np.linalg.norm(collide_fast(sw(f), plan) - sw(Q)) <= 5e-12 * s


def test_projection_kills_invariant_moments():
    plan, f = _case(16, a1=4, a2=4)
    Q = collide_fast(f, plan)
    Qc = project(Q, plan.grid)
    U = moments(Qc, plan.grid)
    Ua = moments(np.abs(Q), plan.grid)
    assert np.all(np.abs(U) <= 1e-14 * np.abs(Ua).max() * 10)
    # the projection is the minimum-norm correction: idempotent, and small here
    assert np.linalg.norm(project(Qc, plan.grid) - Qc) <= 1e-14 * np.linalg.norm(Q) * 10


def test_oracle_snapshot_regression():
    with open(os.path.join(GOLDEN, "oracle_snapshot_n8.json")) as fh:
        gold = json.load(fh)
    plan = make_plan(gold["n"], gold["L"], gold["R"], a1=4, a2=4, C=0.25)
    f = fks_inputs.maxwellian_mixture(gold["n"], gold["L"], 1, seed=3)[0]
    Q = collide_fast(f, plan)
    for smp in gold["samples"]:
        assert abs(Q[tuple(smp["index"])] - smp["Q"]) <= 1e-13 * gold["norm"]

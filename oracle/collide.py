"""Fourier-Galerkin collision operator Q(f, f), two independent FP64 evaluators.

Test infrastructure only (see the package header).

O-direct (collide_direct) is the plain definition, eq. CF1 of Appendix A:
    Qhat_k = sum_{l + m = k} beta(l, m) fhat_l fhat_m,
    beta(l, m) = B_F(l, m) - B_F(m, m),
with B_F replaced by its separable quadrature sum_t alpha_t(l) alpha'_t(m) and
B_F(m, m) by lambda(m) (same quadrature), l, m, k all in the truncated mode set
(Galerkin projection).  Then Q(v_j) = sum_k Qhat_k e^{i xi_k . v_j}.  Its cost
is O(N^6 T); it is only run on small grids.

O-fast (collide_fast) is the fast evaluation of the same sum (Appendix A, the
convolution structure of the separable expansion): for every separable term t,
    A_t(v) = sum_l alpha_t(l) fhat_l e^{i xi_l.v},   B_t(v) = sum_m alpha'_t(m) fhat_m e^{i xi_m.v},
are synthesised on a padded grid of P >= 3N/2 points per axis (linear, not
cyclic, convolution over the kept modes), the gain is G = sum_t A_t B_t, the
loss L = f_N * (sum_m lambda(m) fhat_m e^{i xi_m.v}), and Qhat_k is the
coefficient of G - L for the kept modes k.  Because alpha_t, alpha'_t are real
and even and fhat is Hermitian, A_t and B_t are real, so one complex synthesis of
alpha_t fhat + i alpha'_t fhat gives both (packed=True); packed=False does two
separate syntheses as a check of that packing.
"""

import numpy as np
import scipy.fft as sfft

from .grid import fourier_coefficients, synthesize
from .tables import Plan


def _pair_slices(kidx, K, Kh):
    """Index ranges of l and m = k - l (both kept) for one axis, m reversed."""
    lo = max(0, kidx + Kh - (K - 1))
    hi = min(K - 1, kidx + Kh)
    m_hi = kidx + Kh - lo
    m_lo = kidx + Kh - hi
    l_sl = slice(lo, hi + 1)
    m_sl = slice(m_hi, m_lo - 1 if m_lo > 0 else None, -1)
    return l_sl, m_sl


def collide_direct_hat(fh: np.ndarray, plan: Plan) -> np.ndarray:
    """Qhat on the kept modes by the O(N^6) double sum of eq. CF1."""
    K = fh.shape[0]
    Kh = K // 2
    Qh = np.zeros_like(fh)
    A, Ap, lam = plan.A, plan.Ap, plan.lam
    for a in range(K):
        la, ma = _pair_slices(a, K, Kh)
        for b in range(K):
            lb, mb = _pair_slices(b, K, Kh)
            for c in range(K):
                lc, mc = _pair_slices(c, K, Kh)
                # beta(l, k - l) for every admissible l, elementwise aligned
                gain = (A[:, la, lb, lc] * Ap[:, ma, mb, mc]).sum(axis=0)
                beta = gain - lam[ma, mb, mc]
                Qh[a, b, c] = np.sum(beta * fh[la, lb, lc] * fh[ma, mb, mc])
    return Qh


def collide_direct(f: np.ndarray, plan: Plan, return_imag=False):
    g = plan.grid
    fh = fourier_coefficients(f, g)
    Qh = collide_direct_hat(fh, plan)
    Qc = synthesize(Qh, g.xi, g.v)
    if return_imag:
        return Qc.real, np.abs(Qc.imag).max()
    return Qc.real


def _padded_synthesis(coef: np.ndarray, k: np.ndarray, P: int) -> np.ndarray:
    """sum_k coef_k e^{i xi_k . v'_p} on the padded nodes v'_p = -L + p 2L/P.

    xi_k . v'_p = -pi (k1+k2+k3) + 2 pi k.p / P, so this is an inverse DFT of
    size P (times P^3) of coef_k (-1)^{k1+k2+k3} placed at index k mod P.
    """
    sign = (-1.0) ** (k[:, None, None] + k[None, :, None] + k[None, None, :])
    buf = np.zeros((P, P, P), dtype=np.complex128)
    idx = np.mod(k, P)
    buf[np.ix_(idx, idx, idx)] = coef * sign
    return sfft.ifftn(buf, workers=1) * (P ** 3)


def _padded_analysis(G: np.ndarray, k: np.ndarray, P: int) -> np.ndarray:
    """P^-3 sum_p G(v'_p) e^{-i xi_k . v'_p} for the kept modes k."""
    F = sfft.fftn(G, workers=1)
    idx = np.mod(k, P)
    sign = (-1.0) ** (k[:, None, None] + k[None, :, None] + k[None, None, :])
    return F[np.ix_(idx, idx, idx)] * sign / (P ** 3)


def collide_fast_hat(fh: np.ndarray, plan: Plan, P=None, packed=True) -> np.ndarray:
    g = plan.grid
    P = plan.P if P is None else P
    k = g.k
    G = np.zeros((P, P, P))
    terms = [(plan.A[t], plan.Ap[t]) for t in range(plan.n_terms)]
    terms.append((-np.ones_like(plan.lam), plan.lam))     # the loss, with its sign
    for a_w, b_w in terms:
        if packed:
            Z = _padded_synthesis(a_w * fh + 1j * (b_w * fh), k, P)
            G += Z.real * Z.imag
        else:
            Az = _padded_synthesis(a_w * fh, k, P)
            Bz = _padded_synthesis(b_w * fh, k, P)
            G += Az.real * Bz.real
    return _padded_analysis(G, k, P)


def collide_fast(f: np.ndarray, plan: Plan, P=None, packed=True, return_imag=False):
    g = plan.grid
    fh = fourier_coefficients(f, g)
    Qh = collide_fast_hat(fh, plan, P=P, packed=packed)
    Qc = synthesize(Qh, g.xi, g.v)
    if return_imag:
        return Qc.real, np.abs(Qc.imag).max()
    return Qc.real


def collide_fast_batch(fs: np.ndarray, plan: Plan, P=None) -> np.ndarray:
    """O-fast over a batch of cells, fs shape (C, n, n, n)."""
    return np.stack([collide_fast(fs[c], plan, P=P) for c in range(fs.shape[0])])


def loss_field(f: np.ndarray, plan: Plan) -> np.ndarray:
    """L(v_j) = f_N(v_j) * sum_m lambda(m) fhat_m e^{i xi_m.v_j} (the loss half of Q)."""
    g = plan.grid
    fh = fourier_coefficients(f, g)
    fN = synthesize(fh, g.xi, g.v).real
    nu = synthesize(plan.lam * fh, g.xi, g.v).real
    return fN * nu

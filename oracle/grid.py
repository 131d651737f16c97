"""Velocity grid, Fourier modes, coefficients and synthesis (FP64).

Test infrastructure only (see the package header).

Conventions (paper Section 2.1 "equally spaced" DVM grid, and Appendix A
Fourier expansion of the periodised f):
  * velocity points v_j = -L + j*dv, dv = 2L/n, j = 0..n-1 per axis;
  * modes k in the symmetric set {-n/2+1, ..., n/2-1} per axis (the Nyquist
    plane is dropped so every real f has a Hermitian coefficient set);
  * wave numbers xi_k = pi*k/L (the paper's T = pi gives xi = k);
  * coefficients fhat_k = (2L)^-3 * integral f e^{-i xi_k.v} dv, evaluated
    with the rectangle rule on the grid, i.e. (1/n^3) sum_j f(v_j) e^{-i xi_k.v_j};
  * synthesis f(v) = sum_k fhat_k e^{+i xi_k.v}.
Everything is written with the explicit physical phases e^{+-i xi_k.v}; no
shifted-FFT shortcut is used here.
"""

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Grid:
    n: int          # points per axis
    L: float        # box half-width, grid on [-L, L)
    dv: float       # grid step 2L/n
    v: np.ndarray   # (n,) 1D velocity nodes
    k: np.ndarray   # (n-1,) signed modes -n/2+1..n/2-1
    xi: np.ndarray  # (n-1,) wave numbers pi*k/L


def make_grid(n: int, L: float) -> Grid:
    if n % 2 or n < 4:
        raise ValueError("n must be even and >= 4")
    dv = 2.0 * L / n
    v = -L + np.arange(n) * dv
    k = np.arange(-n // 2 + 1, n // 2)
    xi = np.pi * k / L
    return Grid(n=n, L=float(L), dv=dv, v=v, k=k, xi=xi)


def _axis_forward_matrix(g: Grid) -> np.ndarray:
    """E[a, j] = exp(-i xi_a v_j) / n  (one axis of the rectangle-rule transform)."""
    return np.exp(-1j * np.outer(g.xi, g.v)) / g.n


def _axis_synthesis_matrix(xi: np.ndarray, v: np.ndarray) -> np.ndarray:
    """S[j, a] = exp(+i xi_a v_j)."""
    return np.exp(1j * np.outer(v, xi))


def fourier_coefficients(f: np.ndarray, g: Grid) -> np.ndarray:
    """fhat[a,b,c] for modes (k_a, k_b, k_c); f has shape (n, n, n) (Appendix A)."""
    E = _axis_forward_matrix(g)
    out = np.einsum("aj,jkl->akl", E, f.astype(np.complex128))
    out = np.einsum("bk,akl->abl", E, out)
    out = np.einsum("cl,abl->abc", E, out)
    return out


def synthesize(coef: np.ndarray, xi: np.ndarray, v: np.ndarray) -> np.ndarray:
    """sum_k coef_k exp(i xi_k . v) evaluated on the tensor grid v x v x v."""
    S = _axis_synthesis_matrix(xi, v)
    out = np.einsum("ja,abc->jbc", S, coef)
    out = np.einsum("kb,jbc->jkc", S, out)
    out = np.einsum("lc,jkc->jkl", S, out)
    return out


def mode_vectors(g: Grid) -> np.ndarray:
    """xi vectors of all modes, shape (n-1, n-1, n-1, 3)."""
    X, Y, Z = np.meshgrid(g.xi, g.xi, g.xi, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def velocity_vectors(g: Grid) -> np.ndarray:
    """velocity vectors of all grid points, shape (n, n, n, 3)."""
    X, Y, Z = np.meshgrid(g.v, g.v, g.v, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)

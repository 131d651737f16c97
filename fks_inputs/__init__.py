"""Seeded synthetic inputs shared by the oracle checks, the GPU tests and the bench.

This module only samples distribution functions on the velocity grid; it holds
none of the collision method's arithmetic.  Grid convention: v_j = -L + j*(2L/n),
j = 0..n-1 per axis, arrays indexed [cell][i][j][k] with k fastest (v_z).

Recipes (stated with the workloads they stand for):
  * maxwellian_mixture: batches of two-Maxwellian mixtures, densities
    U[0.5, 1.5], mean velocities N(0, 1)^3, temperatures U[0.5, 2]; the spread of
    states a space-inhomogeneous FKS run sees in its cells.
  * perturbed_maxwellians: f = (1 - a) M1 + a M2, a ~ U[0, 0.3], each Maxwellian
    drawn with the mixture laws above (near-equilibrium surrogate training data).
  * sod_box / wave_box: periodic spatial boxes of cells in local equilibrium
    (the 3D Sod explosion initial state of the paper's Section 5, and a
    sinusoidal density perturbation of a unit Maxwellian).
  * bkw_initial: the Bobylev-Krook-Wu profile for Maxwell molecules.
  * mlp_init: seeded initial weights of the surrogate network (random inputs of its
    training, drawn here so that the device and the reference start alike).
"""

import numpy as np


def velocity_axis(n, L):
    return -L + np.arange(n) * (2.0 * L / n)


def maxwellian_on_grid(n, L, rho, u, T):
    """rho (C,), u (C,3), T (C,) -> (C, n, n, n) float64."""
    v = velocity_axis(n, L)
    rho = np.asarray(rho, dtype=np.float64).reshape(-1)
    u = np.asarray(u, dtype=np.float64).reshape(-1, 3)
    T = np.asarray(T, dtype=np.float64).reshape(-1)
    gx = np.exp(-(v[None, :] - u[:, 0:1]) ** 2 / (2.0 * T[:, None]))
    gy = np.exp(-(v[None, :] - u[:, 1:2]) ** 2 / (2.0 * T[:, None]))
    gz = np.exp(-(v[None, :] - u[:, 2:3]) ** 2 / (2.0 * T[:, None]))
    norm = rho * (2.0 * np.pi * T) ** -1.5
    return norm[:, None, None, None] * gx[:, :, None, None] * gy[:, None, :, None] * gz[:, None, None, :]


def mixture_params(n_cells, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 1.5, (n_cells, 2))
    u = rng.standard_normal((n_cells, 2, 3))
    T = rng.uniform(0.5, 2.0, (n_cells, 2))
    return rho, u, T


def maxwellian_mixture(n, L, n_cells, seed=1701, chunk=256):
    """(n_cells, n, n, n) float64 two-Maxwellian mixtures from the seeded laws."""
    rho, u, T = mixture_params(n_cells, seed)
    out = np.empty((n_cells, n, n, n), dtype=np.float64)
    for c0 in range(0, n_cells, chunk):
        c1 = min(n_cells, c0 + chunk)
        out[c0:c1] = (maxwellian_on_grid(n, L, rho[c0:c1, 0], u[c0:c1, 0], T[c0:c1, 0])
                      + maxwellian_on_grid(n, L, rho[c0:c1, 1], u[c0:c1, 1], T[c0:c1, 1]))
    return out


def perturbed_maxwellians(n, L, n_cells, seed=1, amp=0.3):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 1.5, (n_cells, 2))
    u = rng.standard_normal((n_cells, 2, 3))
    T = rng.uniform(0.5, 2.0, (n_cells, 2))
    a = rng.uniform(0.0, amp, n_cells)
    m1 = maxwellian_on_grid(n, L, rho[:, 0], u[:, 0], T[:, 0])
    m2 = maxwellian_on_grid(n, L, rho[:, 1], u[:, 1], T[:, 1])
    return (1.0 - a)[:, None, None, None] * m1 + a[:, None, None, None] * m2


def perturbed_maxwellians_device(n, L, n_cells, seed=1, amp=0.3, device="cuda", dtype=None):
    """perturbed_maxwellians with the same seeded parameters, evaluated on a torch device
    (large training sets without the host round trip).  Returns (n_cells, n, n, n)."""
    import torch
    dtype = torch.float32 if dtype is None else dtype
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.5, 1.5, (n_cells, 2))
    u = rng.standard_normal((n_cells, 2, 3))
    T = rng.uniform(0.5, 2.0, (n_cells, 2))
    a = rng.uniform(0.0, amp, n_cells)
    v = torch.as_tensor(velocity_axis(n, L), dtype=torch.float64, device=device)
    out = torch.zeros((n_cells, n, n, n), dtype=torch.float64, device=device)
    w = np.stack([1.0 - a, a], axis=1)
    for m in range(2):
        uu = torch.as_tensor(u[:, m], device=device)
        TT = torch.as_tensor(T[:, m], device=device)[:, None]
        g = [torch.exp(-(v[None, :] - uu[:, d:d + 1]) ** 2 / (2.0 * TT)) for d in range(3)]
        norm = torch.as_tensor(w[:, m] * rho[:, m] * (2.0 * np.pi * T[:, m]) ** -1.5, device=device)
        out += norm[:, None, None, None] * g[0][:, :, None, None] * g[1][:, None, :, None] * g[2][:, None, None, :]
    return out.to(dtype)


def mlp_init(sizes, seed):
    """Seeded initial parameters of a multilayer perceptron with layer sizes `sizes`:
    W1, b1, W2, b2, ... with weights [out][in] drawn He-uniform U(-sqrt(6/fan_in),
    sqrt(6/fan_in)) (the last layer scaled by 0.1) and zero biases, FP64."""
    rng = np.random.default_rng(seed)
    params = []
    for i in range(len(sizes) - 1):
        bound = np.sqrt(6.0 / sizes[i])
        W = rng.uniform(-bound, bound, (sizes[i + 1], sizes[i]))
        if i == len(sizes) - 2:
            W *= 0.1
        params += [W, np.zeros(sizes[i + 1])]
    return params


def wave_box(n, L, shape, amp=0.1, rho0=1.0, T0=1.0):
    """Cells of a periodic box [0,2)^3 (dx = 2/nx): f = (1 + amp sin(pi x1)) M_{1,0,1}(v).

    Returns (nx*ny*nz, n, n, n) float64, cells in C order of shape."""
    nx, ny, nz = shape
    dx = 2.0 / nx
    x1 = (np.arange(nx) + 0.5) * dx
    M = maxwellian_on_grid(n, L, [rho0], [[0.0, 0.0, 0.0]], [T0])[0]
    dens = 1.0 + amp * np.sin(np.pi * x1)
    out = np.empty((nx, ny, nz, n, n, n))
    out[:] = M
    out *= dens[:, None, None, None, None, None]
    return out.reshape(nx * ny * nz, n, n, n)


def sod_box(n, L, shape):
    """3D explosion state on [0,2)^3: rho=1, T=5 inside the ball |x-(1,1,1)|<0.2, rho=0.125, T=4 outside."""
    nx, ny, nz = shape
    xs = [(np.arange(m) + 0.5) * (2.0 / m) for m in shape]
    X, Y, Z = np.meshgrid(*xs, indexing="ij")
    inside = ((X - 1) ** 2 + (Y - 1) ** 2 + (Z - 1) ** 2) < 0.04
    rho = np.where(inside, 1.0, 0.125).reshape(-1)
    T = np.where(inside, 5.0, 4.0).reshape(-1)
    u = np.zeros((rho.size, 3))
    return maxwellian_on_grid(n, L, rho, u, T)


def bkw_initial(n, L, t0=5.5):
    """BKW profile for Maxwell molecules (density 1, temperature 1) at time t0."""
    v = velocity_axis(n, L)
    K = 1.0 - np.exp(-t0 / 6.0)
    r2 = v[:, None, None] ** 2 + v[None, :, None] ** 2 + v[None, None, :] ** 2
    c = 0.5 * (2.0 * np.pi * K) ** -1.5
    return c * np.exp(-r2 / (2.0 * K)) * ((5.0 * K - 3.0) / K + (1.0 - K) * r2 / K ** 2)

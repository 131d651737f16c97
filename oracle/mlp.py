"""FP64 reference of the Fourier-mode MLP surrogate (forward, backward, Adam).

Test infrastructure only (see the package header).  Not part of the paper: the learned
surrogate of the collision operator is an addition of this project; this module is the
plain reference its GPU training kernels are checked against.

Network: x (features) -> h1 = silu(x W1^T + b1) -> h2 = silu(h1 W2^T + b2) -> y = h2 W3^T + b3,
weights stored [out][in] (row-major), silu(z) = z sigma(z).
Loss: mean squared error over all outputs, L = sum (y - t)^2 / (batch * n_out).
Backward written out by the chain rule:
    dy = 2 (y - t) / (batch n_out);  dW3 = dy^T h2;  db3 = sum_rows dy;  dh2 = dy W3;
    dz2 = dh2 silu'(z2);  dW2 = dz2^T h1; ...;  silu'(z) = s (1 + z (1 - s)), s = sigma(z).
Adam (Kingma & Ba): m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
    p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""

import numpy as np


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def init_params(sizes, seed):
    """He-uniform weights [out][in] and zero biases: the seeded input generator shared
    with the device runs (fks_inputs.mlp_init)."""
    from fks_inputs import mlp_init
    return mlp_init(sizes, seed)


def forward(params, x):
    cache = [x]
    h = x
    n_layers = len(params) // 2
    zs = []
    for i in range(n_layers):
        W, b = params[2 * i], params[2 * i + 1]
        z = h @ W.T + b
        zs.append(z)
        h = silu(z) if i < n_layers - 1 else z
        cache.append(h)
    return h, (cache, zs)


def loss_and_grads(params, x, t):
    y, (cache, zs) = forward(params, x)
    n = y.size
    loss = float(np.sum((y - t) ** 2) / n)
    grads = [None] * len(params)
    d = 2.0 * (y - t) / n
    n_layers = len(params) // 2
    for i in reversed(range(n_layers)):
        W = params[2 * i]
        h_in = cache[i]
        grads[2 * i] = d.T @ h_in
        grads[2 * i + 1] = d.sum(axis=0)
        if i > 0:
            d = (d @ W) * dsilu(zs[i - 1])
    return loss, grads


class Adam:
    def __init__(self, params, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        out = []
        for p, g, m, v in zip(params, grads, self.m, self.v):
            m *= self.b1
            m += (1 - self.b1) * g
            v *= self.b2
            v += (1 - self.b2) * g * g
            mh = m / (1 - self.b1 ** self.t)
            vh = v / (1 - self.b2 ** self.t)
            out.append(p - self.lr * mh / (np.sqrt(vh) + self.eps))
        return out


# ---- surrogate inputs and checks -------------------------------------------------------
def mean_velocity(f, L):
    """u = sum v f / sum f on the velocity grid of f (n, n, n)."""
    from .grid import make_grid
    v = make_grid(f.shape[0], L).v
    m = f.sum()
    return np.array([np.tensordot(f.sum(axis=(1, 2)), v, 1), np.tensordot(f.sum(axis=(0, 2)), v, 1),
                     np.tensordot(f.sum(axis=(0, 1)), v, 1)]) / m


def spectral_shift(f, delta, L):
    """g(v) = f(v + delta) for the Fourier interpolant of the grid samples f (n, n, n)
    (the Nyquist modes dropped, as in the method's mode set), one axis after the other."""
    n = f.shape[0]
    k = np.arange(n // 2 + 1)
    g = np.asarray(f, dtype=np.float64)
    for ax in range(3):
        F = np.fft.rfft(g, axis=ax)
        ph = np.exp(1j * np.pi * k * delta[ax] / L)
        ph[n // 2] = 0.0
        shape = [1, 1, 1]
        shape[ax] = n // 2 + 1
        g = np.fft.irfft(F * ph.reshape(shape), n=n, axis=ax)
    return g


def features(f, L, modes, center=False):
    """Network input of one cell: Re, Im (interleaved) of fhat_k / fhat_0 for
    k in [-modes/2, modes/2 - 1]^3 (k_z fastest), fhat the Appendix A coefficients of
    the grid samples f (n, n, n) (with center: of f(v + u), u the mean velocity, i.e.
    fhat_k e^{i xi_k.u}); and the density rho = (2L)^3 fhat_0."""
    from .grid import fourier_coefficients, make_grid
    n = f.shape[0]
    g = make_grid(n, L)
    fh = fourier_coefficients(f, g)
    if center:
        u = mean_velocity(f, L)
        X, Y, Z = np.meshgrid(g.xi, g.xi, g.xi, indexing="ij")
        fh = fh * np.exp(1j * (X * u[0] + Y * u[1] + Z * u[2]))
    c = n // 2 - 1                       # index of k = 0
    mh = modes // 2
    sub = fh[c - mh:c + mh, c - mh:c + mh, c - mh:c + mh] / fh[c, c, c]
    x = np.empty(2 * sub.size)
    x[0::2] = sub.real.ravel()
    x[1::2] = sub.imag.ravel()
    rho = float((2.0 * L) ** 3 * fh[c, c, c].real)
    return x, rho


def moment_indicator(q, L):
    """max over phi in (1, v_x, v_y, v_z, |v|^2/2) of |sum phi q| / sum |phi| |q| on the
    velocity grid of q (n, n, n): zero for an operator that conserves mass, momentum and
    energy (Section 3 macroscopic variables)."""
    from .grid import make_grid
    n = q.shape[0]
    v = make_grid(n, L).v
    vx, vy, vz = np.meshgrid(v, v, v, indexing="ij")
    r = 0.0
    for phi in (np.ones_like(vx), vx, vy, vz, 0.5 * (vx * vx + vy * vy + vz * vz)):
        r = max(r, abs(np.sum(phi * q)) / np.sum(np.abs(phi) * np.abs(q)))
    return r

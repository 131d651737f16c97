"""Error measures of the GPU parity tests (relative L2 over a batch and per cell)."""

import numpy as np


def rel(a, b):
    """Relative L2 error of a against b over everything."""
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def cell_errors(q, ref, floor=None):
    """Per-cell relative L2 errors ||q_c - ref_c|| / ||ref_c|| of batches [cells][n][n][n].

    floor (optional, per cell): a norm to use where ||ref_c|| is smaller, e.g. the norm of
    the loss half L for a cell at equilibrium, where Q nearly vanishes."""
    q = np.asarray(q).reshape(len(q), -1)
    ref = np.asarray(ref).reshape(len(ref), -1)
    den = np.linalg.norm(ref, axis=1)
    if floor is not None:
        den = np.maximum(den, np.asarray(floor, dtype=np.float64))
    return np.linalg.norm(q - ref, axis=1) / den


def loss_floor(fs, op, frac=0.1):
    """Per-cell floor frac * ||L|| (L the oracle's loss half of Q).  FP32 rounding of the
    gain and loss terms leaves an error proportional to their size, so a cell close to
    equilibrium, where Q = G - L nearly cancels, is measured against a fraction of ||L||."""
    from oracle.collide import loss_field
    return np.array([frac * np.linalg.norm(loss_field(np.asarray(f, dtype=np.float64), op)) for f in fs])


def assert_parity(q, ref, tol, label="", floor=None):
    """Batch relative L2 and the per-cell maximum both within tol; prints median and max."""
    batch = rel(np.asarray(q), np.asarray(ref))
    per = cell_errors(q, ref, floor)
    print(f"{label} rel-L2 batch {batch:.3e}, per cell median {np.median(per):.3e} max {per.max():.3e}",
          flush=True)
    assert batch <= tol, (label, batch)
    assert per.max() <= tol, (label, per.max(), int(per.argmax()))
    return batch, per

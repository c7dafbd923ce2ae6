"""Small statistics helpers for the tests (no lattice arithmetic here)."""
import numpy as np


def batch_mean_err(x, n_batches=20):
    """Mean and standard error from non-overlapping batch means (axis 0)."""
    x = np.asarray(x)
    n = (x.shape[0] // n_batches) * n_batches
    b = x[:n].reshape((n_batches, n // n_batches) + x.shape[1:]).mean(axis=1)
    return x[:n].mean(axis=0), b.std(axis=0, ddof=1) / np.sqrt(n_batches)


def circ_dist(a, b):
    """|wrap(a - b)| on the circle."""
    d = np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64)
    return np.abs((d + np.pi) % (2 * np.pi) - np.pi)

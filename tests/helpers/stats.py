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


def check_sigma(z, dof, k_sigma=3.0, alpha=1e-3):
    """Multiple-comparison check of normalised differences z (|difference| /
    combined standard error, each error estimated with dof degrees of
    freedom): with p = P(|t_dof| > k_sigma), the number of |z| above k_sigma
    may be at most the smallest k with P(Binomial(N, p) > k) < alpha, and no
    |z| may exceed the Bonferroni bound t_dof quantile at 1 - alpha / (2 N).
    Returns (ok, count above k_sigma, allowed count, largest |z|, bound)."""
    from scipy import stats

    z = np.abs(np.ravel(np.asarray(z, float)))
    N = z.size
    p = 2 * stats.t.sf(k_sigma, dof)
    allowed = 0
    while stats.binom.sf(allowed, N, p) >= alpha:
        allowed += 1
    bound = stats.t.isf(alpha / (2 * N), dof)
    count = int(np.sum(z > k_sigma))
    zmax = float(z.max()) if N else 0.0
    return count <= allowed and zmax <= bound, count, allowed, zmax, float(bound)

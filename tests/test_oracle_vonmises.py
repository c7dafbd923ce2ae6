"""Oracle von Mises sampler (Best--Fisher 1979) pins.

The draws are compared with the exact von Mises density
exp(kappa cos psi) / (2 pi I_0(kappa)): a chi-square test over 64 bins of
exactly integrated probabilities, and the circular moments
E[cos psi] = I_1/I_0, E[cos 2 psi] = I_2/I_0.
"""
import numpy as np
import pytest
from scipy import integrate, special
from scipy.stats import chi2

N = 200_000


def _bin_probs(kappa, nb=64):
    edges = np.linspace(-np.pi, np.pi, nb + 1)
    norm = 2 * np.pi * special.ive(0, kappa)
    f = lambda x: np.exp(kappa * (np.cos(x) - 1.0)) / norm
    return np.array([integrate.quad(f, edges[i], edges[i + 1])[0] for i in range(nb)]), edges


@pytest.mark.parametrize("kappa", [0.0, 1e-8, 0.5, 3.0, 6.0, 20.0])
def test_vonmises_histogram(orc, kappa):
    psi, attempts = orc.vonmises_many(kappa, N, seed=17, key_id=int(kappa * 10) + 1)
    assert np.all(np.isfinite(psi))
    assert np.all(np.abs(psi) <= np.pi)
    p, edges = _bin_probs(kappa)
    counts, _ = np.histogram(psi, bins=edges)
    expect = p * N
    keep = expect > 5
    stat = np.sum((counts[keep] - expect[keep]) ** 2 / expect[keep])
    dof = keep.sum() - 1
    assert chi2.sf(stat, dof) > 1e-4, (kappa, stat, dof)
    # Best--Fisher envelope efficiency is above 0.65 for every kappa
    assert attempts / N < 1.6


@pytest.mark.parametrize("kappa", [0.5, 3.0, 6.0, 20.0])
def test_vonmises_moments(orc, kappa):
    psi, _ = orc.vonmises_many(kappa, N, seed=99, key_id=int(kappa * 10))
    for m in (1, 2):
        exact = special.iv(m, kappa) / special.iv(0, kappa)
        c = np.cos(m * psi)
        err = c.std() / np.sqrt(N)
        assert abs(c.mean() - exact) < 5 * err, (kappa, m, c.mean(), exact)
    s = np.sin(psi)
    assert abs(s.mean()) < 5 * s.std() / np.sqrt(N)


def test_vonmises_moment_values_kappa3_kappa6():
    # I_1/I_0 and I_2/I_0 at kappa = 3 and 6 (40-digit mpmath values)
    import mpmath as mp

    for kappa, m1, m2 in [(3, 0.809985293956505, 0.460009804028997), (6, 0.912359304352915, 0.695880231882362)]:
        assert abs(float(mp.besseli(1, kappa) / mp.besseli(0, kappa)) - m1) < 1e-14
        assert abs(float(mp.besseli(2, kappa) / mp.besseli(0, kappa)) - m2) < 1e-14


def test_naive_rho_cancels_at_small_kappa():
    # Why the oracle uses the rearranged envelope parameter: the textbook
    # rho = (tau - sqrt(2 tau)) / (2 kappa) loses every digit at kappa = 1e-8.
    k = 1e-8
    tau = 1 + np.sqrt(1 + 4 * k * k)
    naive = (tau - np.sqrt(2 * tau)) / (2 * k)
    s = np.sqrt(1 + 4 * k * k)
    good = 2 * k * tau / ((s + 1) * (tau + np.sqrt(2 * tau)))
    assert naive == 0.0
    assert abs(good - k / 2) < 1e-20

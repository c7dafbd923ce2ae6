"""Exact finite-volume results of 2D compact U(1) on an L x T torus.

With N = L*T plaquettes, the plaquette angles are independent up to the single
constraint that their sum vanishes mod 2 pi, so for integer charges q_p
    < prod_p exp(i q_p theta_p) > = sum_n prod_p I_{n+q_p}(beta) / sum_n I_n(beta)^N.
P^dagger(x) P(x+r) is the product of the r*T plaquettes of the strip between the
two lines (all with charge +1).  These are closed forms (Bessel sums), computed
here with mpmath, independent of any simulation code.
"""
import mpmath as mp

mp.mp.dps = 40
_NMAX = 60


_cache = {}


def _I(n, beta):
    """Modified Bessel I_n(beta); I_{-n} = I_n for integer n."""
    key = (abs(n), mp.mpf(beta))
    if key not in _cache:
        _cache[key] = mp.besseli(abs(n), mp.mpf(beta))
    return _cache[key]


def _sum(beta, factors):
    """sum_n prod (I_{n+q}^power) over factors [(q, power), ...]."""
    tot = mp.mpf(0)
    for n in range(-_NMAX, _NMAX + 1):
        term = mp.mpf(1)
        for q, pw in factors:
            if pw:
                term *= _I(n + q, beta) ** pw
        tot += term
    return tot


def Z(beta, N):
    return _sum(beta, [(0, N)])


def plaquette(beta, L, T):
    N = L * T
    return float(_sum(beta, [(0, N - 1), (1, 1)]) / Z(beta, N))


def polyakov_corr(beta, L, T, r):
    N, A = L * T, r * T
    return float(_sum(beta, [(0, N - A), (1, A)]) / Z(beta, N))


def insertion(beta, L, T, r, inside, sign):
    """< P^dagger P exp(sign * i theta_p) > for one plaquette p inside / outside the strip."""
    N, A = L * T, r * T
    if inside:
        f = [(0, N - A), (1, A - 1), (1 + sign, 1)]
    else:
        f = [(0, N - A - 1), (1, A), (sign, 1)]
    return float(_sum(beta, f) / Z(beta, N))

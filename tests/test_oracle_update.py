"""Oracle link-update pins: staple against the action, overrelaxation invariants,
gauge covariance of heatbath + overrelaxation, the heatbath's conditional
distribution in a frozen environment, and a brute-force checkerboard validator.
"""
import itertools

import numpy as np
import pytest
from scipy import integrate, special
from scipy.stats import chi2

from helpers.stats import circ_dist


def _coords(L, site):
    c = []
    for n in L:
        c.append(site % n)
        site //= n
    return c


def _site(L, c):
    s = 0
    for k in reversed(range(len(L))):
        s = s * L[k] + (c[k] % L[k])
    return s


def _random_lattice(orc, d, L, beta, seed=1, key_id=0):
    lat = orc.Lattice(d, L, beta, seed=seed, key_id=key_id)
    lat.init(1)
    return lat


def _all_plaquettes(lat):
    d, V = lat.d, lat.V
    return np.array([[lat.plaq_angle(s, a, b) for a, b in itertools.combinations(range(d), 2)] for s in range(V)])


@pytest.mark.parametrize("d,L", [(4, [4, 4, 4, 4]), (2, [6, 4])])
def test_staple_reproduces_local_action(orc, d, L):
    """sum over the plaquettes that contain the link of cos(theta_P) = |A| cos(theta + arg A)."""
    lat = _random_lattice(orc, d, L, 1.0, seed=5)
    th0 = lat.links()
    rng = np.random.default_rng(0)
    for _ in range(6):
        site, mu = int(rng.integers(lat.V)), int(rng.integers(d))
        lid = mu + d * site
        P0 = _all_plaquettes(lat)
        th = th0.copy()
        th[lid] += 0.3
        lat.set_links(th)
        changed = np.abs(np.sin((_all_plaquettes(lat) - P0) / 2)) > 1e-9
        assert changed.sum() == 2 * (d - 1)
        lat.set_links(th0)
        A = lat.staple(site, mu)
        for val in (th0[lid], 0.0, 1.234, -2.9):
            th = th0.copy()
            th[lid] = val
            lat.set_links(th)
            P = _all_plaquettes(lat)
            lhs = np.cos(P[changed]).sum()
            rhs = abs(A) * np.cos(val + np.angle(A))
            assert abs(lhs - rhs) < 1e-12
        lat.set_links(th0)


def test_overrelaxation_invariants(orc):
    lat = _random_lattice(orc, 4, [4, 4, 4, 4], 1.0, seed=8)
    rng = np.random.default_rng(1)
    for _ in range(20):
        site, mu = int(rng.integers(lat.V)), int(rng.integers(4))
        lid = mu + 4 * site
        A = lat.staple(site, mu)
        t0 = lat.links()[lid]
        lat.overrelax_link(site, mu)
        t1 = lat.links()[lid]
        assert abs((np.exp(1j * t1) * A).real - (np.exp(1j * t0) * A).real) < 1e-13
        assert circ_dist(t1, t0) > 0 or abs(np.sin(t0 + np.angle(A))) < 1e-12
        lat.overrelax_link(site, mu)
        assert circ_dist(lat.links()[lid], t0) < 1e-13


def _gauge_transform(d, L, th, alpha):
    """theta'_mu(x) = theta_mu(x) + alpha(x) - alpha(x + mu)."""
    out = th.copy()
    V = int(np.prod(L))
    for s in range(V):
        c = _coords(L, s)
        for mu in range(d):
            cp = list(c)
            cp[mu] += 1
            out[mu + d * s] = th[mu + d * s] + alpha[s] - alpha[_site(L, cp)]
    return out


@pytest.mark.parametrize("d,L,beta", [(4, [4, 4, 4, 4], 1.0), (2, [6, 4], 1.5)])
@pytest.mark.parametrize("kind,tau", [(0, 0), (1, 0), (0, 2), (1, 4)])
def test_gauge_covariance_of_pass(orc, d, L, beta, kind, tau):
    """Updating the gauge-transformed links with the same random numbers gives the
    gauge transform of the updated links.  One pass at a time: overrelaxation
    amplifies rounding-level differences about 30x per pass (arg A moves by
    delta/|A| when a staple link moves by delta), so longer comparisons would
    measure that amplification rather than the update's correctness."""
    lat1 = _random_lattice(orc, d, L, beta, seed=21, key_id=3)
    lat1.sweeps(2)
    th = lat1.links()
    alpha = np.random.default_rng(4).uniform(-np.pi, np.pi, int(np.prod(L)))
    lat2 = orc.Lattice(d, L, beta, seed=21, key_id=3)
    lat2.set_links(_gauge_transform(d, L, th, alpha))
    lat2.counter = lat1.counter
    P_before = _all_plaquettes(lat1)
    assert np.max(circ_dist(_all_plaquettes(lat2), P_before)) < 1e-12  # plaquettes are invariant
    lat1.pass_(kind, tau)
    lat2.pass_(kind, tau)
    expect = _gauge_transform(d, L, lat1.links(), alpha)
    # within a pass, the eight phases already feed each other's rounding
    # differences forward (measured up to ~2e-12 for one overrelaxation pass)
    assert np.max(circ_dist(lat2.links(), expect)) < 1e-11


def test_heatbath_conditional_distribution(orc):
    """With the environment frozen, theta + arg A ~ von Mises(0, beta |A|)."""
    beta = 1.3
    lat = _random_lattice(orc, 4, [4, 4, 4, 4], beta, seed=31)
    site, mu = 77, 2
    A = lat.staple(site, mu)
    kappa = beta * abs(A)
    N = 40_000
    vals = np.empty(N)
    lid = mu + 4 * site
    for i in range(N):
        lat.counter = i
        lat.heatbath_link(site, mu)
        vals[i] = lat.links()[lid]
    psi = (vals + np.angle(A) + np.pi) % (2 * np.pi) - np.pi
    edges = np.linspace(-np.pi, np.pi, 33)
    norm = 2 * np.pi * special.ive(0, kappa)
    f = lambda x: np.exp(kappa * (np.cos(x) - 1.0)) / norm
    p = np.array([integrate.quad(f, edges[i], edges[i + 1])[0] for i in range(32)])
    counts, _ = np.histogram(psi, bins=edges)
    keep = p * N > 5
    stat = np.sum((counts[keep] - p[keep] * N) ** 2 / (p[keep] * N))
    assert chi2.sf(stat, keep.sum() - 1) > 1e-4


def _staple_map(L, d):
    """Brute force: for every link, the set of other links that share a plaquette with it."""
    out = {}
    for y in range(int(np.prod(L))):
        cy = _coords(L, y)
        for a, b in itertools.combinations(range(d), 2):
            ca = list(cy)
            ca[a] += 1
            cb = list(cy)
            cb[b] += 1
            links = {(y, a), (_site(L, ca), b), (_site(L, cb), a), (y, b)}
            for l in links:
                out.setdefault(l, set()).update(links - {l})
    return out


@pytest.mark.parametrize("L", [[4, 4, 4, 4], [2, 2, 2, 4]])
def test_checkerboard_schedule(orc, L):
    """Each phase writes exactly the non-frozen links of one (mu, parity), and no
    link written in a phase lies in the staple of another link of that phase."""
    d = 4
    V = int(np.prod(L))
    lat = _random_lattice(orc, d, L, 1.0, seed=2)
    smap = _staple_map(L, d)
    for mu in range(d):
        for p in range(2):
            members = [s for s in range(V) if sum(_coords(L, s)) % 2 == p]
            mset = {(s, mu) for s in members}
            for s in members:
                assert not (smap[(s, mu)] & mset)
            for tau in (0, 2, 4):
                before = lat.links()
                lat.counter = lat.counter + 1  # fresh random numbers for every trial
                lat.phase(0, mu, p, tau)
                after = lat.links()
                changed = {(i // d, i % d) for i in np.nonzero(after != before)[0]}
                expect = {(s, mu) for s in members
                          if not (tau > 1 and mu < 3 and _coords(L, s)[3] % tau == 0)}
                assert changed == expect, (mu, p, tau)


def test_overrelaxation_conditioning(orc):
    """The dynamics itself amplifies rounding-level differences: links perturbed
    by 1e-15 drift apart by more than 1e-9 within one sweep, almost all of it
    in the overrelaxation passes.  This is why GPU-vs-oracle comparisons of
    whole sweeps use the oracle's own response as their tolerance."""
    from helpers.inputs import random_links

    th = random_links(256, 12)
    a = orc.Lattice(4, [4, 4, 4, 4], 1.0, seed=1)
    b = orc.Lattice(4, [4, 4, 4, 4], 1.0, seed=1)
    a.set_links(th)
    b.set_links(th + np.random.default_rng(0).uniform(-1e-15, 1e-15, th.size))
    devs = []
    for k in range(4):
        a.pass_(0 if k == 0 else 1, 0)
        b.pass_(0 if k == 0 else 1, 0)
        devs.append(circ_dist(a.links(), b.links()).max())
    assert devs[0] < 1e-12
    assert devs[3] > 1e-9 and devs[3] < 1e-4

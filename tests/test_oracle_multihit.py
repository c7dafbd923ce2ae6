"""Oracle analytic multihit (Sec. II.C) of the temporal links in the
correlator averages, pinned to:
 - I_1/I_0 from an independent Bessel implementation (scipy);
 - the conditional mean e^{-i arg A} I_1/I_0(beta|A|) against direct numerical
   integration of e^{i theta} exp(beta Re(e^{i theta} A));
 - unchanged expectations: the exact 2D torus Polyakov correlator (one and two
   levels, including the neighbouring separations where only one end may be
   replaced) and the exact 2D plaquette insertions;
 - smaller errors than the plain estimator on the same chain.
"""
import numpy as np
import pytest
from scipy import integrate, special

from helpers import exact2d as E
from helpers.stats import batch_mean_err


def test_bessel_ratio_matches_scipy(orc):
    for k in [0.0, 1e-9, 1e-3, 0.2, 0.9, 1.7, 3.3, 6.0, 11.0, 25.0, 60.0, 100.0]:
        want = 0.0 if k == 0 else special.ive(1, k) / special.ive(0, k)
        assert abs(orc.bessel_ratio(k) - want) <= 2e-15 * max(want, 1e-300), k


def test_link_mean_is_conditional_expectation(orc):
    beta = 1.4
    lat = orc.Lattice(4, [4, 4, 4, 4], beta, seed=71)
    lat.init(1)
    for site, mu in [(5, 3), (100, 0), (201, 2)]:
        A = lat.staple(site, mu)
        w = lambda th: np.exp(beta * (np.cos(th) * A.real - np.sin(th) * A.imag) - beta * abs(A))
        z = integrate.quad(w, -np.pi, np.pi, epsabs=1e-14, epsrel=1e-13)[0]
        re = integrate.quad(lambda th: np.cos(th) * w(th), -np.pi, np.pi, epsabs=1e-14, epsrel=1e-13)[0] / z
        im = integrate.quad(lambda th: np.sin(th) * w(th), -np.pi, np.pi, epsabs=1e-14, epsrel=1e-13)[0] / z
        m = lat.link_mean(site, mu)
        assert abs(m - complex(re, im)) < 1e-12, (site, mu, m, re, im)


def _series(orc, L, beta, spec, n_conf, seed):
    lat = orc.Lattice(2, L, beta, seed=seed)
    lat.init(1)
    lat.sweeps(100)
    out = []
    for _ in range(n_conf):
        out.append(spec.unpack(lat.multilevel(spec)))
        lat.sweeps(1)
    return out


@pytest.mark.parametrize("levels", [[(2, 10, 1)], [(4, 3, 1), (2, 4, 1)]], ids=["one_level", "two_levels"])
def test_multihit_correlator_exact_2d(orc, levels):
    L, T, beta = 6, 8, 1.5
    rs = [1, 2, 3, 5]  # 1 and 5 are neighbours on the periodic axis of extent 6
    mh = orc.MLSpec(levels=levels, r=rs, dirs=[0], multihit=True)
    pl = orc.MLSpec(levels=levels, r=rs, dirs=[0])
    Cm = np.array([x["C"].real for x in _series(orc, [L, T], beta, mh, 1500, seed=72)])
    Cp = np.array([x["C"].real for x in _series(orc, [L, T], beta, pl, 1500, seed=72)])
    mm, em = batch_mean_err(Cm)
    mp, ep = batch_mean_err(Cp)
    for i, r in enumerate(rs):
        exact = E.polyakov_corr(beta, L, T, r)
        assert abs(mm[i] - exact) < 4 * em[i], (r, mm[i], em[i], exact)
    # both ends replaced at the non-neighbouring separations: smaller errors
    assert em[1] < ep[1] and em[2] < ep[2]


def test_multihit_insertions_exact_2d(orc):
    beta, L, T, r = 2.0, 6, 4, 2
    probes = [(0, 0, 0, 1), (2, 0, 0, 0)]
    spec = orc.MLSpec(levels=[(2, 10, 1)], r=[r], dirs=[0], probes=probes, comps=[0], multihit=True)
    res = _series(orc, [L, T], beta, spec, 3000, seed=73)
    CO = np.array([x["CO"][0, :, 0, :] for x in res])
    pp = E.polyakov_corr(beta, L, T, r)
    for ip, inside in enumerate([True, False]):
        ap = E.insertion(beta, L, T, r, inside, +1)
        am = E.insertion(beta, L, T, r, inside, -1)
        m, e = batch_mean_err(CO[:, ip, 0].real)
        assert abs(m - 2 * beta * (pp - 0.5 * (ap + am))) < 4 * e
        m, e = batch_mean_err(CO[:, ip, 1].imag)
        assert abs(m - np.sqrt(beta) * 0.5 * (am - ap)) < 4 * e

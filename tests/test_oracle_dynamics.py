"""Oracle Monte-Carlo dynamics pinned to closed forms.

 - 2D compact U(1) on a finite torus: exact plaquette, multilevel Polyakov
   correlator and plaquette insertions from Bessel sums (helpers/exact2d.py).
 - 4D strong coupling: <cos theta_P> = u + O(u^5), u = I_1(beta)/I_0(beta).
 - beta = 0: uniform links, every correlator vanishes.
All streams are seeded, so each test's outcome is fixed; tolerances are 4
standard errors from batch means.
"""
import numpy as np
import pytest
from scipy import special

from helpers import exact2d as E
from helpers.stats import batch_mean_err


def _plaquette_series(orc, d, L, beta, n_therm, n_meas, seed, tau=0):
    lat = orc.Lattice(d, L, beta, seed=seed)
    lat.init(1)
    lat.sweeps(n_therm, 3, tau)
    vals = []
    for _ in range(n_meas):
        lat.sweeps(1, 3, tau)
        vals.append(lat.plaquette_means())
    return np.array(vals)


@pytest.mark.parametrize("L,beta", [([4, 4], 2.0), ([6, 4], 1.5), ([4, 4], 0.7)])
def test_2d_plaquette_exact(orc, L, beta):
    vals = _plaquette_series(orc, 2, L, beta, 200, 20000, seed=3)[:, 0]
    m, e = batch_mean_err(vals)
    exact = E.plaquette(beta, L[0], L[1])
    assert abs(m - exact) < 4 * e, (m, e, exact)


def _ml_series(orc, d, L, beta, spec, n_conf, seed, n_between=1, n_therm=100):
    lat = orc.Lattice(d, L, beta, seed=seed)
    lat.init(1)
    lat.sweeps(n_therm)
    out = []
    for _ in range(n_conf):
        out.append(spec.unpack(lat.multilevel(spec)))
        lat.sweeps(n_between)
    return out


@pytest.mark.parametrize("L,beta,n_conf", [([4, 4], 2.0, 3000), ([4, 4], 1.0, 3000), ([8, 8], 2.0, 1500)])
def test_2d_multilevel_polyakov_correlator_exact(orc, L, beta, n_conf):
    spec = orc.MLSpec(levels=[(2, 10, 1)], r=[1, 2], dirs=[0])
    res = _ml_series(orc, 2, L, beta, spec, n_conf, seed=11)
    C = np.array([r["C"] for r in res])
    m, e = batch_mean_err(C.real)
    for i, r in enumerate([1, 2]):
        exact = E.polyakov_corr(beta, L[0], L[1], r)
        assert abs(m[i] - exact) < 4 * e[i], (r, m[i], e[i], exact)


def test_2d_multilevel_two_levels_exact(orc):
    spec = orc.MLSpec(levels=[(4, 4, 1), (2, 5, 1)], r=[1, 2], dirs=[0])
    res = _ml_series(orc, 2, [4, 8], 2.0, spec, 1500, seed=12)
    C = np.array([r["C"] for r in res])
    m, e = batch_mean_err(C.real)
    for i, r in enumerate([1, 2]):
        exact = E.polyakov_corr(2.0, 4, 8, r)
        assert abs(m[i] - exact) < 4 * e[i], (r, m[i], e[i], exact)


def test_2d_insertions_exact(orc):
    """<P^dagger P O> for O = 2 beta (1 - cos theta_p) and sqrt(beta) sin theta_p,
    with the plaquette p inside the strip (mid-plane probe) or outside it."""
    beta, L, T, r = 2.0, 6, 4, 2
    # mid-plane (inside the strip), just right of it, just left of it
    probes = [(0, 0, 0, 1), (2, 0, 0, 0), (-1, 0, 0, 0)]
    spec = orc.MLSpec(levels=[(2, 10, 1)], r=[r], dirs=[0], probes=probes, comps=[0])
    res = _ml_series(orc, 2, [L, T], beta, spec, 3000, seed=13)
    CO = np.array([x["CO"][0, :, 0, :] for x in res])  # [conf, probe, kind]
    pp = E.polyakov_corr(beta, L, T, r)
    for ip, inside in enumerate([True, False, False]):
        ap = E.insertion(beta, L, T, r, inside, +1)
        am = E.insertion(beta, L, T, r, inside, -1)
        exact_sq = 2 * beta * (pp - 0.5 * (ap + am))
        exact_lin_im = np.sqrt(beta) * 0.5 * (am - ap)  # <P^dagger P sin theta_p> is imaginary
        m, e = batch_mean_err(CO[:, ip, 0].real)
        assert abs(m - exact_sq) < 4 * e, ("sq", ip, m, e, exact_sq)
        m, e = batch_mean_err(CO[:, ip, 1].imag)
        assert abs(m - exact_lin_im) < 4 * e, ("lin", ip, m, e, exact_lin_im)
        m, e = batch_mean_err(CO[:, ip, 1].real)
        assert abs(m) < 4 * e + 1e-12


@pytest.mark.parametrize("beta", [0.1, 0.2])
def test_4d_strong_coupling_plaquette(orc, beta):
    vals = _plaquette_series(orc, 4, [4, 4, 4, 4], beta, 50, 1500, seed=5)
    m, e = batch_mean_err(vals.mean(axis=1))
    u = special.iv(1, beta) / special.iv(0, beta)
    assert abs(m - u) < max(4 * e, 10 * u**5), (m, e, u)


def test_4d_beta_zero(orc):
    vals = _plaquette_series(orc, 4, [4, 4, 4, 4], 0.0, 2, 400, seed=6)
    m, e = batch_mean_err(vals.mean(axis=1))
    assert abs(m) < 4 * e
    spec = orc.MLSpec(levels=[(2, 4, 1)], r=[1, 2], dirs=[0, 1, 2])
    res = _ml_series(orc, 4, [4, 4, 4, 4], 0.0, spec, 200, seed=7, n_therm=2)
    C = np.array([x["C"] for x in res])
    m, e = batch_mean_err(C.real)
    assert np.all(np.abs(m) < 4 * e)


def test_4d_multilevel_correlator_strong_coupling(orc):
    """<P^dagger P(r=1)> = u^(r N_t) (1 + c u^4) on 6^3 x 4 at beta = 0.5.  The first
    correction comes from deforming the r x N_t sheet by one cube, c ~ 2 (d-2)
    (r N_t) plus the edge terms, about 16-30; the tolerance allows 15 %."""
    beta = 0.5
    u = special.iv(1, beta) / special.iv(0, beta)
    spec = orc.MLSpec(levels=[(2, 40, 1)], r=[1], dirs=[0, 1, 2])
    res = _ml_series(orc, 4, [6, 6, 6, 4], beta, spec, 60, seed=8, n_therm=20)
    C = np.array([x["C"][0].real for x in res])
    m, e = batch_mean_err(C, n_batches=10)
    lead = u**4
    assert abs(m - lead) < 4 * e + 0.15 * lead, (m, e, lead)
    assert m > lead  # every correction adds surfaces with positive weight

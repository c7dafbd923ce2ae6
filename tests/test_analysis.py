"""Host estimators and analysis (no GPU), pinned to identities, closed forms
and synthetic data with known answers.

* jackknife error of a mean equals the standard error s / sqrt(n) exactly;
* the connected insertion ratios of synthetic records;
* V(r) = -ln<P^dagger P>/N_t and the potential fit recover V_0, sigma, gamma;
* records whose correlators lie far below the range of FP64 (mantissa and
  binary exponent per separation) give the exact ln<P^dagger P> and the same
  ratios as the plain values scaled into range (40-digit mpmath sums);
* the lattice Green function at the origin is Watson's integral / 2 (closed
  form in Gamma functions); G(r) -> 1/(4 pi r); rbar -> r - 1/2;
* r_0 is exact for a Coulomb-plus-linear potential when rbar makes the
  discrete Coulomb force exact;
* the profile ansatz integrates to w^2 = s in its Gaussian limits, and a fit
  recovers its parameters;
* the tree-level effective-string width reduces to the paper's zero- and
  finite-temperature forms in the limits u -> infinity and u -> 0.
"""
from math import gamma, pi, sqrt

import numpy as np
import pytest

from paper_1309_3859_amd import analysis as A


def test_jackknife_of_mean_is_standard_error():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(37, 3))
    est, err = A.jackknife(x, lambda s: s.mean(axis=0))
    assert np.allclose(est, x.mean(axis=0))
    assert np.allclose(err, x.std(axis=0, ddof=1) / np.sqrt(len(x)), rtol=1e-12)


def _records(rng, n, R, P, Nc):
    recs = []
    for _ in range(n):
        recs.append({"C": rng.uniform(0.5, 1.0, R) + 1j * rng.normal(0, 1e-3, R),
                     "CO": rng.normal(size=(R, P, Nc, 2)) + 1j * rng.normal(size=(R, P, Nc, 2)),
                     "vac_sq": rng.uniform(0.5, 1.5, 6)})
    return recs


def test_field_profile_ratios():
    rng = np.random.default_rng(1)
    recs = _records(rng, 12, 3, 2, 2)
    comps, dirs = [0, 4], [1]
    out, err = A.field_profile(recs, comps, dirs)
    C = np.mean([r["C"].real for r in recs], axis=0)
    CO = np.mean([r["CO"] for r in recs], axis=0)
    vac = np.mean([r["vac_sq"] for r in recs], axis=0)
    v = [vac[A.orientation(c, 1)] for c in comps]
    # axis y: frame (y, z, x); E_par is E_y, B_perp1 (plaquette P_{perp2 par} = P_xy) is B_z
    assert A.orientation(0, 1) == 1 and A.orientation(4, 1) == 5
    assert np.allclose(out[..., 0, 0], CO.real[..., 0] / C[:, None, None] - np.array(v)[None, None, :])
    assert np.allclose(out[..., 1, 0], CO.imag[..., 1] / C[:, None, None])
    assert np.all(err > 0)


def test_scaled_records_below_fp64_range():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    rng = np.random.default_rng(4)
    n, R, P, Nc = 9, 2, 2, 2
    recs, scaled = [], []
    for _ in range(n):
        ex = rng.integers(-2100, -2090, R)
        cm = rng.uniform(0.5, 1.0, R) + 1j * rng.normal(0, 1e-3, R)
        com = rng.normal(size=(R, P, Nc, 2)) + 1j * rng.normal(size=(R, P, Nc, 2))
        zero = np.zeros(R, complex)
        recs.append({"C": zero, "CO": np.zeros_like(com), "C_mant": cm, "CO_mant": com, "exp": ex,
                     "vac_sq": rng.uniform(0.5, 1.5, 6)})
        # the same record scaled by 2^2095 into range (ratios are unchanged)
        scaled.append({"C": np.ldexp(cm.real, ex + 2095) + 1j * np.ldexp(cm.imag, ex + 2095),
                       "CO": np.ldexp(com.real, ex[:, None, None, None] + 2095)
                       + 1j * np.ldexp(com.imag, ex[:, None, None, None] + 2095),
                       "vac_sq": recs[-1]["vac_sq"]})
    lc, lerr = A.log_correlator(recs)
    for ir in range(R):
        mean = mp.fsum(mp.mpf(float(r["C_mant"][ir].real)) * mp.mpf(2) ** int(r["exp"][ir]) for r in recs) / n
        assert abs(lc[ir] - float(mp.log(mean))) < 1e-12 * abs(float(mp.log(mean)))
    assert np.all(np.isfinite(lerr)) and np.all(lerr > 0)
    V, _ = A.potential(recs, 4)
    assert np.allclose(V, -lc / 4, rtol=1e-14)
    out, err = A.field_profile(recs, [0, 3])
    want, werr = A.field_profile(scaled, [0, 3])
    assert np.allclose(out, want, rtol=1e-12, atol=0)
    assert np.allclose(err, werr, rtol=1e-9, atol=0)


def test_potential_and_fit():
    nt, V0, sigma, gam = 8, 0.3, 0.18, pi / 12
    r = np.arange(1, 9)
    V = V0 + sigma * r - gam / r
    recs = [{"C": np.exp(-nt * V) * (1 + 1e-3 * k)} for k in range(-3, 4)]
    Vm, err = A.potential(recs, nt)
    assert np.allclose(Vm, V, atol=1e-6)
    fit = A.fit_potential(r, V)
    assert np.allclose([fit["V0"], fit["sigma"], fit["gamma"]], [V0, sigma, gam], atol=1e-10)
    fit2 = A.fit_potential(r, V, gamma=pi / 12)
    assert abs(fit2["sigma"] - sigma) < 1e-10


def test_lattice_green_function():
    watson = sqrt(6) / (96 * pi ** 3) * gamma(1 / 24) * gamma(5 / 24) * gamma(7 / 24) * gamma(11 / 24)
    assert abs(watson - 0.505462019717) < 1e-11
    assert abs(A.lattice_green(0) - watson / 2) < 1e-10
    assert abs(4 * pi * 16 * A.lattice_green(16) - 1) < 2e-3
    assert abs(A.rbar_tree(16) - 15.5) < 0.05
    assert 1.0 < A.rbar_tree(2) < 1.5


def test_sommer_r0_exact_for_coulomb_plus_linear():
    sigma, gam = 0.1, 0.3
    r = np.arange(1, 12)
    V = sigma * r - gam / r
    # V(r) - V(r-1) = sigma + gam / (r (r-1)): F = f1 + f2 / rbar^2 holds exactly with rbar = sqrt(r (r-1))
    r0 = A.sommer_r0(r, V, rbar=lambda x: np.sqrt(x * (x - 1)))
    assert abs(r0 - np.sqrt((1.65 - gam) / sigma)) < 1e-10
    # the default and the tree-level choice give nearby values on the same data
    assert abs(A.sommer_r0(r, V) - r0) < 0.1 * r0
    assert abs(A.sommer_r0(r, V, rbar=A.rbar_tree) - r0) < 0.1 * r0


def test_profile_ansatz_width():
    s = 3.7
    assert abs(A.width2_from_ansatz(1.0, 0.0, 0.0, s) - s) < 1e-8
    assert abs(A.width2_from_ansatz(2.0, 0.4, 0.4, s) - s) < 1e-8
    assert A.width2_from_ansatz(1.0, 1.0, 0.0, s) < s  # a sharper core narrows the tube
    x2 = np.array([p1 * p1 + p2 * p2 for p1 in range(-6, 7) for p2 in range(-6, 7)], float)
    true = (0.8, 0.5, 0.2, 5.0)
    popt = A.fit_profile(x2, A.profile_ansatz(x2, *true), p0=(1.0, 0.3, 0.1, 4.0))
    assert np.allclose(A.profile_ansatz(x2, *popt), A.profile_ansatz(x2, *true), atol=1e-8)
    # the lattice second moment approaches the continuum one for a wide grid
    g = A.profile_ansatz(x2, 1.0, 0.0, 0.0, 2.0)
    p1 = [p for p in range(-6, 7) for _ in range(13)]
    p2 = [q for _ in range(13) for q in range(-6, 7)]
    assert abs(A.flux_tube_width2(g, p1, p2) - 2.0) < 1e-3


def test_string_width_limits():
    sigma, rho0, d = 0.2, 0.6, 4
    # zero temperature (u -> infinity): (d-2)/(2 pi sigma) log(r/rho0)
    r, T = 6.0, 1e-4
    assert abs(A.width2_string(r, sigma, rho0, T, d) - (d - 2) / (2 * pi * sigma) * np.log(r / rho0)) < 1e-10
    # high temperature (u -> 0): (d-2)/(2 pi sigma) log(1/(4 T rho0)) + (d-2)/(4 sigma) T r
    r, T = 40.0, 0.25
    hi = (d - 2) / (2 * pi * sigma) * np.log(1 / (4 * T * rho0)) + (d - 2) / (4 * sigma) * T * r
    assert abs(A.width2_string(r, sigma, rho0, T, d) - hi) < 1e-8
    # a fit to exact widths recovers sigma and rho0
    rr = np.arange(2, 13, dtype=float)
    w2 = A.width2_string(rr, 0.18, 0.4, 1 / 8.0)
    fit = A.fit_width(rr, w2, 1 / 8.0)
    assert abs(fit["sigma"] - 0.18) < 1e-6 and abs(fit["rho0"] - 0.4) < 1e-6


def test_plaquette_susceptibility_estimator():
    rng = np.random.default_rng(3)
    x = rng.normal(0.6, 0.01, 4000)
    chi, err = A.plaquette_susceptibility(x, 1000, n_blocks=20)
    assert abs(chi - 1000 * x.var()) < 1e-9
    assert 0 < err < 0.2 * chi
    # the sample variance of i.i.d. draws estimates sigma^2: chi ~ N sigma^2
    assert abs(chi - 1000 * 1e-4) < 5 * err


def test_peak_position():
    b = np.linspace(0.95, 1.05, 11)
    assert abs(A.peak_position(b, 3.0 - 40 * (b - 1.003) ** 2) - 1.003) < 1e-12
    g = np.exp(-((b - 1.012) / 0.03) ** 2)
    assert abs(A.peak_position(b, g, n_points=3) - 1.012) < 2e-3


def test_gamma_method_on_processes_with_known_autocorrelation():
    """AR(1) x_t = phi x_{t-1} + sqrt(1 - phi^2) e_t has rho(t) = phi^t, so
    tau_int = (1 + phi) / (2 (1 - phi)) and the error of the mean is
    sqrt(2 tau_int / n); for independent Gaussian draws of variance s^2 the
    susceptibility N s^2 has the error N s^2 sqrt(2 / n) and tau_int = 1/2."""
    rng = np.random.default_rng(11)
    n = 400_000
    for phi in (0.0, 0.5, 0.8, 0.95):
        e = rng.normal(size=n)
        x = np.empty(n)
        x[0] = e[0]
        c = np.sqrt(1 - phi * phi)
        for t in range(1, n):
            x[t] = phi * x[t - 1] + c * e[t]
        sigma, tint, dtint, W = A.gamma_method(x)
        want = (1 + phi) / (2 * (1 - phi))
        assert abs(tint - want) < max(3 * dtint, 0.02), (phi, tint, want, dtint)
        assert abs(sigma - np.sqrt(2 * want / n)) < 0.05 * np.sqrt(2 * want / n)
        assert W > 0
    s, N = 0.01, 1000
    x = rng.normal(0.6, s, n)
    chi, sig, tint, _, _ = A.susceptibility_gamma(x, N)
    assert abs(chi - N * s * s) < 4 * sig
    assert abs(sig - N * s * s * np.sqrt(2 / n)) < 0.05 * sig
    assert abs(tint - 0.5) < 0.02

"""Host-side estimators of the multilevel measurements (arXiv 1309.3859,
Sec. II.C.3 and III.C): ratios of configuration averages and jackknife errors.

Input: records from ``Context.results()`` unpacked with ``Spec.unpack`` -- one
per outer multilevel configuration.
  <P^dagger P>(r)            = mean_i Re C_i(r)
  <O_sq>_{P^dagger P}(r, x0) = mean_i Re CO_i / mean_i Re C_i - <O_sq>_vacuum
  <O_lin>_{P^dagger P}(r, x0) = mean_i Im CO_i / mean_i Re C_i
(<P^dagger P O_lin> is imaginary by charge conjugation; its real part is
reported as a check.)  Errors are delete-one jackknife over configurations.
"""
from __future__ import annotations

from typing import Callable, Optional, Sequence

import numpy as np

# absolute orientation of frame component c for charge axis mu:
# E_i -> i, B_x -> 3, B_y -> 4, B_z -> 5
def orientation(comp: int, mu: int) -> int:
    return (mu + comp) % 3 if comp < 3 else 3 + (mu + comp - 3) % 3


def jackknife(samples: np.ndarray, estimator: Callable[[np.ndarray], np.ndarray]):
    """Delete-one jackknife: (estimate on all samples, standard error)."""
    samples = np.asarray(samples)
    n = samples.shape[0]
    full = estimator(samples)
    if n < 2:
        return full, np.full_like(np.asarray(full, dtype=float), np.nan)
    reps = np.array([estimator(np.delete(samples, i, axis=0)) for i in range(n)])
    err = np.sqrt((n - 1) / n * np.sum((reps - reps.mean(axis=0)) ** 2, axis=0))
    return full, err


def block_means(samples: np.ndarray, n_blocks: Optional[int]):
    """Means of n_blocks consecutive equal blocks of the samples (axis 0; a
    tail shorter than a block is dropped), or the samples themselves if
    n_blocks is None.  Estimators that are functions of means, jackknifed over
    block means, absorb the autocorrelation of consecutive configurations."""
    x = np.asarray(samples)
    if n_blocks is None:
        return x
    b = x.shape[0] // n_blocks
    if b < 1:
        raise ValueError("fewer samples than blocks")
    return x[: b * n_blocks].reshape((n_blocks, b) + x.shape[1:]).mean(axis=1)


def common_scale(records: Sequence[dict]):
    """C [n, R] and CO [n, R, P, Nc, 2] of every record as mantissas relative
    to one binary exponent per separation (the largest of the records'), and
    that exponent [R]: value = mantissa * 2^E.  Records without exponents are
    taken as they are (E = 0)."""
    if not records or "exp" not in records[0]:
        C = np.array([rec["C"] for rec in records])
        CO = np.array([rec["CO"] for rec in records]) if records and "CO" in records[0] else None
        return C, CO, np.zeros(C.shape[1] if C.ndim > 1 else 0, dtype=np.int64)
    ex = np.array([rec["exp"] for rec in records])  # [n, R]
    E = ex.max(axis=0)
    sh = ex - E[None, :]

    def rescale(m, k):
        return np.ldexp(m.real, k) + 1j * np.ldexp(m.imag, k)

    C = np.array([rescale(rec["C_mant"], sh[i]) for i, rec in enumerate(records)])
    CO = np.array([rescale(rec["CO_mant"], sh[i][:, None, None, None]) for i, rec in enumerate(records)])
    return C, CO, E


def correlator(records: Sequence[dict], n_blocks: Optional[int] = None):
    """<P^dagger P>(r) with jackknife errors (over blocks of consecutive
    records if n_blocks is given)."""
    C = np.array([rec["C"].real for rec in records])
    return jackknife(block_means(C, n_blocks), lambda x: x.mean(axis=0))


def log_correlator(records: Sequence[dict], n_blocks: Optional[int] = None):
    """ln <P^dagger P>(r) with jackknife errors, formed from the mantissas and
    exponents of the records, so it stays finite where <P^dagger P> itself is
    below the range of FP64."""
    C, _, E = common_scale(records)
    return jackknife(block_means(C.real, n_blocks), lambda x: np.log(x.mean(axis=0)) + E * np.log(2.0))


def field_profile(records: Sequence[dict], comps: Sequence[int], dirs: Sequence[int] = (0,),
                  n_blocks: Optional[int] = None):
    """Connected insertions <O>_{P^dagger P}[r, probe, comp, kind] (kind 0:
    2 beta (1 - Re P), kind 1: sqrt(beta) Im P) with jackknife errors (over
    blocks of consecutive records if n_blocks is given).  The ratios are
    formed from mantissas on a common exponent per separation, so they hold
    where the correlator is below the range of FP64."""
    C, CO, _ = common_scale(records)
    C = C.real  # [n, R]
    vac = np.array([rec["vac_sq"] for rec in records])  # [n, 6]
    n = C.shape[0]
    packed = np.concatenate([C.reshape(n, -1), CO.real.reshape(n, -1), CO.imag.reshape(n, -1), vac], axis=1)
    R = C.shape[1]
    shp = CO.shape[1:]
    m = int(np.prod(shp))

    def est(x):
        c = x[:, :R].mean(axis=0)
        re = x[:, R:R + m].mean(axis=0).reshape(shp)
        im = x[:, R + m:R + 2 * m].mean(axis=0).reshape(shp)
        v = x[:, R + 2 * m:].mean(axis=0)
        v_comp = np.array([np.mean([v[orientation(cc, mu)] for mu in dirs]) for cc in comps])
        out = np.empty(shp + (2,))
        out[..., 0, 0] = re[..., 0] / c[:, None, None] - v_comp[None, None, :]
        out[..., 1, 0] = im[..., 1] / c[:, None, None]
        out[..., 0, 1] = im[..., 0] / c[:, None, None]  # checks: imaginary part of the O_sq ratio
        out[..., 1, 1] = re[..., 1] / c[:, None, None]  # and real part of the O_lin ratio
        return out

    return jackknife(block_means(packed, n_blocks), est)


def flux_tube_width2(profile: np.ndarray, p1: Sequence[int], p2: Sequence[int]):
    """Second moment of a transverse profile, w^2 = sum x^2 F / sum F
    (Sec. II.B, eq. for w^2(r/2)), over the probe positions given."""
    x2 = np.asarray(p1, float) ** 2 + np.asarray(p2, float) ** 2
    return float(np.sum(x2 * profile) / np.sum(profile))


# ---------------------------------------------------------------------------
# Potential, Sommer scale, profile ansatz and effective-string width
# (arXiv 1309.3859: eq. for V(r), Sec. II.A; r_0, Sec. II.D "Scale setting";
# profile ansatz and width, Sec. III.C; tree-level widening, Sec. I.B).
# ---------------------------------------------------------------------------
def potential(records: Sequence[dict], nt: int):
    """V(r) = -ln <P^dagger P>(r) / N_t with jackknife errors (the Polyakov
    correlator at temperature 1/N_t decays as exp(-N_t V)); from the
    mantissas and exponents, so it holds where the correlator underflows."""
    C, _, E = common_scale(records)
    return jackknife(C.real, lambda x: -(np.log(x.mean(axis=0)) + E * np.log(2.0)) / nt)


def fit_potential(r, V, err=None, gamma: Optional[float] = None):
    """Weighted least squares of V(r) = V_0 + sigma r - gamma / r; gamma free,
    or fixed (for d = 4 the Luscher value is pi / 12).  Returns a dict with
    V0, sigma, gamma."""
    r = np.asarray(r, float)
    V = np.asarray(V, float)
    w = np.ones_like(r) if err is None else 1.0 / np.asarray(err, float)
    if gamma is None:
        A = np.stack([np.ones_like(r), r, -1.0 / r], axis=1)
        coef = np.linalg.lstsq(A * w[:, None], V * w, rcond=None)[0]
        return {"V0": coef[0], "sigma": coef[1], "gamma": coef[2]}
    A = np.stack([np.ones_like(r), r], axis=1)
    coef = np.linalg.lstsq(A * w[:, None], (V + gamma / r) * w, rcond=None)[0]
    return {"V0": coef[0], "sigma": coef[1], "gamma": float(gamma)}


def lattice_green(r: int) -> float:
    """Lattice Coulomb Green function on the cubic lattice,
    G(r) = int d^3k/(2 pi)^3 cos(k_1 r) / (4 sum_j sin^2(k_j/2)).  With
    1/D = int_0^inf exp(-t D) dt the Brillouin-zone integral factorises into
    modified Bessel functions: G(r) = int_0^inf exp(-6t) I_r(2t) I_0(2t)^2 dt,
    evaluated with the exponentially scaled ive.  G(r) -> 1/(4 pi r) at large r."""
    from scipy.integrate import quad
    from scipy.special import ive

    f = lambda t: ive(abs(r), 2 * t) * ive(0, 2 * t) ** 2
    return float(quad(f, 0, 50, limit=400)[0] + quad(f, 50, np.inf, limit=400)[0])


def rbar_tree(r: int) -> float:
    """Tree-level improved distance of the force F(rbar) = V(r) - V(r-1):
    rbar = [4 pi (G(r-1) - G(r))]^(-1/2), so that the lattice Coulomb force is
    exactly 1/(4 pi rbar^2).  (The printed formula's sign and prefactor are
    read so that rbar -> r - 1/2 at large r.)"""
    return float((4 * np.pi * (lattice_green(r - 1) - lattice_green(r))) ** -0.5)


def sommer_r0(r, V, rbar: Optional[Callable[[int], float]] = None, c: float = 1.65):
    """Sommer scale r_0 with r_0^2 F(r_0) = c: for consecutive pairs of
    forces F(rbar_r) = V(r) - V(r-1), F(rbar_{r+1}) = V(r+1) - V(r), solve
    F = f1 + f2 / rbar^2 and take the pair whose interval contains r_0.
    rbar defaults to r - 1/2; pass rbar_tree for the tree-level choice."""
    r = [int(x) for x in r]
    V = np.asarray(V, float)
    rb = rbar or (lambda x: x - 0.5)
    best = None
    for i in range(1, len(r) - 1):
        if r[i] - r[i - 1] != 1 or r[i + 1] - r[i] != 1:
            continue
        a, b = rb(r[i]), rb(r[i + 1])
        Fa, Fb = V[i] - V[i - 1], V[i + 1] - V[i]
        f2 = (Fa - Fb) / (1 / a ** 2 - 1 / b ** 2)
        f1 = Fa - f2 / a ** 2
        if f1 <= 0 or c <= f2:
            continue
        r0 = float(np.sqrt((c - f2) / f1))
        if best is None or (a <= r0 <= b):
            best = r0
            if a <= r0 <= b:
                break
    return best


def profile_ansatz(x2, C1, C2, C3, s):
    """C_1 exp(-x^2/s) (1 + C_2 exp(-x^2/s)) / (1 + C_3 exp(-x^2/s))."""
    g = np.exp(-np.asarray(x2, float) / s)
    return C1 * g * (1 + C2 * g) / (1 + C3 * g)


def fit_profile(x2, y, err=None, p0=(1.0, 0.0, 0.0, 4.0)):
    """Least-squares fit of the profile ansatz to a transverse profile."""
    from scipy.optimize import curve_fit

    popt, _ = curve_fit(profile_ansatz, np.asarray(x2, float), np.asarray(y, float), p0=p0,
                        sigma=None if err is None else np.asarray(err, float), maxfev=20000)
    return popt


def width2_from_ansatz(C1, C2, C3, s):
    """w^2 = int d^2x x^2 f / int d^2x f for the ansatz f over the whole
    transverse plane; with t = x^2, d^2x = pi dt, so w^2 = int t f dt / int f dt."""
    from scipy.integrate import quad

    f = lambda t: profile_ansatz(t, C1, C2, C3, s)
    top = quad(lambda t: t * f(t), 0, np.inf, limit=200)[0]
    bot = quad(f, 0, np.inf, limit=200)[0]
    return top / bot


def log_eta_ratio(u: float, terms: int = 200) -> float:
    """log( eta(2 i u) / eta(i u)^2 ) with the Dedekind eta function
    eta(tau) = q^(1/24) prod_n (1 - q^n), q = exp(2 pi i tau), for u > 0."""
    q1 = np.exp(-2 * np.pi * u)
    n = np.arange(1, terms + 1)
    log_eta = lambda q, lq: lq / 24 + np.sum(np.log1p(-q ** n))
    return float(log_eta(q1 ** 2, -4 * np.pi * u) - 2 * log_eta(q1, -2 * np.pi * u))


def width2_string(r, sigma, rho0, T, d: int = 4):
    """Tree-level effective-string width at the mid-plane,
    w^2(r/2) = (d-2)/(2 pi sigma) log(r/rho0) + (d-2)/(pi sigma) log(eta(2iu)/eta(iu)^2),
    u = 1/(2 T r)."""
    r = np.atleast_1d(np.asarray(r, float))
    out = np.array([(d - 2) / (2 * np.pi * sigma) * np.log(x / rho0)
                    + (d - 2) / (np.pi * sigma) * log_eta_ratio(1.0 / (2 * T * x)) for x in r])
    return out if out.size > 1 else float(out[0])


def fit_width(r, w2, T, err=None, d: int = 4, p0=(0.2, 0.5)):
    """Fit sigma and rho0 of width2_string to measured widths at temperature T."""
    from scipy.optimize import curve_fit

    f = lambda x, sigma, rho0: width2_string(x, sigma, rho0, T, d)
    popt, _ = curve_fit(f, np.asarray(r, float), np.asarray(w2, float), p0=p0,
                        sigma=None if err is None else np.asarray(err, float), maxfev=20000)
    return {"sigma": popt[0], "rho0": popt[1]}


# ---------------------------------------------------------------------------
# Plaquette susceptibility and its peak (the paper locates beta_c at the peak
# of the plaquette susceptibility on 24^3 x 4, Sec. II.D and III.A).
# ---------------------------------------------------------------------------
def plaquette_susceptibility(series, n_plaquettes: int, n_blocks: int = 20):
    """chi = N_P (<P^2> - <P>^2) of the lattice-averaged plaquette P of each
    configuration (series[i]), with a blocked jackknife error (blocks of
    consecutive configurations absorb the autocorrelation)."""
    x = np.asarray(series, float)
    n = len(x) // n_blocks * n_blocks
    blocks = x[:n].reshape(n_blocks, -1)

    def est(b):
        v = b.reshape(-1)
        return n_plaquettes * (np.mean(v * v) - np.mean(v) ** 2)

    return jackknife(blocks, est)


def gamma_method(series, grad: Optional[Callable[[np.ndarray], np.ndarray]] = None, S: float = 1.5):
    """Error of a function f of the means of a Monte-Carlo time series, with
    its integrated autocorrelation time (Wolff, Comput. Phys. Commun. 156
    (2004) 143, "Monte Carlo errors with less errors").

    series: [n] or [n, k] (k primary observables per configuration, in
    Monte-Carlo order); grad(means) -> df/da_alpha (default: the mean of a
    single observable).  The fluctuations are projected on the gradient,
        delta_i = sum_alpha f_alpha (a_{alpha,i} - abar_alpha),
    their autocorrelation function Gamma(t) is summed up to the window W
    chosen automatically: W is the first t where
        exp(-t / tau) - tau / sqrt(t n) < 0,  tau = S / ln((2 tau_int(t) + 1) / (2 tau_int(t) - 1)),
    and  tau_int = 1/2 + sum_{t=1}^{W} Gamma(t) / Gamma(0),  sigma^2 = 2 tau_int Gamma(0) / n.
    Returns (sigma, tau_int, d tau_int, W)."""
    a = np.asarray(series, float)
    if a.ndim == 1:
        a = a[:, None]
    n = a.shape[0]
    mean = a.mean(axis=0)
    g = np.ones(a.shape[1]) if grad is None else np.asarray(grad(mean), float)
    d = (a - mean) @ g
    # Gamma(t) for every t at once from the power spectrum of the zero-padded series
    m = 1 << int(np.ceil(np.log2(2 * n)))
    f = np.fft.rfft(d, m)
    gam = np.fft.irfft(f * np.conj(f), m)[:n] / (n - np.arange(n))
    if gam[0] <= 0:
        return 0.0, 0.5, 0.0, 0
    tint = 0.5
    W = 0
    for t in range(1, n // 2):
        tint += gam[t] / gam[0]
        if tint <= 0.5:
            W = t
            break
        tau = S / np.log((2 * tint + 1) / (2 * tint - 1))
        if np.exp(-t / tau) - tau / np.sqrt(t * n) < 0:
            W = t
            break
    else:
        W = n // 2 - 1
    tint = max(tint, 0.5)
    sigma = np.sqrt(2 * tint * gam[0] / n)
    dtint = tint * np.sqrt(4 * (W + 0.5 - tint) / n)
    return float(sigma), float(tint), float(dtint), int(W)


def susceptibility_gamma(series, n_plaquettes: int):
    """chi = N_P (<P^2> - <P>^2) of a series of lattice-averaged plaquettes,
    with its error and integrated autocorrelation time from gamma_method
    (gradient N_P (-2 <P>, 1) on the primary observables (P, P^2)).
    Returns (chi, sigma, tau_int, d tau_int, W)."""
    x = np.asarray(series, float)
    a = np.stack([x, x * x], axis=1)
    m = a.mean(axis=0)
    chi = n_plaquettes * (m[1] - m[0] ** 2)
    sigma, tint, dtint, W = gamma_method(a, lambda mm: n_plaquettes * np.array([-2.0 * mm[0], 1.0]))
    return float(chi), sigma, tint, dtint, W


def peak_position(betas, chi, n_points: int = 5):
    """Vertex of the parabola fitted (least squares) through the n_points
    values of chi(beta) around its largest one."""
    b = np.asarray(betas, float)
    c = np.asarray(chi, float)
    order = np.argsort(b)
    b, c = b[order], c[order]
    i = int(np.argmax(c))
    lo = max(0, min(i - n_points // 2, len(b) - n_points))
    bb, cc = b[lo:lo + n_points], c[lo:lo + n_points]
    a2, a1, _ = np.polyfit(bb, cc, 2)
    return float(-a1 / (2 * a2))


def phase_mask(ns: Sequence[int], nt: int, mu: int, parity: int, tau: int = 0) -> np.ndarray:
    """Links one checkerboard phase updates, as a boolean mask over the
    canonical link view (element mu + 4 (x + Nx (y + Ny (z + Nz t)))):
    direction mu at the sites of the given parity, without the frozen spatial
    links of the layers t = 0 mod tau when tau > 1 (Sec. II.C.1)."""
    nx, ny, nz = ns
    t, z, y, x = np.meshgrid(np.arange(nt), np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    sites = (x + y + z + t) % 2 == parity
    if mu < 3 and tau > 1:
        sites &= t % tau != 0
    mask = np.zeros((nt, nz, ny, nx, 4), dtype=bool)
    mask[..., mu] = sites
    return mask.reshape(-1)


def acceptance_rate(before: np.ndarray, after: np.ndarray, ns: Sequence[int], nt: int, mu: int, parity: int,
                    tau: int = 0) -> float:
    """Acceptance rate of one Metropolis phase (Sec. II): the fraction of the
    phase's links whose angle changed between the two canonical views."""
    m = phase_mask(ns, nt, mu, parity, tau)
    return float(np.mean(before[m] != after[m]))

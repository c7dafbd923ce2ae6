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

from typing import Callable, Sequence

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


def correlator(records: Sequence[dict]):
    """<P^dagger P>(r) with jackknife errors."""
    C = np.array([rec["C"].real for rec in records])
    return jackknife(C, lambda x: x.mean(axis=0))


def field_profile(records: Sequence[dict], comps: Sequence[int], dirs: Sequence[int] = (0,)):
    """Connected insertions <O>_{P^dagger P}[r, probe, comp, kind] (kind 0:
    2 beta (1 - Re P), kind 1: sqrt(beta) Im P) with jackknife errors."""
    C = np.array([rec["C"].real for rec in records])  # [n, R]
    CO = np.array([rec["CO"] for rec in records])  # [n, R, P, Nc, 2]
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

    return jackknife(packed, est)


def flux_tube_width2(profile: np.ndarray, p1: Sequence[int], p2: Sequence[int]):
    """Second moment of a transverse profile, w^2 = sum x^2 F / sum F
    (Sec. II.B, eq. for w^2(r/2)), over the probe positions given."""
    x2 = np.asarray(p1, float) ** 2 + np.asarray(p2, float) ** 2
    return float(np.sum(x2 * profile) / np.sum(profile))

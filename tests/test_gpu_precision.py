"""Precision study on the two-level preset (32^3 x 8, beta = 1): FP32 link
storage and arithmetic against the FP64 path, which itself agrees with the
oracle within 1e-12 per phase (test_gpu_parity.py).

* one sweep from the same hot start and counters: after each pass, the FP32
  links' deviation from the FP64 links, next to what the FP64 dynamics alone
  does to the FP32-rounded start (the overrelaxation passes amplify any
  rounding-level difference, so this is the yardstick);
* one measurement without updates on the same links (the FP32 run holds them
  rounded): every estimate's error against the FP64 run's;
* the precision study proper: FP32 and FP64 chains of the full preset from
  the same seed, every observable's difference against the combined
  statistical error (the FP64 path stands for the oracle at this size).
"""
import sys

import numpy as np
import pytest

from helpers.stats import circ_dist

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1309_3859_amd import configs, u1ml

    u1ml.lib()
    return u1ml, configs


def _q(d):
    return {"median": float(np.median(d)), "q999": float(np.quantile(d, 0.999)), "max": float(d.max())}


def test_one_sweep_fp32_against_fp64(env):
    u1, configs = env
    s64, _ = configs.c3_precision(u1.FP64, n_outer=1, n_inner=1)
    s32, _ = configs.c3_precision(u1.FP32, n_outer=1, n_inner=1)
    c64 = u1.Context(s64)
    c64.init_links(u1.HOT)
    th0 = c64.links(0)
    c32 = u1.Context(s32)
    c32.init_links(u1.HOT)
    assert np.array_equal(c32.links(0), th0.astype(np.float32).astype(np.float64))
    cr = u1.Context(s64)  # FP64 dynamics from the FP32-rounded start
    cr.init_links(u1.COLD)
    cr.set_links(th0.astype(np.float32).astype(np.float64))
    for kind, name in [(0, "heatbath"), (1, "overrelaxation 1"), (1, "overrelaxation 2"), (1, "overrelaxation 3")]:
        for c in (c64, c32, cr):
            for mu in range(4):
                for par in (0, 1):
                    c.phase(kind, mu, par, 0, 0)
        ref = c64.links(0)
        d32, dr = circ_dist(c32.links(0), ref), circ_dist(cr.links(0), ref)
        say(name, "FP32 vs FP64", _q(d32), "FP64 from rounded start", _q(dr))
        # FP32 arithmetic adds little to what the dynamics itself makes of FP32
        # rounding (the heatbath draws from the same Philox words in both
        # precisions; arg A moves by delta / |A| when a staple link moves by delta)
        assert np.median(d32) < 10 * np.median(dr) + 1e-6
        assert np.quantile(d32, 0.999) < 10 * np.quantile(dr, 0.999) + 1e-5


def test_one_measurement_fp32_against_fp64(env):
    """Estimates of one measurement without updates: the FP32 path (links
    rounded to FP32, sincos in FP32, FP64 accumulators and products) against
    the FP64 path on the same links."""
    u1, configs = env
    out = {}
    th = None
    for prec in (u1.FP64, u1.FP32):
        spec, _ = configs.c3_precision(prec, n_outer=1, n_inner=1)
        spec.levels = [(4, 1, 0), (2, 1, 0)]
        c = u1.Context(spec)
        c.init_links(u1.HOT)
        if th is None:
            c.sweeps(20)
            th = c.links(0)
        else:
            c.set_links(th)
        c.multilevel()
        out[prec] = spec.unpack(c.results()[0][0])
    a, b = out[u1.FP32], out[u1.FP64]
    rel_c = np.abs(a["C"] - b["C"]) / np.abs(b["C"])
    co_scale = np.abs(b["CO"]).max(axis=(1, 2, 3))  # per separation
    rel_co = (np.abs(a["CO"] - b["CO"]).max(axis=(1, 2, 3))) / co_scale
    rel_vac = np.abs(a["vac_sq"] - b["vac_sq"]) / np.abs(b["vac_sq"])
    say("C(r) relative error per r", np.array2string(rel_c, precision=2))
    say("CO relative to its scale per r", np.array2string(rel_co, precision=2))
    say("vacuum <O_sq> relative error", np.array2string(rel_vac, precision=2))
    assert rel_c.max() < 1e-4
    assert rel_co.max() < 1e-4
    assert rel_vac.max() < 1e-5


def test_precision_study_chains(env):
    """FP32 and FP64 chains of the preset (20 outer x 50 inner updates per
    configuration, 40 configurations, two full sweeps between them) from the
    same seed, independent after thermalisation.  The host estimators on each
    chain: <P^dagger P>(r), ln <P^dagger P>(r), the connected insertions of
    the six components (both kinds and their checks) and the vacuum
    plaquettes, with jackknife errors over 20 blocks; the normalised
    differences |FP32 - FP64| / sigma pass the 3-sigma check with its
    multiple-comparison allowance.  The logarithm exists only where every
    jackknife replicate of the mean correlator is positive; at the largest
    separations the 40 configurations leave <P^dagger P> compatible with
    zero, so ln <P^dagger P> is compared at the separations where it is
    defined in both chains (<P^dagger P> itself at every separation).  The
    table of differences is printed."""
    from helpers.stats import check_sigma
    from paper_1309_3859_amd import analysis as A

    u1, configs = env
    n_conf, nb = 40, 20
    rec = {}
    for prec in (u1.FP32, u1.FP64):
        spec, sched = configs.c3_precision(prec, max_configs=n_conf)
        say("precision chain", prec, spec.levels)
        c = u1.Context(spec)
        c.init_links(sched["start"])
        c.sweeps(30)
        for _ in range(n_conf):
            # full-lattice sweeps between configurations also renew the frozen
            # boundary links, so that the configurations are not all
            # conditioned on the same boundaries
            c.sweeps(2)
            c.multilevel()
        r = c.results()
        rec[prec] = [spec.unpack(r[k][0]) for k in range(r.shape[0])]
        c.close()
    zs = []
    for name, est in [("<P+P>(r)", lambda rs: A.correlator(rs, n_blocks=nb)),
                      ("ln <P+P>(r)", lambda rs: A.log_correlator(rs, n_blocks=nb)),
                      ("<O>_P+P[r, comp, kind]", lambda rs: A.field_profile(rs, spec.comps, spec.dirs, n_blocks=nb)),
                      ("vacuum <O_sq>", lambda rs: A.jackknife(
                          A.block_means(np.array([x["vac_sq"] for x in rs]), nb), lambda v: v.mean(axis=0)))]:
        (m32, e32), (m64, e64) = est(rec[u1.FP32]), est(rec[u1.FP64])
        m32, e32, m64, e64 = (np.asarray(v, float) for v in (m32, e32, m64, e64))
        defined = np.isfinite(m32) & np.isfinite(e32) & np.isfinite(m64) & np.isfinite(e64)
        if name.startswith("ln"):
            say(f"{name}: defined in both chains at {int(defined.sum())} of {defined.size} separations")
            assert defined.sum() >= 4
            m32, e32, m64, e64 = m32[defined], e32[defined], m64[defined], e64[defined]
        else:
            assert defined.all(), name
        z = np.abs(m32 - m64) / np.sqrt(e32 ** 2 + e64 ** 2 + 1e-300)
        rel = np.abs(e64 / np.where(m64 == 0, 1.0, m64))
        say(f"{name}: n = {z.size}, max |FP32 - FP64|/sigma {z.max():.2f}, median {np.median(z):.2f}, "
            f"above 3: {int(np.sum(z > 3))}; median relative FP64 error {np.median(rel):.2e}")
        zs.append(np.ravel(z))
    ok, count, allowed, zmax, bound = check_sigma(np.concatenate(zs), nb - 1)
    say("all", sum(z.size for z in zs), "above 3 sigma", count, "allowed", allowed, "largest", zmax, "bound", bound)
    assert ok

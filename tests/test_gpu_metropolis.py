"""GPU parity of the Metropolis update (the paper's own update, Sec. II)
against the oracle, through the C ABI:
 - every checkerboard phase from identical links and counters (FP64 within
   1e-12 with identical accept decisions; FP32 storage within 2e-5 with at
   most a few decisions flipped by FP32 rounding of the acceptance test);
 - Metropolis-only trajectories (sweeps and a multilevel configuration)
   within 1e-9 in FP64;
 - equilibrium: with Metropolis + 3 overrelaxation passes the plaquette
   agrees with the heatbath chain's within 4 combined standard errors.
"""
import sys

import numpy as np
import pytest

from helpers.inputs import random_links, random_links_fp32
from paper_1309_3859_amd import analysis as A
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
    from oracle import oracle as O
    from paper_1309_3859_amd import u1ml

    u1ml.lib()
    O.build()
    return u1ml, O


DELTA = 1.3


def _pair(u1, O, ns, nt, beta, prec, levels=((2, 1, 1),), n_or=3):
    spec = u1.Spec(ensembles=[u1.Ens(ns, nt, beta, seed=51, key_id=4)], levels=list(levels), r=[1],
                   precision=prec, n_or=n_or, update=u1.UPDATE_METROPOLIS, metro_delta=DELTA)
    ctx = u1.Context(spec)
    ctx.init_links(u1.HOT)
    ref = O.Lattice(4, list(ns) + [nt], beta, seed=51, key_id=4)
    ref.set_update(2, DELTA)
    return spec, ctx, ref


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_metropolis_phases(env, prec):
    u1, O = env
    p = u1.FP64 if prec == "fp64" else u1.FP32
    spec, ctx, ref = _pair(u1, O, (6, 4, 4), 4, 1.1, p)
    V = 6 * 4 * 4 * 4
    th = random_links(V, 7) if p == u1.FP64 else random_links_fp32(V, 7)
    for tau in (0, 2):
        for mu in range(4):
            for par in (0, 1):
                ctx.set_links(th)
                ctx.set_counter(9 + mu)
                ref.set_links(th)
                ref.counter = 9 + mu
                ctx.phase(u1.METROPOLIS, mu, par, tau)
                ref.phase(2, mu, par, tau)
                d = circ_dist(ctx.links(0), ref.links())
                moved = int(np.count_nonzero(circ_dist(ref.links(), th) > 0))
                if p == u1.FP64:
                    assert d.max() < 1e-12, (tau, mu, par, d.max())
                    # identical decisions, so identical acceptance rates
                    args = ((6, 4, 4), 4, mu, par, tau)
                    assert A.acceptance_rate(th, ctx.links(0), *args) == A.acceptance_rate(th, ref.links(), *args)
                else:
                    assert int(np.count_nonzero(d > 2e-5)) <= 2, (tau, mu, par)
                assert moved > 0
    say(prec, "phases ok")


def test_metropolis_trajectories(env):
    u1, O = env
    spec, ctx, ref = _pair(u1, O, (4, 4, 4), 8, 1.0, u1.FP64, levels=((4, 2, 1), (2, 2, 1)), n_or=0)
    ref.set_links(ctx.links(0))
    ctx.sweeps(3)
    ref.sweeps(3, 0)
    assert np.max(circ_dist(ctx.links(0), ref.links())) < 1e-9
    assert ctx.counter(0) == ref.counter == 3
    th0 = ctx.links(0)
    ctx.multilevel()
    got = spec.unpack(ctx.results()[0][0])
    ospec = O.MLSpec(levels=spec.levels, r=spec.r, n_or=0)
    want = ospec.unpack(ref.multilevel(ospec))
    assert np.max(np.abs(got["C"] - want["C"])) < 1e-9
    assert np.max(circ_dist(ctx.links(0), ref.links())) < 1e-9


def test_metropolis_equilibrium_matches_heatbath(env):
    u1, O = env
    series = {}
    for upd in (u1.UPDATE_HEATBATH, u1.UPDATE_METROPOLIS):
        spec = u1.Spec(ensembles=[u1.Ens((6, 6, 6), 6, 1.0, seed=61)], levels=[(2, 1, 1)], r=[1],
                       precision=u1.FP64, n_or=3, update=upd, metro_delta=DELTA)
        ctx = u1.Context(spec)
        ctx.init_links(u1.HOT)
        ctx.sweeps(100)
        vals = []
        for _ in range(600):
            ctx.sweeps(1)
            vals.append(np.mean(ctx.plaquette()))
        v = np.array(vals)
        series[upd] = (v.mean(), A.gamma_method(v)[0])
    (m1, e1), (m2, e2) = series[u1.UPDATE_HEATBATH], series[u1.UPDATE_METROPOLIS]
    say("plaquette heatbath", m1, e1, "metropolis", m2, e2)
    assert abs(m1 - m2) < 3 * np.hypot(e1, e2)

"""More observables on the same kernels, through the C ABI:
 - the field in the plane of the charges (probes with longitudinal offsets
   l = -3 .. r + 3 and transverse offsets p1, E_par and E_perp1), history and
   spectral forms, one measurement without updates, against the oracle on the
   same links (FP64 1e-12);
 - a batched coupling scan: the plaquette susceptibility of replicas at
   beta = 0.9, 1.0 and 1.1 in one batch from the per-sweep plaquettes, with
   autocorrelation-aware errors (Gamma method), against the oracle's chains
   within 3 combined standard errors.
"""
import json
import os
import sys

import numpy as np
import pytest

from paper_1309_3859_amd import analysis as A

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
    from paper_1309_3859_amd import configs, u1ml

    u1ml.lib()
    O.build()
    return u1ml, O, configs


@pytest.mark.parametrize("form", [1, 2], ids=["history", "spectral"])
def test_in_plane_map(env, form):
    u1, O, configs = env
    spec, sched = configs.in_plane_map(r=4, margin=3, width=3, ns=10, nt=4, n_inner=1)
    spec.levels = [(2, 1, 0)]
    spec.precision = u1.FP64
    spec.form = form
    ctx = u1.Context(spec)
    assert ctx.plan["form"] == form
    ctx.init_links(sched["start"])
    ctx.sweeps(3)
    ctx.multilevel()
    got = spec.unpack(ctx.results()[0][0])
    e = spec.ensembles[0]
    ref = O.Lattice(4, list(e.ns) + [e.nt], e.beta, seed=e.seed)
    ref.set_links(ctx.links(0))
    ospec = O.MLSpec(levels=spec.levels, r=spec.r, dirs=spec.dirs, probes=spec.probes, comps=spec.comps)
    want = ospec.unpack(ref.multilevel(ospec))
    d = float(np.max(np.abs(got["CO"] - want["CO"])))
    say("in-plane map form", form, "probes", len(spec.probes), "max |dCO|", d)
    assert d < 1e-12 * max(1.0, float(np.abs(want["CO"]).max()))


def test_beta_scan_susceptibility(env):
    """The plaquette susceptibility on 4^4 at beta = 0.9, 1.0 (near this
    volume's pseudo-critical coupling) and 1.1: eight replicas per coupling in
    one batch, 10000 sweeps each after 200, errors and integrated
    autocorrelation times from the Gamma method; against the oracle's own
    chains (four of 20000 sweeps per coupling, stored by
    tests/golden/make_susceptibility.py) within 3 combined standard errors."""
    u1, O, configs = env
    with open(os.path.join(os.path.dirname(__file__), "golden", "susceptibility_4x4.json")) as f:
        gold = json.load(f)
    betas = [float(b) for b in gold["betas"]]
    n_rep, n = 8, 10000
    n_plaq = gold["n_plaquettes"]
    ens = [u1.Ens((4, 4, 4), 4, b, seed=300 + k, key_id=k) for b in betas for k in range(n_rep)]
    spec = u1.Spec(ensembles=ens, levels=[(2, 1, 1)], r=[1], precision=u1.FP64, n_or=gold["n_or"])
    ctx = u1.Context(spec)
    ctx.init_links(u1.HOT)
    ctx.sweeps(gold["therm"])
    series = np.empty((n, len(ens)))
    for i in range(n):
        ctx.sweeps(1)
        series[i] = ctx.plaquette().mean(axis=1)
    for j, b in enumerate(betas):
        res = [A.susceptibility_gamma(series[:, j * n_rep + k], n_plaq) for k in range(n_rep)]
        chi = float(np.mean([r[0] for r in res]))
        sig = float(np.sqrt(np.sum([r[1] ** 2 for r in res])) / n_rep)
        tau = max(r[2] for r in res)
        ref = gold["betas"][str(b)]
        say(f"beta {b}: GPU chi {chi:.4f} +- {sig:.4f} (tau_int <= {tau:.2f}), "
            f"oracle {ref['chi']:.4f} +- {ref['sigma']:.4f}")
        # chains of at least 100 tau_int, where the Gamma-method error is reliable
        assert n >= 100 * tau and gold["sweeps"] >= 100 * max(c["tau_int"] for c in ref["chains"])
        assert abs(chi - ref["chi"]) < 3 * np.hypot(sig, ref["sigma"])

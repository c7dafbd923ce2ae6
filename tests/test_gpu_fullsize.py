"""Parity at the workloads' full sizes, in the launch configuration bench.py
times (autotuned work-group size, HIP graphs on).

For each preset lattice: (1) sampled checkerboard phases (a heatbath phase in
the inner slabs and an overrelaxation phase of the temporal links), every link
of the full lattice compared with the oracle from identical links; (2) one
multilevel configuration without updates (k = 0, one measurement), where every
estimate is compared with the oracle's on the same links.  The largest preset
uses its on-axis probe here: its full transverse map needs the replay form.
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
    from oracle import oracle as O
    from paper_1309_3859_amd import configs, u1ml

    u1ml.lib()
    O.build()
    return u1ml, O, configs


def _preset(configs, name):
    if name == "c5":
        return configs.c5_largest(n_outer=1, n_inner=1, full_map=False)
    if name == "c3":
        return configs.c3_precision(n_outer=1, n_inner=1)
    return configs.PRESETS[name]()


def _oracle_for(O, e):
    return O.Lattice(4, list(e.ns) + [e.nt], e.beta, seed=e.seed, key_id=e.key_id)


@pytest.mark.parametrize("name", ["c2", "c3", "c4", "c5"])
def test_full_size_phases(env, name):
    u1, O, configs = env
    spec, sched = _preset(configs, name)
    ctx = u1.Context(spec)
    ctx.init_links(sched["start"])
    tune = ctx.autotune()
    ctx.sweeps(2)
    tau = spec.levels[-1][0]
    tol = 1e-12 if spec.precision == u1.FP64 else 2e-5
    for ens in sorted({0, len(spec.ensembles) - 1}):
        e = spec.ensembles[ens]
        th0 = ctx.links(ens)
        cnt = ctx.counter(ens)
        for kind, mu, parity, t in [(0, 1, 0, tau), (1, 3, 1, 0)]:
            say(name, "ensemble", ens, "block", tune["chosen_block"], "phase", kind, mu, parity, t)
            ctx.set_links(th0, ens)
            ref = _oracle_for(O, e)
            ref.set_links(th0)
            ref.counter = cnt
            ctx.phase(kind, mu, parity, t)
            ref.phase(kind, mu, parity, t)
            d = circ_dist(ctx.links(ens), ref.links())
            bad = int(np.count_nonzero(d > tol))
            say("  max", float(d.max()), "beyond tolerance", bad, "of", d.size)
            assert bad <= max(2, d.size // 100000)  # rare accept/reject flips only
            if spec.precision == u1.FP64:
                assert bad == 0


@pytest.mark.parametrize("name", ["c2", "c3", "c4", "c5"])
def test_full_size_measurement_chain(env, name):
    u1, O, configs = env
    spec, sched = _preset(configs, name)
    spec.levels = [(lv[0], 1, 0) for lv in spec.levels]  # one measurement, no updates
    spec.max_configs = 1
    ctx = u1.Context(spec)
    ctx.init_links(sched["start"])
    ctx.autotune()
    ctx.sweeps(2)
    say(name, "multilevel k=0")
    ctx.multilevel()
    res = ctx.results()[0]
    ospec = O.MLSpec(levels=spec.levels, r=spec.r, dirs=spec.dirs, probes=spec.probes, comps=spec.comps,
                     n_or=spec.n_or)
    for ens in sorted({0, len(spec.ensembles) - 1}):
        e = spec.ensembles[ens]
        ref = _oracle_for(O, e)
        ref.set_links(ctx.links(ens))
        want = ospec.unpack(ref.multilevel(ospec))
        got = spec.unpack(res[ens])
        dc = np.max(np.abs(got["C"] - want["C"]))
        say("  ensemble", ens, "max |dC|", dc)
        assert dc < 1e-12
        if spec.probes:
            rel = 1e-12 if spec.precision == u1.FP64 else 2e-5
            dco = np.max(np.abs(got["CO"] - want["CO"]))
            say("  max |dCO|", dco, "scale", np.abs(want["CO"]).max())
            assert dco < rel * max(1.0, np.abs(want["CO"]).max())
        tol_v = 1e-12 if spec.precision == u1.FP64 else 1e-6
        assert np.max(np.abs(got["vac_sq"] - want["vac_sq"])) < tol_v


def test_measurement_at_large_spatial_volume(env):
    """256^3 x 4 (N_sigma = 2^24 sites, beyond the 24-bit range of a direct
    site decode): one configuration without updates (n = 1, k = 0) equals
    the plain definitions on the same links, C(r) = mean_x conj P(x) P(x + r e_x)
    and the vacuum <O_sq> = 2 beta (1 - <cos theta_P>) of the plaquette kernel."""
    u1, O, configs = env
    ns, nt, beta = 256, 4, 1.0
    spec = u1.Spec(ensembles=[u1.Ens((ns, ns, ns), nt, beta, seed=12)], levels=[(2, 1, 0)], r=[1, 2, 5], dirs=[0],
                   precision=u1.FP32, max_configs=1)
    say("large spatial volume", ns, nt)
    ctx = u1.Context(spec)
    ctx.init_links(u1.HOT)
    ctx.multilevel()
    got = spec.unpack(ctx.results()[0, 0])
    plaq = ctx.plaquette()[0]
    th = ctx.links(0).reshape(nt, ns, ns, ns, 4)  # [t][z][y][x][mu]
    ctx.close()
    P = np.exp(1j * th[..., 3].sum(axis=0))  # [z][y][x]
    del th
    for i, r in enumerate(spec.r):
        want = np.mean(np.conj(P) * np.roll(P, -r, axis=2))
        assert abs(got["C"][i] - want) < 1e-12, (r, got["C"][i], want)
    # FP32 plaquette angles and sines in the measurement, FP64 in the plaquette kernel
    assert np.max(np.abs(got["vac_sq"] - 2 * beta * (1 - plaq))) < 2e-6


def test_update_phases_at_the_largest_lattice(env):
    """322^3 x 8 in FP32, the largest cube the planner accepts: 4.27 GB of
    links, so the kernels' 32-bit byte offsets reach 2^32 - 2.2e7 (the odd
    temporal links, updated here, are the last array).  An overrelaxation
    phase keeps the total action, the same phase applied twice restores every
    plaquette mean, and a heatbath phase raises the temporal plaquettes and
    leaves every angle in range."""
    u1, O, configs = env
    ns, nt = 322, 8
    spec = u1.Spec(ensembles=[u1.Ens((ns, ns, ns), nt, 1.0, seed=13)], levels=[(2, 1, 0)], r=[1], dirs=[0],
                   precision=u1.FP32, max_configs=1)
    info = u1.plan(spec)
    assert 2 ** 31 < 16 * ns ** 3 * nt <= info["link_bytes"] < 2 ** 32
    say("largest lattice", ns, nt, info["ws_bytes"])
    ctx = u1.Context(spec)
    ctx.init_links(u1.HOT)
    p0 = ctx.plaquette()[0]
    ctx.phase(u1.OVERRELAX, 3, 1)
    p1 = ctx.plaquette()[0]
    ctx.phase(u1.OVERRELAX, 3, 1)
    p2 = ctx.plaquette()[0]
    ctx.phase(u1.HEATBATH, 3, 1)
    p3 = ctx.plaquette()[0]
    bad = ctx.health()
    ctx.close()
    say("plaquettes", p0, p1, p2, p3)
    assert abs(p1.sum() - p0.sum()) < 1e-6
    assert np.max(np.abs(p1 - p0)) > 1e-6  # it moved action between the three temporal orientations (~1/sqrt(V))
    assert np.max(np.abs(p2 - p0)) < 1e-6
    assert p3[:3].sum() > p0[:3].sum() + 0.05
    assert np.array_equal(p3[3:], p0[3:])  # spatial plaquettes hold no temporal link
    assert bad == 0

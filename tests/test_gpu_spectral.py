"""Parity of the spectral form of the insertion estimators (plane transforms
over the plane orthogonal to the charge axis; two levels replay each
configuration), through the C ABI.

* against the history form on the same device trajectory (same links, same
  counters), one and two levels, several axes, probes of both modes and
  several probe groups, plane extents taking every radix of the plane FFT and
  extents taking the direct sums: every estimate within FP64 rounding of the
  contraction order;
* after a two-level configuration the links and counters equal those of the
  history form (the replay restores the start and repeats the trajectory);
* against the oracle's independent FP64 chain (heatbath-only trajectories,
  whose GPU/oracle link agreement is at the 1e-12 level);
* the largest preset's full 441-probe map at full size (48^3 x 12, FP32
  links), one measurement without updates, sampled probes against the oracle.
"""
import sys

import numpy as np
import pytest

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


def _disk(rad, mode=1, l=0):
    return [(l, p1, p2, mode) for p1 in range(-rad, rad + 1) for p2 in range(-rad, rad + 1) if p1 * p1 + p2 * p2 <= rad * rad]


def _run(u1, spec, form, start_seed_sweeps=2):
    spec.form = form
    ctx = u1.Context(spec)
    assert ctx.plan["form"] == (u1.FORM_SPECTRAL if form == u1.FORM_SPECTRAL else u1.FORM_HISTORY)
    ctx.init_links(u1.HOT)
    ctx.sweeps(start_seed_sweeps)
    ctx.multilevel()
    res = ctx.results()[0]
    links = [ctx.links(e) for e in range(len(spec.ensembles))]
    cnt = [ctx.counter(e) for e in range(len(spec.ensembles))]
    return res, links, cnt


def _compare(spec, ra, rb, rel):
    for e in range(len(spec.ensembles)):
        a, b = spec.unpack(ra[e]), spec.unpack(rb[e])
        scale = max(1.0, float(np.abs(a["CO"]).max()))
        d = float(np.abs(a["CO"] - b["CO"]).max())
        say("  ensemble", e, "max |dCO|", d, "scale", scale, "max |dC|", float(np.abs(a["C"] - b["C"]).max()))
        assert d <= rel * scale
        assert np.allclose(a["C"], b["C"], rtol=0, atol=1e-14)
        assert np.allclose(a["vac_sq"], b["vac_sq"], rtol=0, atol=1e-14)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_spectral_one_level_matches_history(env, prec):
    u1, O, _ = env
    mk = lambda: u1.Spec(ensembles=[u1.Ens((6, 6, 6), 4, 1.0, seed=11), u1.Ens((8, 6, 6), 6, 0.9, seed=12, key_id=3)],
                         levels=[(2, 3, 1)], r=[1, 2, 3], dirs=[0, 1, 2],
                         probes=_disk(2) + [(1, 0, 1, 0), (-1, 1, 0, 0), (0, -2, 1, 0)], comps=list(range(6)),
                         precision=u1.FP64 if prec == "fp64" else u1.FP32, n_or=3)
    say("one level", prec)
    rh, lh, ch = _run(u1, mk(), u1.FORM_HISTORY)
    rs, ls, cs = _run(u1, mk(), u1.FORM_SPECTRAL)
    for a, b in zip(lh, ls):
        assert np.array_equal(a, b)
    assert ch == cs
    _compare(mk(), rh, rs, 1e-12)


def test_spectral_transform_sizes_match_history(env):
    """Plane extents that take every radix of the plane FFT (4, 2, 3, 5) and
    extents with a prime factor above 5 (14), which take the direct sums."""
    u1, O, _ = env
    mk = lambda: u1.Spec(ensembles=[u1.Ens((6, 10, 14), 4, 1.0, seed=13), u1.Ens((12, 20, 8), 4, 0.95, seed=14, key_id=2)],
                         levels=[(2, 2, 1)], r=[1, 3], dirs=[0, 1, 2], probes=_disk(1) + [(2, 1, -1, 0)],
                         comps=[0, 2, 4], precision=u1.FP64, n_or=2)
    say("transform sizes")
    rh, lh, ch = _run(u1, mk(), u1.FORM_HISTORY)
    rs, ls, cs = _run(u1, mk(), u1.FORM_SPECTRAL)
    for a, b in zip(lh, ls):
        assert np.array_equal(a, b)
    _compare(mk(), rh, rs, 1e-12)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_spectral_two_levels_replay_matches_history(env, prec):
    u1, O, _ = env
    mk = lambda: u1.Spec(ensembles=[u1.Ens((6, 6, 6), 8, 1.0, seed=21)], levels=[(4, 2, 1), (2, 3, 1)], r=[1, 2],
                         dirs=[0, 2], probes=_disk(1) + [(2, 1, -1, 0)], comps=[0, 1, 3, 5],
                         precision=u1.FP64 if prec == "fp64" else u1.FP32, n_or=2)
    say("two levels", prec)
    rh, lh, ch = _run(u1, mk(), u1.FORM_HISTORY)
    rs, ls, cs = _run(u1, mk(), u1.FORM_SPECTRAL)
    for a, b in zip(lh, ls):
        assert np.array_equal(a, b)  # the replay left the links where one pass leaves them
    assert ch == cs
    _compare(mk(), rh, rs, 1e-12)


def test_spectral_two_levels_against_oracle(env):
    u1, O, _ = env
    spec = u1.Spec(ensembles=[u1.Ens((4, 4, 4), 8, 1.0, seed=31)], levels=[(4, 2, 1), (2, 2, 1)], r=[1, 2],
                   dirs=[0, 1], probes=_disk(1) + [(1, 1, 1, 0)], comps=list(range(6)), precision=u1.FP64, n_or=0,
                   form=u1.FORM_SPECTRAL)
    ctx = u1.Context(spec)
    ctx.init_links(u1.HOT)
    ctx.sweeps(1)
    th0, cnt = ctx.links(0), ctx.counter(0)
    ctx.multilevel()
    got = spec.unpack(ctx.results()[0][0])
    e = spec.ensembles[0]
    ref = O.Lattice(4, list(e.ns) + [e.nt], e.beta, seed=e.seed, key_id=e.key_id)
    ref.set_links(th0)
    ref.counter = cnt
    ospec = O.MLSpec(levels=spec.levels, r=spec.r, dirs=spec.dirs, probes=spec.probes, comps=spec.comps, n_or=0)
    want = ospec.unpack(ref.multilevel(ospec))
    scale = max(1.0, float(np.abs(want["CO"]).max()))
    d = float(np.abs(got["CO"] - want["CO"]).max())
    say("vs oracle: max |dCO|", d, "scale", scale, "max |dC|", float(np.abs(got["C"] - want["C"]).max()))
    assert d < 1e-9 * scale
    assert np.max(np.abs(got["C"] - want["C"])) < 1e-10
    assert np.max(np.abs(got["vac_sq"] - want["vac_sq"])) < 1e-10


def test_full_map_of_largest_preset_sampled(env):
    """48^3 x 12, two levels, 441 probes x 19 r x 6 components in the spectral
    form at full size; one measurement without updates, so the estimates are
    functions of the links alone; sampled probes and separations against the
    oracle on the same links."""
    u1, O, configs = env
    spec, sched = configs.c5_largest(n_outer=1, n_inner=1, full_map=True)
    spec.levels = [(4, 1, 0), (2, 1, 0)]
    ctx = u1.Context(spec)
    say("C5 full map: form", ctx.plan["form"], "workspace", ctx.plan["ws_bytes"])
    assert ctx.plan["form"] == u1.FORM_SPECTRAL
    ctx.init_links(sched["start"])
    ctx.sweeps(2)
    ctx.multilevel()
    got = spec.unpack(ctx.results()[0][0])
    pick_p = [spec.probes.index(p) for p in [(0, 0, 0, 1), (0, 12, 0, 1), (0, 0, -12, 1), (0, 8, 8, 1),
                                              (0, -5, 7, 1)]]
    pick_r = [0, 9, 18]  # r = 2, 11, 20
    e = spec.ensembles[0]
    ref = O.Lattice(4, list(e.ns) + [e.nt], e.beta, seed=e.seed, key_id=e.key_id)
    ref.set_links(ctx.links(0))
    ospec = O.MLSpec(levels=spec.levels, r=[spec.r[i] for i in pick_r], dirs=spec.dirs,
                     probes=[spec.probes[i] for i in pick_p], comps=spec.comps, n_or=spec.n_or)
    want = ospec.unpack(ref.multilevel(ospec))
    sub = got["CO"][np.ix_(pick_r, pick_p)]
    scale = max(1.0, float(np.abs(want["CO"]).max()))
    d = float(np.abs(sub - want["CO"]).max())
    say("  sampled max |dCO|", d, "scale", scale)
    assert d < 2e-5 * scale
    assert np.max(np.abs(got["C"][pick_r] - want["C"])) < 1e-12

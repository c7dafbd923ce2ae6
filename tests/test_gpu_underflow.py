"""Slab products below the range of FP64 (Sec. II.C.2-3): on many thin slabs
the per-site correlator products prod_S [T](S) fall far below 2^-1074, where
a plain FP64 product is zero.  The GPU records mantissas relative to 2^E(r)
and E(r), like the oracle; both are compared on the same start and counters
(heatbath-only sweeps, so the two trajectories stay within rounding), in the
history and spectral forms, one and two levels.  Sizes: 2^3 x 3200 (1600
thin slabs, E(r) near -1400) and 4 x 2^2 x 3200 (complex estimates at r = 1, 2,
E(r) near -1440 and -1520)."""
import sys

import numpy as np
import pytest

from helpers.inputs import random_links

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


CASES = [
    ((2, 2, 2), 3200, [(2, 3, 1)], [1]),
    ((2, 2, 2), 3200, [(4, 2, 1), (2, 2, 1)], [1]),
    ((4, 2, 2), 3200, [(2, 3, 1)], [1, 2]),
]


def _rel(m_a, e_a, m_b, e_b):
    """|a - b| / |b| for a = m_a 2^e_a, b = m_b 2^e_b (per separation)."""
    a = np.ldexp(m_a.real, e_a - e_b) + 1j * np.ldexp(m_a.imag, e_a - e_b)
    return np.abs(a - m_b) / np.abs(m_b)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_products_below_fp64_range_match_oracle(env, case):
    u1, O = env
    ns, nt, levels, r = CASES[case]
    V = int(np.prod(ns)) * nt
    probes, comps = [(0, 0, 0, 1)], [0, 3]
    th = random_links(V, 31)
    rec = {}
    for form in (u1.FORM_HISTORY, u1.FORM_SPECTRAL):
        say("underflow case", ns, nt, levels, "form", form)
        spec = u1.Spec(ensembles=[u1.Ens(ns, nt, 1.0, seed=9)], levels=levels, r=r, dirs=[0], probes=probes,
                       comps=comps, precision=u1.FP64, n_or=0, form=form)
        ctx = u1.Context(spec)
        ctx.set_links(th)
        ctx.set_counter(4)
        ctx.multilevel()
        rec[form] = spec.unpack(ctx.results()[0, 0])
        ctx.close()
    ref = O.Lattice(4, list(ns) + [nt], 1.0, seed=9)
    ref.set_links(th)
    ref.counter = 4
    ospec = O.MLSpec(levels=levels, r=r, dirs=[0], probes=probes, comps=comps, n_or=0)
    want = ospec.unpack(ref.multilevel(ospec))
    say("  oracle E(r)", want["exp"], "C mantissa", want["C_mant"])
    assert np.all(want["exp"] < -1074)  # the plain FP64 products are zero
    assert np.all(want["C"] == 0)
    for form, got in rec.items():
        say("  form", form, "E(r)", got["exp"])
        # E(r) is decided in FP64 on both sides from inputs equal up to rounding
        assert np.all(np.abs(got["exp"] - want["exp"]) <= 1)
        dc = _rel(got["C_mant"], got["exp"], want["C_mant"], want["exp"])
        ex = got["exp"][:, None, None, None]
        dco = _rel(got["CO_mant"], ex, want["CO_mant"], want["exp"][:, None, None, None])
        say("  max rel |dC|", dc.max(), "max rel |dCO|", dco.max())
        assert dc.max() < 1e-6
        assert dco.max() < 1e-6
    # the two forms run the same trajectory: identical correlators, insertions to rounding
    h, s = rec[u1.FORM_HISTORY], rec[u1.FORM_SPECTRAL]
    assert np.array_equal(h["exp"], s["exp"])
    assert np.array_equal(h["C_mant"], s["C_mant"])
    d = np.abs(h["CO_mant"] - s["CO_mant"]).max() / np.abs(h["CO_mant"]).max()
    say("  history vs spectral max rel |dCO|", d)
    assert d < 1e-12

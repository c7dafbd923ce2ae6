"""A batch run as two, three or four lanes on as many streams (two is the
default for two or more ensembles) gives the same links, counters and
estimates, bit for bit, as the whole batch on one stream: one and two levels,
history and spectral forms (the spectral two-level replay copies and clears
only its own lane's ensembles), and a lane count changed between
configurations continues the same chain."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def u1():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1309_3859_amd import u1ml

    u1ml.lib()
    return u1ml


def _disk1():
    return [(0, 0, 0, 1), (0, 1, 0, 1), (0, -1, 0, 1), (0, 0, 1, 1), (0, 0, -1, 1)]


def _spec(u1, levels, form):
    return u1.Spec(ensembles=[u1.Ens((6, 6, 6), 8, 1.0, seed=41), u1.Ens((4, 4, 4), 8, 0.95, seed=42, key_id=1),
                              u1.Ens((8, 6, 6), 8, 1.02, seed=43, key_id=2)],
                   levels=levels, r=[1, 2], dirs=[0, 1], probes=_disk1(), comps=[0, 3], precision=u1.FP32, n_or=2,
                   form=form, max_configs=2)


def _run(u1, spec, lanes):
    ctx = u1.Context(spec)
    ctx.set_lanes(lanes)
    ctx.init_links(u1.HOT)
    ctx.sweeps(3)
    ctx.multilevel()
    ctx.multilevel()
    res = ctx.results()
    links = [ctx.links(e) for e in range(len(spec.ensembles))]
    cnt = [ctx.counter(e) for e in range(len(spec.ensembles))]
    return res, links, cnt


@pytest.mark.parametrize("levels", [[(2, 3, 1)], [(4, 2, 1), (2, 2, 1)]], ids=["one_level", "two_levels"])
@pytest.mark.parametrize("form", [1, 2], ids=["history", "spectral"])
@pytest.mark.parametrize("lanes", [2, 3])
def test_lanes_bit_identical(u1, levels, form, lanes):
    say("lanes", lanes, levels, "form", form)
    r1, l1, c1 = _run(u1, _spec(u1, levels, form), 1)
    r2, l2, c2 = _run(u1, _spec(u1, levels, form), lanes)
    assert c1 == c2
    for a, b in zip(l1, l2):
        assert np.array_equal(a, b)
    assert np.array_equal(r1, r2)


def _spec5(u1):
    return u1.Spec(ensembles=[u1.Ens((6, 6, 6), 8, 1.0, seed=41), u1.Ens((4, 4, 4), 8, 0.95, seed=42, key_id=1),
                              u1.Ens((8, 6, 6), 8, 1.02, seed=43, key_id=2), u1.Ens((4, 4, 4), 4, 0.99, seed=44, key_id=3),
                              u1.Ens((6, 4, 4), 6, 1.01, seed=45, key_id=4)],
                   levels=[(2, 2, 1)], r=[1, 2], dirs=[0], probes=_disk1(), comps=[0, 3], precision=u1.FP32, n_or=2,
                   form=1, max_configs=3)


def test_lane_count_changed_between_configurations(u1):
    """Five ensembles: four lanes, then one, then three, one configuration
    each, equal bit for bit to the same three configurations on one lane."""
    def run(seq):
        spec = _spec5(u1)
        ctx = u1.Context(spec)
        ctx.init_links(u1.HOT)
        for n in seq:
            ctx.set_lanes(n)
            ctx.sweeps(1)
            ctx.multilevel()
        return ctx.results(), [ctx.links(e) for e in range(5)], [ctx.counter(e) for e in range(5)]

    say("lanes 4, 1, 3 against 1, 1, 1")
    ra, la, ca = run([4, 1, 3])
    rb, lb, cb = run([1, 1, 1])
    assert ca == cb
    for a, b in zip(la, lb):
        assert np.array_equal(a, b)
    assert ra.shape[0] == 3
    assert np.array_equal(ra, rb)


def test_set_lanes_rejects_bad_counts(u1):
    spec = u1.Spec(ensembles=[u1.Ens((4, 4, 4), 4, 1.0)], levels=[(2, 1, 1)], r=[1])
    ctx = u1.Context(spec)
    for bad in (0, 2, 5):
        with pytest.raises(u1.U1MLError):
            ctx.set_lanes(bad)
    ctx.set_lanes(1)
    c5 = u1.Context(_spec5(u1))
    for bad in (0, 5, 6):
        with pytest.raises(u1.U1MLError):
            c5.set_lanes(bad)
    for ok in (4, 3, 2, 1):
        c5.set_lanes(ok)


@pytest.mark.parametrize("lanes", [1, 2, 3])
def test_results_ring_keeps_every_configuration(u1, lanes):
    """Three configurations left in the device ring equal the same three
    configurations copied out one at a time (every ring slot holds its own
    record, for every ensemble of the batch)."""
    mk = lambda cap: _spec(u1, [(2, 2, 1)], 1)
    a = mk(3)
    a.max_configs = 3
    ca = u1.Context(a)
    ca.set_lanes(lanes)
    ca.init_links(u1.HOT)
    for _ in range(3):
        ca.multilevel()
    ring = ca.results()
    b = mk(1)
    b.max_configs = 1
    cb = u1.Context(b)
    cb.set_lanes(lanes)
    cb.init_links(u1.HOT)
    one = []
    for _ in range(3):
        cb.multilevel()
        one.append(cb.results()[0])
    assert ring.shape[0] == 3
    for k in range(3):
        assert np.array_equal(ring[k], one[k]), k
    assert not np.array_equal(one[0], one[1])

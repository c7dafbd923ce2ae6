"""The streaming-model byte count of a checkerboard phase (u1ml_phase_bytes,
the numerator of the bench line's roofline) against an independent count:
the distinct link angles the phase reads (the staples of every updated link,
plus its own angle for overrelaxation and Metropolis) and the links it writes,
enumerated here site by site (Sec. II, the staple sum; Sec. II.C.1, the frozen
layers).  Also pins the closed forms of a full-lattice phase (heatbath 8 words
per update, overrelaxation 9) and the C4 figure of the dominant kernel."""
import itertools

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def u1():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1309_3859_amd import u1ml

    u1ml.lib()
    return u1ml


def _count(ns, nt, kind, mu, parity, tau):
    """(distinct words read, words written) of one phase, by enumeration."""
    ext = list(ns) + [nt]

    def link(site, d):
        return (tuple(site), d)

    def shift(site, d, s):
        out = list(site)
        out[d] = (out[d] + s) % ext[d]
        return out

    reads, writes = set(), set()
    for site in itertools.product(*[range(n) for n in ext]):
        if sum(site) % 2 != parity:
            continue
        if mu < 3 and tau > 1 and site[3] % tau == 0:
            continue
        writes.add(link(site, mu))
        if kind != 0:
            reads.add(link(site, mu))
        for nu in range(4):
            if nu == mu:
                continue
            xm, xn, xmn = shift(site, mu, 1), shift(site, nu, 1), shift(site, nu, -1)
            xmmn = shift(xm, nu, -1)
            reads.update({link(xm, nu), link(xn, mu), link(site, nu), link(xmn, nu), link(xmmn, nu), link(xmn, mu)})
    return len(reads), len(writes)


@pytest.mark.parametrize("ns,nt", [((4, 6, 4), 4), ((2, 4, 4), 8)])
@pytest.mark.parametrize("precision", [0, 1])
def test_phase_bytes_match_enumeration(u1, ns, nt, precision):
    spec = u1.Spec(ensembles=[u1.Ens(ns, nt, 1.0)], levels=[(4, 1, 1), (2, 1, 1)], r=[1], precision=precision)
    ctx = u1.Context(spec)
    word = 8 if precision == 0 else 4
    V = int(np.prod(ns)) * nt
    for kind, mu, parity, tau in itertools.product((0, 1, 2), range(4), (0, 1), (0, 2, 4)):
        b, u = ctx.phase_bytes(kind, mu, parity, tau)
        r, w = _count(ns, nt, kind, mu, parity, tau)
        assert (b, u) == ((r + w) * word, w), (kind, mu, parity, tau)
        if tau == 0:  # full lattice: 8 words per heatbath update, 9 with the own angle
            assert u == V // 2 and b == (8 if kind == 0 else 9) * word * u


def test_c4_dominant_kernel_bytes(u1):
    from paper_1309_3859_amd import configs

    spec, _ = configs.c4_batched()
    b, u = u1.Context(spec).phase_bytes(1, 0, 0, 2)
    assert (b, u) == (19_719_168, 410_816)

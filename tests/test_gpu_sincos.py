"""The library's FP64 sine and cosine (Cody-Waite reduction by pi/2 in three
parts and degree-5 polynomials in r^2 fitted by a Remez exchange) against
libm through numpy on the arguments the library meets: angle sums of up to
four links (|x| <= 4 pi), pi u for u in (0, 1), slab sums of temporal links
(|x| <= N_t pi), with multiples of pi/4 and pi/2 and their neighbours where
the reduction changes quadrant.  Bound: 2 ulp of 1 (4.4e-16) absolute, and
at most 1 ulp relative for |result| >= 1/2."""
import sys

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


def test_sincos_within_two_ulp(u1):
    import torch

    rng = np.random.default_rng(11)
    k = np.arange(-64, 65)
    edges = np.concatenate([k * np.pi / 4, k * np.pi / 2])
    x = np.concatenate([rng.uniform(-4 * np.pi, 4 * np.pi, 400_000), np.pi * rng.uniform(0, 1, 100_000),
                        rng.uniform(-40 * np.pi, 40 * np.pi, 100_000), edges, np.nextafter(edges, 1e9),
                        np.nextafter(edges, -1e9), [0.0, -0.0, 1e-300, -1e-300, 1e-9, 4096.5]])
    s, c = u1.sincos_fill(torch.from_numpy(x).cuda())
    s, c = s.cpu().numpy(), c.cpu().numpy()
    es, ec = np.abs(s - np.sin(x)), np.abs(c - np.cos(x))
    print("max abs err sin", es.max(), "cos", ec.max(), flush=True)
    assert es.max() <= 4.5e-16 and ec.max() <= 4.5e-16
    for got, ref in ((s, np.sin(x)), (c, np.cos(x))):
        big = np.abs(ref) >= 0.5
        ulp = np.spacing(np.abs(ref[big]))
        assert np.all(np.abs(got[big] - ref[big]) <= ulp)
    assert s[-6] == 0.0 and c[-6] == 1.0

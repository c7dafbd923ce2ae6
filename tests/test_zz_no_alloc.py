"""The allocation-free plaquette call (u1ml_plaquette_noalloc: partial sums
in the library's static scratch, output in device memory, no allocation and
no synchronisation) against u1ml_plaquette on the same links, bit for bit:
two calls in a row, the second on a smaller batch, so the second reads
none of the first call's partial sums; and the limit on the batch size."""
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
    from paper_1309_3859_amd import u1ml

    u1ml.lib()
    return u1ml, torch


def _ctx(u1, shapes, precision):
    ens = [u1.Ens(ns, nt, 0.95 + 0.01 * j, seed=13, key_id=j) for j, (ns, nt) in enumerate(shapes)]
    spec = u1.Spec(ensembles=ens, levels=[(2, 1, 1)], r=[1], precision=precision, n_or=1)
    c = u1.Context(spec)
    c.init_links(u1.HOT)
    c.sweeps(2)
    return c


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_noalloc_plaquette_equals_plaquette(env, precision):
    u1, torch = env
    big = [((8, 8, 8), 8), ((6, 6, 6), 4), ((10, 8, 6), 6), ((4, 4, 4), 8), ((12, 12, 12), 4)]
    small = [((4, 4, 4), 4), ((6, 4, 4), 2)]
    for shapes in (big, small):
        say("noalloc plaquette", precision, shapes)
        c = _ctx(u1, shapes, precision)
        want = c.plaquette()
        out = torch.full((len(shapes) * 6,), float("nan"), dtype=torch.float64, device="cuda")
        c.plaquette_noalloc(out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().reshape(len(shapes), 6)
        assert np.array_equal(got, want), np.abs(got - want).max()
        c.close()


def test_noalloc_plaquette_limits(env):
    u1, torch = env
    c = _ctx(u1, [((2, 2, 2), 2)] * 33, 1)
    out = torch.zeros(33 * 6, dtype=torch.float64, device="cuda")
    with pytest.raises(u1.U1MLError):
        c.plaquette_noalloc(out)
    c.close()
    spec = u1.Spec(ensembles=[u1.Ens((4, 4, 4), 4, 1.0)], levels=[(2, 1, 1)], r=[1])
    c = u1.Context(spec)
    with pytest.raises(u1.U1MLError):  # links never set
        c.plaquette_noalloc(torch.zeros(6, dtype=torch.float64, device="cuda"))
    c.close()

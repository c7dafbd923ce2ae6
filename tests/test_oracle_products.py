"""Oracle slab products and final estimators beyond the range of FP64.

The correlator is a product over slabs of slab averages whose modulus is
below one (Sec. II.C.2), so on a lattice of many slabs it falls below the
smallest FP64 number; the oracle carries every product as a mantissa and a
binary exponent and stores C and CO as mantissas relative to 2^E(r), E(r) the
largest exponent of the per-site products.  Pinned here against:
  - the exact value of a product of 1000 factors 1e-3 (log10 = -3000, where
    the plain FP64 product is zero);
  - products and the final sums of Sec. II.C.2-3 evaluated in 40-digit
    arbitrary-exponent arithmetic (mpmath) on synthetic slab averages;
  - the plain FP64 definition where nothing leaves the range.
"""
import math

import mpmath as mp
import numpy as np


def _log10(m: complex, e: int) -> float:
    return math.log10(abs(m)) + e * math.log10(2.0)


def test_product_of_1000_factors_1e_minus_3(orc):
    assert np.prod(np.full(1000, 1e-3)) == 0.0  # the plain FP64 product underflows
    m, e = orc.scaled_product(np.full(1000, 1e-3))
    assert 1.0 <= max(abs(m.real), abs(m.imag)) < 2.0
    assert abs(_log10(m, e) + 3000.0) < 1e-11
    assert m.imag == 0.0 and m.real > 0


def test_products_against_arbitrary_precision(orc):
    rng = np.random.default_rng(11)
    n = 400
    mod = 10.0 ** rng.uniform(-5, 0, n)
    z = mod * np.exp(1j * rng.uniform(-np.pi, np.pi, n))
    m, e = orc.scaled_product(z)
    mp.mp.dps = 40
    exact = mp.mpc(1)
    for v in z:
        exact *= mp.mpc(float(v.real), float(v.imag))
    got = mp.mpc(m.real, m.imag) * mp.mpf(2) ** e
    assert abs(got - exact) / abs(exact) < 1e-12
    # rescaling every factor by 2^k moves only the exponent, by n k
    m2, e2 = orc.scaled_product(z * 2.0 ** 7)
    assert m2 == m and e2 == e + 7 * n


def _synthetic(rng, shape, lo, hi):
    mod = 10.0 ** rng.uniform(lo, hi, shape)
    return mod * np.exp(1j * rng.uniform(-np.pi, np.pi, shape))


def _exact_estimates(at, ato, nsig, nt):
    """C(r) and CO(r, p, c, k) of Sec. II.C.2-3 in mpmath from the averages."""
    mp.mp.dps = 40
    nd, nr, S, _ = at.shape
    C = []
    CO = np.empty(ato.shape[1:5], dtype=object)
    for ir in range(nr):
        tot = mp.mpc(0)
        P = {}
        for d in range(nd):
            for x in range(nsig):
                p = mp.mpc(1)
                for s in range(S):
                    p *= mp.mpc(float(at[d, ir, s, x].real), float(at[d, ir, s, x].imag))
                P[d, x] = p
                tot += p
        C.append(tot / (nsig * nd))
        for idx in np.ndindex(*ato.shape[2:5]):
            acc = mp.mpc(0)
            for d in range(nd):
                for x in range(nsig):
                    for s in range(S):
                        a = mp.mpc(float(at[d, ir, s, x].real), float(at[d, ir, s, x].imag))
                        b = ato[(d, ir) + idx + (s, x)]
                        acc += mp.mpc(float(b.real), float(b.imag)) * P[d, x] / a
            CO[(ir,) + idx] = acc / (nsig * nd * nt)
    return C, CO


def test_final_estimators_beyond_fp64_range(orc):
    """300 slabs of averages with moduli 1e-4..1e-2: every per-site product is
    near 1e-900, far below FP64; mantissa * 2^E(r) equals the exact sums."""
    rng = np.random.default_rng(5)
    nsig, nt, S = 8, 600, 300
    spec = orc.MLSpec(levels=[(2, 1, 1)], r=[1, 2], dirs=[0, 1], probes=[(0, 0, 0, 0)], comps=[0, 3])
    at = _synthetic(rng, (2, 2, S, nsig), -4, -2)
    ato = _synthetic(rng, (2, 2, 1, 2, 2, S, nsig), -1, 0.5)
    out = spec.unpack(orc.ml_finalize(spec, nsig, nt, at, ato))
    C, CO = _exact_estimates(at, ato, nsig, nt)
    for ir in range(2):
        assert out["C"][ir] == 0.0  # the plain value is not representable
        E = int(out["exp"][ir])
        assert E < -2500
        got = mp.mpc(out["C_mant"][ir].real, out["C_mant"][ir].imag) * mp.mpf(2) ** E
        assert abs(got - C[ir]) <= 1e-12 * abs(C[ir])
        # E(r) is the largest binary exponent of the per-site products
        exps = [orc.scaled_product(at[d, ir, :, x])[1] for d in range(2) for x in range(nsig)]
        assert E == max(exps)
        for idx in np.ndindex(1, 2, 2):
            v = out["CO_mant"][(ir,) + idx]
            got = mp.mpc(v.real, v.imag) * mp.mpf(2) ** E
            want = CO[(ir,) + idx]
            assert abs(got - want) <= 1e-12 * abs(want)


def test_final_estimators_equal_plain_products_in_range(orc):
    rng = np.random.default_rng(6)
    nsig, nt, S = 12, 8, 4
    spec = orc.MLSpec(levels=[(2, 1, 1)], r=[1, 3], dirs=[0, 2], probes=[(1, 0, 1, 0), (0, 0, 0, 1)],
                      comps=[1, 5])
    at = _synthetic(rng, (2, 2, S, nsig), -1, 0)
    ato = _synthetic(rng, (2, 2, 2, 2, 2, S, nsig), -1, 0.5)
    out = spec.unpack(orc.ml_finalize(spec, nsig, nt, at, ato))
    P = np.prod(at, axis=2)  # [d, r, x]
    C = P.sum(axis=(0, 2)) / (nsig * 2)
    np.testing.assert_allclose(out["C"], C, rtol=1e-14, atol=0)
    W = P[:, :, None, :] / at  # [d, r, S, x]: products over the other slabs
    CO = np.einsum("drpcksx,drsx->rpck", ato, W) / (nsig * 2 * nt)
    np.testing.assert_allclose(out["CO"], CO, rtol=1e-13, atol=0)

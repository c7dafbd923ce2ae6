"""Oracle multilevel estimators: exact special cases.

 - n = 1, k = 0: every slab average is the single current value, so the
   estimators reduce to the plain definitions of the paper (Sec. II.B-C):
   C(r) = mean_x,mu P^dagger(x) P(x + r mu) with P the product of temporal
   links, and CO = mean_x,mu P^dagger P (1/N_t) sum_t O(x0, t).  Those plain
   definitions are evaluated here with numpy, from the link array.
 - two levels with n_2 = 1, k_2 = 0 equal one level of thickness 4.
 - C(N_s - r) = conj C(r) for every configuration.
 - P^dagger(x) P(x + r mu) = product of the plaquettes P_{mu t} of the strip.
"""
import numpy as np
import pytest

FRAME_PLANES = {  # frame component -> (a, b) in terms of (e_par, e_perp1, e_perp2, t)
    0: ("par", "t"), 1: ("p1", "t"), 2: ("p2", "t"),
    3: ("p1", "p2"), 4: ("p2", "par"), 5: ("par", "p1"),
}


def _fields(th, L):
    """Link angles as an array [mu, t, z, y, x] (x fastest in the site index)."""
    Nx, Ny, Nz, Nt = L
    return th.reshape(Nt, Nz, Ny, Nx, 4).transpose(4, 0, 1, 2, 3)


def _axis(mu):
    return 3 - mu  # x -> 3, y -> 2, z -> 1, t -> 0 in [t, z, y, x]


def _plaq(U, a, b):
    """theta_a(y) + theta_b(y + a) - theta_a(y + b) - theta_b(y) on the whole lattice."""
    return U[a] + np.roll(U[b], -1, _axis(a)) - np.roll(U[a], -1, _axis(b)) - U[b]


def _polyakov(U):
    return np.prod(np.exp(1j * U[3]), axis=0)  # [z, y, x]


def _plain_estimates(th, L, beta, r_list, dirs, probes, comps):
    U = _fields(th, L)
    P = _polyakov(U)
    Nt = L[3]
    C = np.zeros(len(r_list), complex)
    CO = np.zeros((len(r_list), len(probes), len(comps), 2), complex)
    for mu in dirs:
        e = {"par": mu, "p1": (mu + 1) % 3, "p2": (mu + 2) % 3, "t": 3}
        for ir, r in enumerate(r_list):
            PP = np.conj(P) * np.roll(P, -r, _axis(mu) - 1)
            C[ir] += PP.mean()
            for ic, c in enumerate(comps):
                a, b = (e[k] for k in FRAME_PLANES[c])
                thp = _plaq(U, a, b)
                Osq = (2 * beta * (1 - np.cos(thp))).sum(axis=0)  # sum over t, [z, y, x]
                Olin = (np.sqrt(beta) * np.sin(thp)).sum(axis=0)
                spans = c in (0, 4, 5)
                for ip, (l, p1, p2, mode) in enumerate(probes):
                    ll = l + (((r - 1) // 2 if spans else r // 2) if mode else 0)
                    sh = [0, 0, 0]
                    sh[_axis(e["par"]) - 1] -= ll
                    sh[_axis(e["p1"]) - 1] -= p1
                    sh[_axis(e["p2"]) - 1] -= p2
                    for kind, O in enumerate((Osq, Olin)):
                        Oy = np.roll(O, sh, axis=(0, 1, 2))
                        CO[ir, ip, ic, kind] += (PP * Oy).mean() / Nt
    return C / len(dirs), CO / len(dirs)


PROBES = [(0, 0, 0, 1), (1, 1, 0, 1), (0, -1, 2, 0), (2, 0, 1, 1)]


@pytest.mark.parametrize("levels,L", [
    ([(2, 1, 0)], [4, 4, 6, 4]),
    ([(4, 1, 0)], [6, 4, 4, 8]),
    ([(4, 1, 0), (2, 1, 0)], [4, 6, 4, 8]),
])
def test_single_measurement_reduces_to_plain_definitions(orc, levels, L):
    beta = 1.1
    lat = orc.Lattice(4, L, beta, seed=3)
    lat.init(1)
    lat.sweeps(2)
    th = lat.links()
    r_list = [1, 2, 3]
    spec = orc.MLSpec(levels=levels, r=r_list, dirs=[0, 1, 2], probes=PROBES, comps=list(range(6)))
    got = spec.unpack(lat.multilevel(spec))
    assert np.array_equal(lat.links(), th)  # k = 0: nothing was updated
    C, CO = _plain_estimates(th, L, beta, r_list, [0, 1, 2], PROBES, list(range(6)))
    np.testing.assert_allclose(got["C"], C, rtol=0, atol=1e-13)
    np.testing.assert_allclose(got["CO"], CO, rtol=0, atol=1e-12)
    # vacuum <O>: the plain plaquette means per absolute orientation
    U = _fields(th, L)
    planes = [(0, 3), (1, 3), (2, 3), (1, 2), (2, 0), (0, 1)]
    for o, (a, b) in enumerate(planes):
        thp = _plaq(U, a, b)
        assert abs(got["vac_sq"][o] - (2 * beta * (1 - np.cos(thp))).mean()) < 1e-13
        assert abs(got["vac_lin"][o] - (np.sqrt(beta) * np.sin(thp)).mean()) < 1e-13


def test_two_levels_with_trivial_inner_level_equal_one_thick_level(orc):
    L, beta = [4, 4, 4, 8], 1.0
    a = orc.Lattice(4, L, beta, seed=9, key_id=2)
    a.init(1)
    a.sweeps(3)
    b = orc.Lattice(4, L, beta, seed=9, key_id=2)
    b.set_links(a.links())
    b.counter = a.counter
    kw = dict(r=[1, 2], dirs=[0, 2], probes=PROBES[:2], comps=[0, 3, 4])
    two = orc.MLSpec(levels=[(4, 5, 1), (2, 1, 0)], **kw)
    one = orc.MLSpec(levels=[(4, 5, 1)], **kw)
    ra, rb = two.unpack(a.multilevel(two)), one.unpack(b.multilevel(one))
    assert np.array_equal(a.links(), b.links())
    np.testing.assert_allclose(ra["C"], rb["C"], rtol=0, atol=1e-14)
    np.testing.assert_allclose(ra["CO"], rb["CO"], rtol=0, atol=1e-13)


def test_correlator_reflection(orc):
    """C(N_s - r) = conj C(r) per configuration (P^dagger(x) P(x - r) summed over x)."""
    L = [6, 6, 6, 4]
    lat = orc.Lattice(4, L, 1.0, seed=4)
    lat.init(1)
    lat.sweeps(3)
    spec = orc.MLSpec(levels=[(2, 3, 1)], r=[1, 2, 3, 4, 5], dirs=[0, 1])
    C = spec.unpack(lat.multilevel(spec))["C"]
    for r in (1, 2):
        assert abs(C[6 - r - 1] - np.conj(C[r - 1])) < 1e-15 + 1e-12 * abs(C[r - 1])


def test_polyakov_pair_equals_strip_of_plaquettes(orc):
    L = [4, 6, 4, 4]
    lat = orc.Lattice(4, L, 1.0, seed=6)
    lat.init(1)
    th = lat.links()
    P = _polyakov(_fields(th, L))
    Nsig = L[0] * L[1] * L[2]
    for mu in range(3):
        for r in (1, 2):
            for xs in (0, 5, 17):
                x, y, z = xs % L[0], (xs // L[0]) % L[1], xs // (L[0] * L[1])
                c = [x, y, z]
                c2 = list(c)
                c2[mu] = (c2[mu] + r) % L[mu]
                lhs = np.conj(P[z, y, x]) * P[c2[2], c2[1], c2[0]]
                ang = 0.0
                for k in range(r):
                    ck = list(c)
                    ck[mu] = (ck[mu] + k) % L[mu]
                    sk = ck[0] + L[0] * (ck[1] + L[1] * ck[2])
                    for t in range(L[3]):
                        ang += lat.plaq_angle(sk + Nsig * t, mu, 3)
                assert abs(lhs - np.exp(1j * ang)) < 1e-12

"""ctypes binding of the FP64 CPU oracle (``libu1oracle.so``).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow reference that the GPU
library is checked against.  Only the test-suite, ``__graft_entry__.smoke()`` and
the benchmark's CPU-baseline leg may import this module.  It never imports the
GPU package and the GPU package never imports it.

Paper: Amado, Cardoso, Bicudo, arXiv 1309.3859 (Sec. II, II.C, Algorithm 1).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libu1oracle.so")
_lib = None

DOM_HB, DOM_INIT, DOM_METRO, DOM_TEST = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with plain gcc (no FP contraction)."""
    args = ["make", "-C", _HERE]
    if force:
        args.insert(1, "-B")
    subprocess.run(args, check=True, stdout=subprocess.DEVNULL)
    return _LIB_PATH


class _Spec(C.Structure):
    _fields_ = [
        ("n_levels", C.c_int),
        ("tau", C.c_int * 2),
        ("n_iter", C.c_int * 2),
        ("k_sweeps", C.c_int * 2),
        ("n_or", C.c_int),
        ("n_dirs", C.c_int),
        ("dirs", C.c_int * 3),
        ("n_r", C.c_int),
        ("r", C.POINTER(C.c_int)),
        ("n_probe", C.c_int),
        ("probe", C.POINTER(C.c_int)),
        ("n_comp", C.c_int),
        ("comp", C.POINTER(C.c_int)),
        ("multihit", C.c_int),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        u32, dbl, i32, lng, vp = C.c_uint32, C.c_double, C.c_int, C.c_long, C.c_void_p
        pd = C.POINTER(C.c_double)
        L.orc_philox4x32_10.argtypes = [C.POINTER(u32), C.POINTER(u32), C.POINTER(u32)]
        L.orc_vonmises.argtypes = [dbl, C.POINTER(u32), u32, u32, u32, C.POINTER(i32)]
        L.orc_vonmises.restype = dbl
        L.orc_vonmises_many.argtypes = [dbl, u32, u32, u32, u32, u32, lng, pd, C.POINTER(lng)]
        L.orc_create.argtypes = [i32, C.POINTER(i32), dbl, u32, u32]
        L.orc_create.restype = vp
        L.orc_destroy.argtypes = [vp]
        L.orc_init.argtypes = [vp, i32]
        L.orc_get_links.argtypes = [vp, pd]
        L.orc_set_links.argtypes = [vp, pd]
        L.orc_get_counter.argtypes = [vp]
        L.orc_get_counter.restype = u32
        L.orc_set_counter.argtypes = [vp, u32]
        L.orc_staple.argtypes = [vp, lng, i32, pd, pd]
        L.orc_heatbath_link.argtypes = [vp, lng, i32]
        L.orc_overrelax_link.argtypes = [vp, lng, i32]
        L.orc_metropolis_link.argtypes = [vp, lng, i32]
        L.orc_set_update.argtypes = [vp, i32, dbl]
        L.orc_bessel_ratio.argtypes = [dbl]
        L.orc_bessel_ratio.restype = dbl
        L.orc_link_mean.argtypes = [vp, lng, i32, pd, pd]
        L.orc_phase.argtypes = [vp, i32, i32, i32, i32]
        L.orc_pass.argtypes = [vp, i32, i32]
        L.orc_sweeps.argtypes = [vp, i32, i32, i32]
        L.orc_plaq_angle.argtypes = [vp, lng, i32, i32]
        L.orc_plaq_angle.restype = dbl
        L.orc_plaquette_means.argtypes = [vp, pd]
        L.orc_ml_result_size.argtypes = [C.POINTER(_Spec)]
        L.orc_ml_result_size.restype = lng
        L.orc_scaled_product.argtypes = [lng, pd, pd, pd, pd, C.POINTER(lng)]
        L.orc_ml_finalize.argtypes = [C.POINTER(_Spec), lng, i32, i32, pd, pd, pd]
        L.orc_ml_finalize.restype = i32
        L.orc_multilevel.argtypes = [vp, C.POINTER(_Spec), pd]
        L.orc_multilevel.restype = i32
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def philox(ctr, key) -> np.ndarray:
    """One Philox4x32-10 block: 4 uint32 words for counter ``ctr`` and key ``key``."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def bessel_ratio(kappa: float) -> float:
    """I_1(kappa) / I_0(kappa) (continued fraction)."""
    return lib().orc_bessel_ratio(kappa)


def vonmises(kappa: float, key, c0: int, c1: int, domain: int = DOM_TEST):
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    n = C.c_int(0)
    psi = lib().orc_vonmises(float(kappa), k, c0, c1, domain, C.byref(n))
    return psi, n.value


def vonmises_many(kappa: float, n: int, seed: int = 0, key_id: int = 0, c0_start: int = 0,
                  c1: int = 0, domain: int = DOM_TEST):
    out = np.empty(n, dtype=np.float64)
    tot = C.c_long(0)
    lib().orc_vonmises_many(float(kappa), seed, key_id, c0_start, c1, domain, n, _dptr(out), C.byref(tot))
    return out, tot.value


class MLSpec:
    """Multilevel measurement specification (levels outer first)."""

    def __init__(self, levels, r, dirs=(0,), probes=(), comps=(), n_or=3, multihit=False):
        self.levels = [tuple(lv) for lv in levels]  # (tau, n_iter, k_sweeps)
        self.r = [int(v) for v in r]
        self.dirs = [int(v) for v in dirs]
        self.probes = [tuple(int(u) for u in p) for p in probes]  # (l, p1, p2, mode)
        self.comps = [int(v) for v in comps]
        self.n_or = int(n_or)
        self.multihit = bool(multihit)

    def _struct(self):
        s = _Spec()
        s.n_levels = len(self.levels)
        for i, (tau, n, k) in enumerate(self.levels):
            s.tau[i], s.n_iter[i], s.k_sweeps[i] = tau, n, k
        s.n_or = self.n_or
        s.n_dirs = len(self.dirs)
        for i, d in enumerate(self.dirs):
            s.dirs[i] = d
        self._r = (C.c_int * max(1, len(self.r)))(*self.r)
        flat = [v for p in self.probes for v in p]
        self._p = (C.c_int * max(1, len(flat)))(*flat)
        self._c = (C.c_int * max(1, len(self.comps)))(*self.comps)
        s.n_r, s.r = len(self.r), self._r
        s.n_probe, s.probe = len(self.probes), self._p
        s.n_comp, s.comp = len(self.comps), self._c
        s.multihit = int(self.multihit)
        return s

    def result_size(self) -> int:
        return 2 * len(self.r) + 4 * len(self.r) * len(self.probes) * len(self.comps) + 12 + len(self.r)

    def unpack(self, out: np.ndarray) -> dict:
        """Split one configuration's doubles into C[r], CO[r,probe,comp,kind],
        vacuum and the binary exponents E[r]: "C" and "CO" are the values
        (mantissa * 2^E[r], zero where that underflows), "C_mant", "CO_mant"
        the stored mantissas."""
        nr, npb, nc = len(self.r), len(self.probes), len(self.comps)
        C_ = out[: 2 * nr].reshape(nr, 2)
        CO = out[2 * nr: 2 * nr + 4 * nr * npb * nc].reshape(nr, npb, nc, 2, 2)
        base = 2 * nr + 4 * nr * npb * nc
        ex = out[base + 12: base + 12 + nr].astype(np.int64)
        cm = C_[:, 0] + 1j * C_[:, 1]
        com = CO[..., 0] + 1j * CO[..., 1]
        scale = lambda m, e: np.ldexp(m.real, e) + 1j * np.ldexp(m.imag, e)
        return {
            "C": scale(cm, ex),
            "CO": scale(com, ex[:, None, None, None]),
            "C_mant": cm,
            "CO_mant": com,
            "exp": ex,
            "vac_sq": out[base: base + 6].copy(),
            "vac_lin": out[base + 6: base + 12].copy(),
        }


def scaled_product(factors):
    """Product of complex factors as (mantissa, binary exponent), rescaled after
    every factor; mantissa max(|re|, |im|) in [1, 2)."""
    z = np.ascontiguousarray(np.asarray(factors, dtype=np.complex128))
    re, im = np.ascontiguousarray(z.real), np.ascontiguousarray(z.imag)
    mr, mi, ex = C.c_double(), C.c_double(), C.c_long()
    lib().orc_scaled_product(z.size, _dptr(re), _dptr(im), C.byref(mr), C.byref(mi), C.byref(ex))
    return complex(mr.value, mi.value), int(ex.value)


def ml_finalize(spec: "MLSpec", n_sigma: int, nt: int, at: np.ndarray, ato: np.ndarray) -> np.ndarray:
    """The oracle's final estimators from given slab averages
    at[dir, r, slab, x] and ato[dir, r, probe, comp, kind, slab, x] (complex)."""
    s = spec._struct()
    n = lib().orc_ml_result_size(C.byref(s))
    out = np.zeros(n, dtype=np.float64)
    at = np.ascontiguousarray(at, dtype=np.complex128)
    ato = np.ascontiguousarray(ato if np.size(ato) else np.zeros(1), dtype=np.complex128)
    n_slabs = at.shape[2]
    rc = lib().orc_ml_finalize(C.byref(s), n_sigma, nt, n_slabs, at.ctypes.data_as(C.POINTER(C.c_double)),
                               ato.ctypes.data_as(C.POINTER(C.c_double)), _dptr(out))
    if rc != 0:
        raise ValueError(f"oracle finalize: code {rc}")
    return out


class Lattice:
    """One ensemble in the oracle: links, update counter, key (seed, key_id)."""

    def __init__(self, d: int, L, beta: float, seed: int = 1, key_id: int = 0):
        self.d = int(d)
        self.L = [int(v) for v in L]
        assert len(self.L) == self.d
        arr = (C.c_int * 4)(*(self.L + [1] * (4 - self.d)))
        self._h = lib().orc_create(self.d, arr, float(beta), seed, key_id)
        if not self._h:
            raise ValueError("oracle: bad lattice")
        self.beta = float(beta)
        self.V = int(np.prod(self.L))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_destroy(h)
            self._h = None

    def init(self, start: int):
        lib().orc_init(self._h, int(start))

    def links(self) -> np.ndarray:
        out = np.empty(self.V * self.d, dtype=np.float64)
        lib().orc_get_links(self._h, _dptr(out))
        return out

    def set_links(self, th: np.ndarray):
        th = np.ascontiguousarray(th, dtype=np.float64)
        assert th.size == self.V * self.d
        lib().orc_set_links(self._h, _dptr(th))

    @property
    def counter(self) -> int:
        return int(lib().orc_get_counter(self._h))

    @counter.setter
    def counter(self, v: int):
        lib().orc_set_counter(self._h, int(v))

    def staple(self, site: int, mu: int):
        a, b = C.c_double(), C.c_double()
        lib().orc_staple(self._h, site, mu, C.byref(a), C.byref(b))
        return a.value + 1j * b.value

    def heatbath_link(self, site: int, mu: int):
        lib().orc_heatbath_link(self._h, site, mu)

    def overrelax_link(self, site: int, mu: int):
        lib().orc_overrelax_link(self._h, site, mu)

    def metropolis_link(self, site: int, mu: int):
        lib().orc_metropolis_link(self._h, site, mu)

    def link_mean(self, site: int, mu: int) -> complex:
        re, im = C.c_double(), C.c_double()
        lib().orc_link_mean(self._h, site, mu, C.byref(re), C.byref(im))
        return complex(re.value, im.value)

    def set_update(self, kind: int, delta: float = 0.0):
        """Stochastic update of sweeps and multilevel: 0 heatbath, 2 Metropolis
        with proposal step delta (the paper's update, Sec. II)."""
        lib().orc_set_update(self._h, kind, delta)

    def phase(self, kind: int, mu: int, parity: int, tau: int = 0):
        lib().orc_phase(self._h, kind, mu, parity, tau)

    def pass_(self, kind: int, tau: int = 0):
        lib().orc_pass(self._h, kind, tau)

    def sweeps(self, n: int, n_or: int = 3, tau: int = 0):
        lib().orc_sweeps(self._h, n, n_or, tau)

    def plaq_angle(self, site: int, a: int, b: int) -> float:
        return lib().orc_plaq_angle(self._h, site, a, b)

    def plaquette_means(self) -> np.ndarray:
        out = np.zeros(6, dtype=np.float64)
        lib().orc_plaquette_means(self._h, _dptr(out))
        return out

    def multilevel(self, spec: MLSpec) -> np.ndarray:
        s = spec._struct()
        n = lib().orc_ml_result_size(C.byref(s))
        out = np.zeros(n, dtype=np.float64)
        rc = lib().orc_multilevel(self._h, C.byref(s), _dptr(out))
        if rc != 0:
            raise ValueError(f"oracle multilevel: invalid spec (code {rc})")
        return out

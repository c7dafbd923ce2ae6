"""Python binding of libu1ml (the C ABI in include/u1ml.h).

Argument marshalling only: every step of the multilevel path runs in the HIP
kernels of libu1ml.so.  PyTorch provides the device workspace and the stream.
If the library is not built, the first call into it raises ImportError: there
is no CPU fallback.

Paper: Amado, Cardoso, Bicudo, arXiv 1309.3859 (Sec. II, II.C, Algorithm 1).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libu1ml.so")

FP64, FP32 = 0, 1
COLD, HOT = 0, 1
HEATBATH, OVERRELAX, METROPOLIS = 0, 1, 2
UPDATE_HEATBATH, UPDATE_METROPOLIS = 0, 1
FORM_AUTO, FORM_HISTORY, FORM_SPECTRAL = 0, 1, 2
STATUS = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EDEVICE", 4: "ESTATE", 5: "ENOTSUP"}


class U1MLError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Ensemble(C.Structure):
    _fields_ = [("ns", C.c_int * 3), ("nt", C.c_int), ("beta", C.c_double), ("seed", C.c_uint32),
                ("key_id", C.c_uint32)]


class _Level(C.Structure):
    _fields_ = [("tau", C.c_int), ("n_iter", C.c_int), ("k_sweeps", C.c_int)]


class _Probe(C.Structure):
    _fields_ = [("l", C.c_int), ("p1", C.c_int), ("p2", C.c_int), ("mode", C.c_int)]


class _Problem(C.Structure):
    _fields_ = [
        ("n_ens", C.c_int), ("ens", C.POINTER(_Ensemble)), ("precision", C.c_int), ("n_or", C.c_int),
        ("n_levels", C.c_int), ("levels", _Level * 2), ("n_dirs", C.c_int), ("dirs", C.c_int * 3),
        ("n_r", C.c_int), ("r", C.POINTER(C.c_int)), ("n_probe", C.c_int), ("probes", C.POINTER(_Probe)),
        ("n_comp", C.c_int), ("comps", C.POINTER(C.c_int)), ("max_configs", C.c_int), ("form", C.c_int),
        ("update", C.c_int), ("metro_delta", C.c_double), ("multihit", C.c_int), ("ins_kernel", C.c_int),
    ]


class _PlanInfo(C.Structure):
    _fields_ = [
        ("ws_bytes", C.c_size_t), ("link_bytes", C.c_size_t), ("history_bytes", C.c_size_t),
        ("average_bytes", C.c_size_t), ("outer_bytes", C.c_size_t), ("result_bytes", C.c_size_t),
        ("scratch_bytes", C.c_size_t), ("paper_running_bytes", C.c_size_t), ("n_doubles_per_config", C.c_long),
        ("updates_per_config", C.c_long), ("updates_per_sweep", C.c_long), ("form", C.c_int),
        ("spectral_bytes", C.c_size_t), ("launches_per_config", C.c_long), ("est_history_ms", C.c_double),
        ("est_spectral_ms", C.c_double), ("ins_slots", C.c_int),
    ]


class _TuneReport(C.Structure):
    _fields_ = [("n_candidates", C.c_int), ("block", C.c_int * 8), ("us_per_sweep", C.c_double * 8),
                ("chosen_block", C.c_int)]


_lib = None


def lib():
    """Load libu1ml.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1309_3859_amd.build`")
    L = C.CDLL(LIB_PATH)
    st, vp, i32, u32, dbl, sz = C.c_int, C.c_void_p, C.c_int, C.c_uint32, C.c_double, C.c_size_t
    pd = C.POINTER(C.c_double)
    sigs = {
        "u1ml_plan": [C.POINTER(_Problem), C.POINTER(_PlanInfo)],
        "u1ml_create": [C.POINTER(_Problem), vp, sz, vp, C.POINTER(vp)],
        "u1ml_destroy": [vp],
        "u1ml_init_links": [vp, i32],
        "u1ml_sweeps": [vp, i32],
        "u1ml_phase": [vp, i32, i32, i32, i32, i32],
        "u1ml_multilevel": [vp],
        "u1ml_copy_results": [vp, pd, sz, C.POINTER(sz)],
        "u1ml_get_links": [vp, i32, pd, sz],
        "u1ml_set_links": [vp, i32, pd, sz],
        "u1ml_get_counter": [vp, i32, C.POINTER(u32)],
        "u1ml_set_counter": [vp, i32, u32],
        "u1ml_plaquette": [vp, pd],
        "u1ml_plaquette_noalloc": [vp, vp],
        "u1ml_health": [vp, C.POINTER(C.c_uint64)],
        "u1ml_autotune": [vp, C.POINTER(_TuneReport)],
        "u1ml_set_block": [vp, i32],
        "u1ml_set_graphs": [vp, i32],
        "u1ml_set_lanes": [vp, i32],
        "u1ml_time_phase": [vp, i32, i32, i32, i32, i32, pd],
        "u1ml_time_phase_lane": [vp, i32, i32, i32, i32, i32, i32, pd, pd, C.POINTER(C.c_long)],
        "u1ml_phase_bytes": [vp, i32, i32, i32, i32, pd, C.POINTER(C.c_long)],
        "u1ml_philox_fill": [u32, u32, u32, u32, u32, u32, sz, vp, vp],
        "u1ml_vonmises_fill": [dbl, i32, u32, u32, u32, u32, sz, vp, vp, vp],
        "u1ml_sincos_fill": [vp, sz, vp, vp, vp],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = st
    L.u1ml_status_str.argtypes = [C.c_int]
    L.u1ml_status_str.restype = C.c_char_p
    L.u1ml_last_error.argtypes = [vp]
    L.u1ml_last_error.restype = C.c_char_p
    _lib = L
    return L


def _check(status: int, ctx=None):
    if status != 0:
        msg = lib().u1ml_last_error(ctx).decode(errors="replace")
        raise U1MLError(status, msg)


# ---------------------------------------------------------------------------
# Problem description
# ---------------------------------------------------------------------------
@dataclass
class Ens:
    ns: Tuple[int, int, int]
    nt: int
    beta: float
    seed: int = 1
    key_id: int = 0

    @property
    def volume(self) -> int:
        return self.ns[0] * self.ns[1] * self.ns[2] * self.nt


@dataclass
class Spec:
    """Multilevel problem: ensembles, levels (tau, n_iter, k_sweeps) outer
    first, charge axes, separations, probes (l, p1, p2, mode), components."""

    ensembles: List[Ens]
    levels: List[Tuple[int, int, int]]
    r: Sequence[int]
    dirs: Sequence[int] = (0,)
    probes: Sequence[Tuple[int, int, int, int]] = ()
    comps: Sequence[int] = ()
    precision: int = FP64
    n_or: int = 3
    max_configs: int = 1
    form: int = 0  # FORM_AUTO
    update: int = 0  # UPDATE_HEATBATH
    metro_delta: float = 1.0
    multihit: bool = False
    ins_kernel: int = 0  # history-form insertion contraction: 0 auto, 1 vector, 2 matrix cores
    _keep: list = field(default_factory=list, repr=False)

    def struct(self) -> _Problem:
        p = _Problem()
        ens = (_Ensemble * len(self.ensembles))()
        for i, e in enumerate(self.ensembles):
            ens[i].ns[0], ens[i].ns[1], ens[i].ns[2] = e.ns
            ens[i].nt, ens[i].beta, ens[i].seed, ens[i].key_id = e.nt, e.beta, e.seed, e.key_id
        r = (C.c_int * max(1, len(self.r)))(*self.r)
        pr = (_Probe * max(1, len(self.probes)))()
        for i, (l, p1, p2, mode) in enumerate(self.probes):
            pr[i].l, pr[i].p1, pr[i].p2, pr[i].mode = l, p1, p2, mode
        cp = (C.c_int * max(1, len(self.comps)))(*self.comps)
        self._keep[:] = [ens, r, pr, cp]
        p.n_ens, p.ens = len(self.ensembles), ens
        p.precision, p.n_or = self.precision, self.n_or
        p.n_levels = len(self.levels)
        for i, (tau, n, k) in enumerate(self.levels):
            p.levels[i].tau, p.levels[i].n_iter, p.levels[i].k_sweeps = tau, n, k
        p.n_dirs = len(self.dirs)
        for i, d in enumerate(self.dirs):
            p.dirs[i] = d
        p.n_r, p.r = len(self.r), r
        p.n_probe, p.probes = len(self.probes), pr
        p.n_comp, p.comps = len(self.comps), cp
        p.max_configs = self.max_configs
        p.form = self.form
        p.update = self.update
        p.metro_delta = self.metro_delta
        p.multihit = int(bool(self.multihit))
        p.ins_kernel = int(self.ins_kernel)
        return p

    def n_doubles_per_config(self) -> int:
        R, Np, Nc = len(self.r), len(self.probes), len(self.comps)
        return 2 * R + 4 * R * Np * Nc + 12 + R

    def unpack(self, rec: np.ndarray) -> dict:
        """One ensemble's record: C[r], CO[r, probe, comp, kind] as values
        (mantissa * 2^E[r], zero where that underflows), the stored mantissas
        "C_mant", "CO_mant", the binary exponents "exp" and the vacuum sums."""
        R, Np, Nc = len(self.r), len(self.probes), len(self.comps)
        Cv = rec[: 2 * R].reshape(R, 2)
        CO = rec[2 * R: 2 * R + 4 * R * Np * Nc].reshape(R, Np, Nc, 2, 2)
        b = 2 * R + 4 * R * Np * Nc
        ex = rec[b + 12: b + 12 + R].astype(np.int64)
        cm = Cv[:, 0] + 1j * Cv[:, 1]
        com = CO[..., 0] + 1j * CO[..., 1]

        def scale(m, e):
            return np.ldexp(m.real, e) + 1j * np.ldexp(m.imag, e)

        return {"C": scale(cm, ex), "CO": scale(com, ex[:, None, None, None]), "C_mant": cm, "CO_mant": com,
                "exp": ex, "vac_sq": rec[b: b + 6].copy(), "vac_lin": rec[b + 6: b + 12].copy()}


def plan(spec: Spec) -> dict:
    info = _PlanInfo()
    _check(lib().u1ml_plan(C.byref(spec.struct()), C.byref(info)))
    return {k: getattr(info, k) for k, _ in _PlanInfo._fields_}


def _stream_handle(stream) -> Optional[int]:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Context:
    """One libu1ml context: a torch-owned device workspace and a HIP stream."""

    def __init__(self, spec: Spec, device="cuda", stream=None):
        import torch

        self.spec = spec
        self.plan = plan(spec)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.ws = torch.empty(self.plan["ws_bytes"], dtype=torch.uint8, device=device)
        h = C.c_void_p()
        _check(lib().u1ml_create(C.byref(spec.struct()), C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                 C.c_void_p(_stream_handle(self.stream)), C.byref(h)))
        self._h = h
        self.n_ens = len(spec.ensembles)
        self.nd = self.plan["n_doubles_per_config"]
        self._n_lanes = min(self.n_ens, 4 if spec.precision == FP64 else 2)  # the library's default

    def close(self):
        if getattr(self, "_h", None):
            lib().u1ml_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _c(self, status):
        _check(status, self._h)

    def init_links(self, start: int):
        self._c(lib().u1ml_init_links(self._h, start))

    def sweeps(self, n: int):
        self._c(lib().u1ml_sweeps(self._h, n))

    def phase(self, kind: int, mu: int, parity: int, tau: int = 0, pass_offset: int = 0):
        self._c(lib().u1ml_phase(self._h, kind, mu, parity, tau, pass_offset))

    def multilevel(self):
        self._c(lib().u1ml_multilevel(self._h))

    def results(self, max_configs: Optional[int] = None) -> np.ndarray:
        """Copy and clear the results ring: array [config, ensemble, n_doubles]."""
        cap = (max_configs or self.spec.max_configs) * self.n_ens * self.nd
        buf = np.zeros(cap, dtype=np.float64)
        n = C.c_size_t(0)
        self._c(lib().u1ml_copy_results(self._h, buf.ctypes.data_as(C.POINTER(C.c_double)), cap, C.byref(n)))
        k = n.value // (self.n_ens * self.nd)
        return buf[: k * self.n_ens * self.nd].reshape(k, self.n_ens, self.nd)

    def links(self, ens: int = 0) -> np.ndarray:
        V = self.spec.ensembles[ens].volume
        out = np.empty(4 * V, dtype=np.float64)
        self._c(lib().u1ml_get_links(self._h, ens, out.ctypes.data_as(C.POINTER(C.c_double)), out.size))
        return out

    def set_links(self, th: np.ndarray, ens: int = 0):
        th = np.ascontiguousarray(th, dtype=np.float64)
        self._c(lib().u1ml_set_links(self._h, ens, th.ctypes.data_as(C.POINTER(C.c_double)), th.size))

    def counter(self, ens: int = 0) -> int:
        v = C.c_uint32()
        self._c(lib().u1ml_get_counter(self._h, ens, C.byref(v)))
        return int(v.value)

    def set_counter(self, value: int, ens: int = 0):
        self._c(lib().u1ml_set_counter(self._h, ens, value))

    def plaquette(self) -> np.ndarray:
        out = np.zeros(6 * self.n_ens, dtype=np.float64)
        self._c(lib().u1ml_plaquette(self._h, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out.reshape(self.n_ens, 6)

    def plaquette_noalloc(self, out):
        """Plaquette means into the float64 device tensor `out` (n_ens * 6
        elements), asynchronously on the context's stream; the library's
        static scratch holds the partial sums."""
        self._c(lib().u1ml_plaquette_noalloc(self._h, C.c_void_p(out.data_ptr())))
        return out

    def health(self) -> int:
        v = C.c_uint64()
        self._c(lib().u1ml_health(self._h, C.byref(v)))
        return int(v.value)

    def autotune(self) -> dict:
        rep = _TuneReport()
        self._c(lib().u1ml_autotune(self._h, C.byref(rep)))
        n = rep.n_candidates
        return {"block": list(rep.block[:n]), "us_per_sweep": list(rep.us_per_sweep[:n]),
                "chosen_block": rep.chosen_block}

    def set_block(self, block: int):
        self._c(lib().u1ml_set_block(self._h, block))

    def set_graphs(self, enable: bool):
        self._c(lib().u1ml_set_graphs(self._h, int(bool(enable))))

    def set_lanes(self, n_lanes: int):
        self._c(lib().u1ml_set_lanes(self._h, int(n_lanes)))
        self._n_lanes = int(n_lanes)

    def time_phase(self, kind: int, mu: int, parity: int, tau: int, n_rep: int) -> float:
        us = C.c_double()
        self._c(lib().u1ml_time_phase(self._h, kind, mu, parity, tau, n_rep, C.byref(us)))
        return us.value

    def time_phase_lane(self, lane: int, kind: int, mu: int, parity: int, tau: int, n_rep: int):
        """(us per launch, bytes, updates) of one lane's launch of a phase."""
        us, b, u = C.c_double(), C.c_double(), C.c_long()
        self._c(lib().u1ml_time_phase_lane(self._h, lane, kind, mu, parity, tau, n_rep, C.byref(us), C.byref(b),
                                           C.byref(u)))
        return us.value, b.value, u.value

    @property
    def n_lanes(self) -> int:
        return self._n_lanes

    def phase_bytes(self, kind: int, mu: int, parity: int, tau: int):
        b, u = C.c_double(), C.c_long()
        self._c(lib().u1ml_phase_bytes(self._h, kind, mu, parity, tau, C.byref(b), C.byref(u)))
        return b.value, u.value


def philox_fill(key, ctr, n: int, device="cuda"):
    """Device Philox4x32-10 blocks (ctr[0] + i, ctr[1], ctr[2], ctr[3]) as a torch uint32 [n, 4] view."""
    import torch

    out = torch.empty(4 * n, dtype=torch.int32, device=device)
    _check(lib().u1ml_philox_fill(key[0], key[1], ctr[0], ctr[1], ctr[2], ctr[3], n, C.c_void_p(out.data_ptr()),
                                  C.c_void_p(_stream_handle(None))))
    return out.view(n, 4)


def vonmises_fill(kappa: float, n: int, precision: int = FP64, seed: int = 0, key_id: int = 0, c0: int = 0,
                  c1: int = 0, device="cuda"):
    """n device draws of the heatbath's von Mises sampler; returns (psi, attempts) torch tensors."""
    import torch

    out = torch.empty(n, dtype=torch.float64, device=device)
    att = torch.empty(n, dtype=torch.int32, device=device)
    _check(lib().u1ml_vonmises_fill(float(kappa), precision, seed, key_id, c0, c1, n, C.c_void_p(out.data_ptr()),
                                    C.c_void_p(att.data_ptr()), C.c_void_p(_stream_handle(None))))
    return out, att


def sincos_fill(x):
    """The library's FP64 sine and cosine of the float64 device tensor x;
    returns (sin x, cos x) as torch tensors."""
    import torch

    x = x.contiguous()
    s = torch.empty_like(x)
    c = torch.empty_like(x)
    _check(lib().u1ml_sincos_fill(C.c_void_p(x.data_ptr()), x.numel(), C.c_void_p(s.data_ptr()),
                                  C.c_void_p(c.data_ptr()), C.c_void_p(_stream_handle(None))))
    return s, c

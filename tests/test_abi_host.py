"""Host-side checks of libu1ml that need no GPU: the shared library loads and
exports every call include/u1ml.h declares, and the pure-host planner
validates problems and sizes the workspace (including the paper's worked
memory example)."""
import json
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def u1():
    from paper_1309_3859_amd import build, u1ml

    if not os.path.exists(u1ml.LIB_PATH):
        build.build()
    u1ml.lib()
    return u1ml


def test_library_exports_every_declared_call(u1):
    hdr = open(os.path.join(ROOT, "include", "u1ml.h")).read()
    declared = set(re.findall(r"\b(u1ml_[a-z_0-9]+)\s*\(", hdr))
    lib = u1.lib()
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", u1.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (u1ml_[a-z_0-9]+)", out))
    assert declared == exported


def _spec(u1, **kw):
    base = dict(ensembles=[u1.Ens((4, 4, 4), 4, 1.0)], levels=[(2, 10, 1)], r=[1, 2], dirs=[0],
                probes=[(0, 0, 0, 1)], comps=[0])
    base.update(kw)
    return u1.Spec(**base)


BAD = [
    ("odd extent", dict(ens=((5, 4, 4), 4, 1.0))),
    ("extent 0", dict(ens=((0, 4, 4), 4, 1.0))),
    ("nt not multiple of tau", dict(ens=((4, 4, 4), 6, 1.0), levels=[(4, 2, 1)])),
    ("nan beta", dict(ens=((4, 4, 4), 4, float("nan")))),
    ("negative beta", dict(ens=((4, 4, 4), 4, -1.0))),
    ("r >= Ns", dict(r=[4])),
    ("r = 0", dict(r=[0])),
    ("tau 1", dict(levels=[(1, 2, 1)])),
    ("outer not multiple", dict(ens=((4, 4, 4), 12, 1.0), levels=[(6, 2, 1), (4, 2, 1)])),
    ("n_iter 0", dict(levels=[(2, 0, 1)])),
    ("k negative", dict(levels=[(2, 2, -1)])),
    ("probe too far", dict(probes=[(0, 2, 0, 1)])),
    ("bad component", dict(comps=[6])),
    ("bad axis", dict(dirs=[3])),
    ("repeated axis", dict(dirs=[0, 0])),
    ("probes without comps", dict(comps=[])),
    ("bad form", dict(form=3)),
    # a 66 x 66 plane orthogonal to the x axis holds more than 4096 sites
    ("spectral plane too large", dict(ens=((2, 66, 66), 4, 1.0), r=[1], form=2)),
    # limits of the kernels' index arithmetic
    ("Ns^3 / 2 >= 2^24", dict(ens=((324, 324, 324), 2, 1.0), r=[1])),
    ("Nt >= 2^22", dict(ens=((2, 2, 2), 1 << 22, 1.0), r=[1])),
    ("FP32 links of one ensemble >= 4 GiB", dict(ens=((256, 256, 256), 16, 1.0), r=[1], precision=1)),
    ("FP64 links of one ensemble >= 4 GiB", dict(ens=((256, 256, 256), 8, 1.0), r=[1], precision=0)),
]


@pytest.mark.parametrize("name,kw", BAD, ids=[b[0] for b in BAD])
def test_planner_rejects_invalid_problems(u1, name, kw):
    kw = dict(kw)
    if "ens" in kw:
        ns, nt, beta = kw.pop("ens")
        kw["ensembles"] = [u1.Ens(ns, nt, beta)]
    with pytest.raises(u1.U1MLError) as ei:
        u1.plan(_spec(u1, **kw))
    assert ei.value.status == 1  # EINVAL
    assert str(ei.value).strip() != "EINVAL:"


@pytest.mark.parametrize("ns,nt,precision", [((256, 256, 256), 14, 1), ((256, 256, 256), 6, 0),
                                             ((322, 322, 322), 8, 1), ((2, 2, 2), (1 << 22) - 2, 1)])
def test_planner_accepts_lattices_at_the_limits(u1, ns, nt, precision):
    info = u1.plan(_spec(u1, ensembles=[u1.Ens(ns, nt, 1.0)], r=[1], probes=[], comps=[], precision=precision))
    assert info["link_bytes"] >= 4 * ns[0] * ns[1] * ns[2] * nt * (4 if precision else 8)


def test_planner_accepts_presets_and_counts_updates(u1):
    from paper_1309_3859_amd import configs

    spec, _ = configs.c1_plain_fp64()
    p = u1.plan(spec)
    # C1 by brute force: per sweep (1 + 3 passes), each pass updates every
    # temporal link and the spatial links off the frozen layers t = 0 mod 2
    L = 4
    per_pass = sum(1 for t in range(L) for _ in range(L ** 3)) + 3 * sum(
        1 for t in range(L) if t % 2 for _ in range(L ** 3))
    assert p["updates_per_config"] == 10 * 4 * per_pass == 25600
    assert p["updates_per_sweep"] == 4 * 4 * L ** 4
    assert p["n_doubles_per_config"] == spec.n_doubles_per_config()
    for name in ("c2", "c3", "c4", "replicas"):
        s, _ = configs.PRESETS[name]()
        assert u1.plan(s)["ws_bytes"] < 16 * 2**30
    # replicas: N copies of one lattice plan N times its updates
    one = u1.plan(configs.replicas(n_ens=1)[0])["updates_per_config"]
    # per sweep of 4 passes at tau = 2: every temporal link (V) and the spatial links of half the slices (3V/2)
    V = 24 ** 3 * 8
    assert u1.plan(configs.replicas(n_ens=32)[0])["updates_per_config"] == 32 * one == 32 * 50 * 4 * (V + 3 * V // 2)


def test_paper_memory_example(u1):
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_memory_example.json")))
    spec = u1.Spec(ensembles=[u1.Ens(tuple(g["ns"]), g["nt"], 1.0)], levels=[(g["tau"], 1, 1)], r=[1], dirs=[0])
    p = u1.plan(spec)
    assert p["paper_running_bytes"] == g["bytes"]
    assert round(g["bytes"] / 2**20) == g["paper_states_MB"]
    # the paper's "1.7 MB" is one link direction in FP64; the library stores all four
    spec64 = u1.Spec(ensembles=[u1.Ens(tuple(g["ns"]), g["nt"], 1.0)], levels=[(2, 1, 1)], r=[1], precision=u1.FP64)
    assert u1.plan(spec64)["link_bytes"] == 4 * g["link_bytes_one_direction"]


def test_workspace_too_small_is_rejected_before_any_device_call(u1):
    import ctypes as C

    spec = _spec(u1)
    h = C.c_void_p()
    st = u1.lib().u1ml_create(C.byref(spec.struct()), C.c_void_p(256), 16, None, C.byref(h))
    assert st == 1 and not h.value
    assert b"workspace too small" in u1.lib().u1ml_last_error(None)


def test_contraction_form_selection(u1):
    """The planner keeps the per-site history form while its averages fit and
    switches to the spectral form for the full transverse map of the largest
    preset, whose per-site averages would need about a terabyte."""
    from paper_1309_3859_amd import configs

    s2, _ = configs.c2_fp32_profiles()
    p2 = u1.plan(s2)
    assert p2["form"] == u1.FORM_HISTORY and p2["spectral_bytes"] == 0
    s5, _ = configs.c5_largest()
    p5 = u1.plan(s5)
    assert p5["form"] == u1.FORM_SPECTRAL
    assert p5["average_bytes"] < 2**30 and p5["ws_bytes"] < 16 * 2**30
    # the spectral sections: weights W (3 thick slabs) and G (6 thin slabs),
    # plane spectra of the 19 T fields and 12 O rows, spectral sums of 19 r x 6
    # components x 2 kinds x 1 probe group over 48 x 48 planes, one link copy,
    # and one measurement's slab phases (double2) and 12 O rows (FP32) in
    # plane-major order
    nsig, R = 48 ** 3, 19
    want = 16 * (R * 3 * nsig + R * 6 * nsig + 6 * R * nsig + 6 * 12 * nsig + 6 * R * 6 * 2 * 48 * 48) \
        + p5["link_bytes"] + 16 * 6 * nsig + 4 * 6 * 12 * nsig
    assert abs(p5["spectral_bytes"] - want) <= 6 * 256
    s5.form = u1.FORM_HISTORY
    assert u1.plan(s5)["average_bytes"] > 10 ** 12
    # forcing the spectral form on a small problem is allowed
    s2.form = u1.FORM_SPECTRAL
    assert u1.plan(s2)["form"] == u1.FORM_SPECTRAL


def test_contraction_form_follows_the_cost_estimates(u1):
    """AUTO takes the form with the smaller estimated device time.  The
    estimates order the forms as measured on MI355X (ms per configuration,
    history / spectral): 24^3x8 with 9 probes 11.5 / 18.0, the in-plane map
    18.1 / 19.4, 48^3x12 at 2 x 10 updates with 1 probe 8.8 / 21.5 and with
    8 probes 39.9 / 21.6; without probes there is nothing to estimate."""
    from paper_1309_3859_amd import configs

    cases = []
    s, _ = configs.c2_fp32_profiles()
    cases.append((s, u1.FORM_HISTORY))
    s, _ = configs.in_plane_map()
    cases.append((s, u1.FORM_HISTORY))
    s, _ = configs.c5_largest(n_outer=2, n_inner=10, full_map=False)
    cases.append((s, u1.FORM_HISTORY))
    s, _ = configs.c5_largest(n_outer=2, n_inner=10)
    s.probes = s.probes[:8]
    cases.append((s, u1.FORM_SPECTRAL))
    for spec, want in cases:
        p = u1.plan(spec)
        assert p["est_history_ms"] > 0 and p["est_spectral_ms"] > 0
        assert p["form"] == want, (p["est_history_ms"], p["est_spectral_ms"])
        assert (p["est_spectral_ms"] < p["est_history_ms"]) == (want == u1.FORM_SPECTRAL)
    p4 = u1.plan(configs.c4_batched()[0])
    assert p4["est_history_ms"] == 0 and p4["est_spectral_ms"] == -1
    # a plane of more than 4096 sites leaves the history form whatever it costs
    spec = u1.Spec(ensembles=[u1.Ens((2, 66, 66), 4, 1.0)], levels=[(2, 10, 1)], r=[1], probes=[(0, 0, 0, 1)],
                   comps=[0], precision=u1.FP32)
    p = u1.plan(spec)
    assert p["form"] == u1.FORM_HISTORY and p["est_spectral_ms"] == -1


def test_large_bodies_are_launched_directly(u1):
    """Multilevel bodies above 8192 kernel launches are not captured into a
    single graph (the planner reports the launch count); the headline batch
    and the one-level presets stay captured."""
    from paper_1309_3859_amd import configs

    n = {k: u1.plan(configs.PRESETS[k]()[0])["launches_per_config"] for k in ("c1", "c2", "c3", "c4", "c5")}
    # C4: 50 measurements x (1 sweep of 4 passes x 8 phases + 1 measurement) + contraction and products
    assert 50 * 33 < n["c4"] <= 8192
    assert n["c2"] <= 8192 and n["c1"] <= 8192
    assert n["c3"] > 8192
    # C5 (two levels, spectral, replayed): two passes of 40 x (32 + 100 x 33) launches
    assert n["c5"] > 2 * 40 * (32 + 100 * 33)


def test_insertion_kernel_choice(u1):
    """The history form's insertion sums run on the vector kernel (slot blocks
    of 9, 6, 3 or 1 for FP64 O rows, 3 or 1 for FP32 ones, the fewest empty
    slots) or on the matrix cores (blocks of 8), whichever is estimated
    faster: on the 24^3x8 workload with 9 probes x 6 components x 11
    separations the vector kernel (1.5 ms per launch on MI355X against 3.3
    ms); either can be asked for, and the matrix-core kernel only where its
    chunk fits LDS (the estimate does not take it otherwise)."""
    from paper_1309_3859_amd import configs

    spec, _ = configs.c2_fp32_profiles()
    auto = u1.plan(spec)
    assert auto["ins_slots"] == 3
    spec.precision = u1.FP64
    assert u1.plan(spec)["ins_slots"] == 9
    spec.precision = u1.FP32
    spec.ins_kernel = 2
    mf = u1.plan(spec)
    assert mf["ins_slots"] == 8 and mf["est_history_ms"] > auto["est_history_ms"]
    spec.ins_kernel = 1
    assert u1.plan(spec)["ins_slots"] == 3
    spec.ins_kernel = 3
    with pytest.raises(u1.U1MLError, match="EINVAL"):
        u1.plan(spec)
    # no probes: no insertion kernel; the spectral form: none either
    assert u1.plan(configs.c4_batched()[0])["ins_slots"] == 0
    s, _ = configs.c5_largest(n_outer=2, n_inner=10)
    p = u1.plan(s)
    assert p["form"] == u1.FORM_SPECTRAL and p["ins_slots"] == 0

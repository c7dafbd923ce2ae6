"""GPU path (libu1ml through its C ABI) against the FP64 CPU oracle.

Element-wise parity on identical inputs wherever the two follow the same
arithmetic: Philox blocks bit-exact, von Mises draws, every checkerboard
phase (both update kinds, every direction and parity, frozen masks),
plaquettes, the multilevel measurement and estimator chain.  Overrelaxation
amplifies rounding-level differences (about 30x per pass, measured on the
oracle itself), so whole trajectories are compared with heatbath-only sweeps,
and the full dynamics statistically.
"""
import itertools
import sys

import numpy as np
import pytest

from helpers.inputs import random_links, random_links_fp32
from helpers.stats import circ_dist

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
    return u1ml, O, torch


def _ctx(u1, ns, nt, beta=1.0, levels=((4, 1, 1), (2, 1, 1)), precision=0, n_or=3, seed=1, key_id=0, **kw):
    spec = u1.Spec(ensembles=[u1.Ens(tuple(ns), nt, beta, seed=seed, key_id=key_id)], levels=list(levels),
                   r=kw.pop("r", [1]), dirs=kw.pop("dirs", [0]), probes=kw.pop("probes", ()),
                   comps=kw.pop("comps", ()), precision=precision, n_or=n_or, max_configs=kw.pop("max_configs", 4),
                   ins_kernel=kw.pop("ins_kernel", 0))
    return spec, u1.Context(spec)


def test_philox_bit_exact(env):
    u1, O, torch = env
    for key in [(0, 0), (1, 2), (0xDEADBEEF, 0x12345678)]:
        for ctr in [(0, 0, 0, 0), (123456, 7, 3, 0), (0xFFFFFFF0, 1, 2, 3)]:
            say("philox", key, ctr)
            dev = u1.philox_fill(key, ctr, 2048).cpu().numpy().view(np.uint32)
            ref = np.array([O.philox(((ctr[0] + i) & 0xFFFFFFFF, ctr[1], ctr[2], ctr[3]), key) for i in range(2048)])
            assert np.array_equal(dev, ref)


@pytest.mark.parametrize("kappa", [0.0, 1e-8, 0.5, 3.0, 6.0, 20.0])
def test_vonmises_fp64_draws_match_oracle(env, kappa):
    u1, O, torch = env
    say("vonmises fp64", kappa)
    n = 20000
    psi, att = u1.vonmises_fill(kappa, n, precision=u1.FP64, seed=17, key_id=5, c0=100, c1=3)
    ref, _ = O.vonmises_many(kappa, n, seed=17, key_id=5, c0_start=100, c1=3, domain=O.DOM_TEST)
    psi = psi.cpu().numpy()
    att = att.cpu().numpy()
    # psi = arccos(f) amplifies a 1-ulp difference in f by 1/|sin psi|, so the
    # well-conditioned comparison is on cos(psi) (= f) and on the sign
    same = np.abs(np.cos(psi) - np.cos(ref)) < 1e-14
    same &= (np.sign(psi) == np.sign(ref)) | (np.abs(psi) < 1e-6)
    assert np.count_nonzero(~same) <= 2  # an accept/reject decision may flip at rounding level
    assert np.all(att > 0)


@pytest.mark.parametrize("kappa", [0.5, 3.0, 20.0])
def test_vonmises_fp32_statistics(env, kappa):
    from scipy import special

    u1, O, torch = env
    say("vonmises fp32", kappa)
    n = 400_000
    psi, att = u1.vonmises_fill(kappa, n, precision=u1.FP32, seed=3, key_id=9)
    psi = psi.cpu().numpy()
    assert np.all(np.abs(psi) <= np.pi + 1e-6)
    for m in (1, 2):
        c = np.cos(m * psi)
        exact = special.iv(m, kappa) / special.iv(0, kappa)
        assert abs(c.mean() - exact) < 5 * c.std() / np.sqrt(n) + 1e-6
    assert att.float().mean().item() < 1.6


def test_init_matches_oracle(env):
    u1, O, torch = env
    for ns, nt in [((4, 4, 4), 4), ((6, 4, 2), 8)]:
        spec, ctx = _ctx(u1, ns, nt, seed=11, key_id=2)
        ref = O.Lattice(4, list(ns) + [nt], 1.0, seed=11, key_id=2)
        for start in (0, 1):
            say("init", ns, nt, start)
            ctx.init_links(start)
            ref.init(start)
            assert np.array_equal(ctx.links(0), ref.links())
            assert ctx.counter(0) == 0


GEOMS = [((4, 4, 4), 4), ((6, 4, 2), 8)]


@pytest.mark.parametrize("ns,nt", GEOMS)
@pytest.mark.parametrize("precision", [0, 1])
def test_every_phase_matches_oracle(env, ns, nt, precision):
    """Each checkerboard phase from identical links and counter: FP64 within
    1e-12 on the circle; FP32 storage within 2e-5 (hardware sin/cos), with
    heatbath accept/reject flips counted apart (at most a few)."""
    u1, O, torch = env
    V = int(np.prod(ns)) * nt
    spec, ctx = _ctx(u1, ns, nt, beta=1.1, precision=precision, seed=7, key_id=1)
    ref = O.Lattice(4, list(ns) + [nt], 1.1, seed=7, key_id=1)
    th0 = random_links_fp32(V, 5) if precision else random_links(V, 5)
    worst = 0.0
    flips = 0
    for kind, mu, p, tau in itertools.product((0, 1), range(4), (0, 1), (0, 2, 4)):
        say("phase", precision, ns, nt, kind, mu, p, tau)
        ctx.set_links(th0)
        ctx.set_counter(9)
        ref.set_links(th0)
        ref.counter = 9
        ctx.phase(kind, mu, p, tau)
        ref.phase(kind, mu, p, tau)
        d = circ_dist(ctx.links(0), ref.links())
        if precision == 0:
            assert d.max() < 1e-12, (kind, mu, p, tau, d.max())
        else:
            big = d > 2e-5
            flips += int(big.sum())
            worst = max(worst, float(d[~big].max()))
    if precision:
        say("fp32 phases: worst", worst, "flips", flips)
        assert flips <= 3


@pytest.mark.parametrize("precision", [0, 1])
def test_heatbath_at_zero_coupling(env, precision):
    """beta = 0, the degenerate case of the update: every link has kappa = 0
    and its new angle is uniform from the first Philox word.  Each heatbath
    phase equals the oracle's (FP64 within 1e-12, FP32 storage within 2e-5),
    and a full sweep leaves angles uniform on [-pi, pi) (Kolmogorov-Smirnov)."""
    from scipy import stats

    u1, O, torch = env
    ns, nt = (6, 4, 4), 4
    V = int(np.prod(ns)) * nt
    spec, ctx = _ctx(u1, ns, nt, beta=0.0, precision=precision, seed=17, key_id=3)
    ref = O.Lattice(4, list(ns) + [nt], 0.0, seed=17, key_id=3)
    th0 = random_links_fp32(V, 8) if precision else random_links(V, 8)
    tol = 1e-12 if precision == 0 else 2e-5
    for mu, p, tau in itertools.product(range(4), (0, 1), (0, 2)):
        ctx.set_links(th0)
        ctx.set_counter(4)
        ref.set_links(th0)
        ref.counter = 4
        ctx.phase(0, mu, p, tau)
        ref.phase(0, mu, p, tau)
        d = circ_dist(ctx.links(0), ref.links())
        assert d.max() < tol, (mu, p, tau, d.max())
    big = u1.Spec(ensembles=[u1.Ens((8, 8, 8), 8, 0.0, seed=18)], levels=[(2, 1, 1)], r=[1], precision=precision,
                  n_or=0)
    c2 = u1.Context(big)
    c2.init_links(u1.COLD)
    c2.sweeps(1)
    th = c2.links(0)
    assert stats.kstest((th + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-3


@pytest.mark.parametrize("precision", [0, 1])
def test_plaquette_matches_oracle(env, precision):
    u1, O, torch = env
    ns, nt = (6, 4, 2), 8
    V = int(np.prod(ns)) * nt
    spec, ctx = _ctx(u1, ns, nt, precision=precision)
    ref = O.Lattice(4, list(ns) + [nt], 1.0)
    th = random_links_fp32(V, 8)
    ctx.set_links(th)
    ref.set_links(th)
    say("plaquette", precision)
    assert np.max(np.abs(ctx.plaquette()[0] - ref.plaquette_means())) < 1e-13


def test_sweep_parity_per_pass_fp64(env):
    """One full sweep (1 heatbath + 3 overrelaxation passes) from identical
    links.  The heatbath pass agrees within 1e-12.  Overrelaxation amplifies
    any rounding-level difference (arg A moves by delta/|A|), so after each
    pass the GPU-vs-oracle deviation is bounded by 10x the deviation between
    the oracle and itself started from links perturbed by 1e-15."""
    u1, O, torch = env
    ns, nt = (4, 4, 4), 4
    spec, ctx = _ctx(u1, ns, nt, beta=1.0, levels=[(2, 1, 1)])
    ref = O.Lattice(4, [4, 4, 4, 4], 1.0, seed=1)
    pert = O.Lattice(4, [4, 4, 4, 4], 1.0, seed=1)
    th = random_links(256, 12)
    ctx.set_links(th)
    ref.set_links(th)
    pert.set_links(th + np.random.default_rng(0).uniform(-1e-15, 1e-15, th.size))
    devs, own = [], []
    for k in range(4):
        for mu in range(4):
            for p in range(2):
                ctx.phase(0 if k == 0 else 1, mu, p, 0, 0)
        ref.pass_(0 if k == 0 else 1, 0)
        pert.pass_(0 if k == 0 else 1, 0)
        devs.append(float(circ_dist(ctx.links(0), ref.links()).max()))
        own.append(float(circ_dist(pert.links(), ref.links()).max()))
    say("per-pass max deviation gpu-oracle", devs, "oracle-perturbed oracle", own)
    assert devs[0] < 1e-12
    for d, o in zip(devs, own):
        assert d <= 10 * o + 1e-13


def test_first_sweep_of_c1_within_1e12(env):
    """The bar on its own workload: C1 (4^3 x 4, beta = 1, cold start, Philox
    seed 1), the first full FP64 sweep (1 heatbath + 3 overrelaxation passes)
    through u1ml_sweeps; every link angle within 1e-12 of the oracle's.  From
    the cold start the staple sums are large, so the passes amplify rounding
    little (the oracle against itself from links perturbed by 1e-15: at most
    2.1e-13 after the sweep)."""
    u1, O, torch = env
    spec, ctx = _ctx(u1, (4, 4, 4), 4, beta=1.0, levels=[(2, 10, 1)], seed=1)
    ref = O.Lattice(4, [4, 4, 4, 4], 1.0, seed=1)
    ctx.init_links(u1.COLD)
    ref.init(0)
    ctx.sweeps(1)
    ref.sweeps(1, n_or=3)
    d = circ_dist(ctx.links(0), ref.links())
    say("C1 first sweep: max |d theta|", d.max(), "counter", ctx.counter(0), ref.counter)
    assert ctx.counter(0) == ref.counter == 1
    assert d.max() < 1e-12


def _multilevel_pair(env, ns, nt, levels, n_or, r, dirs, probes, comps, beta=1.0, seed=3, precision=0, start_seed=21,
                     ins_kernel=0):
    u1, O, torch = env
    V = int(np.prod(ns)) * nt
    spec, ctx = _ctx(u1, ns, nt, beta=beta, levels=levels, n_or=n_or, r=r, dirs=dirs, probes=probes, comps=comps,
                     seed=seed, precision=precision, ins_kernel=ins_kernel)
    ref = O.Lattice(4, list(ns) + [nt], beta, seed=seed)
    th = random_links_fp32(V, start_seed) if precision else random_links(V, start_seed)
    ctx.set_links(th)
    ctx.set_counter(4)
    ref.set_links(th)
    ref.counter = 4
    ctx.multilevel()
    got = spec.unpack(ctx.results()[0, 0])
    ospec = O.MLSpec(levels=levels, r=r, dirs=dirs, probes=probes, comps=comps, n_or=n_or)
    want = ospec.unpack(ref.multilevel(ospec))
    return got, want, ctx, ref


PROBES = [(0, 0, 0, 1), (1, 1, -1, 1), (-1, 2, 1, 0)]


@pytest.mark.parametrize("levels", [[(2, 3, 0)], [(4, 2, 0), (2, 3, 0)], [(4, 3, 0)], [(8, 2, 0)],
                                    [(8, 2, 0), (4, 2, 0)]])
@pytest.mark.parametrize("precision", [0, 1])
def test_measurement_and_estimators_match_oracle(env, levels, precision):
    """k = 0: no updates, so both sides measure the same links; the whole
    measurement -> slab average -> combine -> product -> sum chain is compared.
    The last two cases are the degenerate slabs: one slab of the whole time
    extent (the product over the other slabs is empty), and one thick slab
    holding two thin ones."""
    say("measurement parity", levels, precision)
    got, want, _, _ = _multilevel_pair(env, (6, 6, 8), 8, levels, 3, [1, 2, 3], [0, 1, 2], PROBES, list(range(6)),
                                       precision=precision)
    tol_c = 1e-12
    tol_o = 1e-12 if precision == 0 else 1e-5
    assert np.max(np.abs(got["C"] - want["C"])) < tol_c
    assert np.max(np.abs(got["CO"] - want["CO"])) < tol_o * max(1.0, np.abs(want["CO"]).max())
    assert np.max(np.abs(got["vac_sq"] - want["vac_sq"])) < (1e-12 if precision == 0 else 1e-6)
    assert np.max(np.abs(got["vac_lin"] - want["vac_lin"])) < (1e-12 if precision == 0 else 1e-6)


# (probes, components): the history-form contraction groups (probe, component)
# slots sharing (l, mode, spans) in blocks of 9, 6, 3 or 1, whichever leaves
# the fewest empty slots (the larger on a tie); these cases reach each block
# size (9: 9 probes x 3 components per spans class; 6: 2 probes x 3; 3: 1 probe
# x 3; 1: one slot)
SLOT_CASES = {
    "blocks_of_9": ([(0, p1, p2, 1) for p1 in (-1, 0, 1) for p2 in (-1, 0, 1)], [0, 1, 2, 3, 4, 5]),
    "blocks_of_9_one_r": ([(0, p1, p2, 1) for p1 in (-1, 0, 1) for p2 in (-1, 0, 1)], [0, 1, 2, 3, 4, 5], [2]),
    "blocks_of_6": ([(1, 0, 0, 1), (1, 1, 1, 1)], [0, 1, 2, 3, 4, 5]),
    "blocks_of_3": ([(-1, 1, 0, 0)], [0, 1, 2, 3, 4, 5]),
    "block_of_1": ([(0, 1, 1, 1)], [4]),
}


@pytest.mark.parametrize("case", sorted(SLOT_CASES))
@pytest.mark.parametrize("ns,dirs", [((8, 6, 6), [0]), ((6, 8, 6), [1]), ((8, 8, 8), [0, 1, 2])])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("kernel", [1, 2])
def test_insertion_contraction_slot_blocks_match_oracle(env, case, ns, dirs, precision, kernel):
    """The history-form insertion averages for every slot-block size of the
    vector kernel (kernel 1: 9, 6, 3 and 1 with FP64 and FP32 O rows, the
    planner's choice for each case) and the matrix-core kernel's blocks of 8
    slots
    (kernel 2, several blocks per work-group on these short lines), along a
    contiguous axis (x: chunks copied straight into LDS) and strided ones
    (y, z), against the oracle on the same links (no updates)."""
    probes, comps = SLOT_CASES[case][:2]
    r = SLOT_CASES[case][2] if len(SLOT_CASES[case]) > 2 else [1, 2, 3]
    say("slot blocks", case, ns, dirs, precision, kernel)
    got, want, ctx, _ = _multilevel_pair(env, ns, 8, [(2, 5, 0)], 3, r, dirs, probes, comps,
                                         precision=precision, ins_kernel=kernel)
    assert ctx.plan["form"] == env[0].FORM_HISTORY
    assert (ctx.plan["ins_slots"] == 8) == (kernel == 2), ctx.plan["ins_slots"]
    tol_o = 1e-12 if precision == 0 else 1e-5
    assert np.max(np.abs(got["C"] - want["C"])) < 1e-12
    assert np.max(np.abs(got["CO"] - want["CO"])) < tol_o * max(1.0, np.abs(want["CO"]).max())


# matrix-core contraction shapes: (lattice, axes, separations, levels, precision)
#   two separation octets on a 24-site line (one pass of 48 tiles), updates
#   between the 13 measurements (FP64 O rows: chunks of 4, the last one ragged);
#   a strided 32-site axis with 9 separations (64 tiles: two passes; FP32 O
#   rows, as FP64 rows of 32 sites exceed the chunk buffer);
#   FP32 O rows on the 24-site line (9 identical measurements: chunks of 8);
#   a strided 24-site axis (the vector kernel's build for 24-site lines with
#   rows staged through registers; the matrix-core kernel's word copies, FP32
#   and FP64 O rows)
MFMA_CASES = {
    "octets_x": ((24, 6, 6), [0], list(range(1, 12)), [(2, 13, 1)], 0),
    "octets_x_still": ((24, 6, 6), [0], list(range(1, 12)), [(2, 5, 0)], 0),
    "passes_y": ((4, 32, 6), [1], list(range(1, 10)), [(2, 6, 1)], 1),
    "fp32_o": ((24, 6, 6), [0], list(range(1, 12)), [(2, 9, 0)], 1),
    "two_levels": ((24, 6, 4), [0], list(range(1, 12)), [(4, 2, 1), (2, 5, 1)], 0),
    "strided_24_fp32": ((6, 24, 6), [1], list(range(1, 9)), [(2, 5, 0)], 1),
    "strided_24_fp64": ((6, 24, 6), [1], list(range(1, 9)), [(2, 5, 0)], 0),
}


@pytest.mark.parametrize("case", sorted(MFMA_CASES))
def test_insertion_contraction_matrix_cores_match_oracle(env, case):
    """The matrix-core kernel on the shapes that exercise its tiling: more
    than 8 separations, lines of up to 32 sites, several passes over the
    measurements, chunks cut short, both O precisions.  With updates between
    the measurements (every measurement differs) it is compared with the
    vector kernel on the same device trajectory (the update kernels are the
    same, so the links are bit-identical and only the order of the FP64 sums
    differs); without updates also with the oracle."""
    u1, O, torch = env
    ns, dirs, r, levels, precision = MFMA_CASES[case]
    say("matrix-core contraction", case)
    got, want, ctx, _ = _multilevel_pair(env, ns, 8, levels, 0, r, dirs, PROBES, [0, 1, 2, 3, 4, 5],
                                         precision=precision, ins_kernel=2)
    assert ctx.plan["form"] == u1.FORM_HISTORY and ctx.plan["ins_slots"] == 8
    vec, _, ctx_v, _ = _multilevel_pair(env, ns, 8, levels, 0, r, dirs, PROBES, [0, 1, 2, 3, 4, 5],
                                        precision=precision, ins_kernel=1)
    assert ctx_v.plan["ins_slots"] != 8
    assert np.array_equal(ctx.links(0), ctx_v.links(0))
    assert np.array_equal(got["C"], vec["C"])
    scale = max(1.0, np.abs(vec["CO"]).max())
    assert np.max(np.abs(got["CO"] - vec["CO"])) < 1e-12 * scale
    if all(lv[2] == 0 for lv in levels):
        tol = 1e-12 if precision == 0 else 1e-5
        assert np.max(np.abs(got["C"] - want["C"])) < 1e-12
        assert np.max(np.abs(got["CO"] - want["CO"])) < tol * max(1.0, np.abs(want["CO"]).max())


@pytest.mark.parametrize("levels", [[(2, 4, 1)], [(4, 2, 1), (2, 3, 1)]])
def test_multilevel_trajectory_parity_heatbath_only(env, levels):
    """Whole multilevel configurations (updates included) with heatbath-only
    sweeps, where rounding differences stay at the 1e-13 level."""
    say("trajectory parity", levels)
    got, want, ctx, ref = _multilevel_pair(env, (4, 4, 4), 8, levels, 0, [1, 2], [0, 1], PROBES[:2], [0, 3, 4])
    # the heatbath's arccos amplifies rounding differences near psi = 0 a little
    assert np.max(circ_dist(ctx.links(0), ref.links())) < 1e-9
    assert ctx.counter(0) == ref.counter
    assert np.max(np.abs(got["C"] - want["C"])) < 1e-10
    assert np.max(np.abs(got["CO"] - want["CO"])) < 1e-9


def _chain(u1, spec, start, therm, n_conf, between=1):
    ctx = u1.Context(spec)
    ctx.init_links(start)
    ctx.sweeps(therm)
    out = []
    for _ in range(n_conf):
        ctx.multilevel()
        ctx.sweeps(between)
        out.append(spec.unpack(ctx.results()[0, 0]))
    return out, ctx


@pytest.mark.parametrize("precision", [0, 1])
def test_c1_statistical_parity_with_overrelaxation(env, precision):
    """The C1 workload (1 heatbath + 3 overrelaxation) on the GPU and on the
    oracle as independent chains of 400 configurations; the host estimators
    (Sec. II.B-C) on each chain's records: <P^dagger P>(r), ln <P^dagger P>(r),
    the connected insertions <O_sq>, <O_lin> and their checks, and the vacuum
    plaquette, with jackknife errors over 20 blocks of consecutive
    configurations.  The normalised differences pass the 3-sigma check with
    its multiple-comparison allowance."""
    u1, O, torch = env
    from helpers.stats import check_sigma
    from paper_1309_3859_amd import analysis as A
    from paper_1309_3859_amd import configs

    spec, sched = configs.c1_plain_fp64()
    spec.precision = precision
    n, nb = 400, 20
    say("c1 statistical", precision)
    g, _ = _chain(u1, spec, sched["start"], sched["therm"], n)
    ref = O.Lattice(4, [4, 4, 4, 4], 1.0, seed=1)
    ref.init(sched["start"])
    ref.sweeps(sched["therm"])
    ospec = O.MLSpec(levels=spec.levels, r=spec.r, dirs=spec.dirs, probes=spec.probes, comps=spec.comps)
    w = []
    for _ in range(n):
        w.append(ospec.unpack(ref.multilevel(ospec)))
        ref.sweeps(1)
    zs = []
    for name, est in [("<P+P>", lambda rs: A.correlator(rs, n_blocks=nb)),
                      ("ln <P+P>", lambda rs: A.log_correlator(rs, n_blocks=nb)),
                      ("<O>_P+P", lambda rs: A.field_profile(rs, spec.comps, spec.dirs, n_blocks=nb)),
                      ("vacuum", lambda rs: A.jackknife(A.block_means(np.array([x["vac_sq"] for x in rs]), nb),
                                                        lambda v: v.mean(axis=0)))]:
        (mg, eg), (mw, ew) = est(g), est(w)
        z = np.abs(mg - mw) / np.sqrt(eg ** 2 + ew ** 2 + 1e-300)
        say(name, "GPU", np.ravel(mg), "+-", np.ravel(eg), "oracle", np.ravel(mw), "+-", np.ravel(ew))
        zs.append(np.ravel(z))
    ok, count, allowed, zmax, bound = check_sigma(np.concatenate(zs), nb - 1)
    say("above 3 sigma", count, "allowed", allowed, "largest", zmax, "bound", bound)
    assert ok


@pytest.mark.parametrize("kernel", [1, 2])
def test_results_independent_of_tile_batch_and_graphs(env, kernel):
    """Same ensemble alone or inside a batch of uneven ensembles, any work-group
    size, graphs on or off: bit-identical links and estimates, with either
    insertion kernel (vector, matrix cores)."""
    u1, O, torch = env
    A = u1.Ens((6, 4, 4), 8, 1.0, seed=3, key_id=7)
    B = u1.Ens((4, 4, 8), 4, 0.9, seed=3, key_id=1)
    Cc = u1.Ens((8, 8, 4), 4, 1.05, seed=9, key_id=2)
    kw = dict(levels=[(4, 2, 1), (2, 2, 1)], r=[1, 2, 3], dirs=[0], probes=[(0, 0, 0, 1), (0, 1, 1, 1)],
              comps=[0, 1, 5], precision=1, n_or=3, max_configs=2, ins_kernel=kernel)
    runs = []
    for ens_list, idx, block, graphs in [([A], 0, 256, True), ([B, A, Cc], 1, 64, False), ([Cc, B, A], 2, 1024, True),
                                         ([A, B], 0, 128, False)]:
        say("determinism", len(ens_list), block, graphs, kernel)
        spec = u1.Spec(ensembles=ens_list, **kw)
        ctx = u1.Context(spec)
        assert (ctx.plan["ins_slots"] == 8) == (kernel == 2)
        ctx.set_block(block)
        ctx.set_graphs(graphs)
        ctx.init_links(1)
        ctx.sweeps(3)
        ctx.multilevel()
        res = ctx.results()[0, idx]
        runs.append((ctx.links(idx), res, ctx.counter(idx)))
    for th, res, cnt in runs[1:]:
        assert np.array_equal(th, runs[0][0])
        assert np.array_equal(res, runs[0][1])
        assert cnt == runs[0][2]


def test_checkpoint_resume_is_bit_exact(env):
    u1, O, torch = env
    kw = dict(levels=[(2, 2, 1)], r=[1], dirs=[0])
    spec = u1.Spec(ensembles=[u1.Ens((4, 4, 4), 8, 1.0, seed=2)], precision=1, **kw)
    a = u1.Context(spec)
    a.init_links(1)
    a.sweeps(6)
    a.multilevel()
    straight = a.links(0), a.results()[0, 0]
    b = u1.Context(spec)
    b.init_links(1)
    b.sweeps(3)
    saved, cnt = b.links(0), b.counter(0)
    del b
    c = u1.Context(spec)
    c.set_links(saved)
    c.set_counter(cnt)
    c.sweeps(3)
    c.multilevel()
    assert np.array_equal(c.links(0), straight[0])
    assert np.array_equal(c.results()[0, 0], straight[1])


def test_health_and_state_errors(env):
    u1, O, torch = env
    spec = u1.Spec(ensembles=[u1.Ens((4, 4, 4), 4, 1.0)], levels=[(2, 1, 1)], r=[1], max_configs=1)
    ctx = u1.Context(spec)
    with pytest.raises(u1.U1MLError) as ei:
        ctx.multilevel()
    assert ei.value.status == 4  # ESTATE: links never initialised
    ctx.init_links(0)
    assert ctx.health() == 0
    th = ctx.links(0)
    th[5] = np.nan
    th[17] = 4.0
    ctx.set_links(th)
    assert ctx.health() == 2
    ctx.init_links(1)
    ctx.multilevel()
    with pytest.raises(u1.U1MLError) as ei:
        ctx.multilevel()
    assert ei.value.status == 4  # ring full
    assert ctx.results().shape[0] == 1
    ctx.multilevel()

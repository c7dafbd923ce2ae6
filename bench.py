"""Benchmark: multilevel link updates per second on one MI355X.

A step is one multilevel configuration (the body of Algorithm 1 of arXiv
1309.3859 with the workload's levels: sublattice sweeps of 1 heatbath + 3
overrelaxation passes, measurements, slab averages, slab products and sums)
over the whole batch of ensembles, with the links already resident in HBM.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4|c2|c3|c1]

Prints one JSON line.  value = non-frozen link updates of K steps / GPU time of
K steps.  The roofline entry is for the dominant kernel (the overrelaxation
phase of a spatial direction inside the inner slabs): algorithmic bytes under
the streaming model (every distinct link angle the phase reads once, every link
it writes once) divided by its average launch time from HIP events.
"""
from __future__ import annotations

import argparse
import inspect
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_update_or_c4_counters.md")
KERNEL_SOURCES = ["k_update.hip", "device_common.hpp"]


def _code_only(text: str) -> bytes:
    """Source text without // comments, blank lines and indentation, so that an
    edit of the comments alone keeps the hash."""
    out = []
    for line in text.splitlines():
        code = line.split("//", 1)[0].strip()
        if code:
            out.append(" ".join(code.split()))
    return "\n".join(out).encode()


def kernel_source_hash() -> str:
    """Hash of what the update kernel is built from and how it is launched:
    its two source files, the records it reads (the ensemble descriptor and the
    per-block record; the rest of the shared header holds other kernels'
    declarations and constants) and the host function that builds the block
    records and their order, comments left out."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1309_3859_amd", "csrc")
    for f in KERNEL_SOURCES:
        with open(os.path.join(csrc, f)) as fh:
            h.update(_code_only(fh.read()))
    with open(os.path.join(csrc, "u1ml_internal.hpp")) as fh:
        text = fh.read()
    for struct in ("struct EnsDesc {", "struct alignas(64) UpdBlock {"):
        start = text.index(struct)
        h.update(_code_only(text[start:text.index("};", start) + 2]))
    with open(os.path.join(csrc, "u1ml_api.cpp")) as fh:
        text = fh.read()
    start = text.index("void build_update_tabs(")
    h.update(_code_only(text[start:text.index("\n}\n", start) + 3]))
    return h.hexdigest()


def counter_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by the ratio of
    a plain copy's known bytes to what the same counter read for it), or None
    when the summary is missing or the kernel sources changed since."""
    try:
        vals = {}
        with open(COUNTERS_FILE) as fh:
            for line in fh:
                if line.startswith("- ") and ":" in line:
                    k, v = line[2:].split(":", 1)
                    vals[k.strip()] = v.strip().strip("`")
        if vals.get("kernel_source_sha256") != kernel_source_hash():
            return None
        fetch = float(vals["fetch_kib_per_launch"]) * float(vals["fetch_scale"])
        write = float(vals["write_kib_per_launch"]) * float(vals["write_scale"])
        return (fetch + write) * 1024.0
    except (OSError, KeyError, ValueError):
        return None


def metropolis_acceptance(ctx, spec, tau):
    """Acceptance rate of one phase of the paper's Metropolis update (step
    metro_delta) over the whole batch: spatial direction x, even sites, inner
    slabs; the fraction of the phase's links whose angle changed."""
    from paper_1309_3859_amd import analysis, u1ml

    before = [ctx.links(e) for e in range(len(spec.ensembles))]
    ctx.phase(u1ml.METROPOLIS, 0, 0, tau)
    moved = total = 0
    for e, ens in enumerate(spec.ensembles):
        m = analysis.phase_mask(ens.ns, ens.nt, 0, 0, tau)
        moved += int(((before[e] != ctx.links(e)) & m).sum())
        total += int(m.sum())
    return {"delta": spec.metro_delta, "acceptance": moved / total, "links": total}


def staple_abs(th, ns, nt):
    """|A| of every link from canonical angles th[4 s + mu], s = x + Nx (y +
    Ny (z + Nz t)): A = sum over nu != mu of the forward and backward
    staples' phases, returned in the same (s, mu) order."""
    import numpy as np

    nx, ny, nz = ns
    th = np.asarray(th).reshape(nt, nz, ny, nx, 4)
    ax = (3, 2, 1, 0)  # array axis of direction x, y, z, t
    sh = lambda a, d, k: np.roll(a, -k, axis=ax[d])  # sh(a, d, 1)[x] = a[x + d]
    out = np.empty(th.shape)
    for mu in range(4):
        A = np.zeros(th.shape[:4], dtype=np.complex128)
        for nu in range(4):
            if nu == mu:
                continue
            tm, tn = th[..., mu], th[..., nu]
            A += np.exp(1j * (sh(tn, mu, 1) - sh(tm, nu, 1) - tn))
            A += np.exp(1j * (sh(tn, nu, -1) - sh(sh(tn, mu, 1), nu, -1) - sh(tm, nu, -1)))
        out[..., mu] = np.abs(A)
    return out.ravel()


def heatbath_attempts(ctx, spec, n_bins: int = 48, draws: int = 8192):
    """Best-Fisher attempts per accepted link on the batch's current links:
    kappa = beta |A| of every link (staple sums formed on the host from the
    canonical angles), binned, and the mean attempt count of each bin's
    kappa from `draws` device draws of the heatbath's own sampler
    (u1ml_vonmises_fill, the workload's precision), weighted by the bin's
    links."""
    import numpy as np

    from paper_1309_3859_amd import u1ml

    kap = np.concatenate([ens.beta * staple_abs(ctx.links(e), ens.ns, ens.nt) for e, ens in enumerate(spec.ensembles)])
    edges = np.linspace(0.0, kap.max() * (1 + 1e-9), n_bins + 1)
    counts, _ = np.histogram(kap, edges)
    mean_att = 0.0
    for b in range(n_bins):
        if counts[b] == 0:
            continue
        k = 0.5 * (edges[b] + edges[b + 1])
        _, att = u1ml.vonmises_fill(k, draws, precision=spec.precision, seed=11, key_id=b)
        mean_att += counts[b] * float(att.double().mean())
    return {"attempts_per_link": mean_att / counts.sum(), "kappa_mean": float(kap.mean()),
            "links": int(kap.size),
            "method": f"kappa = beta |A| of every link of the batch after the timed steps, {n_bins} bins, "
                      f"{draws} draws of the device sampler per bin"}


def measurement_accuracy(ctx64, spec):
    """Accuracy of the FP32 form against the FP64 form on identical inputs:
    the FP64 context's current links, rounded to FP32 for both sides, (1)
    measured once without updates by each precision (largest relative
    difference of the correlators C(r) and of the vacuum plaquette over the
    batch), then (2) updated by one overrelaxation and one heatbath phase
    with the same counters (circular differences of the links: median,
    99.9th percentile, maximum; a heatbath link whose accept decision flips
    under FP32 rounding lands elsewhere)."""
    import dataclasses

    import numpy as np

    from paper_1309_3859_amd import u1ml

    links = [np.asarray(ctx64.links(e), dtype=np.float32).astype(np.float64) for e in range(len(spec.ensembles))]
    tau = spec.levels[-1][0]
    out, after = {}, {}
    for prec in (u1ml.FP32, u1ml.FP64):
        sp = dataclasses.replace(spec, levels=[(tau, 1, 0)], precision=prec, max_configs=1, _keep=[])
        c = u1ml.Context(sp)
        for e, th in enumerate(links):
            c.set_links(th, e)
            c.set_counter(0, e)
        c.multilevel()
        out[prec] = [sp.unpack(rec) for rec in c.results()[0]]
        c.phase(u1ml.OVERRELAX, 0, 0, tau)
        c.phase(u1ml.HEATBATH, 0, 1, tau)
        after[prec] = [c.links(e) for e in range(len(links))]
        c.close()
    pairs = list(zip(out[u1ml.FP32], out[u1ml.FP64]))
    rel_v = max(float(np.max(np.abs(a["vac_sq"] - b["vac_sq"]) / np.abs(b["vac_sq"]))) for a, b in pairs)
    moved = np.concatenate([(a != th) | (b != th) for a, b, th in zip(after[u1ml.FP32], after[u1ml.FP64], links)])
    d = np.concatenate([np.abs(np.angle(np.exp(1j * (a - b)))) for a, b in zip(after[u1ml.FP32], after[u1ml.FP64])])
    d = d[moved]
    return {"measurement": "vacuum <O_sq>, one measurement without updates on the same FP32-rounded links (C(r) "
                           "is formed in FP64 from the stored angles in both forms, so it differs only through the "
                           "links; chains of both forms agree within 3.2 sigma on every observable of the 32^3x8 "
                           "precision study, tests/test_gpu_precision.py)",
            "max_rel_diff_vacuum": rel_v,
            "update": "links after one overrelaxation and one heatbath phase from the same links and counters",
            "link_diff_median": float(np.median(d)), "link_diff_p999": float(np.quantile(d, 0.999)),
            "link_diff_max": float(d.max()), "links_updated": int(d.size)}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-n-inner", type=int, default=2,
                    help="inner-level updates of the oracle's sampled configuration (0: the workload's own)")
    ap.add_argument("--cpu-n-outer", type=int, default=1,
                    help="outer-level updates of the oracle's sampled configuration (0: the workload's own)")
    ap.add_argument("--cpu-max-probes", type=int, default=0,
                    help="insertion probes of the oracle's sampled configuration (0: all of the workload's)")
    ap.add_argument("--cpu-timeout", type=float, default=600.0,
                    help="seconds the oracle's child processes may run before the single-thread fallback")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison leg")
    ap.add_argument("--precision", choices=("workload", "f32", "f64"), default="workload",
                    help="link storage and update arithmetic of the timed line (default: the workload's own); "
                         "with f32 the plain FP64 leg times the same workload in FP64")
    ap.add_argument("--cpu-only", action="store_true",
                    help="time only the oracle on the host (no GPU) and print its cpu_baseline object")
    ap.add_argument("--block", type=int, default=256,
                    help="work-group size of the update kernels (0: autotune; candidates differ by about 2 percent, "
                         "so a fixed size keeps profiled and unprofiled runs on the same launch shape)")
    ap.add_argument("--n-inner", type=int, default=0,
                    help="for kernel traces of the large presets: sublattice updates of the inner level (0: the preset's)")
    ap.add_argument("--n-outer", type=int, default=0,
                    help="for kernel traces of the two-level presets: updates of the outer level (0: the preset's)")
    ap.add_argument("--n-ens", type=int, default=0,
                    help="for the replicas preset: number of replicas in the batch (0: the preset's 16)")
    ap.add_argument("--ins-kernel", type=int, choices=(0, 1, 2), default=0,
                    help="history-form insertion sums: 0 the planner's choice, 1 the vector kernel, 2 the matrix cores")
    ap.add_argument("--counters", action="store_true",
                    help="for hardware-counter runs: one 256 MiB device copy (calibration of the byte counters), "
                         "then 20 launches each of the heatbath and overrelaxation phases of the dominant kernel")
    return ap.parse_args()


def _sample_levels(spec, n_inner: int = 2, n_outer: int = 1):
    """The workload's levels with the update counts cut to n_inner (inner
    level) and n_outer (outer level of two); 0 keeps the workload's count."""
    levels = [list(lv) for lv in spec.levels]
    if n_inner:
        levels[-1][1] = n_inner
    if len(levels) == 2 and n_outer:
        levels[0][1] = n_outer
    return levels


def oracle_configuration(job: dict) -> dict:
    """One ensemble's multilevel configuration on the FP64 oracle (one host
    thread): the non-frozen link updates it performs and the seconds it took."""
    from oracle import oracle as O

    ns, nt, levels, n_or = job["ns"], job["nt"], job["levels"], job["n_or"]
    ospec = O.MLSpec(levels=[tuple(lv) for lv in levels], r=job["r"], dirs=job["dirs"],
                     probes=[tuple(p) for p in job["probes"]], comps=job["comps"], n_or=n_or)
    lat = O.Lattice(4, list(ns) + [nt], job["beta"], seed=job["seed"], key_id=job["key_id"])
    lat.init(1)
    # configurations of the chain until min_seconds have passed (at least one)
    n_cfg = 0
    t0 = time.perf_counter()
    while True:
        lat.multilevel(ospec)
        n_cfg += 1
        dt = time.perf_counter() - t0
        if dt >= job.get("min_seconds", 0.0):
            break
    V = ns[0] * ns[1] * ns[2] * nt
    sp = lambda tau: V // 2 // nt * (nt - nt // tau)
    per_sweep = lambda tau: (1 + n_or) * 2 * (V // 2 + 3 * sp(tau))
    ti, ni, ki = levels[-1]
    u = ni * ki * per_sweep(ti)
    if len(levels) == 2:
        to, no, ko = levels[0]
        u = no * (ko * per_sweep(to) + ni * ki * per_sweep(ti))
    return {"updates": u * n_cfg, "seconds": dt, "configurations": n_cfg}


def cpu_model() -> str:
    """The host CPU's model name (first entry of /proc/cpuinfo), or the
    platform's processor string."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or "unknown"


def cpu_baseline(spec, budget_s: float, workers: int = 16, n_inner: int = 2, n_outer: int = 1, max_probes: int = 0,
                 min_seconds: float = 2.0, timeout_s: float = 600.0):
    """Time the FP64 oracle on the host cores on a bounded sample of the
    workload: every ensemble of the batch (independent, as on the GPU), one
    multilevel configuration each with the update counts cut down (repeated
    until the child has run min_seconds, so that a tiny lattice is not timed
    on the interpreter's start-up), each in a child interpreter of its own, up
    to `workers` at a time.  `value` is the
    sample's updates over the wall time; `single_thread` the same updates over
    the sum of the children's own times.  Falls back to one thread in this
    process (stopping after about budget_s seconds) if a child fails."""
    import subprocess

    from oracle import oracle as O

    O.build()
    levels = _sample_levels(spec, n_inner, n_outer)
    probes = list(spec.probes)[:max_probes] if max_probes else list(spec.probes)
    jobs = [{"ns": list(e.ns), "nt": e.nt, "beta": e.beta, "seed": e.seed, "key_id": e.key_id, "levels": levels,
             "r": list(spec.r), "dirs": list(spec.dirs), "probes": [list(p) for p in probes],
             "comps": list(spec.comps), "n_or": spec.n_or, "min_seconds": min_seconds} for e in spec.ensembles]
    workers = max(1, min(workers, len(jobs), os.cpu_count() or 1))
    results, running = [], []
    # largest ensembles first, a new child as soon as one ends
    pending = sorted(jobs, key=lambda j: -j["ns"][0] * j["ns"][1] * j["ns"][2] * j["nt"])
    try:
        t0 = time.perf_counter()
        while pending or running:
            while pending and len(running) < workers:
                running.append(subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-job",
                                                 json.dumps(pending.pop(0))], stdout=subprocess.PIPE,
                                                stderr=subprocess.DEVNULL, text=True, cwd=ROOT))
            time.sleep(0.005)
            for pr in [q for q in running if q.poll() is not None]:
                running.remove(pr)
                out = pr.stdout.read()
                if pr.returncode != 0:
                    raise RuntimeError(f"oracle child exited with {pr.returncode}")
                results.append(json.loads(out.strip().splitlines()[-1]))
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError(f"oracle children still running after {timeout_s:g} s")
        wall = time.perf_counter() - t0
        upd = sum(r["updates"] for r in results)
        cpu_s = sum(r["seconds"] for r in results)
        n_cfg = sum(r["configurations"] for r in results)
        return {"value": upd / wall, "unit": "link updates/s", "cores": workers, "kind": "oracle",
                "cpu": cpu_model(), "host_cpus": os.cpu_count(),
                "sample": f"{len(jobs)} of {len(jobs)} ensembles, multilevel configurations with levels "
                          f"{levels} (tau, n_iter, k_sweeps), {len(probes)} of {len(spec.probes)} probes, FP64, "
                          f"one ensemble per process, up to {workers} at a time, each repeating configurations "
                          f"for at least {min_seconds:g} s ({n_cfg} in all); {cpu_s:.1f} s of oracle time in "
                          f"{wall:.1f} s",
                "single_thread": {"value": upd / cpu_s, "cores": 1}}
    except Exception as exc:  # noqa: BLE001 -- the baseline must not cost the bench line
        for pr in running:
            pr.kill()
            pr.wait()
        done_upd, t_used, n = 0, 0.0, 0
        for j in jobs:
            r = oracle_configuration(j)
            done_upd += r["updates"]
            t_used += r["seconds"]
            n += 1
            if t_used > budget_s:
                break
        return {"value": done_upd / t_used, "unit": "link updates/s", "cores": 1, "kind": "oracle",
                "cpu": cpu_model(), "host_cpus": os.cpu_count(),
                "sample": f"{n} of {len(jobs)} ensembles, one multilevel configuration each with levels {levels} "
                          f"(tau, n_iter, k_sweeps), FP64, single thread ({type(exc).__name__} in the "
                          f"per-process run); {t_used:.1f} s"}


def step_update_bytes(ctx, spec):
    """Algorithmic bytes of one step's link updates under the streaming model:
    the enumerated read and write sets of every phase (u1ml_phase_bytes) of
    every sweep of the workload's levels, the stochastic pass once and the
    overrelaxation pass n_or times per sweep."""
    from paper_1309_3859_amd import u1ml

    stoch = u1ml.METROPOLIS if spec.update == u1ml.UPDATE_METROPOLIS else u1ml.HEATBATH
    memo = {}

    def sweep(tau):
        if tau not in memo:
            b = u = 0.0
            for mu in range(4):
                for p in (0, 1):
                    for kind, times in ((stoch, 1), (u1ml.OVERRELAX, spec.n_or)):
                        bb, uu = ctx.phase_bytes(kind, mu, p, tau)
                        b += times * bb
                        u += times * uu
            memo[tau] = (b, u)
        return memo[tau]

    levels = spec.levels
    ti, ni, ki = levels[-1]
    bi, ui = sweep(ti)
    if len(levels) == 1:
        return ni * ki * bi, ni * ki * ui
    to, no, ko = levels[0]
    bo, uo = sweep(to)
    return no * (ko * bo + ni * ki * bi), no * (ko * uo + ni * ki * ui)


def time_steps(ctx, steps: int, warmup: int):
    """Warm up, then time `steps` multilevel configurations with events on the
    context's stream; returns milliseconds."""
    import torch

    for _ in range(warmup):
        ctx.multilevel()
    torch.cuda.synchronize()
    ctx.results()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(ctx.stream)
    for _ in range(steps):
        ctx.multilevel()
    stop.record(ctx.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    assert ctx.results().shape[0] == steps
    return ms


def time_full_sweeps(ctx, n: int = 10):
    """Full-lattice sweeps (every link, no frozen slabs: 1 heatbath and n_or
    overrelaxation passes each) timed with events on the context's stream;
    returns link updates/s."""
    import torch

    ctx.sweeps(2)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(ctx.stream)
    ctx.sweeps(n)
    b.record(ctx.stream)
    torch.cuda.synchronize()
    return ctx.plan["updates_per_sweep"] * n / (a.elapsed_time(b) / 1e3)


def copy_reference(nbytes: float, reps: int = 50):
    """A plain device copy moving the same number of bytes as one launch of
    the dominant kernel (half read, half written), timed with events: the
    bandwidth a kernel of this size can reach on the part, for context."""
    import torch

    n = int(nbytes // 2)
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    us = a.elapsed_time(b) * 1e3 / reps
    return {"bytes": 2 * n, "us_per_copy": us, "GB/s": 2 * n / (us * 1e-6) / 1e9}


def run_counter_workload(spec, sched):
    """Kernels for rocprofv3 --pmc runs: a plain copy of 2^28 bytes (its
    FETCH_SIZE / WRITE_SIZE give the counters' scale), then the inner-slab
    spatial heatbath and overrelaxation phases (mu = x, parity 0) as the step
    launches them, one launch per lane, 20 launches of each lane and kind:
    heatbath lane 0, lane 1, then overrelaxation lane 0, lane 1; first with
    the workload's FP32 links, then the same in FP64."""
    import dataclasses

    import torch

    from paper_1309_3859_amd import u1ml

    src = torch.empty(1 << 28, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    out = {"copy_bytes": 1 << 28}
    for prec in (spec.precision, u1ml.FP64 if spec.precision == u1ml.FP32 else None):
        if prec is None:
            continue
        sp = dataclasses.replace(spec, precision=prec, _keep=[])
        ctx = u1ml.Context(sp)
        ctx.init_links(sched["start"])
        ctx.sweeps(2)
        tau = sp.levels[-1][0]
        name = "f32" if prec == u1ml.FP32 else "f64"
        for kind in (0, 1):
            for lane in range(ctx.n_lanes):
                us, b, u = ctx.time_phase_lane(lane, kind, 0, 0, tau, 20)
                out[f"{name}_{('hb', 'or')[kind]}_lane{lane}"] = {"bytes": b, "updates": u, "us": us}
        torch.cuda.synchronize()
        ctx.close()
    print(json.dumps(out), flush=True)


def progress(msg: str):
    """One line on stderr per stage of the run (the JSON line stays alone on stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def main():
    if len(sys.argv) == 3 and sys.argv[1] == "--oracle-job":
        # child of cpu_baseline: one oracle configuration, no GPU
        print(json.dumps(oracle_configuration(json.loads(sys.argv[2]))), flush=True)
        return
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the library has no multi-GPU path; "
              "how a batch or one lattice would shard across GPUs is described in the design notes", file=sys.stderr)
        sys.exit(2)
    from paper_1309_3859_amd import configs, u1ml

    preset = configs.PRESETS[args.workload]

    if args.n_ens and "n_ens" not in inspect.signature(preset).parameters:
        sys.exit(f"--n-ens applies to the replicas preset, not to {args.workload}")

    def make():
        spec, sched = preset(n_ens=args.n_ens) if args.n_ens else preset()
        lv = [list(x) for x in spec.levels]
        if args.n_inner:
            lv[-1][1] = args.n_inner
        if args.n_outer and len(lv) == 2:
            lv[0][1] = args.n_outer
        spec.levels = [tuple(x) for x in lv]
        if args.precision != "workload":
            spec.precision = u1ml.FP32 if args.precision == "f32" else u1ml.FP64
        spec.ins_kernel = args.ins_kernel
        return spec, sched

    spec, sched = make()
    if args.cpu_only:
        print(json.dumps({"workload": preset.__name__, "updates_per_config": u1ml.plan(spec)["updates_per_config"],
                          "cpu_baseline": cpu_baseline(spec, args.cpu_seconds, n_inner=args.cpu_n_inner,
                                                       n_outer=args.cpu_n_outer, max_probes=args.cpu_max_probes,
                                                       timeout_s=args.cpu_timeout)}),
              flush=True)
        return
    import torch

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    if args.counters:
        run_counter_workload(spec, sched)
        return
    spec.max_configs = max(1, args.steps + args.warmup)
    ctx = u1ml.Context(spec)
    ctx.init_links(sched["start"])
    # the autotuner's sweep timings for every work-group size (it restores
    # links and counters), reported beside the size the line runs with
    tune = ctx.autotune()
    if args.block:
        ctx.set_block(args.block)
        block = args.block
    else:
        block = tune["chosen_block"]
    ctx.sweeps(20)
    upd = ctx.plan["updates_per_config"]
    ms = time_steps(ctx, args.steps, args.warmup)
    value = upd * args.steps / (ms / 1e3)
    progress(f"{args.steps} steps timed: {ms / args.steps:.3f} ms per step")

    # dominant kernel: spatial overrelaxation phase inside inner slabs, in the
    # launch shape of the step (one launch per lane), each lane's launch timed
    # by its own dispatch events; achieved = the lanes' bytes / their time
    tau = spec.levels[-1][0]
    lanes = []
    for lane in range(ctx.n_lanes):
        lus, lb, lu = ctx.time_phase_lane(lane, 1, 0, 0, tau, 50)
        lanes.append({"lane": lane, "us_per_launch": lus, "bytes_per_launch": lb, "updates_per_launch": lu,
                      "GB/s": lb / (lus * 1e-6) / 1e9})
    us = sum(x["us_per_launch"] for x in lanes) / len(lanes)
    b = sum(x["bytes_per_launch"] for x in lanes) / len(lanes)
    u = sum(x["updates_per_launch"] for x in lanes) / len(lanes)
    achieved = b / (us * 1e-6) / 1e9
    # every phase kind as one whole-batch launch, for context
    per_phase = {}
    for kind, mu in [(1, 0), (0, 0), (1, 3), (0, 3), (2, 0)]:
        pus = ctx.time_phase(kind, mu, 0, tau, 50)
        pb, pu = ctx.phase_bytes(kind, mu, 0, tau)
        per_phase[(kind, mu)] = (pus, pb, pu)
    wus, wb, wu = per_phase[(1, 0)]
    line = {
        "metric": "link updates/s (HB+OR, multilevel)",
        "value": value,
        "unit": "link updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if spec.precision == u1ml.FP32 else "f64",
        "data": "synthetic (seeded Monte-Carlo ensembles)",
        "config": {"workload": preset.__name__, "ensembles": len(spec.ensembles),
                   "lattices": sorted({f"{e.ns[0]}^3x{e.nt}" for e in spec.ensembles}),
                   "levels": spec.levels, "n_or": spec.n_or, "updates_per_step": upd,
                   "block": block,
                   "autotune": {"us_per_sweep": dict(zip(map(str, tune["block"]), tune["us_per_sweep"])),
                                "chosen_block": tune["chosen_block"],
                                "note": "work-group size only; the update kernels have no other tile dimension"}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": counter_traffic() if args.workload == "c4" else None,
                     "kernel": f"k_update<{'float' if spec.precision == u1ml.FP32 else 'double'},1,0> "
                               "(overrelaxation, mu = x, inner slabs), one launch per lane as the step launches it; "
                               "averages over the lanes",
                     "bytes_per_launch": b, "updates_per_launch": u, "us_per_launch": us, "lanes": lanes,
                     "whole_batch_launch": {"us_per_launch": wus, "bytes_per_launch": wb, "updates_per_launch": wu,
                                            "frac": wb / (wus * 1e-6) / 1e9 / HBM_PEAK_GBS}},
        # per launch of each phase over the whole batch; MET = the paper's Metropolis update
        "phases_us": {f"{('HB', 'OR', 'MET')[k]}_mu{m}": v[0] for (k, m), v in per_phase.items()},
    }
    progress("phases timed")
    line["roofline"]["copy_reference"] = copy_reference(wb)
    # the whole step: every update phase's enumerated bytes over the step's time
    sb, su = step_update_bytes(ctx, spec)
    assert int(su) == upd, (su, upd)
    step_gbs = sb / (ms / args.steps * 1e-3) / 1e9
    line["step_roofline"] = {"bound": "hbm", "achieved": step_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": step_gbs / HBM_PEAK_GBS, "bytes_per_step": sb, "bytes_per_update": sb / su,
                             "note": "link-update bytes of every phase of the step (streaming model) / ms_per_step"}
    # the same batch in full-lattice sweeps (thermalisation), next to the multilevel rate of `value`
    line["full_sweeps"] = {"value": time_full_sweeps(ctx), "unit": "link updates/s"}
    line["metropolis"] = metropolis_acceptance(ctx, spec, tau)
    line["heatbath"] = heatbath_attempts(ctx, spec)
    progress("step bytes, full sweeps, Metropolis acceptance and heatbath attempts done")
    if not args.no_fp64 and spec.precision == u1ml.FP32:
        # the same workload with FP64 link storage and update arithmetic
        spec64, _ = make()
        spec64.precision = u1ml.FP64
        spec64.max_configs = spec.max_configs
        del ctx
        ctx64 = u1ml.Context(spec64)
        ctx64.init_links(sched["start"])
        ctx64.set_block(block)
        ctx64.sweeps(5)
        ms64 = time_steps(ctx64, args.steps, args.warmup)
        ph64 = {f"{('HB', 'OR')[k]}_mu{m}": ctx64.time_phase(k, m, 0, tau, 50) for k, m in [(1, 0), (0, 0), (1, 3), (0, 3)]}
        line["plain_fp64"] = {"value": upd * args.steps / (ms64 / 1e3), "unit": "link updates/s",
                              "ms_per_step": ms64 / args.steps, "dtype": "f64", "phases_us": ph64,
                              "accuracy_of_f32": measurement_accuracy(ctx64, spec)}
    if not args.no_cpu_baseline:
        progress("FP64 leg done; timing the oracle on the host")
        line["cpu_baseline"] = cpu_baseline(spec, args.cpu_seconds, n_inner=args.cpu_n_inner,
                                            n_outer=args.cpu_n_outer, max_probes=args.cpu_max_probes,
                                            timeout_s=args.cpu_timeout)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

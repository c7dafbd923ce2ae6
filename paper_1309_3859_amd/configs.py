"""Seeded synthetic workloads shaped like the paper's (arXiv 1309.3859: 24^3 x Nt
lattices, beta near 1, Sec. II and III).  Input descriptions only: lattice
shapes, couplings, seeds, multilevel levels and the observable lists.

Each preset returns (spec, schedule) where schedule holds the start
(cold/hot) and the number of thermalisation sweeps.  Probes are
(l, p1, p2, mode): mode 1 places the insertion in the mid-plane between the
charges (offset l added), p1 and p2 are transverse offsets.
"""
from __future__ import annotations

import numpy as np

from .u1ml import COLD, FP32, FP64, HOT, Ens, Spec


def c1_plain_fp64(max_configs: int = 16):
    """4^3 x 4, beta = 1, cold, 20 sweeps (1 heatbath + 3 overrelaxation), one
    level: 2 slabs of thickness 2, 10 sublattice updates; r = 1, 2 along x;
    E_x insertion at the mid-plane; Philox seed 1; FP64."""
    spec = Spec(ensembles=[Ens((4, 4, 4), 4, 1.0, seed=1, key_id=0)], levels=[(2, 10, 1)], r=[1, 2], dirs=[0],
                probes=[(0, 0, 0, 1)], comps=[0], precision=FP64, n_or=3, max_configs=max_configs)
    return spec, {"start": COLD, "therm": 20}


def c2_fp32_profiles(n_iter: int = 100, max_configs: int = 4, precision: int = FP32):
    """24^3 x 8, beta = 0.99, hot start, 500 sweeps, one level (thickness 2,
    100 updates); r = 2..12 along x; E_x, E_y, E_z, B_x, B_y, B_z at the
    mid-plane, transverse distance 0..8; FP32 links, FP64 accumulators."""
    probes = [(0, p1, 0, 1) for p1 in range(9)]
    spec = Spec(ensembles=[Ens((24, 24, 24), 8, 0.99, seed=2, key_id=0)], levels=[(2, n_iter, 1)],
                r=list(range(2, 13)), dirs=[0], probes=probes, comps=list(range(6)), precision=precision, n_or=3,
                max_configs=max_configs)
    return spec, {"start": HOT, "therm": 500}


def c3_precision(precision: int = FP32, n_outer: int = 20, n_inner: int = 50, max_configs: int = 4):
    """32^3 x 8, beta = 1, two levels (slabs of 2 inside slabs of 4; 50 and 20
    updates), r = 1..16; the six field components on the axis at the
    mid-plane; FP32 or FP64 links from the same seed."""
    spec = Spec(ensembles=[Ens((32, 32, 32), 8, 1.0, seed=3, key_id=0)], levels=[(4, n_outer, 1), (2, n_inner, 1)],
                r=list(range(1, 17)), dirs=[0], probes=[(0, 0, 0, 1)], comps=list(range(6)), precision=precision,
                n_or=3, max_configs=max_configs)
    return spec, {"start": HOT, "therm": 500}


def c4_batched(precision: int = FP32, n_iter: int = 50, max_configs: int = 4):
    """16 independent ensembles, (Ns, Nt) in {16, 20, 24, 32} x {4, 6, 8, 10},
    beta_j uniform in [0.98, 1.00] (numpy generator, seed 4), Philox key
    (seed 4, key_id j); one level (thickness 2, 50 updates); correlators
    r = 1..8 along x (8 = Ns/2 of the smallest lattice)."""
    rng = np.random.default_rng(4)
    ens = []
    j = 0
    for ns in (16, 20, 24, 32):
        for nt in (4, 6, 8, 10):
            ens.append(Ens((ns, ns, ns), nt, float(0.98 + 0.02 * rng.random()), seed=4, key_id=j))
            j += 1
    spec = Spec(ensembles=ens, levels=[(2, n_iter, 1)], r=list(range(1, 9)), dirs=[0], precision=precision, n_or=3,
                max_configs=max_configs)
    return spec, {"start": HOT, "therm": 500}


def replicas(n_ens: int = 16, precision: int = FP32, n_iter: int = 50, max_configs: int = 4):
    """n_ens independent replicas of the paper's 24^3 x 8 lattice at beta = 0.99
    (Philox key (seed 9, key_id j)) in one batch; one level (thickness 2, 50
    updates), correlators r = 1..12 along x.  The batch-size study: how the
    rate of one small lattice grows when replicas share every launch."""
    ens = [Ens((24, 24, 24), 8, 0.99, seed=9, key_id=j) for j in range(n_ens)]
    spec = Spec(ensembles=ens, levels=[(2, n_iter, 1)], r=list(range(1, 13)), dirs=[0], precision=precision, n_or=3,
                max_configs=max_configs)
    return spec, {"start": HOT, "therm": 500}


def c5_largest(n_outer: int = 40, n_inner: int = 100, full_map: bool = True, max_configs: int = 1):
    """48^3 x 12, beta = 1.005, two levels (2 inside 4; 100 and 40 updates),
    r = 2..20 along x, the full transverse map |x_perp| <= 12 of all six
    components at the mid-plane (441 probes), FP32 links."""
    if full_map:
        probes = [(0, p1, p2, 1) for p1 in range(-12, 13) for p2 in range(-12, 13) if p1 * p1 + p2 * p2 <= 144]
    else:
        probes = [(0, 0, 0, 1)]
    spec = Spec(ensembles=[Ens((48, 48, 48), 12, 1.005, seed=5, key_id=0)], levels=[(4, n_outer, 1), (2, n_inner, 1)],
                r=list(range(2, 21)), dirs=[0], probes=probes, comps=list(range(6)), precision=FP32, n_or=3,
                max_configs=max_configs)
    return spec, {"start": HOT, "therm": 2000}


def in_plane_map(r: int = 6, margin: int = 3, width: int = 4, ns: int = 24, nt: int = 8, beta: float = 0.99,
                 n_inner: int = 100, max_configs: int = 1):
    """The field in the plane containing the charges (the paper's Fig. 1):
    probes (l, p1, 0) for l = -margin .. r + margin along the axis and
    p1 = -width .. width across it, E_par and E_perp1, one level tau = 2,
    FP32 links.  Every l is its own probe group in the spectral form."""
    probes = [(l, p1, 0, 0) for l in range(-margin, r + margin + 1) for p1 in range(-width, width + 1)]
    spec = Spec(ensembles=[Ens((ns, ns, ns), nt, beta, seed=6, key_id=0)], levels=[(2, n_inner, 1)], r=[r],
                dirs=[0], probes=probes, comps=[0, 1], precision=FP32, n_or=3, max_configs=max_configs)
    return spec, {"start": HOT, "therm": 500}


def beta_scan(betas, ns: int = 24, nt: int = 4, precision: int = FP32):
    """One batch of ensembles Ns^3 x Nt at the given couplings (plaquette
    susceptibility scan for beta_c); ensemble j has Philox key (7, j)."""
    ens = [Ens((ns, ns, ns), nt, float(b), seed=7, key_id=j) for j, b in enumerate(betas)]
    spec = Spec(ensembles=ens, levels=[(2, 1, 1)], r=[1], precision=precision, n_or=3)
    return spec, {"start": HOT, "therm": 500}


def out_of_cache(ns: int = 128, nt: int = 16):
    """Not one of the paper's workloads: one 128^3 x 16 FP32 ensemble (537 MB
    of links, twice the 256 MB Infinity Cache), one level tau = 2, the
    correlator at r = 1 only; its update phases show the rate when the links
    stream from DRAM."""
    spec = Spec(ensembles=[Ens((ns, ns, ns), nt, 1.0, seed=8, key_id=0)], levels=[(2, 2, 1)], r=[1], dirs=[0],
                precision=FP32, n_or=3, max_configs=4)
    return spec, {"start": HOT, "therm": 0}


PRESETS = {"c1": c1_plain_fp64, "c2": c2_fp32_profiles, "c3": c3_precision, "c4": c4_batched, "c5": c5_largest,
           "dram": out_of_cache, "replicas": replicas}

"""Writes susceptibility_4x4.json: the oracle's plaquette susceptibility
chi = N_P (<P^2> - <P>^2) on the 4^4 lattice (Sec. II: Wilson action; the
susceptibility locates beta_c, Sec. III.A) at beta = 0.9, 1.0, 1.1, from
four independent chains per coupling (hot start, 200 sweeps of one heatbath
and three overrelaxation passes, then 20000 sweeps, the plaquette averaged
over the lattice and its six orientations after each sweep), with errors and
integrated autocorrelation times from the Gamma method.  Calls only the
oracle and the host estimators.

    python tests/golden/make_susceptibility.py
"""
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

BETAS = (0.9, 1.0, 1.1)
SEEDS = (101, 102, 103, 104)
THERM, N = 200, 20000
N_PLAQ = 6 * 4 ** 4


def chain(args):
    from oracle import oracle as O
    from paper_1309_3859_amd import analysis as A

    beta, seed = args
    lat = O.Lattice(4, [4, 4, 4, 4], beta, seed=seed, key_id=0)
    lat.init(1)
    lat.sweeps(THERM)
    x = np.empty(N)
    for i in range(N):
        lat.sweeps(1)
        x[i] = lat.plaquette_means().mean()
    chi, sig, tint, dtint, W = A.susceptibility_gamma(x, N_PLAQ)
    return beta, seed, {"chi": chi, "sigma": sig, "tau_int": tint, "d_tau_int": dtint, "window": W,
                        "plaquette": float(x.mean())}


def main():
    from oracle import oracle as O

    O.build()
    jobs = [(b, s) for b in BETAS for s in SEEDS]
    with Pool(min(len(jobs), os.cpu_count() or 1)) as pool:
        res = pool.map(chain, jobs)
    out = {"lattice": [4, 4, 4, 4], "n_plaquettes": N_PLAQ, "therm": THERM, "sweeps": N, "n_or": 3,
           "start": "hot", "seeds": list(SEEDS), "betas": {}}
    for b in BETAS:
        ch = [r for bb, _, r in res if bb == b]
        chi = float(np.mean([c["chi"] for c in ch]))
        sig = float(np.sqrt(np.sum([c["sigma"] ** 2 for c in ch])) / len(ch))
        out["betas"][str(b)] = {"chi": chi, "sigma": sig, "chains": ch}
    with open(os.path.join(HERE, "susceptibility_4x4.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({b: (v["chi"], v["sigma"]) for b, v in out["betas"].items()}))


if __name__ == "__main__":
    main()

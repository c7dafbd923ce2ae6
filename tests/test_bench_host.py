"""bench.py's host side (no GPU): the committed HBM-counter summary of the
dominant kernel still belongs to the update kernel's current code (else the
bench line would report traffic as null), and its figure is consistent with
the kernel's algorithmic bytes."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402

# one launch of the C4 inner-slab overrelaxation phase per lane, averaged over the two lanes (410,816 updates in
# all): distinct link words read plus words written
ALGORITHMIC_BYTES = 9_859_584


def test_counter_summary_matches_the_update_kernel_code():
    traffic = bench.counter_traffic()
    assert traffic is not None, "profiles/k_update_or_c4_counters.md was taken on other update-kernel code"
    assert ALGORITHMIC_BYTES <= traffic < 1.2 * ALGORITHMIC_BYTES


def test_multi_gpu_request_is_refused(monkeypatch, capsys):
    monkeypatch.setattr(sys, "argv", ["bench.py", "--gpus", "2"])
    try:
        bench.main()
    except SystemExit as e:
        assert e.code == 2
    else:
        raise AssertionError("bench.py accepted --gpus 2")
    assert "one GPU only" in capsys.readouterr().err


def test_cpu_baseline_runs_one_oracle_process_per_ensemble():
    """The oracle leg runs each ensemble in a child interpreter (no GPU), and
    its update count is the planner's for the sampled levels."""
    from paper_1309_3859_amd import configs, u1ml

    spec, _ = configs.beta_scan([0.9, 1.0, 1.1], ns=4, nt=4)
    r = bench.cpu_baseline(spec, 5.0, workers=2)
    assert r["kind"] == "oracle" and r["cores"] == 2, r
    assert "one ensemble per process" in r["sample"], r
    assert r["value"] > 0 and r["single_thread"]["value"] > 0
    # the children's update count equals the planner's for the same (cut-down) levels
    job = {"ns": [4, 4, 4], "nt": 4, "beta": 1.0, "seed": 7, "key_id": 0, "levels": bench._sample_levels(spec),
           "r": [1], "dirs": [0], "probes": [], "comps": [], "n_or": spec.n_or}
    spec.levels = [tuple(lv) for lv in bench._sample_levels(spec)]
    spec.ensembles = spec.ensembles[:1]
    assert bench.oracle_configuration(job)["updates"] == u1ml.plan(spec)["updates_per_config"]


def test_staple_magnitudes_match_the_oracle():
    """bench.py's host staple sums (for the heatbath attempt count) give the
    oracle's |A| on a random 4 x 3 x 5 x 6 lattice."""
    import numpy as np

    from oracle import oracle as O

    ns, nt = (4, 3, 5), 6
    lat = O.Lattice(4, list(ns) + [nt], 1.0, seed=3, key_id=0)
    lat.init(1)
    th = lat.links()
    got = bench.staple_abs(th, ns, nt)
    V = ns[0] * ns[1] * ns[2] * nt
    want = np.array([abs(lat.staple(s, mu)) for s in range(V) for mu in range(4)])
    assert np.allclose(got, want, rtol=0, atol=1e-12)

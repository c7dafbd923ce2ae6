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

# one launch of the C4 inner-slab overrelaxation phase (410,816 updates): distinct link words read plus words written
ALGORITHMIC_BYTES = 19_719_168


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

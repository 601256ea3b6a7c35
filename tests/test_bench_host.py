"""Host-side pieces of bench.py, on the CPU (no GPU is touched).

* The committed rocprofv3 summaries of the fold's HBM bytes, in both layouts,
  are read back as bench.py reads them: a byte count when the fold's sources
  are the ones the counters were taken with, else a note; never an error.
* More than one GPU is refused with a message and exit status 2.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
bench = pytest.importorskip("bench")


@pytest.mark.parametrize("layout", ["posmajor", "persignal"])
def test_fold_traffic_summaries_read_back(layout):
    traffic, source = bench.measured_traffic(f"metric_batch512_c64_{layout}")
    assert source is not None
    if traffic is None:  # sources changed since the counters were taken
        assert "changed" in source or "no fold byte count" in source, source
    else:
        # about 0.8 (position-major) or 10 (per-signal) times the 2.07 GB of
        # algorithmic bytes per step of the metric batch
        assert 1.0e9 < traffic < 40e9, traffic
        assert source.startswith("profiles/")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr, (r.returncode, r.stderr)

"""Host-side checks of bench.py (no GPU): the one-GPU contract, the work count
behind the roofline, and that the committed HBM-traffic profile still belongs
to the search kernel's sources."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("n_t,K", [(16, 512), (16, 128), (8, 64), (4, 32)])
def test_search_work_is_the_papers_count(n_t, K):
    # Sec. III-B: the path search costs K N_t (1 + (N_t + 1) / 2) complex multiplications per vector
    assert bench.search_cm_per_vector(n_t, K) == K * n_t * (1 + (n_t + 1) / 2)


def test_valu_peak():
    # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz x 2 flop per FMA (no packed fp32)
    assert abs(bench.PEAK_VALU_TFLOPS - 78.6432) < 1e-9


def test_traffic_profile_belongs_to_the_sources():
    rec = json.load(open(os.path.join(ROOT, bench.TRAFFIC_FILE)))
    value, src = bench.search_traffic(512)
    assert value is not None, src   # a stale profile means the counters must be taken again
    assert value == rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    assert rec["source_files"] == bench.SEARCH_SOURCES
    assert bench.search_traffic(256)[0] is None

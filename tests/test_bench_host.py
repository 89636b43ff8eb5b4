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
    # MI355X's published fp32 vector peak: 256 CUs x 4 SIMDs x 2.4 GHz x 64 flop per clock
    assert abs(bench.PEAK_VALU_TFLOPS - 157.2864) < 1e-9


def test_traffic_is_reported_only_for_the_profiled_sources(tmp_path):
    # bench.py reports the committed HBM-traffic profile only while the search
    # kernel's sources hash to what the profile recorded, and null otherwise
    rec = json.load(open(os.path.join(ROOT, bench.TRAFFIC_FILE)))
    assert rec["source_files"] == bench.SEARCH_SOURCES
    fresh = dict(rec, source_sha256=bench.sources_sha256(bench.SEARCH_SOURCES))
    p = tmp_path / "fresh.json"
    p.write_text(json.dumps(fresh))
    value, _ = bench.search_traffic(512, str(p))
    assert value == rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    assert bench.search_traffic(256, str(p))[0] is None
    stale = dict(rec, source_sha256="0" * 64)
    p.write_text(json.dumps(stale))
    value, why = bench.search_traffic(512, str(p))
    assert value is None and "changed" in why


def test_rzf_powers_match_the_oracle():
    """The l = 0 reference of the RZF-gain report: ||W s_pi||^2 from the packed
    W and the level order equals the oracle's dense computation."""
    torch = pytest.importorskip("torch")
    import collections

    import numpy as np

    import vpgen
    from oracle import vp_oracle as O
    wl = vpgen.make("t", 6, 8, 3, 5, 64, 0.1, 16, seed=9)
    Ws, perms = [], []
    want = []
    for sc in range(wl.n_sc):
        p = O.preprocess(wl.H[sc], wl.alpha)
        W = np.asarray(p.W)
        Ws.append(np.concatenate([W[j:, j] for j in range(wl.N)]))   # packed lower, column-major
        perms.append(np.asarray(p.perm))
        for j in range(wl.n_sym):
            v = sc * wl.n_sym + j
            want.append(np.linalg.norm(W @ wl.s[np.asarray(p.perm), v]) ** 2)
    Prep = collections.namedtuple("Prep", "W perm")
    prep = Prep(torch.from_numpy(np.array(Ws)), torch.from_numpy(np.array(perms).astype(np.uint8)))
    got = bench.rzf_powers(prep, torch.from_numpy(wl.s), wl.n_sym).numpy()
    np.testing.assert_allclose(got, np.array(want), rtol=1e-12)


def test_counters_are_reported_only_for_the_profiled_sources(tmp_path):
    # the clock / VALU-issue record is reported while the search sources hash
    # to the recorded value, and not at all for a stale hash or an old format
    rec = json.load(open(os.path.join(ROOT, bench.COUNTERS_FILE)))
    assert rec["source_files"] == bench.SEARCH_SOURCES
    fresh = dict(rec, source_sha256=bench.sources_sha256(bench.SEARCH_SOURCES))
    p = tmp_path / "fresh.json"
    p.write_text(json.dumps(fresh))
    got = bench.search_counters(512, str(p))
    assert got["simd_clocks_per_valu_instr"] == rec["simd_clocks_per_valu_instr"]
    assert got["issue_vs_fma_stream"] == rec["issue_vs_fma_stream"]
    assert bench.search_counters(256, str(p)) == {}
    p.write_text(json.dumps(dict(rec, source_sha256="0" * 64)))
    assert bench.search_counters(512, str(p)) == {}
    old = {k: v for k, v in fresh.items() if k != "simd_clocks_per_valu_instr"}
    p.write_text(json.dumps(old))
    assert bench.search_counters(512, str(p)) == {}


def test_clocks_per_valu_instruction(tmp_path):
    # pmcsum: shader clock = GRBM_GUI_ACTIVE / 8 XCDs over the dispatch time,
    # SIMD clocks per VALU instruction = 1024 SIMDs x those clocks / SQ_INSTS_VALU,
    # both averaged over the kernel's dispatches (counters summed per dispatch)
    import sqlite3

    from paper_2602_12098_amd import pmcsum
    db = tmp_path / "run_results.db"
    con = sqlite3.connect(db)
    con.execute("create table counters_collection (kernel_name text, dispatch_id int, counter_name text, "
                "value real, duration real)")
    rows = []
    for did, (cycles, valu) in enumerate([(2.0e6, 5.12e8), (2.4e6, 6.144e8)]):
        dur_ns = 1.0e6   # 1 ms
        for xcd in range(8):   # GRBM_GUI_ACTIVE is read per XCD and summed
            rows.append(("k_x<16>", did, "GRBM_GUI_ACTIVE", cycles, dur_ns))
        rows.append(("k_x<16>", did, "SQ_INSTS_VALU", valu, dur_ns))
        rows.append(("k_other", did, "SQ_INSTS_VALU", 1.0, dur_ns))
    con.executemany("insert into counters_collection values (?, ?, ?, ?, ?)", rows)
    con.commit()
    con.close()
    ghz, cpi, valu, n, dur = pmcsum.clocks_per_valu(str(db), r"k_x")
    assert n == 2 and abs(dur - 1e-3) < 1e-15
    assert abs(ghz - 2.2) < 1e-12                       # mean cycles 2.2e6 over 1 ms
    assert abs(valu - 5.632e8) < 1e-3
    assert abs(cpi - 1024 * 2.2e6 / 5.632e8) < 1e-12    # = 4.0


def test_fma_stream_reference_builds(tmp_path):
    # the issue-rate reference of the VALU counters compiles for gfx950 (hipcc
    # cross-compiles without a GPU) and its loop is plain v_fmac_f32, no packed FP32
    import shutil
    import subprocess

    if shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("no hipcc")
    from paper_2602_12098_amd import valuref
    exe = valuref.build(str(tmp_path))
    assert os.path.exists(exe)
    asm = tmp_path / "fma_stream.s"
    subprocess.run(["hipcc", "-O3", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", "--offload-device-only", "-S", "-o", str(asm),
                    str(tmp_path / "fma_stream.hip")], check=True, capture_output=True)
    text = asm.read_text()
    assert text.count("v_fmac_f32") >= 24 and "v_pk_fma_f32" not in text

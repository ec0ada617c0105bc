"""Host logic of the benchmark (CPU, no GPU): the one-GPU guard, the reader of
the printed [Rational 0] table the shifted-solve leg uses, and the rule that
the recorded HBM traffic is reported only while the kernel sources it was
measured on are unchanged."""
import os
import subprocess
import sys

import numpy as np

import bench
from tests.test_oracle_rational import read_table

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_before_any_gpu_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_rational_reader_matches_the_table():
    A, nu, mu, delta = bench.read_rational()
    t = read_table()
    assert A == t["A"] and delta == t["delta"]
    assert np.array_equal(nu, t["nu"]) and np.array_equal(mu, t["mu"]) and len(nu) == 10


def test_recorded_traffic_follows_the_source_hash(monkeypatch, tmp_path):
    rec = None
    for line in open(os.path.join(ROOT, "profiles", "dhat_schur_c1.md")):
        if line.startswith("traffic-record:"):
            rec = dict(item.split("=", 1) for item in line.split()[1:])
    assert rec is not None and rec["kernel"] == "dhat_f64"
    assert bench.recorded_traffic("dhat_f64") == int(rec["bytes_per_launch"])
    assert bench.recorded_traffic("no_such_kernel") is None
    # any change to a traffic source invalidates the record
    changed = tmp_path / "dirac.hip"
    changed.write_bytes(open(os.path.join(ROOT, bench.TRAFFIC_SOURCES[0]), "rb").read() + b"\n")
    monkeypatch.setattr(bench, "TRAFFIC_SOURCES", (str(changed),) + tuple(bench.TRAFFIC_SOURCES[1:]))
    assert bench.recorded_traffic("dhat_f64") is None


def test_solve_summary_picks_fastest_and_ratios():
    """The summary of a time-to-solution block: FP64 CG, the network leg and the
    fastest converged leg with their speed-ups; failed legs and non-leg entries
    are ignored."""
    tts = {"lattice": "some text",
           "qhat-2": {"network_training": {"pairs": 10},
                      "cg_f64": {"ms_median": 600.0, "status": 0},
                      "fgcr_f32_in_f64": {"ms_median": 150.0, "status": 0},
                      "fgcr_f32_sap_in_f64": {"ms_median": 100.0, "status": 0},
                      "fgcr_f32_nn_in_f64": {"ms_median": 240.0, "status": 0},
                      "fgcr_bf16links_in_f64": {"ms_median": 50.0, "status": 6}},
           "qhat+4": {"fgcr_f32_in_f64": {"ms_median": 150.0, "status": 0}}}
    s = bench.solve_summary(tts)
    assert list(s) == ["qhat-2"]
    row = s["qhat-2"]
    assert row["fastest"] == "fgcr_f32_sap_in_f64" and row["fastest_ms"] == 100.0
    assert row["fastest_speedup_vs_cg_f64"] == 6.0
    assert row["mixed_learned_ms"] == 240.0 and row["mixed_learned_speedup_vs_cg_f64"] == 2.5

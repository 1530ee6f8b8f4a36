"""Host-side logic of bench.py (no GPU): the one-GPU refusal, argument
checks, and the reading of the committed counter profiles into the bench
line's roofline.traffic."""
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("argv,msg", [(["--gpus", "2"], "one GPU only"),
                                      (["--precision", "fp32d", "--method", "carleman"], "sigma form only")])
def test_bench_refuses_before_touching_a_gpu(argv, msg):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert msg in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("precision,method,prefix,unit", [("fp64", "sigma", "pairs", "node"),
                                                          ("fp32", "sigma", "pairs", "node"),
                                                          ("fp32d", "sigma", "pairs", "node"),
                                                          ("fp64", "carleman", "carleman", "dir")])
def test_traffic_is_read_only_from_a_profile_of_this_source(monkeypatch, precision, method, prefix, unit):
    b = _bench()
    name = ("carleman_hs_fp64_batched_q_4096.md" if method == "carleman"
            else f"k_pairs32_zstage_traffic_{precision}.md")
    kv = dict(line.split(": ", 1) for line in open(os.path.join(ROOT, "profiles", name)).read().splitlines()
              if ": " in line)
    per = float(kv[f"{prefix}_fetch_bytes_per_cell_{unit}"]) + float(kv[f"{prefix}_write_bytes_per_cell_{unit}"])
    assert per > 0
    # a profile taken on other sources gives no traffic
    monkeypatch.setattr(b, "q_source_sha256", lambda: "0" * 64)
    assert b.traffic_per_launch(precision, 1000, 10, method) is None
    # on the source it names, bytes per unit x units / launches
    monkeypatch.setattr(b, "q_source_sha256", lambda: kv["source_sha256"].strip())
    assert b.traffic_per_launch(precision, 1000, 10, method) == pytest.approx(per * 100)
    assert b.traffic_per_launch(precision, 1000, 0, method) is None


def test_source_hash_covers_the_collision_sources():
    b = _bench()
    assert b.Q_SOURCES[0] == "bz_q.hip"
    for name in b.Q_SOURCES:
        assert os.path.exists(os.path.join(ROOT, "paper_2409_01910_amd", "csrc", name))
    assert len(b.q_source_sha256()) == 64

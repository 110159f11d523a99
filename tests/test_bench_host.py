"""Host-side logic of bench.py (no GPU): the measured-traffic field is taken
from the committed counter summary only while every source file it was
measured with is unchanged, the multi-GPU request is refused, and the
launch-fill and fast-transform-floor records follow their definitions."""
import hashlib
import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def write_summary(path, digests, value=1.5e8, mode="fp16_scaled"):
    lines = ["# test summary", "traffic_bytes_per_launch dct %.6e" % value]
    lines += ["source_sha256 %s %s" % (f, d) for f, d in digests.items()]
    lines.append("dct_mode %s" % mode)
    path.write_text("\n".join(lines) + "\n")


def current_digests(bench, cls):
    out = {}
    for f in bench.CLASS_SOURCE[cls]:
        p = os.path.join(ROOT, "paper_2203_13675_amd", "csrc", f)
        out[f] = hashlib.sha256(open(p, "rb").read()).hexdigest()
    return out


def test_traffic_used_only_while_sources_match(tmp_path, monkeypatch):
    bench = load_bench()
    summary = tmp_path / "traffic.txt"
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(summary))
    dig = current_digests(bench, "dct")
    write_summary(summary, dig)
    assert bench.measured_traffic("dct", "fp16_scaled", 256) == pytest.approx(1.5e8)
    # another workload, another DCT mode, an unknown class: no figure
    assert bench.measured_traffic("dct", "fp16_scaled", 32) is None
    assert bench.measured_traffic("dct", "split_bf16", 256) is None
    assert bench.measured_traffic("finish", "fp16_scaled", 256) is None
    # any one source digest stale (the kernel file or a header it includes): no figure
    for f in dig:
        stale = dict(dig)
        stale[f] = "0" * 64
        write_summary(summary, stale)
        assert bench.measured_traffic("dct", "fp16_scaled", 256) is None, f
    # a digest missing from the summary: no figure
    partial = dict(dig)
    partial.pop(next(iter(partial)))
    write_summary(summary, partial)
    assert bench.measured_traffic("dct", "fp16_scaled", 256) is None


def test_committed_summary_names_every_source():
    bench = load_bench()
    text = open(bench.TRAFFIC_PROFILE).read()
    for cls in ("dct", "spmv", "update"):
        for f in bench.CLASS_SOURCE[cls]:
            assert "source_sha256 %s " % f in text, f


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_iteration_record():
    bench = load_bench()
    # maps of 100 and 200 px, 5 and 10 iterations, 12 SpMV launches
    rec = bench.iteration_record([(10, 10), (10, 20)], [5, 10], 12)
    work, total = 100 * 5 + 200 * 10, 300
    assert rec["launch_fill"] == pytest.approx(work / (12 * total))
    assert rec["launch_fill_bound"] == pytest.approx(work / (10 * total))
    assert rec["per_map"]["max"] == 10 and rec["per_map"]["min"] == 5
    # no schedule issues fewer launches than the slowest map's iterations, so
    # a measured fill never exceeds the bound; equal maps fill every launch
    assert rec["launch_fill"] <= rec["launch_fill_bound"]
    assert bench.iteration_record([(8, 8), (4, 16)], [7, 7], 7)["launch_fill"] == pytest.approx(1.0)
    assert bench.iteration_record([(8, 8)], [3], 0)["launch_fill"] is None


def test_dct_floor_record():
    bench = load_bench()
    # 24 GB of four-stage traffic is 8 GB at the fast-transform floor: 1 ms at 8 TB/s
    rec = bench.dct_floor_record(24e9, 100.0)
    assert rec["floor_ms_per_step"] == pytest.approx(1.0)
    assert rec["frac"] == pytest.approx(0.01)


def test_small_fp64_case_parses(monkeypatch):
    bench = load_bench()
    monkeypatch.setattr(sys, "argv", ["bench.py", "--workload", "peaks64", "--precision", "fp64"])
    a = bench.parse()
    assert (a.workload, a.precision, a.gpus) == ("peaks64", "fp64", 1)
    monkeypatch.setattr(sys, "argv", ["bench.py"])
    a = bench.parse()
    assert (a.workload, a.precision) == ("batch256", "mixed")

"""Host logic of bench.py (no GPU): the sort period, the refusal of more
than one GPU, and the traffic figure read from the committed counter
summary only while the push sources match it."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_sort_period_is_the_largest_divisor_not_above_the_cap():
    b = _bench()
    assert b.sort_period(64, 16) == 16
    assert b.sort_period(20, 16) == 10
    assert b.sort_period(7, 32) == 7
    assert b.sort_period(13, 4) == 1
    for steps in range(1, 80):
        p = b.sort_period(steps, 16)
        assert steps % p == 0 and p <= 16
        assert all(steps % q for q in range(p + 1, min(16, steps) + 1))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_is_reported_only_for_the_sources_it_was_taken_on(tmp_path, monkeypatch):
    b = _bench()
    src = b.TRAFFIC_FILE.format(workload="c5", precision="fp64")
    text = open(src).read()
    recorded = [l.split(":", 1)[1].strip() for l in text.splitlines()
                if l.startswith("source_hash:")][0]
    got = b.committed_traffic("c5", "fp64")
    if recorded == b.push_source_hash():
        assert got is not None and got > 10.7e9  # at least the algorithmic bytes
    else:
        assert got is None  # counters of other sources: not reported
    # the same summary with another source hash is not used
    text = text.replace(f"source_hash: {recorded}", "source_hash: 0")
    fake = tmp_path / "push_deposit_c5_fp64_traffic.txt"
    fake.write_text(text)
    monkeypatch.setattr(b, "TRAFFIC_FILE", str(tmp_path / "push_deposit_{workload}_{precision}_traffic.txt"))
    assert b.committed_traffic("c5", "fp64") is None

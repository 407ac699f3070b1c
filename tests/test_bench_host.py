"""Host logic of bench.py (CPU): the counter-measured traffic is reported
only for the kernel source it was measured on, the source digest ignores
comments, and a run on more than one GPU is refused."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_strip_comments_keeps_code_only():
    src = "int a; // one\n/* two\n   lines */ int b;\n\n   \nint c;  \n"
    assert bench.strip_comments(src) == "int a;\n int b;\nint c;"
    assert bench.strip_comments("x = 1; /* a */ y = 2;") == "x = 1;  y = 2;"


def test_traffic_follows_the_recorded_source(monkeypatch):
    key = ("a workload", "k_cg_iter_iso<512>")
    digest = bench.kernel_source_digest("k_cg_iter_iso<512>")
    rec = {"fetch_kib": 100.0, "write_kib": 50.0, "src": digest}
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, key, rec)
    want = int(1024 * (100.0 * bench.COUNTER_SCALE["FETCH_SIZE"] + 50.0 * bench.COUNTER_SCALE["WRITE_SIZE"]))
    assert bench.measured_traffic(*key) == want
    # another source (a changed kernel): no figure
    monkeypatch.setitem(bench.MEASURED_TRAFFIC, key, dict(rec, src="0" * 16))
    assert bench.measured_traffic(*key) is None
    # no record: no figure
    assert bench.measured_traffic("no such workload", "k_cg_iter_iso<512>") is None


def test_digest_ignores_comments_but_not_code(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2504_18526_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "k.hip").write_text("int f() { return 1; }  // a\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setitem(bench.TRAFFIC_SOURCES, "k_test", ["k.hip"])
    d0 = bench.kernel_source_digest("k_test<1>")
    (csrc / "k.hip").write_text("/* reworded */\nint f() { return 1; }  // b\n")
    assert bench.kernel_source_digest("k_test<1>") == d0
    (csrc / "k.hip").write_text("int f() { return 2; }\n")
    assert bench.kernel_source_digest("k_test<1>") != d0


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stdout

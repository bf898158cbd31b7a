"""Host-side logic of bench.py (no GPU): the kernel-source hash that gates the
committed counter summaries, the provenance record of a summary, the bytes
formula of the product, and the single-GPU guard."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_source_hash_ignores_comments_and_blank_space(tmp_path, monkeypatch):
    src = tmp_path / "paper_1211_1581_amd" / "csrc"
    src.mkdir(parents=True)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    f = src / "a.hip"
    f.write_text("int f(int x) {\n  return x + 1;  // one\n}\n")
    h1 = bench.kernel_source_hash(("a.hip",))
    f.write_text("int f(int x)\n{\n\n  return x + 1;  /* another\n comment */\n}\n")
    assert bench.kernel_source_hash(("a.hip",)) == h1
    f.write_text("int f(int x) { return x + 2; }\n")
    assert bench.kernel_source_hash(("a.hip",)) != h1
    assert len(h1) == 16


def test_traffic_record_applies_only_on_matching_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    src = tmp_path / "paper_1211_1581_amd" / "csrc"
    src.mkdir(parents=True)
    for name in bench.SPMV_SOURCES:
        (src / name).write_text(f"// {name}\nint {name.replace('.', '_')};\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    cur = bench.kernel_source_hash(bench.SPMV_SOURCES)
    rec = {"source_hash": cur, "bytes_per_launch": 123, "ratio_to_algorithmic": 1.01}
    (prof / "traffic_k_x_w.txt").write_text(json.dumps(rec))
    r = bench.traffic_record("k_x", "w", bench.SPMV_SOURCES)
    assert r["file"] == os.path.join("profiles", "traffic_k_x_w.txt")
    assert r["bytes_per_launch"] == 123 and bench.measured_traffic("k_x", "w", bench.SPMV_SOURCES) == 123
    rec["source_hash"] = "0000000000000000"
    (prof / "traffic_k_x_w.txt").write_text(json.dumps(rec))
    r = bench.traffic_record("k_x", "w", bench.SPMV_SOURCES)
    assert r["bytes_per_launch"] is None and r["bytes_per_launch_then"] == 123
    assert r["taken_on_hash"] == "0000000000000000" and r["current_hash"] == cur
    assert bench.traffic_record("k_y", "w", bench.SPMV_SOURCES)["file"] is None


def test_committed_traffic_summaries_name_their_hash():
    for name in os.listdir(os.path.join(ROOT, "profiles")):
        if name.startswith("traffic_"):
            d = json.load(open(os.path.join(ROOT, "profiles", name)))
            assert len(d["source_hash"]) == 16 and d["bytes_per_launch"] > 0
            assert d["commands"] and all("rocprofv3" in c for c in d["commands"])


def test_spmv_bytes_formula():
    # values and columns per entry, row pointers, x read once, y written once
    n, nnz = 1000, 7000
    assert bench.spmv_bytes(n, nnz) == nnz * 12 + 4 * (n + 1) + 8 * n + 8 * n
    assert bench.spmv_bytes(n, nnz, sv=4, sx=4) == nnz * 8 + 4 * (n + 1) + 4 * n + 4 * n


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr

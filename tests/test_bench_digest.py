"""The code digest that keys the committed traffic counters to the kernels'
code: comment or whitespace edits keep it, code edits change it."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_code_digest_ignores_comments_only(tmp_path):
    b = _bench()
    (tmp_path / "a.hip").write_text("int f(int x) {\n    return x + 1;  // add one\n}\n/* block\n comment */\n")
    d0 = b.code_digest(str(tmp_path), ["a.hip"])
    (tmp_path / "a.hip").write_text("// header\nint f(int x) {\n  return x + 1;   // plus one\n}\n")
    assert b.code_digest(str(tmp_path), ["a.hip"]) == d0
    (tmp_path / "a.hip").write_text("int f(int x) {\n    return x + 2;\n}\n")
    assert b.code_digest(str(tmp_path), ["a.hip"]) != d0



def test_table_key():
    b = _bench()
    assert b.table_key([24, 24, 24], [0, 0, 0]) == "24,24,24/0,0,0"
    assert b.table_key((52, 8, 16), (3, 0, 12)) == "52,8,16/3,0,12"


def _record(tmp_path, code="int f() { return 1; }\n", n=2048):
    (tmp_path / "k.hip").write_text(code)
    b = _bench()
    rec = {"fused": {"sources": ["k.hip"], "n": n, "code_sha256": b.code_digest(str(tmp_path), ["k.hip"]),
                     "bytes_per_launch_by_table": {"24,24,24/0,0,0": 402597622}}}
    import json
    os.makedirs(tmp_path / "profiles", exist_ok=True)
    (tmp_path / "profiles" / "fused_and_split_vortex2048_traffic.json").write_text(json.dumps(rec))
    # a copy of bench.py beside the record, so that it reads this record
    (tmp_path / "bench.py").write_text(open(os.path.join(ROOT, "bench.py")).read())
    spec = importlib.util.spec_from_file_location("bench_copy", str(tmp_path / "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_counted_traffic_keys(tmp_path):
    b = _record(tmp_path)
    assert b.counted_traffic("fused", "24,24,24/0,0,0", 2048) == 402597622
    assert b.counted_traffic("fused", "24,24,24/1,0,0", 2048) is None   # another table
    assert b.counted_traffic("fused", "24,24,24/0,0,0", 1024) is None   # another grid
    assert b.counted_traffic("fused3d", "24,24,24/0,0,0", 2048) is None  # no such record
    (tmp_path / "k.hip").write_text("// a comment\nint f() {   return 1; }\n")
    assert b.counted_traffic("fused", "24,24,24/0,0,0", 2048) == 402597622  # comments only
    (tmp_path / "k.hip").write_text("int f() { return 2; }\n")
    assert b.counted_traffic("fused", "24,24,24/0,0,0", 2048) is None   # the code changed


def test_committed_traffic_record_matches_the_code():
    # the committed counters belong to the kernels as they are now
    b = _bench()
    assert b.counted_traffic("fused", "24,24,24/0,0,0", 2048) is not None
    assert b.counted_traffic("fused3d", "52,52,52/0,0,0", 256) is not None
    assert b.counted_traffic("split", "residual", 2048) is not None


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""

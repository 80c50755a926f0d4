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


"""CPU checks of bench.py's bookkeeping: the committed rocprofv3 summary belongs to the current
device code (so `roofline.traffic` and the executed flops behind `roofline.achieved` are reported),
and the code hash ignores comments only."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_committed_profile_matches_the_device_code():
    b = _bench()
    rec = b.profile_record(b.PROFILE_VJP)
    assert rec, "device code changed since profiles/ was recorded: profile again"
    assert 1e6 < rec["traffic"] < 1e9
    assert 1e8 < rec["executed_flops"] < 1e11


def test_code_hash_ignores_comments_and_blank_lines_only():
    b = _bench()
    src = "int a = 1;  // one\n\n/* block\n comment */int b = 2;\n"
    assert b.code_only(src) == "int a = 1;\nint b = 2;"
    assert b.code_only(src) != b.code_only(src.replace("2", "3"))

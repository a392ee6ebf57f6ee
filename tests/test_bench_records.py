"""bench.py's traffic records: a record's counters are reported only while
the kernel sources hash to the values they were taken with and the run used
one of the record's configurations; comments and whitespace do not change
the hash (host only, no GPU)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _record(tmp_path, text):
    src = tmp_path / "k.hip"
    src.write_text(text)
    rel = os.path.relpath(src, bench.ROOT)
    return rel, bench.code_hash(str(src))


def test_hash_ignores_comments_and_whitespace(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    a.write_text("int f(int x) { return x + 1; }  // one\n")
    b.write_text("/* two */\nint f(int x)\n{\n  return x + 1;\n}\n")
    assert bench.code_hash(str(a)) == bench.code_hash(str(b))
    b.write_text("int f(int x) { return x + 2; }\n")
    assert bench.code_hash(str(a)) != bench.code_hash(str(b))


def test_records_match_by_configuration_and_code(tmp_path):
    rel, h = _record(tmp_path, "kernel body\n")
    t = {"sources_sha256": {rel: h},
         "records": [{"cfg": {"a": 1}, "fetch_kib": 10.0, "write_kib": 5.0},
                     {"cfg": {"a": 2}, "fetch_kib": 20.0, "write_kib": 7.0}],
         "fetch_scale": 2.0, "write_scale": 1.0}
    assert bench.measured_traffic_bytes(t, "cfg", {"a": 1}) == (10.0 * 2 + 5.0) * 1024
    assert bench.measured_traffic_bytes(t, "cfg", {"a": 2}) == (20.0 * 2 + 7.0) * 1024
    assert bench.measured_traffic_bytes(t, "cfg", {"a": 3}) is None
    (tmp_path / "k.hip").write_text("kernel body changed\n")
    assert bench.measured_traffic_bytes(t, "cfg", {"a": 1}) is None


def test_single_record_form(tmp_path):
    rel, h = _record(tmp_path, "x\n")
    t = {"sources_sha256": {rel: h}, "config": {"b": 4}, "fetch_kib": 1.0, "write_kib": 1.0,
         "fetch_scale": 2.0, "write_scale": 1.0}
    assert bench.measured_traffic_bytes(t, "config", {"b": 4}) == 3.0 * 1024
    assert bench.measured_traffic_bytes(t, "config", {"b": 5}) is None

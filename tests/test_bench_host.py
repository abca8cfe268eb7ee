"""Host logic of bench.py (CPU only): the key under which the committed counter summary is used."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_strip_comments_keeps_code_and_literals():
    src = ('int a = 1;   // note\n'
           '/* block\n   comment */ const char *s = "x // y /* z */";\n'
           "\n"
           "char q = '\"'; char r = '\\''; // after\n"
           'int b = "\\"//"[0];\n')
    assert bench.strip_comments(src) == (
        'int a = 1;\n'
        '  const char *s = "x // y /* z */";\n'
        "char q = '\"'; char r = '\\'';\n"
        'int b = "\\"//"[0];')


def test_comment_edits_keep_the_key_and_code_edits_change_it():
    code = "__global__ void k(int *p) {\n  p[0] = 1;  // one\n}\n"
    reworded = ("// header\n/* two\n   lines */\n__global__ void k(int *p) {\n"
                "  p[0] = 1;  // the value one,\n  // reworded\n\n}\n")
    changed = "__global__ void k(int *p) {\n  p[0] = 2;  // one\n}\n"
    assert bench.strip_comments(code) == bench.strip_comments(reworded)
    assert bench.strip_comments(code) != bench.strip_comments(changed)


def test_traffic_is_null_for_another_source_hash_or_index(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(
        '{"source_hash": "0000000000000000", "isa_sample": 1, "kernels": {"smem": {"hbm_bytes_per_launch": 5.0}}}')
    monkeypatch.setattr(bench, "ROOT", tmp_path)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "1111111111111111")
    assert bench.traffic_from_profile("smem", 1.0, 1) is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0000000000000000")
    assert bench.traffic_from_profile("smem", 1.0, 1) == 5.0
    # counters taken with another inverse-SA step describe another index
    assert bench.traffic_from_profile("smem", 1.0, 4) is None


def test_transaction_rates_follow_the_summary_and_the_run(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(
        '{"source_hash": "0000000000000000", "isa_sample": 1, "kernels": {'
        '"smem": {"hbm_bytes_per_launch": 5.0, "l2": {"hit_rate_by_round": [0.1, 0.2], '
        '"hbm_read_requests_by_round": [3000, 1000]}}, '
        '"locate": {"hbm_bytes_per_launch": 7.0, "l2": {"hit_rate": 0.3, "hbm_read_requests_per_launch": 500}}}}')
    monkeypatch.setattr(bench, "ROOT", tmp_path)
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0000000000000000")
    s, lo = bench.profile_entry("smem", 1), bench.profile_entry("locate", 1)
    t = bench.transactions(s, lo, 2.0, 1.0, 1e6)   # 4000 requests in 2 ms, 500 in 1 ms, probe 1e6 / s
    assert t["smem"]["hbm_read_requests_per_step"] == 4000
    assert t["smem"]["requests_per_s"] == 2_000_000 and t["smem"]["frac_of_probe"] == 2.0
    assert t["locate"]["requests_per_s"] == 500_000 and t["locate"]["frac_of_probe"] == 0.5
    assert t["smem"]["l2_hit_rate_by_round"] == [0.1, 0.2] and t["locate"]["l2_hit_rate"] == 0.3
    # no summary for these sources, or one without the L2 figures: nothing is reported
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "1111111111111111")
    assert bench.profile_entry("smem", 1) is None
    assert bench.transactions(None, lo, 2.0, 1.0, 1e6) is None
    assert bench.transactions({"hbm_bytes_per_launch": 5.0}, lo, 2.0, 1.0, 1e6) is None

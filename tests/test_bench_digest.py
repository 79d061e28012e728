"""The source digest that ties the committed rocprofv3 summaries to the
kernel sources: it follows the code and ignores the comments."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_strip_comments_keeps_code_and_literals():
    src = ('int a = 1; // note\n'
           'const char* u = "http://x/*y*/"; /* block\n comment */ char c = \'/\';\n'
           'double d = 2.0 / 3.0;\n')
    out = bench.strip_comments(src)
    assert "note" not in out and "block" not in out and "comment" not in out
    assert '"http://x/*y*/"' in out and "'/'" in out and "2.0 / 3.0" in out
    assert out.count("\n") == src.count("\n") - 1      # the block comment's newline goes


def test_digest_ignores_comments_but_not_code(tmp_path, monkeypatch):
    files = ("paper_2509_12381_amd/csrc/ai.hip", "paper_2509_12381_amd/csrc/schedule.hip",
             "paper_2509_12381_amd/csrc/schedule.h", "include/ai.h")
    for f in files:
        dst = tmp_path / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        dst.write_text(open(os.path.join(bench.ROOT, f), encoding="utf-8").read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.source_digest()
    hip = tmp_path / files[0]
    text = hip.read_text()
    hip.write_text(text + "\n// a new remark\n/* and another */\n")
    assert bench.source_digest() == base
    hip.write_text(text.replace("constexpr int WAVE = 64;", "constexpr int WAVE = 32;", 1))
    assert bench.source_digest() != base

"""The guard of the committed HBM-traffic record (bench.kernel_source_hash):
it follows the code of the pass sources, not their comments or layout."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402


def test_code_only_drops_comments_and_layout():
    src = 'int a = 1; // note\n/* block\n comment */ int  b =\n 2;\nconst char *s = "// kept";\n'
    assert bench._code_only(src) == 'int a = 1; int b = 2; const char *s = "// kept";'
    assert bench._code_only("x /* a */ y") == bench._code_only("x /* b, longer */ y")


def test_code_change_changes_the_hash(tmp_path, monkeypatch):
    src = tmp_path / "k.hpp"
    src.write_text("constexpr int k = 4;  // four\n")
    monkeypatch.setattr(bench, "HERE", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["k.hpp"])
    h0 = bench.kernel_source_hash()
    src.write_text("constexpr int k = 4;\n// a comment added\n")
    assert bench.kernel_source_hash() == h0
    src.write_text("constexpr int k = 5;  // four\n")
    assert bench.kernel_source_hash() != h0

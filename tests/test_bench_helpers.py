"""Host helpers of bench.py: the code hash that keeps a counter summary
valid across comment edits but not across code edits."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_text_drops_comments_only():
    a = 'int x = 1; // one\n/* block\n comment */ const char *s = "// not a comment";\n'
    b = 'int  x = 1;\n   const char *s = "// not a comment"; // other words\n'
    c = 'int x = 2; const char *s = "// not a comment";'
    assert bench.code_text(a) == bench.code_text(b)
    assert bench.code_text(a) != bench.code_text(c)
    assert "// not a comment" in bench.code_text(a)
    assert bench.code_text("char q = '\\''; // x") == "char q = '\\'';"


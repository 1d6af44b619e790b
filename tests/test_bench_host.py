"""Host-side helpers of bench.py: the code digest that ties stored HBM byte
counters to the kernel code they were taken on."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_tokens_drop_comments_and_layout():
    a = "int a = 1; // one\n/* two\n lines */\tint  b;\n"
    b = "int a = 1;\nint b;"
    assert bench.code_tokens(a) == bench.code_tokens(b) == "int a = 1; int b;"


def test_code_tokens_keep_literals():
    src = 'const char* s = "x // y /* z */"; char c = \'"\'; // tail'
    assert bench.code_tokens(src) == \
        'const char* s = "x // y /* z */"; char c = \'"\';'


def test_code_tokens_see_code_changes():
    assert bench.code_tokens("x = a + b;") != bench.code_tokens("x = a - b;")


def test_measured_traffic_is_bytes_or_none():
    v = bench.measured_traffic("dna-1k")
    assert v is None or (isinstance(v, int) and v > 0)
    assert bench.measured_traffic("no-such-workload") is None

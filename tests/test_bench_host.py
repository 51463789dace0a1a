"""Host logic of bench.py (no GPU): the source digest that ties a byte-counter summary under
profiles/ to the kernel sources it was measured on, and the traffic lookup that uses it."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_code_text_ignores_comments_and_layout(bench):
    a = "int x = 1;  // one\n/* block\n comment */ float y = x * 2.0f;\n"
    b = "int x = 1;\nfloat y = x * 2.0f;  // a different comment\n"
    assert bench._code_text(a) == bench._code_text(b) == "int x = 1; float y = x * 2.0f;"


def test_code_text_sees_code_changes(bench):
    a = "int x = 1; float y = x * 2.0f;"
    for b in ("int x = 2; float y = x * 2.0f;", "int x = 1; float y = x * 2.0f; y += 1;",
              "int x = 1; double y = x * 2.0f;"):
        assert bench._code_text(a) != bench._code_text(b)


def test_traffic_summaries_parse(bench):
    # each summary names its kernels, byte counts and the digest of the sources it was taken on;
    # while the sources still match, the lookup returns the recorded bytes, else None
    for wl, precisions in (("blobs128", (0, 1)), ("blobs256", (1,))):
        for prec in precisions:
            t = bench.measured_traffic(wl, prec)
            assert t is None or t > bench.stage_bytes(
                {"blobs128": 128, "blobs256": 256}[wl],
                {"blobs128": 1 << 23, "blobs256": 1 << 25}[wl],
                4 if prec == 1 else 8)["particles"] * 0.5
    assert bench.measured_traffic("no_such_workload", 1) is None

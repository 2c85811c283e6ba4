"""Host logic of bench.py: the code hash that keys the committed counter
summaries to the kernel sources, and the reading of those summaries."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _write(tmp_path, name, text):
    p = tmp_path / name
    p.write_text(text)
    return str(p)


def test_code_hash_ignores_comments_and_blank_lines(tmp_path):
    a = _write(tmp_path, "a.hip", "int f(int x) {\n  return x + 1;\n}\n")
    b = _write(tmp_path, "b.hip", "// f adds one\nint f(int x) {  /* the\n  argument */\n\n"
                                  "  return x + 1;  // plus one\n}\n")
    c = _write(tmp_path, "c.hip", "int f(int x) {\n  return x + 2;\n}\n")
    assert bench.code_hash([a]) == bench.code_hash([b])
    assert bench.code_hash([a]) != bench.code_hash([c])


def test_measured_bytes_follows_the_code(tmp_path):
    src = _write(tmp_path, "k.hip", "__global__ void k() {}\n")
    prof = _write(tmp_path, "p.md", "# summary\n\nleg-source-sha256: %s\nleg-bytes-measured: 1234\n"
                  % bench.code_hash([src]))
    assert bench.measured_bytes(prof, "leg", [src]) == 1234
    assert bench.measured_bytes(prof, "other", [src]) is None
    _write(tmp_path, "k.hip", "// a comment only\n__global__ void k() {}\n")
    assert bench.measured_bytes(prof, "leg", [src]) == 1234
    _write(tmp_path, "k.hip", "__global__ void k() { int x = 0; }\n")
    assert bench.measured_bytes(prof, "leg", [src]) is None


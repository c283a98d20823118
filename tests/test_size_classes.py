"""Size classes of the library's device block cache (`size_class` in
csrc/alloc.hip), compiled for the host with g++ from the library source:
every class holds the request, is at most 25% larger than it (requests above
256 bytes), has the form m * 2^e with m in 4..7, and grows with the request,
so a buffer that grows by the DBuf headroom lands in a class of its own."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1904_08553_amd", "csrc", "alloc.hip")

HARNESS = r"""
#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <random>
%s
static bool form_ok(size_t c) {
  if (c == 256) return true;
  int e = 0;
  while ((c >> e) >= 8) ++e;
  const size_t m = c >> e;
  return (m << e) == c && m >= 4 && m <= 7;
}
int main() {
  std::mt19937_64 rng(5);
  long bad = 0;
  size_t prev = 0;
  for (size_t b = 1; b <= (size_t(1) << 20); ++b) {  // every size up to 1 MiB
    const size_t c = size_class(b);
    if (c < b || !form_ok(c) || c < prev || (b > 256 && 4 * c > 5 * b)) ++bad;
    prev = c;
  }
  for (int i = 0; i < 200000; ++i) {  // random sizes up to 256 GiB
    const size_t b = 1 + size_t(rng() %% (size_t(1) << 38));
    const size_t c = size_class(b);
    if (c < b || !form_ok(c) || (b > 256 && 4 * c > 5 * b)) ++bad;
  }
  printf("bad %%ld\n", bad);
  return bad != 0;
}
"""


def _function_source():
    text = open(SRC).read()
    m = re.search(r"size_t size_class\(size_t bytes\) \{.*?\n\}\n", text, re.S)
    assert m, "size_class not found in alloc.hip"
    return m.group(0)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_size_classes(tmp_path):
    src = tmp_path / "size_class.cpp"
    exe = tmp_path / "size_class"
    src.write_text(HARNESS % _function_source())
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", str(exe), str(src)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "bad 0" in r.stdout

"""The row search of the graph kernels (`find_in_row` in csrc/graph.hip: the
first position in [b, e) whose neighbour id is at least c, by bisection)
compiled for the host with g++ from the kernel source itself, against
std::lower_bound on random sorted rows of 0 to 3,000 entries placed at an
offset, every query inside an exactly sized array under AddressSanitizer
(no probe may leave the row)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1904_08553_amd", "csrc", "graph.hip")

HARNESS = r"""
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>
struct int2 { int x, y; };
#define __device__
#define __forceinline__ inline
%s
int main() {
  std::mt19937 rng(11);
  long bad = 0, cases = 0;
  for (int it = 0; it < 40000; ++it) {
    const int d = (it %% 5 == 0) ? int(rng() %% 3000) : int(rng() %% 70);
    std::vector<int> xs;
    int v = int(rng() %% 5);
    for (int i = 0; i < d; ++i) { v += 1 + int(rng() %% 4); xs.push_back(v); }
    const int pad = int(rng() %% 5);
    std::vector<int2> adj(pad + d);
    for (int i = 0; i < d; ++i) adj[pad + i] = int2{xs[i], 1};
    for (int q = 0; q < 6; ++q) {
      const int c = int(rng() %% (v + 6)) - 1;
      const int want = pad + int(std::lower_bound(xs.begin(), xs.end(), c) - xs.begin());
      const int got = find_in_row(adj.data(), pad, pad + d, c);
      ++cases;
      if (got != want) ++bad;
    }
  }
  printf("cases %%ld bad %%ld\n", cases, bad);
  return bad != 0;
}
"""


def _function_source():
    text = open(SRC).read()
    m = re.search(r"__device__ __forceinline__ int32_t find_in_row\(.*?\n}\n", text, re.S)
    assert m, "find_in_row not found in graph.hip"
    return m.group(0)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_row_search_matches_lower_bound(tmp_path):
    src = tmp_path / "row_search.cpp"
    exe = tmp_path / "row_search"
    src.write_text(HARNESS % _function_source())
    subprocess.run(["g++", "-O1", "-std=c++17", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-o", str(exe), str(src)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "bad 0" in r.stdout

"""The Hilbert index that orders the search's 64-source tiles (csrc/batch.hpp,
hilbert3), compiled for the host with g++: on the 16^3 corner of the grid it is a
bijection onto [0, 4096) and consecutive indices are neighbouring cells (the property
that makes consecutive sources close in space). The order affects only which sources
share a wavefront, never a search's result."""
import os
import re
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
BATCH = os.path.join(os.path.dirname(HERE), "paper_2509_26193_amd", "csrc", "batch.hpp")

HARNESS = r"""
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>
%s
int main() {
  const int K = 16;
  std::vector<int> seen(K * K * K, 0);
  std::vector<int> cx(K * K * K), cy(K * K * K), cz(K * K * K);
  for (int x = 0; x < K; ++x)
    for (int y = 0; y < K; ++y)
      for (int z = 0; z < K; ++z) {
        uint64_t h = hilbert3(x, y, z);
        if (h >= (uint64_t)(K * K * K) || seen[h]++) return 1;
        cx[h] = x; cy[h] = y; cz[h] = z;
      }
  for (int h = 1; h < K * K * K; ++h)
    if (abs(cx[h] - cx[h - 1]) + abs(cy[h] - cy[h - 1]) + abs(cz[h] - cz[h - 1]) != 1) return 2;
  printf("ok\n");
  return 0;
}
"""


def test_hilbert_index_is_a_continuous_bijection(tmp_path):
    src = open(BATCH).read()
    m = re.search(r"__device__ __forceinline__ (uint64_t hilbert3\(.*?\n\})", src, re.S)
    assert m, "hilbert3 not found"
    cpp = tmp_path / "h.cpp"
    cpp.write_text(HARNESS % m.group(1))
    exe = tmp_path / "h"
    subprocess.check_call(["g++", "-O2", "-std=c++17", str(cpp), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.returncode
    assert r.stdout.strip() == "ok"

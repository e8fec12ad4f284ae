"""Where theta <= 1/2 and every position lies in the cube, the search sweep decides the
Barnes-Hut acceptance (Sec. II: a cell of edge l is accepted when l / d < theta, here
l^2 < theta^2 d^2 with l^2 = L^2 4^-dep) by comparing d2 with a precomputed bound
instead of forming theta^2 d2 (csrc/search.hpp, accept_bound and bh_accept_d). The
library's own functions, compiled for the host, must take the same decision as the
product test on every (L^2, theta, depth, d2) tried: squared distances within a few
ulps of each depth's boundary, random ones, and theta = 0 (nothing accepted)."""
import os
import re
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2509_26193_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"

HARNESS = r"""
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <random>
constexpr uint32_t kSkipBits = %(skip)s;
%(code)s
int main() {
  std::mt19937_64 g(7);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  const double thetas[] = {0.0, 1e-3, 0.1, 0.2, 0.25, 0.3, 1.0 / 3.0, 0.45, 0.5};
  long checked = 0, accepted = 0;
  for (int c = 0; c < 400; ++c) {
    // cube edges from 1e-3 to 1e6 um, some of them powers of two
    double edge = pow(10.0, -3.0 + 9.0 * u(g));
    if (c %% 7 == 0) edge = ldexp(1.0, (int)(u(g) * 40) - 10);
    const double L2 = edge * edge;
    const double theta = c < 9 ? thetas[c] : (c %% 3 == 0 ? thetas[c %% 9] : 0.5 * u(g));
    const double theta2 = theta * theta;
    const double D = accept_bound(L2, theta2);
    for (uint32_t dep = 0; dep <= 21; ++dep) {
      const uint32_t meta = dep << kSkipBits;
      const double e2 = edge2_at(L2, meta);
      const double b = edge2_at(D, meta);
      double d2s[64];
      int k = 0;
      double lo = b, hi = b;                      // the bound and its neighbours
      d2s[k++] = b;
      for (int s = 0; s < 6; ++s) {
        lo = nextafter(lo, 0.0);
        hi = nextafter(hi, DBL_MAX);
        d2s[k++] = lo;
        d2s[k++] = hi;
      }
      if (theta2 > 0.0) {                         // around e2 / theta2 as well
        double q = e2 / theta2;
        d2s[k++] = q;
        d2s[k++] = nextafter(q, 0.0);
        d2s[k++] = nextafter(q, DBL_MAX);
      }
      while (k < 64) d2s[k++] = 3.0 * L2 * u(g);  // points of the cube
      for (int j = 0; j < k; ++j) {
        const double d2 = d2s[j];
        if (!(d2 >= 0.0) || d2 > 3.2 * L2) continue;
        const bool want = e2 < theta2 * d2;       // the product test
        const bool got = bh_accept_d(D, d2, meta);
        if (want != got) {
          printf("mismatch L2=%%a theta2=%%a dep=%%u d2=%%a want=%%d\n", L2, theta2, dep, d2,
                 (int)want);
          return 1;
        }
        ++checked;
        accepted += want;
      }
    }
  }
  printf("ok %%ld %%ld\n", checked, accepted);
  return 0;
}
"""


def _function(src, name):
    m = re.search(r"(?:__host__ )?__device__ (?:__forceinline__|inline) (\w+ " + name +
                  r"\(.*?\n\})", src, re.S)
    assert m, name
    return "inline " + m.group(1)


@pytest.mark.skipif(not os.path.exists(CLANG), reason="no clang++")
def test_bound_decides_as_the_product(tmp_path):
    src = open(os.path.join(CSRC, "search.hpp")).read()
    skip = re.search(r"constexpr uint32_t kSkipBits = (\d+);",
                     open(os.path.join(CSRC, "common.hpp")).read()).group(1)
    vec = re.search(r"typedef uint32_t u32x2 [^;]*;", src).group(0)
    code = "\n".join([vec, _function(src, "edge2_at"), _function(src, "accept_bound"),
                      _function(src, "bh_accept_d")])
    cpp = tmp_path / "b.cpp"
    cpp.write_text(HARNESS % dict(skip=skip, code=code))
    exe = tmp_path / "b"
    subprocess.check_call([CLANG, "-O2", "-std=c++17", "-ffp-contract=off", str(cpp), "-o",
                           str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout
    ok, checked, accepted = r.stdout.split()
    assert ok == "ok" and int(checked) > 400_000 and 0 < int(accepted) < int(checked)

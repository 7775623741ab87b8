"""Host-side check of the library's occupied/orbit triple enumeration
(csrc/device_common.hpp), compiled for the host only: the closed-form decode
of a linear index into a sorted triple p >= q >= r must agree with plain
lexicographic enumeration, and unit_triple must reorder pair units as the
pair-unit rule states (p > q = r evaluated as (q, q, p)).  The work tables
are built on the host with these functions, and the kernels use the same
code for units and 8^3 orbit blocks."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2412_18553_amd", "csrc")

PROGRAM = r"""
#include "device_common.hpp"
#include <cstdio>
int main() {
  long n = 0, bad = 0;
  for (int bound : {1, 2, 3, 7, 24, 41, 130}) {
    int64_t u = 0;
    for (int p = 0; p < bound; ++p)
      for (int q = 0; q <= p; ++q)
        for (int r = 0; r <= q; ++r, ++u) {
          int a, b, c;
          sie::decode_sorted_triple(u, bound, a, b, c);
          ++n;
          bad += (a != p || b != q || c != r);
          int i, j, k;
          const bool one = sie::unit_triple(u, bound, true, i, j, k);
          if (p == r) bad += (one || i != p || j != p || k != p);
          else if (q == r) bad += (!one || i != q || j != q || k != p);   // p > q = r
          else if (p == q) bad += (!one || i != p || j != p || k != r);   // p = q > r
          else bad += (one || i != p || j != q || k != r);
          const bool one0 = sie::unit_triple(u, bound, false, i, j, k);
          bad += (one0 || i != p || j != q || k != r);
        }
  }
  std::printf("%ld %ld\n", n, bad);
  return bad != 0;
}
"""


def test_sorted_triple_decode_and_pair_units(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = tmp_path / "enum.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "enum"
    res = subprocess.run([hipcc, "-x", "hip", "--offload-host-only", "-O1", "-std=c++17",
                          "-I", CSRC, "-I", os.path.join(ROOT, "include"), str(src), "-o",
                          str(exe)], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    n, bad = (int(x) for x in out.stdout.split())
    assert n == 389700 and bad == 0, out.stdout

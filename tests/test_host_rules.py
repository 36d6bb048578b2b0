"""Host-side checks of the march epilogue's record rule (compiled with g++,
no GPU): the K minimum-|f| records of Sec. 3.4 / App. B.2."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1911_13225_amd", "csrc")

PROGRAM = r"""
#include <cmath>
#include <cstdio>
#include <limits>
#include "march_rules.h"
using dist::topk_rank;
int main() {
  const float inf = std::numeric_limits<float>::infinity();
  const float nan = std::numeric_limits<float>::quiet_NaN();
  const float rec[4] = {0.1f, 0.2f, 0.2f, inf};
  printf("%d %d %d %d %d %d %d %d\n",
         topk_rank(0.05f, rec, 4),   // new minimum -> 0
         topk_rank(0.2f, rec, 4),    // tie: after the earlier equal records -> 3
         topk_rank(0.3f, rec, 4),    // before the empty record -> 3
         topk_rank(nan, rec, 4),     // NaN is never recorded -> K
         topk_rank(inf, rec, 4),     // infinity likewise -> K
         topk_rank(-nan, rec, 3),    // any NaN -> K
         topk_rank(0.0f, rec, 1),    // K = 1
         topk_rank(1e30f, rec, 3));  // larger than every record -> K
  return 0;
}
"""


def test_topk_rank_rule(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    src = tmp_path / "rules.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "rules"
    subprocess.run([gxx, "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    assert [int(x) for x in out] == [0, 3, 3, 4, 4, 3, 0, 3]

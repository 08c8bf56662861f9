"""Host check of the workgroup renumbering over the XCDs (hm_internal.h xcd_order):
for every launch size it is a bijection of [0, n), and each XCD (hardware linear ids
congruent modulo 8) receives one contiguous range of logical ids in increasing order.
The header is compiled for the host with hipcc; skipped where hipcc is absent."""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = r"""
#include "hm_internal.h"
#include <cstdio>
#include <vector>
int main() {
  for (int n = 1; n <= 6000; ++n) {
    std::vector<int> seen(n, 0);
    for (int b = 0; b < n; ++b) {
      const int l = hm::xcd_order(b, n);
      if (l < 0 || l >= n || seen[l]++) { std::printf("not a bijection at n=%d b=%d\n", n, b); return 1; }
    }
    for (int b = hm::kXcds; b < n; ++b)
      if (hm::xcd_order(b, n) != hm::xcd_order(b - hm::kXcds, n) + 1) {
        std::printf("range not contiguous at n=%d b=%d\n", n, b);
        return 1;
      }
  }
  std::printf("ok\n");
  return 0;
}
"""


def test_xcd_order_is_a_contiguous_bijection(tmp_path):
    if not (Path(HIPCC).exists() or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    src = tmp_path / "order.cpp"
    src.write_text(PROGRAM)
    exe = tmp_path / "order"
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17",
           f"-I{ROOT / 'paper_2303_10102_amd' / 'csrc'}", str(src), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr

"""The multiply-and-shift division the kernels use for runtime divisors,
checked against integer division on the host (same header, host compile)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1603_07008_amd", "csrc")

PROG = r'''
#include <cstdio>
#include <cstdint>
#include "sldg_internal.h"
int main() {
  uint64_t checked = 0, bad = 0;
  auto check = [&](uint32_t d, uint32_t n) {
    sldg::FastDiv f = sldg::FastDiv::make(d);
    ++checked;
    if (f.div(n) != n / d || f.mod(n) != n % d) {
      if (bad < 5) printf("bad d=%u n=%u got %u\n", d, n, f.div(n));
      ++bad;
    }
  };
  uint64_t x = 88172645463325252ull;
  auto rnd = [&]() { x ^= x << 13; x ^= x >> 7; x ^= x << 17; return x; };
  for (uint32_t d = 1; d <= 4096; ++d) {
    for (uint32_t n = 0; n < 3 * d + 5; ++n) check(d, n);
    for (int k = 0; k < 64; ++k) check(d, (uint32_t)(rnd() % 2147483648u));
    check(d, 2147483647u);
    check(d, 2147483647u - (2147483647u % d));
    if (2147483647u % d) check(d, 2147483647u - (2147483647u % d) - 1);
  }
  for (int k = 0; k < 200000; ++k) {
    uint32_t d = 1 + (uint32_t)(rnd() % 2147483647u);
    uint32_t n = (uint32_t)(rnd() % 2147483648u);
    check(d, n);
    uint32_t q = n / d;
    if (q > 0) { check(d, q * d); check(d, q * d - 1); }
  }
  printf("checked=%llu bad=%llu\n", (unsigned long long)checked, (unsigned long long)bad);
  return bad != 0;
}
'''


def test_fastdiv_matches_integer_division():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "fd.cpp")
        exe = os.path.join(d, "fd")
        with open(src, "w") as f:
            f.write(PROG)
        subprocess.check_call([hipcc, "-O2", "-std=c++17", "-I", CSRC, "-I", os.path.join(ROOT, "include"), src, "-o", exe],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        out = subprocess.run([exe], capture_output=True, text=True)
        assert out.returncode == 0, out.stdout
        assert "bad=0" in out.stdout

"""The multiply-shift division used to decode node and cell indices in the
kernels (paper_2212_02362_amd/csrc/sbm_fastdiv.h) equals integer division for
every numerator below 2^31, checked on the host with g++ over all grid
extents up to 20000, the extents of the workloads, and dense numerator
ranges including every multiple-boundary q d - 1, q d, q d + 1."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r'''
#include <cstdio>
#include <cstdint>
#include "sbm_fastdiv.h"
using sbm::FastDiv; using sbm::make_fastdiv;
int main() {
  uint64_t bad = 0, checked = 0;
  const uint32_t ds[] = {1,2,3,4,5,7,9,13,17,33,49,65,97,129,193,257,513,1025,4097,65537,
                         (1u<<20)+1, 1000003u, 2147483647u};
  for (uint32_t d : ds) {
    FastDiv f = make_fastdiv(d);
    for (uint64_t n = 0; n < (1ull << 31); n += (n < (1u << 21) ? 1 : 104729)) {
      ++checked; bad += f.div((uint32_t)n) != n / d; }
    for (uint64_t n = (1ull << 31) - 50000; n < (1ull << 31); ++n) {
      ++checked; bad += f.div((uint32_t)n) != n / d; }
    for (uint64_t q = 1; q * d + 1 < (1ull << 31) && q < 100000; ++q)
      for (int e = -1; e <= 1; ++e) { uint64_t n = q * d + e; ++checked; bad += f.div((uint32_t)n) != n / d; }
  }
  for (uint32_t d = 1; d < 20000; ++d) {
    FastDiv f = make_fastdiv(d);
    const uint64_t cand[5] = {(uint64_t)d - 1, (uint64_t)d, (uint64_t)d * d - 1,
                              (1ull << 31) - 1, (1ull << 31) - d};
    for (uint64_t n : cand) { if (n >= (1ull << 31)) continue; ++checked; bad += f.div((uint32_t)n) != n / d; }
  }
  printf("%llu %llu\n", (unsigned long long)checked, (unsigned long long)bad);
  return bad != 0;
}
'''


def test_fastdiv_exact(tmp_path):
    src = tmp_path / "fd.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "fd"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-I",
                           os.path.join(ROOT, "paper_2212_02362_amd", "csrc"), "-o", str(exe), str(src)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    checked, bad = map(int, out.stdout.split())
    assert out.returncode == 0 and bad == 0 and checked > 10_000_000

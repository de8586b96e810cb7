"""The library's host-side method code (parameter validation, storage sizes, relaxation
blocks; csrc/lbm_method.cpp) built with AddressSanitizer and UndefinedBehaviorSanitizer and
driven through the C entry points by a deterministic fuzzer: valid and invalid enums, dims
from 0 to beyond 2^32 cells, rates inside and outside [0, 2] (NaN and infinities included),
NULL pointers and wrong rate counts.  Every call must return a status and leave an error
text on failure; any memory or undefined-behaviour error aborts the program."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2211_02435_amd", "csrc")

DRIVER = r'''
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <limits>
#include "lbm.h"

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint64_t next() {  // xorshift64*
  state ^= state >> 12; state ^= state << 25; state ^= state >> 27;
  return state * 0x2545F4914F6CDD1Dull;
}
static int pick(int n) { return int(next() % uint64_t(n)); }

int main() {
  const double specials[] = {0.0, 1.0, 2.0, 1.9, 0.7, -0.1, 2.1, std::numeric_limits<double>::quiet_NaN(),
                             std::numeric_limits<double>::infinity(), -std::numeric_limits<double>::infinity()};
  const int64_t dims[] = {1, 2, 3, 5, 64, 70, 512, 0, -1, 65536, 4096, int64_t(1) << 31, int64_t(1) << 40};
  // (the first seven are admissible edge lengths)
  double om[40];
  long ok = 0, bad = 0;
  for (int it = 0; it < 200000; ++it) {
    // even iterations draw inside the admissible ranges (the method restrictions still reject
    // some), odd ones anywhere, out-of-range values included
    const bool in_range = (it % 2) == 0;
    lbm_params p;
    if (lbm_params_default(&p) != LBM_OK) return 2;
    p.stencil = in_range ? pick(4) : pick(6) - 1;
    p.space = in_range ? pick(4) : pick(6) - 1;
    p.equilibrium = in_range ? (pick(4) == 0 ? 1 + pick(2) : 0) : pick(5) - 1;
    p.eq_form = in_range ? pick(3) : pick(5) - 1;
    p.zero_centered = in_range ? (pick(5) != 0) : pick(3) - (pick(4) == 0);
    p.storage = in_range ? pick(3) : pick(5) - 1;
    p.streaming = in_range ? pick(5) : pick(7) - 1;
    p.layout = in_range ? pick(3) : pick(5) - 1;
    p.arithmetic = in_range ? pick(2) : pick(4) - 1;
    p.force_model = in_range ? pick(2) : pick(4) - 1;
    p.basis = in_range ? (pick(4) == 0 ? 1 + pick(2) : 0) : pick(5) - 1;
    p.gravity = in_range ? 0.1 : (pick(3) == 0 ? -0.1 : 0.1 * pick(3));
    p.nx = dims[pick(in_range ? 7 : 13)];
    p.ny = dims[pick(in_range ? 7 : 13)];
    p.nz = (p.stencil == LBM_D2Q9 && in_range) || pick(2) ? 1 : dims[pick(in_range ? 7 : 13)];
    for (int d = 0; d < 3; ++d) {
      p.periodic[d] = in_range || pick(10) != 0;
      p.force[d] = pick(3) == 0 ? 1e-5 * pick(3) : 0.0;
    }
    const int q = p.stencil == LBM_D2Q9 ? 9 : (p.stencil == LBM_D3Q19 ? 19 : (p.stencil == LBM_D3Q15 ? 15 : 27));
    p.n_omegas = (!in_range && pick(8) == 0) ? pick(40) : q;
    for (int i = 0; i < 40; ++i)
      om[i] = (!in_range && pick(6) == 0) ? specials[pick(10)] : 0.5 + 1.4 * double(pick(1000)) / 1000.0;
    p.omegas = (!in_range && pick(20) == 0) ? nullptr : om;
    const lbm_status s = lbm_validate(&p);
    const char *e = lbm_last_error();
    if (!e) return 3;
    if (s != LBM_OK) {
      if (std::strlen(e) == 0) return 4;
      ++bad;
    } else {
      ++ok;
      size_t bytes = 0;
      if (lbm_required_bytes(&p, &bytes) != LBM_OK || bytes == 0) return 5;
      if (lbm_required_bytes(&p, nullptr) != LBM_EINVAL) return 6;
    }
  }
  if (lbm_validate(nullptr) == LBM_OK) return 7;
  if (lbm_params_default(nullptr) == LBM_OK) return 8;
  std::printf("valid %ld invalid %ld\n", ok, bad);
  return 0;
}
'''


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_method_host_code_under_asan_and_ubsan(tmp_path):
    drv = tmp_path / "fuzz.cpp"
    drv.write_text(DRIVER)
    exe = tmp_path / "fuzz"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), str(drv),
           os.path.join(CSRC, "lbm_method.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout, r.stderr[-3000:])
    assert r.returncode == 0, (r.returncode, r.stderr[-3000:])
    valid, invalid = (int(v) for v in r.stdout.split()[1::2])
    assert valid > 1000 and invalid > 1000

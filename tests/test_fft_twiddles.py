"""The block FFT's compile-time twiddle table against the C library's long
double cos and sin: every entry is the correctly rounded float value, except
where the exact value lies within one float rounding of a tie."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2311_00482_amd", "csrc", "fft_twiddles.h")

CHECK = r'''
#include <cmath>
#include <cstdio>
#include "fft_twiddles.h"
using namespace pwbf::fft::detail;
constexpr TwTable kTab{};
int main() {
  int off = 0;
  double worst = 0.0;
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < kTwN / 2; ++k) {
    const long double a = 2.0L * pi * k / kTwN;
    const long double c = cosl(a), s = -sinl(a);
    if ((float)c != kTab.v[k].c || (float)s != kTab.v[k].s) ++off;
    worst = std::fmax(worst, (double)fabsl((long double)kTab.v[k].c - c));
    worst = std::fmax(worst, (double)fabsl((long double)kTab.v[k].s - s));
  }
  std::printf("%d %.6e\n", off, worst);
  return 0;
}
'''


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("tw")
    src = d / "check.cpp"
    src.write_text(CHECK)
    exe = d / "check"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", os.path.dirname(HDR), str(src),
                           "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split()
    return int(out[0]), float(out[1])


def test_table_is_correctly_rounded_but_for_ties(checker):
    off, worst = checker
    # entries of magnitude <= 1: half an ulp is <= 2^-25
    assert worst <= 2.0 ** -25
    assert off <= 2


def test_symmetries_of_the_table():
    # W^0 = 1, W^512 = -i, W^1024 = -1 (cos of a quarter turn is +0 or a tiny value)
    src = r'''
#include <cstdio>
#include "fft_twiddles.h"
using namespace pwbf::fft::detail;
constexpr TwTable kTab{};
int main() {
  std::printf("%a %a %a %a %a %a\n", kTab.v[0].c, kTab.v[0].s, kTab.v[1024].c, kTab.v[1024].s,
              kTab.v[512].c, kTab.v[512].s);
  for (int k = 1; k < 1024; ++k)  // W^(1024 + k) = -i W^k: c' = s, s' = -c
    if (kTab.v[1024 + k].c != kTab.v[k].s || kTab.v[1024 + k].s != -kTab.v[k].c) {
      std::printf("asym %d\n", k);
      return 1;
    }
  return 0;
}
'''
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "s.cpp")
        open(p, "w").write(src)
        subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", os.path.dirname(HDR), p, "-o",
                               os.path.join(d, "s")])
        out = subprocess.run([os.path.join(d, "s")], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    c0, s0, c1024, s1024, c512, s512 = [float.fromhex(v) for v in out.stdout.split()]
    assert (c0, s0) == (1.0, 0.0)
    assert s1024 == -1.0 and abs(c1024) < 1e-7
    assert abs(c512 - 2 ** -0.5) < 6e-8 and abs(s512 + 2 ** -0.5) < 6e-8

"""Host check of the FP32 ordering keys (csrc/alp_keys.h).

The weights pass builds each staged window's screening frame with integer LDS
atomics: the smallest and largest axial coordinate (signed) through
f32_key / f32_of_key, and the largest squared deviation and radius
(non-negative) through the plain bits.  A C++ program compiled on the host
from the same header checks, over random finite floats of every sign and
magnitude (subnormals and zeros included) and all pairs of a sorted sample,
that the keys order exactly like the values, that a key decodes to the value
bit for bit, and that the plain bits of non-negative values order like the
values; and, as a reduction, that the minimum and maximum of random sets taken
through the keys equal the ones taken on the floats.
"""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2609_39443_amd", "csrc")

PROG = r'''
#define ALP_HD inline
#include "alp_keys.h"
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>
using namespace alp;

#define CHECK(cond, ...) do { if (!(cond)) { std::printf(__VA_ARGS__); std::printf("\n"); return 1; } } while (0)

int main() {
  std::mt19937_64 rng(2024);
  std::vector<float> v;
  // random bit patterns (finite ones), both zeros, the extremes, and values
  // of the size the frames see
  for (int i = 0; i < 200000; ++i) {
    uint32_t b = (uint32_t)rng();
    float x;
    std::memcpy(&x, &b, 4);
    if (std::isfinite(x)) v.push_back(x);
  }
  const float special[] = {0.0f, -0.0f, 1e-45f, -1e-45f, 1.17549435e-38f, -1.17549435e-38f,
                           3.40282347e38f, -3.40282347e38f, 1.0f, -1.0f, 0.004f, -0.004f};
  for (float x : special) v.push_back(x);
  std::uniform_real_distribution<float> u(-0.2f, 0.2f);
  for (int i = 0; i < 200000; ++i) v.push_back(u(rng));
  long n = 0;
  for (float x : v) {
    const uint32_t k = f32_key(x);
    CHECK(f32_bits(f32_of_key(k)) == f32_bits(x), "key of %a does not decode to it", (double)x);
    ++n;
  }
  // every pair of a sorted sample of 4000
  std::vector<float> s(v.begin(), v.begin() + 2000);
  s.insert(s.end(), v.end() - 2000, v.end());
  std::sort(s.begin(), s.end());
  for (size_t i = 0; i < s.size(); ++i)
    for (size_t j = i + 1; j < s.size(); ++j) {
      const float a = s[i], b = s[j];
      if (a < b) CHECK(f32_key(a) < f32_key(b), "%a < %a but keys %08x >= %08x", (double)a, (double)b, f32_key(a), f32_key(b));
      if (a == b && f32_bits(a) == f32_bits(b)) CHECK(f32_key(a) == f32_key(b), "equal values, different keys");
      if (a >= 0.0f && b >= 0.0f && a < b) CHECK(f32_bits(a) < f32_bits(b), "bits of %a and %a out of order", (double)a, (double)b);
      ++n;
    }
  // reductions as the frames take them: minimum and maximum through keys
  for (int t = 0; t < 2000; ++t) {
    const int m = 1 + (int)(rng() % 200);
    float lo = INFINITY, hi = -INFINITY;
    uint32_t klo = 0xffffffffu, khi = 0u;
    for (int i = 0; i < m; ++i) {
      const float x = v[rng() % v.size()];
      lo = std::fmin(lo, x);
      hi = std::fmax(hi, x);
      klo = std::min(klo, f32_key(x));
      khi = std::max(khi, f32_key(x));
    }
    // (fmin of +0 and -0 may return either; compare values)
    CHECK(f32_of_key(klo) == lo && f32_of_key(khi) == hi, "set %d: key min / max %a %a against %a %a", t,
          (double)f32_of_key(klo), (double)f32_of_key(khi), (double)lo, (double)hi);
  }
  std::printf("ok %ld\n", n);
  return 0;
}
'''


def test_fp32_keys_order_like_their_values(tmp_path):
    src = tmp_path / "keys.cpp"
    src.write_text(PROG)
    exe = tmp_path / "keys"
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-I", CSRC, str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=240)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok ")
    assert int(out.stdout.split()[1]) > 1000000

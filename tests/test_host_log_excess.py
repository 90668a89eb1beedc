"""The mixed-precision log term on the host (CPU only).

q(d) = d - log(1 + d) in float (log_excess(float) in p1e_device.h, the Neo-Hookean density's
log term in mixed precision) is compiled with g++ from the header's own text, the hardware
reciprocal replaced by a correctly rounded division (the function refines it by a Newton
step either way), and compared with a long double reference: the series
d^2/2 - d^3/3 + ... for |d| < 1e-3 (where d - log1p(d) itself cancels), d - log1p(d)
otherwise. Bounds: 3 float ulps of q for |d| <= 1/4, 12 over (-1, 1e3).
"""

import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(os.path.dirname(HERE), "paper_2109_01158_amd", "csrc", "p1e_device.h")

_DRIVER = r"""
#include <cmath>
#include <cstdio>
#include <random>
static inline float rcpf_(float x) { return 1.0f / x; }
%s
static long double q_ref(long double d) {
  if (fabsl(d) < 1e-3L) {
    long double t = 0, p = d * d;
    for (int k = 2; k < 14; ++k) { t += (k %% 2 == 0 ? 1 : -1) * p / k; p *= d; }
    return t;
  }
  return d - log1pl(d);
}
int main() {
  std::mt19937_64 g(1);
  std::uniform_real_distribution<double> u(0, 1);
  double small = 0, all = 0;
  long n = 0;
  for (long i = 0; i < 2000000; ++i) {
    const double x = u(g);
    float d;
    switch (i %% 4) {
      case 0: d = (float)(-1 + pow(10, -7 * x)); break;     // toward d = -1
      case 1: d = (float)((x * 2 - 1) * 0.5); break;        // |d| < 1/2
      case 2: d = (float)((x * 2 - 1) * pow(10, -8 * u(g))); break;  // near 0
      default: d = (float)pow(10, 3 * x); break;            // up to 1e3
    }
    if (!(d > -1.0f)) continue;
    const long double r = q_ref(d);
    if (r == 0) continue;
    const double e = (double)fabsl((log_excess(d) - r) / r) / 5.9604644775390625e-8;
    if (fabsf(d) <= 0.25f && e > small) small = e;
    if (e > all) all = e;
    ++n;
  }
  printf("%%ld %%.3f %%.3f\n", n, small, all);
}
"""


def _function_text():
    src = open(HEADER).read()
    m = re.search(r"__device__ __forceinline__ float log_excess\(float d\) \{", src)
    assert m, "log_excess(float) not found in p1e_device.h"
    depth, i = 0, m.end() - 1
    for j in range(i, len(src)):
        depth += {"{": 1, "}": -1}.get(src[j], 0)
        if depth == 0:
            body = src[m.start():j + 1]
            break
    body = body.replace("__device__ __forceinline__", "static inline")
    return body.replace("__builtin_amdgcn_rcpf(", "rcpf_(")


@pytest.mark.timeout(300)
def test_float_log_excess_ulps(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    src = tmp_path / "log_excess.cpp"
    src.write_text(_DRIVER % _function_text())
    exe = str(tmp_path / "log_excess")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", str(src), "-o", exe],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True,
                         timeout=120).stdout.split()
    n, small, worst = int(out[0]), float(out[1]), float(out[2])
    print(f"log_excess(float): {n} samples, worst {small:.2f} ulp for |d| <= 1/4, "
          f"{worst:.2f} overall")
    assert n > 1_500_000
    assert small <= 3.0
    assert worst <= 12.0

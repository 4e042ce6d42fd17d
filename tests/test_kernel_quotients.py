"""The kernels form two kinds of quotient without a division instruction
each: x0 / x2 and x1 / x2 of the projection share one correctly rounded
reciprocal 1 / x2, and the running average divides by W + 1 (W = 0 .. 255)
with a table of the correctly rounded reciprocals.  In both, the product
q = a y is corrected once with fused operations, q + (a - b q) y (Markstein).
These checks run that arithmetic in IEEE single precision on the CPU against
the correctly rounded a / b that the oracle's FP32 mirror performs: all
2^23 numerators of a binade for every divisor 1 .. 256 (the quotient's
rounding pattern repeats in every binade of normal numbers), and random
pairs over 40 binades for general divisors (no GPU)."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np

_SRC = r"""
#include <math.h>
#include <stdint.h>
#include <string.h>
static float fb(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
static float quot(float a, float b, float y) {
  volatile float q = a * y;
  volatile float r = fmaf(-q, b, a);
  return fmaf(r, y, q);
}
/* out[0]: mismatches of the table form over b = 1..256, a in [1, 2);
   out[1]: mismatches over n random pairs; out[2]: plain products a * y that
   differ from a / b (the correction is needed at all) */
void check(int64_t* out, int64_t n) {
  out[0] = out[1] = out[2] = 0;
  for (int b = 1; b <= 256; ++b) {
    volatile float bf = (float)b;
    volatile float y = 1.0f / bf;
    for (uint32_t u = 0x3f800000u; u < 0x40000000u; ++u) {
      volatile float a = fb(u);
      volatile float ex = a / bf;
      volatile float pr = a * y;
      out[0] += quot(a, bf, y) != ex;
      out[2] += pr != ex;
    }
  }
  uint64_t s = 0x1905020821ull;
  for (int64_t i = 0; i < n; ++i) {
    s ^= s << 13; s ^= s >> 7; s ^= s << 17;
    uint32_t ub = (uint32_t)(s & 0x7fffff) | ((uint32_t)((s >> 23) % 40 + 107) << 23);
    uint32_t ua = (uint32_t)((s >> 32) & 0x7fffff) | ((uint32_t)(((s >> 55) % 40) + 107) << 23) |
                  ((uint32_t)((s >> 63) & 1) << 31);
    volatile float a = fb(ua), bf = fb(ub);
    volatile float y = 1.0f / bf;
    volatile float ex = a / bf;
    out[1] += quot(a, bf, y) != ex;
  }
}
"""


def test_corrected_quotients_equal_correctly_rounded_division():
    with tempfile.TemporaryDirectory() as d:
        src, lib = os.path.join(d, "q.c"), os.path.join(d, "q.so")
        with open(src, "w") as fh:
            fh.write(_SRC)
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC", src,
                               "-o", lib, "-lm"])
        L = ctypes.CDLL(lib)
        out = np.zeros(3, np.int64)
        L.check(ctypes.c_void_p(out.ctypes.data), ctypes.c_int64(100_000_000))
    assert out[2] > 0, "the plain product must differ somewhere (else the check is vacuous)"
    assert out[0] == 0 and out[1] == 0

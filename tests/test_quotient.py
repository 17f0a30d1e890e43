"""The 3D FD update divides by S_0 = 6 on the GPU as q = RN(x z), z = RN(1/6),
followed by one fused multiply-add correction (q' = fma(fma(-q, 6, x), z, q)).
For a divisor 3 * 2^k this equals the correctly rounded x / 6 for every x with
a normal quotient; here the identity is checked on the CPU in C, against the
plain IEEE division, over seeded random doubles of many binades and every
float significand of two binades.  A variant without the correction step must
fail the same check."""
import os
import subprocess

import pytest

SRC = r"""
#include <math.h>
#include <stdio.h>
#include <stdint.h>
#include <string.h>
static uint64_t st = 0x243F6A8885A308D3ULL;
static uint64_t nx(void) {
    uint64_t z = (st += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
int main(void) {
    const double z = 1.0 / 6.0;
    long bad = 0;
    for (long i = 0; i < 20000000L; ++i) {
        uint64_t m = nx();
        uint64_t bits = (m & 0x000FFFFFFFFFFFFFULL) | ((uint64_t)(1023 + (int)(nx() % 200) - 100) << 52)
                        | (m & 0x8000000000000000ULL);
        double x;
        memcpy(&x, &bits, 8);
        double q = x * z;
#ifdef CORRECT
        q = fma(fma(-q, 6.0, x), z, q);
#endif
        if (q != x / 6.0) ++bad;
    }
    const float zf = 1.0f / 6.0f;
    long badf = 0;
    for (uint32_t mm = 0; mm < (1u << 23); ++mm)
        for (int e = -1; e <= 0; ++e) {
            uint32_t bits = mm | ((uint32_t)(127 + e) << 23);
            float x;
            memcpy(&x, &bits, 4);
            float q = x * zf;
#ifdef CORRECT
            q = fmaf(fmaf(-q, 6.0f, x), zf, q);
#endif
            if (q != x / 6.0f) ++badf;
        }
    printf("%ld %ld\n", bad, badf);
    return 0;
}
"""


def _run(tmp_path, correct):
    c = tmp_path / "q.c"
    c.write_text(SRC)
    exe = tmp_path / ("q1" if correct else "q0")
    flags = ["-DCORRECT"] if correct else []
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math"] + flags
                   + ["-o", str(exe), str(c), "-lm"], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), int(out[1])


def test_corrected_quotient_equals_division(tmp_path):
    assert _run(tmp_path, True) == (0, 0)


def test_uncorrected_quotient_is_caught(tmp_path):
    bad, badf = _run(tmp_path, False)
    assert bad > 0 and badf > 0

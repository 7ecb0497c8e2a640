"""The library's host routines for the modified Bessel functions I_n and K_n
(paper_2203_05933_amd/csrc/vp_bessel.hpp, used at plan time for the modified
Helmholtz operators) against mpmath at 40 digits; CPU only (the header is
compiled with g++ into a small driver)."""
import os
import subprocess
import tempfile

import mpmath
import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2203_05933_amd", "csrc", "vp_bessel.hpp")

DRIVER = r"""
#include "%s"
#include <cstdio>
int main() {
    const double xs[] = {1.0 / 8192, 1.0 / 1024, 0.05, 0.3, 1.0, 2.5, 7.0, 15.0, 30.0, 60.0, 120.0};
    for (double x : xs) {
        long double I[61], K[61];
        vp::bessel_i_all(x, 60, I);
        vp::bessel_k_all(x, 60, K);
        for (int n = 0; n <= 60; n += 3) std::printf("%%.17g %%d %%.21Le %%.21Le\n", x, n, I[n], K[n]);
    }
    return 0;
}
"""


def test_bessel_i_k_match_mpmath():
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "t.cpp"), os.path.join(d, "t")
        with open(src, "w") as fh:
            fh.write(DRIVER % HDR)
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-o", exe, src])
        out = subprocess.check_output([exe], text=True)
    mpmath.mp.dps = 40
    worst = 0.0
    for line in out.splitlines():
        xs, ns, iv, kv = line.split()
        x, n = mpmath.mpf(xs), int(ns)
        for got, ref in ((iv, mpmath.besseli(n, x)), (kv, mpmath.besselk(n, x))):
            worst = max(worst, float(abs(mpmath.mpf(got) - ref) / abs(ref)))
    assert worst < 1e-15, worst

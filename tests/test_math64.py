"""The restricted FP64 logarithm of the step kernel (mc_math64.hpp), compiled
on the host with g++: within 2 ulp of the C library's log over uniform
variates (w + 1/2) 2^-32, their products, and the ends of its domain."""
import os
import subprocess

HARNESS = r'''
#include "mc_math64.hpp"
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
static double ulps(double a, double b) {
    if (a == b) return 0;
    const double u = std::nextafter(std::fabs(b), INFINITY) - std::fabs(b);
    return std::fabs(a - b) / u;
}
int main() {
    std::mt19937_64 rng(3);
    double worst = 0;
    for (long k = 0; k < 4000000; ++k) {
        const double u = ((double)(uint32_t)rng() + 0.5) * 0x1p-32;
        const double v = ((double)(uint32_t)rng() + 0.5) * 0x1p-32;
        worst = std::fmax(worst, ulps(mc::ln_unit(u), std::log(u)));
        worst = std::fmax(worst, ulps(mc::ln_unit(u * v), std::log(u * v)));
        const double w = std::ldexp(0.5 + 0.5 * u, -(int)(rng() % 1000));  // exponents down to 2^-1000
        worst = std::fmax(worst, ulps(mc::ln_unit(w), std::log(w)));
    }
    const double ends[] = {1.0, 0.5, 0x1p-66, 0x1p-1022, 0.70710678118654746, 0.70710678118654757,
                           1.0 - 0x1p-53, 0.9999999};
    for (double x : ends) worst = std::fmax(worst, ulps(mc::ln_unit(x), std::log(x)));
    if (mc::ln_unit(1.0) != 0.0) { std::puts("FAIL ln 1"); return 1; }
    std::printf(worst <= 2.0 ? "OK %.3f\n" : "FAIL %.3f\n", worst);
    return 0;
}
'''


def test_restricted_log_within_two_ulp(tmp_path):
    csrc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2609_31258_amd", "csrc")
    src = tmp_path / "ln_test.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "ln_test"
    subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-I" + csrc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.strip()
    assert out.startswith("OK"), out

"""The restricted FP64 elementary functions of the step kernel
(mc_math64.hpp), compiled on the host with g++ and checked against
extended-precision (x87 long double) references: each within 2 ulp (the
table-driven sine and cosine 2.5) over the arguments the step takes -- uniform variates (w + 1/2) 2^-32 and their
products for the logarithms (series and table-driven, the latter also at both
ends and the centre of every bin), positive ratios over the whole double
range for log1p, uniform turns for the sine and cosine -- and at the ends of
each domain; the seeded square root is correctly rounded from estimates eight
times worse than the hardware's, and the seeded reciprocal within 1 ulp from
such estimates."""
import os
import subprocess

HARNESS = r'''
#include "mc_math64.hpp"
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
// distance in units of the last place of the correctly rounded reference
static double ulps(double a, long double ref) {
    const double b = (double)ref;
    const double u = std::nextafter(std::fabs(b), INFINITY) - std::fabs(b);
    return (double)(std::fabs((long double)a - ref) / u);
}
static long double two_pi_l() { return 2.0L * 3.14159265358979323846264338327950288L; }
int main() {
    mc::LnEntry tab[mc::kLnBins];
    mc::ln_table_fill(tab);
    mc::TurnEntry ttab[mc::kTurnBins];
    mc::turn_table_fill(ttab);
    std::mt19937_64 rng(3);
    double w_ln = 0, w_lnt = 0, w_ln1p = 0, w_sin = 0, w_cos = 0, w_sin2 = 0, w_cos2 = 0, w_st = 0, w_ct = 0;
    for (long k = 0; k < 2000000; ++k) {
        const double u = ((double)(uint32_t)rng() + 0.5) * 0x1p-32;
        const double v = ((double)(uint32_t)rng() + 0.5) * 0x1p-32;
        // logarithm: uniforms, their products, and the whole normal range
        w_ln = std::fmax(w_ln, ulps(mc::ln_pos(u), logl(u)));
        w_ln = std::fmax(w_ln, ulps(mc::ln_pos(u * v), logl((long double)(u * v))));
        const double x = std::ldexp(0.5 + 0.5 * u, (int)(rng() % 2040) - 1020);
        w_ln = std::fmax(w_ln, ulps(mc::ln_pos(x), logl(x)));
        // the table-driven logarithm on the same arguments
        w_lnt = std::fmax(w_lnt, ulps(mc::ln_tab(u, tab), logl(u)));
        w_lnt = std::fmax(w_lnt, ulps(mc::ln_tab(u * v, tab), logl((long double)(u * v))));
        w_lnt = std::fmax(w_lnt, ulps(mc::ln_tab(x, tab), logl(x)));
        // log1p: positive ratios from 2^-1020 to 2^1020, small ratios, and
        // near the bins next to 1 + x = 1 and sqrt 2
        w_ln1p = std::fmax(w_ln1p, ulps(mc::ln1p_tab(x, tab), log1pl(x)));
        const double y = 0.41421356237309503 * (1.0 + (v - 0.5) * 1e-3);
        w_ln1p = std::fmax(w_ln1p, ulps(mc::ln1p_tab(y, tab), log1pl(y)));
        const double z = std::ldexp(1.0 + u, -(int)(rng() % 60));
        w_ln1p = std::fmax(w_ln1p, ulps(mc::ln1p_tab(z, tab), log1pl(z)));
        // sine and cosine of a turn: against the reference on the same exact
        // reduction (all arguments), and against the unreduced extended
        // argument where the result is not near a zero (checks the quadrants)
        double s, c;
        mc::sincos_turn(u, &s, &c);
        const double q = std::rint(4.0 * u);
        const long double t = (long double)u - 0.25L * (long double)q;
        if (t != (long double)(u - 0.25 * q)) { std::puts("FAIL reduction not exact"); return 1; }
        const long double th = two_pi_l() * t;
        const int kq = (int)q & 3;
        const long double st = sinl(th), ct = cosl(th);
        const long double rs = kq == 0 ? st : kq == 1 ? ct : kq == 2 ? -st : -ct;
        const long double rc = kq == 0 ? ct : kq == 1 ? -st : kq == 2 ? -ct : st;
        w_sin = std::fmax(w_sin, ulps(s, rs));
        w_cos = std::fmax(w_cos, ulps(c, rc));
        double st2, ct2;
        mc::sincos_turn_tab(u, ttab, &st2, &ct2);
        w_st = std::fmax(w_st, ulps(st2, rs));
        w_ct = std::fmax(w_ct, ulps(ct2, rc));
        if (mc::cos_turn_tab(u, ttab) != ct2) { std::puts("FAIL cos_turn_tab differs from sincos_turn_tab"); return 1; }
        if (mc::cos_turn(u) != c) { std::puts("FAIL cos_turn differs from sincos_turn"); return 1; }
        const long double ds = sinl(two_pi_l() * u), dc = cosl(two_pi_l() * u);
        if (fabsl(ds) > 0.01L) w_sin2 = std::fmax(w_sin2, ulps(s, ds));
        if (fabsl(dc) > 0.01L) w_cos2 = std::fmax(w_cos2, ulps(c, dc));
    }
    const double ends[] = {1.0, 0.5, 0x1p-66, 0x1p-1022, 0.70710678118654746, 0.70710678118654757,
                           1.0 - 0x1p-53, 0.9999999, 0x1p1000, 1.7976931348623157e308};
    for (double x : ends) w_ln = std::fmax(w_ln, ulps(mc::ln_pos(x), logl(x)));
    for (double x : ends) w_lnt = std::fmax(w_lnt, ulps(mc::ln_tab(x, tab), logl(x)));
    if (mc::ln_pos(1.0) != 0.0 || mc::ln_tab(1.0, tab) != 0.0) { std::puts("FAIL ln 1"); return 1; }
    // every bin of the table, at its ends and centre
    for (int j = 0; j < mc::kLnBins; ++j)
        for (double f : {0.0, 0.5, 1.0 - 0x1p-40}) {
            const double mm = 0.5 + (j + f) / (2.0 * mc::kLnBins);
            w_lnt = std::fmax(w_lnt, ulps(mc::ln_tab(mm, tab), logl(mm)));
            w_lnt = std::fmax(w_lnt, ulps(mc::ln_tab(2 * mm, tab), logl(2 * mm)));
        }
    const double ends1p[] = {0x1p-1074, 0x1p-60, 1e-17, 1e-9, 0.41421356237309492, 0.41421356237309515, 1.0,
                             3.0, 1e15, 0x1p53, 1.7976931348623157e308};
    for (double x : ends1p) w_ln1p = std::fmax(w_ln1p, ulps(mc::ln1p_tab(x, tab), log1pl(x)));
    if (mc::ln1p_tab(0.0, tab) != 0.0 || mc::ln1p_tab(INFINITY, tab) != INFINITY) { std::puts("FAIL ln1p 0 / inf"); return 1; }
    // exact values at the quarter turns
    const double turns[] = {0.0, 0.25, 0.5, 0.75, 1.0};
    const double want_s[] = {0.0, 1.0, 0.0, -1.0, 0.0}, want_c[] = {1.0, 0.0, -1.0, 0.0, 1.0};
    for (int i = 0; i < 5; ++i) {
        double s, c;
        mc::sincos_turn(turns[i], &s, &c);
        if (s != want_s[i] || c != want_c[i]) { std::printf("FAIL turn %g: %g %g\n", turns[i], s, c); return 1; }
        mc::sincos_turn_tab(turns[i], ttab, &s, &c);
        if (s != want_s[i] || c != want_c[i]) { std::printf("FAIL table turn %g: %g %g\n", turns[i], s, c); return 1; }
    }
    // the seeded square root from estimates perturbed by up to 2^-20 (the
    // hardware estimate is within 2^-23): correctly rounded
    std::uniform_real_distribution<double> pert(-1.0, 1.0);
    for (long k = 0; k < 1000000; ++k) {
        const double m = 1.0 + ((double)(uint32_t)rng() + 0.5) * 0x1p-32;
        const double x = std::ldexp(m, (int)(rng() % 2000) - 1000);
        const double r = (double)(1.0L / sqrtl((long double)x)) * (1.0 + pert(rng) * 0x1p-20);
        if (mc::sqrt_seeded(x, r) != std::sqrt(x)) { std::printf("FAIL sqrt %.17g\n", x); return 1; }
    }
    if (mc::sqrt_seeded(0.0, INFINITY) != 0.0) { std::puts("FAIL sqrt 0"); return 1; }
    // the seeded reciprocal from estimates perturbed by up to 2^-20: within 1 ulp
    double w_rcp = 0.0;
    for (long k = 0; k < 1000000; ++k) {
        const double m = 1.0 + ((double)(uint32_t)rng() + 0.5) * 0x1p-32;
        const double x = std::ldexp(m, (int)(rng() % 2000) - 1000);
        const double r = (double)(1.0L / (long double)x) * (1.0 + pert(rng) * 0x1p-20);
        w_rcp = std::fmax(w_rcp, ulps(mc::recip_seeded(x, r), 1.0L / (long double)x));
    }
    if (w_rcp > 1.0) { std::printf("FAIL reciprocal %.3f ulp\n", w_rcp); return 1; }
    // bounds: 2 ulp, and 2.5 for the table sine and cosine (the node's own
    // rounding shows where the result is smaller than the node's value)
    const bool ok = std::fmax(std::fmax(w_ln, w_lnt), w_ln1p) <= 2.0 &&
                    std::fmax(std::fmax(w_sin, w_cos), std::fmax(w_sin2, w_cos2)) <= 2.0 &&
                    std::fmax(w_st, w_ct) <= 2.5;
    std::printf("%s ln %.3f ln(table) %.3f ln1p(table) %.3f sin %.3f cos %.3f sin(unreduced) %.3f cos(unreduced) %.3f "
                "sin(table) %.3f cos(table) %.3f\n",
                ok ? "OK" : "FAIL", w_ln, w_lnt, w_ln1p, w_sin, w_cos, w_sin2, w_cos2, w_st, w_ct);
    return 0;
}
'''


def test_restricted_functions_within_two_ulp(tmp_path):
    csrc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2609_31258_amd", "csrc")
    src = tmp_path / "math64_test.cpp"
    src.write_text(HARNESS)
    exe = tmp_path / "math64_test"
    subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-I" + csrc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.strip()
    print(out)
    assert out.startswith("OK"), out

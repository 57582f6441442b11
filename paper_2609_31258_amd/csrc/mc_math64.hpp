// mc_math64.hpp -- double-precision elementary functions for the arguments
// the FP64 step takes, written from their series, with and without small
// tables (the step keeps its tables in LDS).
//
// The general library functions handle every input (denormals, infinities,
// NaN, arguments of any size) and cost about 100 (logarithm), 130 (log1p) and
// 65 (sine and cosine of pi x) instructions.  The collision loop takes, per
// candidate, three or four logarithms of uniform variates or their products
// in (0, 1], two sine/cosine pairs and a cosine of 2 pi u for uniform u, and
// (in the internal-energy exchange) a log1p of a positive ratio.  These
// restricted versions stay within 2 ulp there (the table-driven sine and
// cosine 2.5; tested on the host against extended-precision references) in
// a fifth to a half of the instructions.
//
//   div_mid(n, d)        n / d for d in [1, 4), |n| < 1 (its quotient step)
//   sqrt_seeded(x, r)    sqrt x from a reciprocal-square-root estimate r
//   recip_seeded(x, r)   1/x from a reciprocal estimate r (within 1 ulp)
//   ln_pos(x)            natural logarithm, x > 0 normal and finite (series)
//   ln_tab(x, tab)       the same from a 256-bin table (ln_table_fill)
//   ln1p_tab(x, tab)     ln(1 + x), x >= 0 (+inf gives +inf), from the table
//   sincos_turn(u, s, c) sin(2 pi u), cos(2 pi u), 0 <= u <= 1 (series)
//   cos_turn(u)          cos(2 pi u), 0 <= u <= 1
//   sincos_turn_tab, cos_turn_tab   the same from a 256-node table
//                        (turn_table_fill)
//
// Plain C++ (host and device).
#pragma once
#include <cmath>
#include <cstdint>
#include <cstring>

#if defined(__HIPCC__)
#define MC_HD __host__ __device__ __forceinline__
#define MC_H __host__ inline
#else
#define MC_HD inline
#define MC_H inline
#endif

namespace mc {

// num / den for den in [1, 4) and |num| < 1, where no operand scaling or
// special case can arise.  On the device: the reciprocal estimate refined by
// two Newton steps, the quotient and one residual correction, which is the
// arithmetic of the compiler's double division without its range scaling and
// fix-up (so the same quotient in four fewer instructions).
MC_HD double div_mid(double num, double den) {
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(den);
    double e = std::fma(-den, r, 1.0);
    r = std::fma(r, e, r);
    e = std::fma(-den, r, 1.0);
    r = std::fma(r, e, r);
    const double q = num * r;
    return std::fma(std::fma(-den, q, num), r, q);
#else
    return num / den;
#endif
}

// sqrt x for x >= 0 (zero or normal) from an estimate r of 1/sqrt(x) with
// relative error below 2^-20 (the hardware estimate is within 2^-23): one
// coupled Newton step for y = sqrt(x) and h = 1/(2 sqrt(x)) (error about
// 1.5 times the square of the estimate's), then one residual correction,
// y + (x - y^2) h, which squares the error again below the final rounding.
MC_HD double sqrt_seeded(double x, double r) {
    double y = x * r, h = 0.5 * r;
    const double e = std::fma(-y, h, 0.5);
    y = std::fma(y, e, y);
    h = std::fma(h, e, h);
    y = std::fma(std::fma(-y, y, x), h, y);
    return x > 0.0 ? y : 0.0;
}

// 1/x for x positive and normal from an estimate r within 2^-20 relative:
// two Newton steps r + r (1 - x r), each squaring the relative error, leave
// it below the final rounding (within one unit in the last place; not
// always the correctly rounded quotient).
MC_HD double recip_seeded(double x, double r) {
    r = std::fma(r, std::fma(-x, r, 1.0), r);
    r = std::fma(r, std::fma(-x, r, 1.0), r);
    return r;
}

// 2 atanh f = 2 (f + f^3/3 + f^5/5 + ...) for f = num / den, |f| <= 0.1716
// (so f^2 <= 0.0295 and ten terms after the first leave a relative
// truncation error below 2^-60).
MC_HD double atanh2(double num, double den) {
    const double f = div_mid(num, den);
    const double g = f * f;
    double p = 1.0 / 21.0;
    p = std::fma(p, g, 1.0 / 19.0);
    p = std::fma(p, g, 1.0 / 17.0);
    p = std::fma(p, g, 1.0 / 15.0);
    p = std::fma(p, g, 1.0 / 13.0);
    p = std::fma(p, g, 1.0 / 11.0);
    p = std::fma(p, g, 1.0 / 9.0);
    p = std::fma(p, g, 1.0 / 7.0);
    p = std::fma(p, g, 1.0 / 5.0);
    p = std::fma(p, g, 1.0 / 3.0);
    // 2 atanh f = 2f + 2f g p, the small part added last
    return std::fma(2.0 * f, g * p, 2.0 * f);
}

// e ln 2 + v, with ln 2 split into a 32-bit head (e * head is exact for every
// exponent of a double) and a tail.
MC_HD double add_e_ln2(int e, double v) {
    const double ln2_hi = 0.6931471806019545;       // round(2^32 ln 2) / 2^32 (32 significant bits)
    const double ln2_lo = -4.2009150726810846e-11;  // ln 2 - ln2_hi
    const double de = (double)e;
    return std::fma(de, ln2_hi, std::fma(de, ln2_lo, v));
}

// ln x = e ln 2 + ln m, x = m 2^e with m in [sqrt(1/2), sqrt(2)), and
// ln m = 2 atanh f with f = (m - 1)/(m + 1), |f| <= 0.1716.
MC_HD double ln_pos(double x) {
    int e;
    double m = std::frexp(x, &e);  // x = m 2^e, m in [1/2, 1)
    if (m < 0.70710678118654752440) {
        m += m;
        --e;
    }
    return add_e_ln2(e, atanh2(m - 1.0, m + 1.0));  // m - 1 and m + 1 are exact
}

// Table-driven logarithm (the step's collision loop, where the table sits in
// LDS).  x = mm 2^e with mm in [1/2, 1) from frexp; bin j (0..255) = the top
// eight fraction bits of mm.  Bins below sqrt(1/2) (j < 106) take the reduced
// argument m = 2 mm and exponent e - 1, the others m = mm; each bin stores
// c_j = (m / mm) / m_j and t_j = ln m_j for its centre m_j (m_j = 1 for the
// two bins next to m = 1, so that ln x is exact in its leading term there).
// Then r = mm c_j - 1 (one rounding; |r| < 2^-8) and
// ln x = (e or e - 1) ln 2 + t_j + ln(1 + r), the last by its series through
// r^7 (relative truncation below 2^-58).
struct LnEntry {
    double c, t;
};
constexpr int kLnBins = 256, kLnDoubled = 106;

// The table, in extended precision on the host (c_j rounded once, t_j the
// logarithm of the centre that c_j stands for).
MC_H void ln_table_fill(LnEntry *tab) {
    for (int j = 0; j < kLnBins; ++j) {
        const long double lo = 0.5L + (long double)j / (2 * kLnBins), centre = lo + 1.0L / (4 * kLnBins);
        const long double scale = j < kLnDoubled ? 2.0L : 1.0L;  // m / mm
        long double mj = scale * centre;
        if (j == 0 || j == kLnBins - 1) mj = 1.0L;                 // bins next to m = 1
        tab[j].c = (double)(scale / mj);
        tab[j].t = (double)logl(scale / (long double)tab[j].c);  // ln of the centre c_j stands for
    }
}

// ln(1 + r) - r = r^2 (-1/2 + r/3 - r^2/4 + ... + r^5/7) for |r| < 2^-8.
MC_HD double log1p_small(double r) {
    double q = 1.0 / 7.0;
    q = std::fma(q, r, -1.0 / 6.0);
    q = std::fma(q, r, 1.0 / 5.0);
    q = std::fma(q, r, -1.0 / 4.0);
    q = std::fma(q, r, 1.0 / 3.0);
    q = std::fma(q, r, -0.5);
    return std::fma(r * r, q, r);
}

// Bin of the frexp mantissa mm in [1/2, 1): its top eight fraction bits.
MC_HD int ln_bin(double mm) {
    uint64_t b;
    std::memcpy(&b, &mm, sizeof b);
    return (int)((b >> 44) & (kLnBins - 1));
}

// ln x for x > 0 normal and finite, with the table above.
MC_HD double ln_tab(double x, const LnEntry *tab) {
    int e;
    const double mm = std::frexp(x, &e);
    const int j = ln_bin(mm);
    const LnEntry en = tab[j];
    const double r = std::fma(mm, en.c, -1.0);
    return add_e_ln2(j < kLnDoubled ? e - 1 : e, en.t + log1p_small(r));
}

// ln(1 + x) for x >= 0 with the table: ln y for y = 1 + x rounded, plus the
// first-order correction (x - (y - 1)) / y for the rounding of y (exact
// subtraction; at most 2^-53 relative to y, so a reciprocal estimate is ample);
// +inf gives +inf.
MC_HD double ln1p_tab(double x, const LnEntry *tab) {
    const double y = 1.0 + x;
    int e;
    const double mm = std::frexp(y, &e);
    const int j = ln_bin(mm);
    const LnEntry en = tab[j];
    const double r = std::fma(mm, en.c, -1.0);
#if defined(__HIP_DEVICE_COMPILE__)
    const double ry = __builtin_amdgcn_rcp(y);
#else
    const double ry = 1.0 / y;
#endif
    const double corr = (x - (y - 1.0)) * ry;
    const double v = add_e_ln2(j < kLnDoubled ? e - 1 : e, en.t + (log1p_small(r) + corr));
    return y < HUGE_VAL ? v : y;
}

// sin(2 pi u) and cos(2 pi u) for 0 <= u <= 1.  q = rint(4u) is the nearest
// quarter turn and t = u - q/4 (exact, |t| <= 1/8); th = 2 pi t is formed with
// 2 pi split into a double head and tail, and |th| <= pi/4.  Taylor series:
// sin th through th^17/17! and cos th through th^16/16!, whose next terms are
// below 2^-62 of the result on that interval.  The quarter turn then swaps
// and signs the pair: (sin, cos)(q pi/2 + th) = (s, c), (c, -s), (-s, -c),
// (-c, s) for q = 0, 1, 2, 3 (mod 4).
MC_HD void sincos_turn(double u, double *sn, double *cs) {
    const double q = std::rint(4.0 * u);
    const double t = std::fma(-0.25, q, u);
    const double two_pi_hi = 6.283185307179586;       // 2 pi rounded to double
    const double two_pi_lo = 2.4492935982947064e-16;  // 2 pi - two_pi_hi
    const double th = std::fma(t, two_pi_hi, t * two_pi_lo);
    const double z = th * th;
    double ps = 1.0 / 355687428096000.0;  // 1/17!
    ps = std::fma(ps, z, -1.0 / 1307674368000.0);
    ps = std::fma(ps, z, 1.0 / 6227020800.0);
    ps = std::fma(ps, z, -1.0 / 39916800.0);
    ps = std::fma(ps, z, 1.0 / 362880.0);
    ps = std::fma(ps, z, -1.0 / 5040.0);
    ps = std::fma(ps, z, 1.0 / 120.0);
    ps = std::fma(ps, z, -1.0 / 6.0);
    const double s = std::fma(th * z, ps, th);
    double pc = 1.0 / 20922789888000.0;  // 1/16!
    pc = std::fma(pc, z, -1.0 / 87178291200.0);
    pc = std::fma(pc, z, 1.0 / 479001600.0);
    pc = std::fma(pc, z, -1.0 / 3628800.0);
    pc = std::fma(pc, z, 1.0 / 40320.0);
    pc = std::fma(pc, z, -1.0 / 720.0);
    pc = std::fma(pc, z, 1.0 / 24.0);
    pc = std::fma(pc, z, -0.5);
    const double c = std::fma(z, pc, 1.0);
    const int k = (int)q & 3;
    const double a = (k & 1) ? c : s, b = (k & 1) ? s : c;
    *sn = (k & 2) ? -a : a;
    *cs = ((k + 1) & 2) ? -b : b;
}

MC_HD double cos_turn(double u) {
    double s, c;
    sincos_turn(u, &s, &c);
    return c;
}

// Table-driven sine and cosine of a turn (the step's collision loop, where
// the table sits in LDS).  Node j = rint(256 u) (mod 256) holds sin and cos of
// 2 pi j / 256 (exact zeros and units at the quarter turns); t = u - j/256 is
// exact and |t| <= 1/512, so d = 2 pi t is at most pi/256 and
// sin(2 pi u) = S_j + S_j (cos d - 1) + C_j sin d and
// cos(2 pi u) = C_j + C_j (cos d - 1) - S_j sin d, with sin d through d^7/7!
// and cos d - 1 through d^6/6! (next terms below 2^-60 of the result).
struct TurnEntry {
    double s, c;
};
constexpr int kTurnBins = 256;

MC_H void turn_table_fill(TurnEntry *tab) {
    const long double two_pi = 6.28318530717958647692528676655900577L;
    for (int j = 0; j < kTurnBins; ++j) {
        tab[j].s = (double)sinl(two_pi * j / kTurnBins);
        tab[j].c = (double)cosl(two_pi * j / kTurnBins);
    }
    tab[0].s = tab[kTurnBins / 2].s = 0.0;  // exact at the quarter turns
    tab[kTurnBins / 4].c = tab[3 * kTurnBins / 4].c = 0.0;
    tab[0].c = tab[kTurnBins / 4].s = 1.0;
    tab[kTurnBins / 2].c = tab[3 * kTurnBins / 4].s = -1.0;
}

MC_HD void sincos_turn_tab(double u, const TurnEntry *tab, double *sn, double *cs) {
    const double q = std::rint(u * (double)kTurnBins);
    const double t = std::fma(q, -1.0 / kTurnBins, u);
    const double two_pi_hi = 6.283185307179586;       // 2 pi rounded to double
    const double two_pi_lo = 2.4492935982947064e-16;  // 2 pi - two_pi_hi
    const double d = std::fma(t, two_pi_hi, t * two_pi_lo);
    const double z = d * d;
    double ps = -1.0 / 5040.0;
    ps = std::fma(ps, z, 1.0 / 120.0);
    ps = std::fma(ps, z, -1.0 / 6.0);
    const double sd = std::fma(d * z, ps, d);
    double pc = -1.0 / 720.0;
    pc = std::fma(pc, z, 1.0 / 24.0);
    pc = std::fma(pc, z, -0.5);
    const double cm1 = z * pc;  // cos d - 1
    const TurnEntry en = tab[(int)q & (kTurnBins - 1)];
    // the node's value plus the small corrections, added last
    *sn = en.s + std::fma(en.s, cm1, en.c * sd);
    *cs = en.c + std::fma(en.c, cm1, -(en.s * sd));
}

MC_HD double cos_turn_tab(double u, const TurnEntry *tab) {
    double s, c;
    sincos_turn_tab(u, tab, &s, &c);
    return c;
}

// Both tables of the FP64 step (8 KB), filled on the host.
struct StepTables {
    LnEntry ln[kLnBins];
    TurnEntry turn[kTurnBins];
};

MC_H void step_tables_fill(StepTables *t) {
    ln_table_fill(t->ln);
    turn_table_fill(t->turn);
}

}  // namespace mc

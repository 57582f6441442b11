// mc_math64.hpp -- double-precision elementary functions for the arguments
// the FP64 step takes, written from their series.
//
// The general library functions handle every input (denormals, infinities,
// NaN, arguments of any size) and cost about 100 (logarithm), 130 (log1p) and
// 65 (sine and cosine of pi x) instructions.  The collision loop takes, per
// candidate, three or four logarithms of uniform variates or their products
// in (0, 1], two sine/cosine pairs and a cosine of 2 pi u for uniform u, and
// (in the internal-energy exchange) a log1p of a positive ratio.  These
// restricted versions stay within 2 ulp there (log1p 2.5; tested on the host
// against extended-precision references) in a third to a half of the
// instructions.
//
//   div_mid(n, d)        n / d for d in [1, 4), |n| < 1 (its quotient step)
//   ln_pos(x)            natural logarithm, x > 0 normal and finite
//   ln1p_pos(x)          ln(1 + x), x >= 0 (+inf gives +inf)
//   sincos_turn(u, s, c) sin(2 pi u), cos(2 pi u), 0 <= u <= 1
//   cos_turn(u)          cos(2 pi u), 0 <= u <= 1
//
// Plain C++ (host and device).
#pragma once
#include <cmath>

#if defined(__HIPCC__)
#define MC_HD __host__ __device__ __forceinline__
#else
#define MC_HD inline
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

// ln(1 + x) for x >= 0.  With y = 1 + x rounded, y = m 2^e as in ln_pos:
// for e = 0 (x < sqrt 2 - 1) ln(1 + x) = 2 atanh(x / (2 + x)) exactly, which
// keeps full relative precision for small x; otherwise ln y plus the
// first-order correction for the rounding of y, (x - (y - 1)) / y, which is at
// most 2^-53 against a result of at least ln(sqrt 2) (a reciprocal estimate is
// ample for it).
MC_HD double ln1p_pos(double x) {
    const double y = 1.0 + x;
    int e;
    double m = std::frexp(y, &e);
    if (m < 0.70710678118654752440) {
        m += m;
        --e;
    }
    const bool small = e == 0;
#if defined(__HIP_DEVICE_COMPILE__)
    const double ry = __builtin_amdgcn_rcp(y);
#else
    const double ry = 1.0 / y;
#endif
    const double corr = small ? 0.0 : (x - (y - 1.0)) * ry;
    const double r = add_e_ln2(e, atanh2(small ? x : m - 1.0, small ? 2.0 + x : m + 1.0) + corr);
    return y < HUGE_VAL ? r : y;
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

}  // namespace mc

// mc_device.hpp -- device-side building blocks of the ion-pack step on gfx950.
//
// Precision policies (P64: FP64 state, math and tables; P32: FP32 math,
// two-float positions and internal energy, BF16 or FP32 tables with a
// per-table scale), the Philox4x32-10 counter generator, uniform and normal
// draws, bilinear table access and the Einstein heat-capacity conversion.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mc_math64.hpp"

namespace mc {

// Exact SI constants and CODATA 2022 values.
constexpr double kB = 1.380649e-23;
constexpr double kQe = 1.602176634e-19;
constexpr double kH = 6.62607015e-34;
constexpr double kNA = 6.02214076e23;
constexpr double kEps0 = 8.8541878188e-12;
constexpr double kDa = 1.66053906892e-27;
constexpr double kPi = 3.14159265358979323846;

enum : int32_t { ST_ACTIVE = 0, ST_TRANSMITTED = 1, ST_ELECTRODE = 2, ST_RADIAL = 3, ST_AXIAL = 4, ST_NUMERIC = 5 };

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64 products
// with multipliers 0xD2511F53 and 0xCD9E8D57, key bumped by the Weyl
// constants 0x9E3779B9 / 0xBB67AE85 after each round.  The key is uniform
// across a wavefront, so the key schedule lives in scalar registers.
// Stream layout: counter = (pack id low 32, step, purpose << 24 | block,
// pack id high 32); purpose 0 = emission, 1 = collisions, 2 = Langevin.
// ---------------------------------------------------------------------------
struct W4 {
    uint32_t w0, w1, w2, w3;
};

// a ^ b ^ c as one three-input bitwise instruction (truth table 0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ W4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)0xD2511F53u * c0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * c2;
        // the first rounds still mix words that are the same across the
        // wavefront (step, purpose and block, the key and what the first
        // products make of them): plain XORs there let the compiler keep those
        // in scalar instructions; the three-input XOR takes the rounds where
        // both mixed words differ per lane
        const uint32_t n0 = r <= 1 ? ((uint32_t)(pb >> 32) ^ c1 ^ k0) : xor3((uint32_t)(pb >> 32), c1, k0);
        const uint32_t n2 = r <= 2 ? ((uint32_t)(pa >> 32) ^ c3 ^ k1) : xor3((uint32_t)(pa >> 32), c3, k1);
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return W4{c0, c1, c2, c3};
}

constexpr uint32_t kPurposeEmit = 0u, kPurposeCollide = 1u, kPurposeLangevin = 2u;

__device__ __forceinline__ W4 draw(int64_t id, int64_t step, uint32_t purpose, uint32_t block, uint32_t k0,
                                   uint32_t k1) {
    return philox((uint32_t)((uint64_t)id), (uint32_t)step, (purpose << 24) | block, (uint32_t)((uint64_t)id >> 32),
                  k0, k1);
}

// ---------------------------------------------------------------------------
// Precision policies.
// ---------------------------------------------------------------------------
// The FP64 step's tables in the block's LDS (logarithm and turn tables):
// loaded by the kernels that take the step (P::prepare_tables), which are
// their only readers.
static __shared__ StepTables g_tables;

struct P64 {
    using T = double;
    static constexpr bool kTwo = false;
    // every thread of the block calls this before the first table read
    // (ln_fast, log1p_, sc2pi_fast, cos2pi_fast)
    static __device__ __forceinline__ void prepare_tables(const StepTables *src) {
        static_assert(sizeof(StepTables) % sizeof(double2) == 0, "tables move in 16-byte pieces");
        const double2 *from = reinterpret_cast<const double2 *>(src);
        double2 *to = reinterpret_cast<double2 *>(&g_tables);
        for (int k = threadIdx.x; k < (int)(sizeof(StepTables) / sizeof(double2)); k += blockDim.x) to[k] = from[k];
        __syncthreads();
    }
    // one 32-bit word -> (0,1): (w + 1/2) 2^-32, exact in double (an add of an
    // inline constant and an exponent shift: no 64-bit constant in a register)
    static __device__ __forceinline__ double u01(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }
    // every call site passes x in (0, 1] (uniform variates and their products)
    static __device__ __forceinline__ double ln(double x) { return ln_pos(x); }
    // the same from the block's table (step kernels, after prepare_ln)
    static __device__ __forceinline__ double ln_fast(double x) { return ln_tab(x, g_tables.ln); }
    // x >= 0 and zero or normal at every call site: the hardware reciprocal
    // square root estimate (within 2^-23) refined by sqrt_seeded
    static __device__ __forceinline__ double sqrt_(double x) { return sqrt_seeded(x, __builtin_amdgcn_rsq(x)); }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
    // 1/x for x positive and normal: the hardware estimate refined by
    // recip_seeded (within 1 ulp)
    static __device__ __forceinline__ double rcp(double x) { return recip_seeded(x, __builtin_amdgcn_rcp(x)); }
    static __device__ __forceinline__ double exp_(double x) { return exp(x); }
    // every call site passes a positive ratio (the Einstein-model inverse,
    // called in the step kernels only, after prepare_ln)
    static __device__ __forceinline__ double log1p_(double x) { return ln1p_tab(x, g_tables.ln); }
    // sin(2 pi u), cos(2 pi u) of uniform variates u in (0, 1): a quarter-turn
    // reduction and two short series instead of the library's general reduction
    static __device__ __forceinline__ void sc2pi(double u, double *s, double *c) { sincos_turn(u, s, c); }
    static __device__ __forceinline__ double cos2pi(double u) { return cos_turn(u); }
    // the same from the block's turn table (step kernels, after prepare_tables)
    static __device__ __forceinline__ void sc2pi_fast(double u, double *s, double *c) {
        sincos_turn_tab(u, g_tables.turn, s, c);
    }
    static __device__ __forceinline__ double cos2pi_fast(double u) { return cos_turn_tab(u, g_tables.turn); }
};

// FP32 form: the hardware transcendental instructions (v_log_f32 = log2,
// v_exp_f32 = 2^x, v_sin/cos_f32 take revolutions, v_sqrt_f32, v_rcp_f32).
struct P32 {
    using T = float;
    static constexpr bool kTwo = true;
    // the top 24 bits of the same word: ((w >> 8) + 1/2) 2^-24, exact in float
    static __device__ __forceinline__ float u01(uint32_t w) {
        return __builtin_fmaf((float)(w >> 8), 0x1p-24f, 0x1p-25f);  // exact
    }
    static __device__ __forceinline__ void prepare_tables(const StepTables *) {}
    static __device__ __forceinline__ float ln(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945f; }
    static __device__ __forceinline__ float ln_fast(float x) { return ln(x); }
    static __device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float exp_(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896f); }
    static __device__ __forceinline__ float log1p_(float x) { return ln(1.0f + x); }
    static __device__ __forceinline__ void sc2pi(float u, float *s, float *c) {
        *s = __builtin_amdgcn_sinf(u);
        *c = __builtin_amdgcn_cosf(u);
    }
    static __device__ __forceinline__ float cos2pi(float u) { return __builtin_amdgcn_cosf(u); }
    static __device__ __forceinline__ void sc2pi_fast(float u, float *s, float *c) { sc2pi(u, s, c); }
    static __device__ __forceinline__ float cos2pi_fast(float u) { return cos2pi(u); }
};

// Error-free sum a + b = s + e (Knuth), for two-float accumulation.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e) {
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// (hi, lo) += d, renormalised.  (The FP64 overload is a plain sum.)
__device__ __forceinline__ void acc2(double &hi, double &, double d) { hi += d; }
__device__ __forceinline__ void acc2(float &hi, float &lo, float d) {
    float s, e;
    two_sum(hi, d, s, e);
    e += lo;
    hi = s + e;
    lo = e - (hi - s);
}

// ---------------------------------------------------------------------------
// Field tables.  Four channels per node, node-interleaved so one bilinear
// gather reads four 32-byte (FP64), 16-byte (FP32) or 8-byte (BF16) nodes.
//   E table:   (E_S,r, E_S,z, E_RF,r, E_RF,z)   E_S = E_DC + V_off E_OFF + E_SC
//   gas table: (u_r, u_z, p, T)
// ---------------------------------------------------------------------------
struct bf16x4 {
    uint16_t a, b, c, d;
};

__device__ __forceinline__ float bf16_to_f(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }

template <class T>
struct Q4 {
    T a, b, c, d;
};

__device__ __forceinline__ Q4<double> load4(const double4 *t, int64_t k, const float *) {
    const double4 v = t[k];
    return Q4<double>{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ Q4<float> load4(const float4 *t, int64_t k, const float *) {
    const float4 v = t[k];
    return Q4<float>{v.x, v.y, v.z, v.w};
}
// BF16 records are read unscaled; gather4 applies the channel scales once,
// after the interpolation (a scale is linear in the record values)
__device__ __forceinline__ Q4<float> load4(const bf16x4 *t, int64_t k, const float *) {
    const bf16x4 v = t[k];
    return Q4<float>{bf16_to_f(v.a), bf16_to_f(v.b), bf16_to_f(v.c), bf16_to_f(v.d)};
}

// Cell location with clamping (constant extension outside the grid).
template <class T>
struct Cell {
    int32_t i, j;
    T f, g;
};

template <class T>
__device__ __forceinline__ Cell<T> locate(T r, T z, T inv_dr, T inv_dz, int32_t nr, int32_t nz) {
    const T ur = r * inv_dr, uz = z * inv_dz;
    T fi = floor(ur), fj = floor(uz);
    fi = fmin(fmax(fi, (T)0), (T)(nr - 2));
    fj = fmin(fmax(fj, (T)0), (T)(nz - 2));
    Cell<T> c;
    c.f = fmin(fmax(ur - fi, (T)0), (T)1);
    c.g = fmin(fmax(uz - fj, (T)0), (T)1);
    c.i = (int32_t)fi;
    c.j = (int32_t)fj;
    return c;
}

// The four nodes of one table cell, (i, j), (i+1, j), (i, j+1), (i+1, j+1).
template <class T>
struct Nodes4 {
    Q4<T> t00, t10, t01, t11;
};

template <class T, class Tab>
__device__ __forceinline__ Nodes4<T> load_nodes(const Tab *tab, const float *sc, int32_t i, int32_t j, int32_t nr) {
    const int64_t k = (int64_t)j * nr + i;
    return Nodes4<T>{load4(tab, k, sc), load4(tab, k + 1, sc), load4(tab, k + nr, sc), load4(tab, k + nr + 1, sc)};
}

// Bilinear interpolation of a cell's nodes at the cell fractions (f, g).
template <class T>
__device__ __forceinline__ Q4<T> interp(const Nodes4<T> &n, const Cell<T> &c) {
    const T w00 = ((T)1 - c.f) * ((T)1 - c.g), w10 = c.f * ((T)1 - c.g);
    const T w01 = ((T)1 - c.f) * c.g, w11 = c.f * c.g;
    Q4<T> o;
    o.a = w00 * n.t00.a + w10 * n.t10.a + w01 * n.t01.a + w11 * n.t11.a;
    o.b = w00 * n.t00.b + w10 * n.t10.b + w01 * n.t01.b + w11 * n.t11.b;
    o.c = w00 * n.t00.c + w10 * n.t10.c + w01 * n.t01.c + w11 * n.t11.c;
    o.d = w00 * n.t00.d + w10 * n.t10.d + w01 * n.t01.d + w11 * n.t11.d;
    return o;
}

template <class T, class Tab>
__device__ __forceinline__ Q4<T> gather4(const Tab *tab, const float *sc, const Cell<T> &c, int32_t nr) {
    Q4<T> q = interp(load_nodes<T>(tab, sc, c.i, c.j, nr), c);
    if constexpr (sizeof(Tab) == sizeof(bf16x4)) {
        q.a *= sc[0];
        q.b *= sc[1];
        q.c *= sc[2];
        q.d *= sc[3];
    }
    return q;
}

// Einstein model inverse: T = theta / ln(1 + s kB theta / U).  FP64 form:
// both quotients by the refined reciprocal (each within one unit in the
// last place) for a normal U, by division for a subnormal one (whose
// reciprocal the hardware estimate does not cover).
template <class P>
__device__ __forceinline__ typename P::T einstein_t(typename P::T e, typename P::T skt, typename P::T theta) {
    using T = typename P::T;
    if constexpr (!P::kTwo) {
        if (e >= 0x1p-1022) return theta * P::rcp(P::log1p_(skt * P::rcp(e)));
    }
    return e > (T)0 ? P::div(theta, P::log1p_(P::div(skt, e))) : (T)0;
}

// Dissociation rate k(T) = A T^p exp(-B / T): Eyring (p = 1, A = kB/h e^{dS/R},
// B = dH/R) or Arrhenius (p = 0, A, B = Ea/kB).
template <class P>
__device__ __forceinline__ typename P::T rate(int32_t kind, typename P::T a, typename P::T b, typename P::T t) {
    using T = typename P::T;
    if (kind == 0 || !(t > (T)0)) return (T)0;
    const T e = P::exp_(-P::div(b, t));
    return kind == 1 ? a * t * e : a * e;
}

// Per-species constants resolved on the host at mc_define_ion/mc_set_operating.
struct Species {
    double m, qm, ccs, alpha, theta, skt, act_a, act_b, e0;
    int32_t act_kind, n_atoms;
};

// 32-bit DPP move of v (row_mask selects the rows that take the moved value;
// lanes whose source is outside the row, and rows not selected, read 0).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, kRowMask, 0xf, true);
}

// Sum of v over the 64 lanes of a wavefront whose lanes are all active, in
// every lane: an inclusive scan within each row of 16 lanes (shifts 1, 2, 4,
// 8), the row totals carried across rows (broadcasts of lanes 15 and 31),
// then lane 63 read into a scalar.  Modulo 2^32.
__device__ __forceinline__ uint32_t wave_total_u32(uint32_t v) {
    v += dpp_u32<0x111, 0xf>(v);  // row_shr:1
    v += dpp_u32<0x112, 0xf>(v);  // row_shr:2
    v += dpp_u32<0x114, 0xf>(v);  // row_shr:4
    v += dpp_u32<0x118, 0xf>(v);  // row_shr:8
    v += dpp_u32<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_u32<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

}  // namespace mc

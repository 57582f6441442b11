// mc_kernels.hpp -- HIP kernels of the ion-pack step (gfx950).
//
//   k_emit      source emission: truncated Gaussian radius, gas-flow plus
//               Maxwellian velocity (Eq. 5 and the Gaussian-source section)
//   k_step      fused per-pack step: RK4 push in E_S + c(t) E_RF (Eqs. 3-4),
//               terminal classification, collisions (Eq. 6, thinning with
//               internal-energy exchange), dissociation hazard (Eq. 7),
//               terminal tallies (Eq. 8)
//   k_deposit   int64 cloud-in-cell deposit (PIC section)
//   k_bake, k_fold  E = -grad(phi) on nodes; folded static field table
//               (k_bake_fold: both in one pass, the space-charge update)
//   k_hit       electrode hit table from the mask and hit distance
//   k_snapshot  read-time tallies of the active population
//
// The library is compiled with FMA contraction within each source
// expression (-ffp-contract=on), so the kernels that inline the same step
// code round alike; the blocks whose results
// must be reproducible bit for bit on any IEEE implementation given the same
// positions (classification, deposit, hit table, histogram bins) switch it
// off locally with `#pragma clang fp contract(off)`.
#pragma once
#include "../../include/mucite.h"
#include "mc_device.hpp"

namespace mc {

template <class T>
struct PackPtrs {
    T *x, *y, *z;      // position (high part in the two-float form)
    T *xl, *yl, *zl;   // low parts (two-float form only)
    T *vx, *vy, *vz;
    T *e, *el;         // internal energy (high, low)
    T *h;              // dissociation hazard H = integral k(T_eff) dt
    double *w;         // weight [real ions]
    int64_t *id, *q;   // pack id (random-stream key), charge [2^-32 e]
    int32_t *tag, *status;
};

// int64 tally block.  Layout of cnt: class_n[6], class_w[6], n_cand, n_coll,
// n_cap, n_clamp, pack_steps, exit_overflow, exit_dropped, exit_count,
// n_langevin, n_exchange.
enum { TC_CLASS_N = 0, TC_CLASS_W = 6, TC_CAND = 12, TC_COLL = 13, TC_CAP = 14, TC_CLAMP = 15, TC_PACKSTEPS = 16,
       TC_EXOVER = 17, TC_EXDROP = 18, TC_EXCOUNT = 19, TC_LANG = 20, TC_EXCH = 21, TC_N = 22 };

// Per-step event counters (pack steps, candidates, collisions, caps, clamps,
// Langevin steps, internal-energy exchanges): each block adds its totals to one of kHotRep replicas,
// one 128-byte line each, so concurrent blocks rarely update the same
// address; readers add the replicas into the counters (fold_hot).
enum { HOT_PACKSTEPS = 0, HOT_CAND = 1, HOT_COLL = 2, HOT_CAP = 3, HOT_CLAMP = 4, HOT_LANG = 5, HOT_EXCH = 6, HOT_N = 7 };
constexpr int kHotRep = 128, kHotStride = 16;
constexpr int64_t kHotLen = (int64_t)kHotRep * kHotStride;

// Offset of the replicated counters in a tally array whose other regions
// take `base` words (rounded up to whole 128-byte lines).
inline int64_t hot_offset(int64_t base) { return (base + kHotStride - 1) / kHotStride * kHotStride; }

inline void fold_hot(const unsigned long long *hot, unsigned long long *cnt) {
    static const int to[HOT_N] = {TC_PACKSTEPS, TC_CAND, TC_COLL, TC_CAP, TC_CLAMP, TC_LANG, TC_EXCH};
    for (int r = 0; r < kHotRep; ++r)
        for (int k = 0; k < HOT_N; ++k) cnt[to[k]] += hot[(int64_t)r * kHotStride + k];
}

struct TallyPtrs {
    unsigned long long *cnt, *exit_bins, *loss_map, *hist_ke, *hist_teff, *hist_r, *hot;
    mc_exit_rec *exits;
    int64_t exit_cap;
};

// ---------------------------------------------------------------------------
// Histogram bins: KE log10 bins over [1e-3, 1e3] eV, T_eff over [0, 5000] K,
// exit radius over [0, r_det]; bin 0 = underflow, last = overflow.  The
// ranges are published by mc_get_tally_layout.
// ---------------------------------------------------------------------------
constexpr double kKeLog10Lo = -3.0, kKeLog10Hi = 3.0, kTeffLo = 0.0, kTeffHi = 5000.0;
constexpr int kKeBins = MC_HIST_KE - 2, kTeffBins = MC_HIST_TEFF - 2, kRBins = MC_HIST_R - 2;

__device__ __forceinline__ int hbin_ke(double ke_ev) {
#pragma clang fp contract(off)
    if (!(ke_ev > 0.0)) return 0;
    const double u = (log10(ke_ev) - kKeLog10Lo) * ((double)kKeBins / (kKeLog10Hi - kKeLog10Lo));
    if (!(u >= 0.0)) return 0;
    if (u >= (double)kKeBins) return kKeBins + 1;
    return 1 + (int)floor(u);
}
__device__ __forceinline__ int hbin_teff(double t) {
#pragma clang fp contract(off)
    const double u = (t - kTeffLo) * ((double)kTeffBins / (kTeffHi - kTeffLo));
    if (!(u >= 0.0)) return 0;
    if (u >= (double)kTeffBins) return kTeffBins + 1;
    return 1 + (int)floor(u);
}
__device__ __forceinline__ int hbin_r(double r, double rdet) {
#pragma clang fp contract(off)
    const double u = r / rdet * (double)kRBins;
    if (!(u >= 0.0)) return 0;
    if (u >= (double)kRBins) return kRBins + 1;
    return 1 + (int)floor(u);
}

__device__ __forceinline__ void atom_add(unsigned long long *p, int64_t v) { atomicAdd(p, (unsigned long long)v); }

__device__ __forceinline__ int64_t fx32(double v) { return (int64_t)rint(ldexp(v, 32)); }

// ---------------------------------------------------------------------------
// Emission.
// ---------------------------------------------------------------------------
template <class P, class Tab>
struct EmitArgs {
    PackPtrs<typename P::T> p;
    const Tab *gtab;
    float gsc[4];
    const Species *sp;
    int64_t slot0, count, id0, step;
    double sigma_r, r_trunc, z_inj, w;
    int64_t q;
    double inv_dr, inv_dz;
    int32_t nr, nz, ion;
    uint32_t k0, k1;
};

template <class P, class Tab>
__device__ __forceinline__ void emit_one(const EmitArgs<P, Tab> &a, int64_t k) {
    using T = typename P::T;
    const int64_t id = a.id0 + k, s = a.slot0 + k;
    const W4 wa = draw(id, a.step, kPurposeEmit, 0u, a.k0, a.k1);
    const W4 wb = draw(id, a.step, kPurposeEmit, 1u, a.k0, a.k1);
    const Species sp = a.sp[a.ion];
    // radius of a Gaussian truncated at r_trunc by inversion, uniform azimuth
    const T sg = (T)a.sigma_r, rt = (T)a.r_trunc;
    const T r = sg * P::sqrt_((T)-2 * P::ln((T)1 - P::u01(wa.w0) * ((T)1 - P::exp_(-P::div(rt * rt, (T)2 * sg * sg)))));
    T sph, cph;
    P::sc2pi(P::u01(wa.w1), &sph, &cph);
    const T z = (T)a.z_inj;
    const Cell<T> c = locate<T>(r, z, (T)a.inv_dr, (T)a.inv_dz, a.nr, a.nz);
    const Q4<T> g = gather4<T>(a.gtab, a.gsc, c, a.nr);
    // gas flow plus the ion's Maxwellian at the local gas temperature
    const T vth = P::sqrt_(P::div((T)kB * g.d, (T)sp.m));
    const T r1 = P::sqrt_((T)-2 * P::ln(P::u01(wa.w2))), r2 = P::sqrt_((T)-2 * P::ln(P::u01(wb.w0)));
    T s1, c1, s2, c2;
    P::sc2pi(P::u01(wa.w3), &s1, &c1);
    P::sc2pi(P::u01(wb.w1), &s2, &c2);
    a.p.x[s] = r * cph;
    a.p.y[s] = r * sph;
    a.p.z[s] = z;
    const T ehi = (T)sp.e0;
    a.p.e[s] = ehi;
    if constexpr (P::kTwo) {
        a.p.xl[s] = 0;
        a.p.yl[s] = 0;
        a.p.zl[s] = 0;
        a.p.el[s] = (T)(sp.e0 - (double)ehi);
    }
    a.p.vx[s] = g.a * cph + vth * r1 * c1;
    a.p.vy[s] = g.a * sph + vth * r1 * s1;
    a.p.vz[s] = g.b + vth * r2 * c2;
    a.p.h[s] = 0;
    a.p.w[s] = a.w;
    a.p.id[s] = id;
    a.p.q[s] = a.q;
    a.p.tag[s] = a.ion;
    a.p.status[s] = ST_ACTIVE;
}

template <class P, class Tab>
__global__ __launch_bounds__(256) void k_emit(EmitArgs<P, Tab> a) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < a.count) emit_one(a, k);
}

// Query owning a block in a multi-query launch: prefix[q] is the first block of
// query q, prefix[nq] the total (uniform per block, so this is scalar code).
__device__ __forceinline__ int block_query(const int32_t *prefix, int32_t nq) {
    int lo = 0, hi = nq - 1;
    const int b = (int)blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <class P, class Tab>
__global__ __launch_bounds__(256) void k_emit_multi(const EmitArgs<P, Tab> *descs, const int32_t *prefix,
                                                    int32_t nq) {
    const int q = block_query(prefix, nq);
    const EmitArgs<P, Tab> &a = descs[q];
    const int64_t k = (int64_t)(blockIdx.x - prefix[q]) * blockDim.x + threadIdx.x;
    if (k < a.count) emit_one(a, k);
}

// ---------------------------------------------------------------------------
// Fused step.
// ---------------------------------------------------------------------------
template <class P, class Tab>
struct StepArgs {
    PackPtrs<typename P::T> p;
    const Tab *etab, *gtab;
    float esc[4], gsc[4];
    const uint8_t *hit;
    const Species *sp;
    TallyPtrs t;
    int64_t n_slots, step;
    double dt, t0, c0, ch, c1;      // c = V_RF cos(2 pi f t + phase) at t0, t0 + dt/2, t0 + dt
    double z_det, r_det, R, inv_dr, inv_dz, mg, exit_bin_dt;
    int32_t nr, nz, n_exit_bins, collisions_on;
    int32_t langevin_on;
    double lv_z_lo, lv_z_hi, lv_switch, lv_dt_ref;  // switch: lambda lv_dt_ref >= lv_switch
    uint32_t k0, k1;
    const StepTables *tables;  // the FP64 step's logarithm and turn tables (device memory)
    // adaptive step kept on the device: the step record written by
    // k_dt_finish -- (t0, dt, c0, ch, c1) of this step, then t0 and c0 of
    // the next -- read in place of the fields above; null with a fixed step
    const double *dyn;
};

// Total field of Eq. 4 at (x, y, z), radial part projected by Eq. 3.
template <class P, class Tab>
__device__ __forceinline__ void efield(const StepArgs<P, Tab> &a, typename P::T x, typename P::T y,
                                       typename P::T z, typename P::T c, typename P::T &ex, typename P::T &ey,
                                       typename P::T &ez) {
    using T = typename P::T;
    const T r = P::sqrt_(x * x + y * y);
    const Cell<T> cl = locate<T>(r, z, (T)a.inv_dr, (T)a.inv_dz, a.nr, a.nz);
    const Q4<T> q = gather4<T>(a.etab, a.esc, cl, a.nr);
    const T er = q.a + c * q.c;
    ez = q.b + c * q.d;
    const T s = r > (T)0 ? P::div(er, r) : (T)0;
    ex = s * x;
    ey = s * y;
}

// Terminal event: int64 tallies (class weights, Eq. 8 exit-current bins,
// loss map, histograms) and one exit record.
template <class P, class Tab>
__device__ __forceinline__ void record_exit(const StepArgs<P, Tab> &a, int64_t s, int32_t cls, int32_t in,
                                            int32_t jn, double x, double y, double z, double vx, double vy,
                                            double vz, double tc, double rc, double eint, double h,
                                            const Species &sp) {
#pragma clang fp contract(off)
    const double w = a.p.w[s];
    const int64_t wfx = fx32(w);
    atom_add(&a.t.cnt[TC_CLASS_N + cls], 1);
    atom_add(&a.t.cnt[TC_CLASS_W + cls], wfx);
    const double ke = 0.5 * sp.m * (vx * vx + vy * vy + vz * vz);
    const double te = eint > 0.0 ? sp.theta / log1p(sp.skt / eint) : 0.0;
    if (cls == ST_ELECTRODE) atom_add(&a.t.loss_map[(int64_t)jn * a.nr + in], wfx);
    if (cls == ST_TRANSMITTED) {
        const double u = tc / a.exit_bin_dt;
        if (u >= 0.0 && u < (double)a.n_exit_bins) atom_add(&a.t.exit_bins[(int64_t)floor(u)], wfx);
        else atom_add(&a.t.cnt[TC_EXOVER], wfx);
        atom_add(&a.t.hist_ke[hbin_ke(ke / kQe)], wfx);
        atom_add(&a.t.hist_teff[hbin_teff(te)], wfx);
        atom_add(&a.t.hist_r[hbin_r(rc, a.r_det)], wfx);
    }
    const unsigned long long slot = atomicAdd(&a.t.cnt[TC_EXCOUNT], 1ull);
    if ((int64_t)slot < a.t.exit_cap) {
        mc_exit_rec *r = &a.t.exits[slot];
        r->id = a.p.id[s];
        r->step = a.step;
        r->cls = cls;
        r->inode = in;
        r->jnode = jn;
        r->tag = a.p.tag[s];
        r->x = x; r->y = y; r->z = z;
        r->vx = vx; r->vy = vy; r->vz = vz;
        r->t_cross = tc;
        r->r_cross = rc;
        r->ke_ev = ke / kQe;
        r->t_eff = te;
        r->h = h;
        r->w = w;
    } else {
        atom_add(&a.t.cnt[TC_EXDROP], 1);
    }
}

// Per thread and step: act, cap and lang are 0 or 1; a pack draws at most
// 8000064 candidates (the loop's cap), so a wavefront's sums stay below 2^29.
struct StepCount {
    uint32_t cand, acc, cap, clamp, act, lang, exch;
};

// Per pack and step.
struct PackCount {
    uint32_t cand, acc, cap, clamp, lang, exch;
};

// Gas at a pack's post-push position ("Gas field and electrode mask
// coupling"): flow velocity projected by Eq. 3, temperature, and n_gas sigma
// of the pack's species (zero where there is no gas).
template <class T>
struct GasAt {
    T ux, uy, uz, tg, ngs;
    bool gas;
};

template <class P, class Tab>
__device__ __forceinline__ GasAt<typename P::T> gas_at(const StepArgs<P, Tab> &a, const Species &sp,
                                                       typename P::T rr, typename P::T x1, typename P::T y1,
                                                       typename P::T z1) {
    using T = typename P::T;
    const T m = (T)sp.m, ccs = (T)sp.ccs;
    const Cell<T> cl = locate<T>(rr, z1, (T)a.inv_dr, (T)a.inv_dz, a.nr, a.nz);
    const Q4<T> g = gather4<T>(a.gtab, a.gsc, cl, a.nr);
    const T sr = rr > (T)0 ? P::div(g.a, rr) : (T)0;
    GasAt<T> o;
    o.ux = sr * x1;
    o.uy = sr * y1;
    o.uz = g.b;
    o.tg = g.d;
    // n_gas * sigma.  FP32 form: evaluated on every lane and then
    // selected, so that all four gas components and the cross-section
    // are read at once rather than behind a branch on the temperature
    // (its quotient is one reciprocal); FP64: the division stays behind
    // the branch, where the compiler keeps it without stack use
    if constexpr (P::kTwo) {
        const T ngs_any = P::div(g.c, (T)kB * (o.tg > (T)0 ? o.tg : (T)1)) * ccs;
        o.ngs = o.tg > (T)0 ? ngs_any : (T)0;
    } else {
        o.ngs = o.tg > (T)0 ? P::div(g.c, (T)kB * o.tg) * ccs : (T)0;
    }
    // (FP32 form: the mass, positive by definition, enters the test so
    // that its read is issued with the gas gather instead of after it)
    o.gas = P::kTwo ? (o.ngs > (T)0) & (bool)isfinite(o.ngs) & (m > (T)0) : o.ngs > (T)0 && isfinite(o.ngs);
    return o;
}

// Whether a pack takes the hybrid Langevin branch this step: the branch is
// on, its post-push z lies in the window (or there is none), and its
// candidate rate lambda = n sigma (s + abar) reaches the switch
// (lambda dt_ref >= lv_switch).
template <class P, class Tab>
__device__ __forceinline__ bool takes_langevin(const StepArgs<P, Tab> &a, double Z1, typename P::T lam) {
    using T = typename P::T;
    return a.langevin_on && (!(a.lv_z_hi > a.lv_z_lo) || (Z1 >= a.lv_z_lo && Z1 < a.lv_z_hi)) &&
           lam * (T)a.lv_dt_ref >= (T)a.lv_switch;
}

// Hybrid Langevin branch: exact Ornstein-Uhlenbeck relaxation of v toward
// the gas velocity over dt, hard-sphere friction rate, Box-Muller normals
// from one block.
template <class P, class Tab>
__device__ __forceinline__ void langevin_relax(const StepArgs<P, Tab> &a, const Species &sp, int64_t id,
                                               uint32_t k0, uint32_t k1, const GasAt<typename P::T> &g,
                                               typename P::T &vx, typename P::T &vy, typename P::T &vz) {
    using T = typename P::T;
    const T dt = (T)a.dt, m = (T)sp.m, mg = (T)a.mg;
    const T fm = P::div(mg, m + mg);
    const W4 w = draw(id, a.step, kPurposeLangevin, 0u, k0, k1);
    const T r0 = P::sqrt_((T)-2 * P::ln_fast(P::u01(w.w0)));
    const T r1 = P::sqrt_((T)-2 * P::ln_fast(P::u01(w.w2)));
    T s0, c0;
    P::sc2pi_fast(P::u01(w.w1), &s0, &c0);
    const T c1 = P::cos2pi_fast(P::u01(w.w3));
    const T ktm = P::div((T)kB * g.tg, m);  // kB T / m (no underflow in FP32)
    const T gam = (T)(16.0 / 3.0) * g.ngs * P::sqrt_(fm * ktm * (T)0.15915494309189535);
    const T f = P::exp_(-gam * dt);
    const T sd = P::sqrt_(ktm * ((T)1 - f * f));
    vx = g.ux + (vx - g.ux) * f + sd * (r0 * c0);
    vy = g.uy + (vy - g.uy) * f + sd * (r0 * s0);
    vz = g.uz + (vz - g.uz) * f + sd * (r1 * c1);
}

// The explicit collision loop of one pack over one step (Eq. 6 and the
// collision paragraph): sequential exponential waits at lambda =
// n sigma (s + abar), partner from the two-branch mixture, acceptance
// |g|/(s + |w|), impulsive hard-sphere update with the internal-energy
// exchange.  Entered with s, lambda and v - u of the post-push state.
template <class P, class Tab>
__device__ __forceinline__ void collide_explicit(const StepArgs<P, Tab> &a, const Species &sp, int64_t id,
                                                 uint32_t k0, uint32_t k1, const GasAt<typename P::T> &g,
                                                 typename P::T ag, typename P::T abar, typename P::T sv,
                                                 typename P::T lam, typename P::T &vx, typename P::T &vy,
                                                 typename P::T &vz, typename P::T &e, typename P::T &el,
                                                 PackCount &pc) {
    using T = typename P::T;
    const T dt = (T)a.dt, m = (T)sp.m, mg = (T)a.mg;
    const T M = m + mg, fm = P::div(mg, M), fi = P::div(m, M), mu = mg * fi;  // no m*mg product (FP32 range)
    const T two_mu = P::div((T)2, mu);
    const T alpha = (T)sp.alpha, skt = (T)sp.skt, theta = (T)sp.theta;
    const T alpha2 = alpha * alpha;
    const T ux = g.ux, uy = g.uy, uz = g.uz, ngs = g.ngs;
    T rx = vx - ux, ry = vy - uy, rz = vz - uz;
    // candidate cap; a non-finite rate ends the loop at once
    const T nexp = lam * dt;
    const int32_t cap = (nexp < (T)1e6) ? 64 + 8 * (int32_t)ceil(nexp) : (nexp >= (T)1e6 ? 8000064 : 0);
    T tleft = dt;
    T inv_lam = P::rcp(lam);  // the waits' scale, refreshed with the rate
    for (int32_t c = 0;; ++c) {
        if (c == cap) {
            ++pc.cap;
            break;
        }
        const W4 wa = draw(id, a.step, kPurposeCollide, (uint32_t)(3 * c), k0, k1);
        const T tau = -P::ln_fast(P::u01(wa.w0)) * inv_lam;
        if (!(tau < tleft)) break;
        tleft -= tau;
        ++pc.cand;
        const W4 wb = draw(id, a.step, kPurposeCollide, (uint32_t)(3 * c + 1), k0, k1);
        // partner thermal velocity: E = |w|^2/(2 a^2) ~ Gamma(3/2) (Maxwellian branch)
        // or Gamma(2) (flux-weighted branch), isotropic direction; no divergent branch
        const bool maxw = P::u01(wa.w1) * (sv + abar) < sv;  // u < s/(s + abar)
        const T cc = P::cos2pi_fast(P::u01(wb.w0));
        const T en = -P::ln_fast(P::u01(wa.w2)) - P::ln_fast(P::u01(wa.w3)) * (maxw ? cc * cc : (T)1);
        const T wn = ag * P::sqrt_((T)2 * en);
        const T ct = (T)2 * P::u01(wb.w1) - (T)1;
        const T st = P::sqrt_(fmax((T)0, (T)1 - ct * ct));
        T sph, cph;
        P::sc2pi_fast(P::u01(wb.w2), &sph, &cph);
        const T wx = wn * st * cph, wy = wn * st * sph, wz = wn * ct;
        const T gx = rx - wx, gy = ry - wy, gz = rz - wz;
        const T g2 = gx * gx + gy * gy + gz * gz;
        // acceptance u (s + |w|) < |g| and the exchange select u (s + |w|) <
        // alpha |g|, both sides non-negative: compared squared, with no root
        const T lhs = P::u01(wb.w3) * (sv + wn);
        const T lhs2 = lhs * lhs;
        if (!(lhs2 < g2)) continue;
        ++pc.acc;
        const W4 wc = draw(id, a.step, kPurposeCollide, (uint32_t)(3 * c + 2), k0, k1);
        // centre of mass of the ion and the partner (lab velocity u + w)
        const T vcx = fi * vx + fm * (ux + wx), vcy = fi * vy + fm * (uy + wy), vcz = fi * vz + fm * (uz + wz);
        const T et = (T)0.5 * mu * g2;
        T etp = et;
        // exchange select: the acceptance residual, uniform given acceptance
        if (lhs2 < alpha2 * g2) {  // residual u (s + |w|)/|g| < alpha
            ++pc.exch;
            const T te = einstein_t<P>(e + el, skt, theta);
            etp = -(T)kB * te * P::ln_fast(P::u01(wc.w2) * P::u01(wc.w3));
            const T de = et - etp;
            if (e + el + de < (T)0) {
                etp = e + el + et;
                e = 0;
                el = 0;
                ++pc.clamp;
            } else {
                acc2(e, el, de);
            }
        }
        const T cchi = (T)2 * P::u01(wc.w0) - (T)1;
        const T schi = P::sqrt_(fmax((T)0, (T)1 - cchi * cchi));
        T sps, cps;
        P::sc2pi_fast(P::u01(wc.w1), &sps, &cps);
        const T f = fm * P::sqrt_(etp * two_mu);
        vx = vcx + f * schi * cps;
        vy = vcy + f * schi * sps;
        vz = vcz + f * cchi;
        rx = vx - ux;
        ry = vy - uy;
        rz = vz - uz;
        sv = P::sqrt_(rx * rx + ry * ry + rz * rz);
        lam = ngs * (sv + abar);
        inv_lam = P::rcp(lam);
    }
}

// Eq. 7: hazard with the post-collision effective temperature.
template <class P, class Tab>
__device__ __forceinline__ void accumulate_hazard(const StepArgs<P, Tab> &a, const Species &sp, int64_t s,
                                                  typename P::T e, typename P::T el) {
    using T = typename P::T;
    const T te = einstein_t<P>(e + el, (T)sp.skt, (T)sp.theta);
    a.p.h[s] = a.p.h[s] + rate<P>(sp.act_kind, (T)sp.act_a, (T)sp.act_b, te) * (T)a.dt;
}

// One pack, one step.  kOneSpecies: every pack carries tag 0 (a context
// that defines one species, or a serving query), so the tag array is not
// read and the species record sits at one address for the whole wavefront
// (read through the scalar cache, not by a vector load that waits for the
// pack's tag: one dependent trip fewer before the push).
template <class P, class Tab, bool kOneSpecies>
__device__ __forceinline__ void step_one(const StepArgs<P, Tab> &a, int64_t s, StepCount &n, uint32_t k0, uint32_t k1) {
    using T = typename P::T;
    PackCount pc{0, 0, 0, 0, 0, 0};
    // the state is read together with the status word rather than after it
    // (one memory round trip fewer before the first field gather; a slot that
    // turns out inactive discards its reads)
    int32_t status = -1, tag = 0;
    T x0 = 0, y0 = 0, z0 = 0, xl = 0, yl = 0, zl = 0, vx0 = 0, vy0 = 0, vz0 = 0;
    // the random-stream key: in the FP32 form read with the state (a read
    // issued where the draws start would stall a Langevin step on memory a
    // second time); the FP64 form reads it where the draws start, which
    // keeps its registers free through the push
    int64_t id = 0;
    if (s < a.n_slots) {
        status = a.p.status[s];
        if constexpr (!kOneSpecies) tag = a.p.tag[s];
        x0 = a.p.x[s];
        y0 = a.p.y[s];
        z0 = a.p.z[s];
        if constexpr (P::kTwo) {
            xl = a.p.xl[s];
            yl = a.p.yl[s];
            zl = a.p.zl[s];
        }
        vx0 = a.p.vx[s];
        vy0 = a.p.vy[s];
        vz0 = a.p.vz[s];
        if constexpr (P::kTwo) id = a.p.id[s];
    }
    if (status == ST_ACTIVE) {
        n.act = 1;
        // the species record by reference, so each field is read where it is
        // used and the dissociation constants hold no registers through the
        // collision loop (at five waves in the FP32 form and three in the FP64
        // form they would spill)
        const Species &sp = a.sp[kOneSpecies ? 0 : tag];
        const T dt = (T)a.dt, qm = (T)sp.qm, hd = (T)0.5 * dt;
        const T xl0 = xl, yl0 = yl, zl0 = zl;

        // ---- classical RK4 on (x, v); stages at t, t + dt/2, t + dt/2, t + dt ----
        T ex, ey, ez;
        efield(a, x0, y0, z0, (T)a.c0, ex, ey, ez);
        T ax = qm * ex, ay = qm * ey, az = qm * ez;
        T sxx = vx0, sxy = vy0, sxz = vz0, svx = ax, svy = ay, svz = az;
        T kx = vx0 + hd * ax, ky = vy0 + hd * ay, kz = vz0 + hd * az;
        efield(a, x0 + (xl + hd * vx0), y0 + (yl + hd * vy0), z0 + (zl + hd * vz0), (T)a.ch, ex, ey, ez);
        ax = qm * ex; ay = qm * ey; az = qm * ez;
        sxx += (T)2 * kx; sxy += (T)2 * ky; sxz += (T)2 * kz;
        svx += (T)2 * ax; svy += (T)2 * ay; svz += (T)2 * az;
        const T k2x = kx, k2y = ky, k2z = kz;
        kx = vx0 + hd * ax; ky = vy0 + hd * ay; kz = vz0 + hd * az;
        efield(a, x0 + (xl + hd * k2x), y0 + (yl + hd * k2y), z0 + (zl + hd * k2z), (T)a.ch, ex, ey, ez);
        ax = qm * ex; ay = qm * ey; az = qm * ez;
        sxx += (T)2 * kx; sxy += (T)2 * ky; sxz += (T)2 * kz;
        svx += (T)2 * ax; svy += (T)2 * ay; svz += (T)2 * az;
        const T k3x = kx, k3y = ky, k3z = kz;
        kx = vx0 + dt * ax; ky = vy0 + dt * ay; kz = vz0 + dt * az;
        efield(a, x0 + (xl + dt * k3x), y0 + (yl + dt * k3y), z0 + (zl + dt * k3z), (T)a.c1, ex, ey, ez);
        ax = qm * ex; ay = qm * ey; az = qm * ez;
        sxx += kx; sxy += ky; sxz += kz;
        svx += ax; svy += ay; svz += az;
        const T d6 = dt / (T)6;
        T x1 = x0, y1 = y0, z1 = z0;
        acc2(x1, xl, d6 * sxx);
        acc2(y1, yl, d6 * sxy);
        acc2(z1, zl, d6 * sxz);
        T vx = vx0 + d6 * svx, vy = vy0 + d6 * svy, vz = vz0 + d6 * svz;

        // ---- terminal classification at the new position ----
        // (the FP64 form performs exactly the IEEE operations of its reference;
        // the two-float form classifies its full-precision position in FP64)
        const double X1 = (double)x1 + (double)xl, Y1 = (double)y1 + (double)yl, Z1 = (double)z1 + (double)zl;
        double r1;
        {
#pragma clang fp contract(off)
        r1 = sqrt(X1 * X1 + Y1 * Y1);
        }
        // the gas at the new position, gathered before the hit test so that
        // the two reads overlap (a pack that turns out terminal discards it;
        // the gather's cell is clamped, so any position reads in bounds)
        GasAt<T> g{};
        if (a.collisions_on) g = gas_at(a, sp, (T)r1, x1, y1, z1);
        int32_t cls = ST_ACTIVE, in = -1, jn = -1;
        double tcross = 0.0, rcross = 0.0;
        {
#pragma clang fp contract(off)
        const double X0 = (double)x0 + (double)xl0, Y0 = (double)y0 + (double)yl0, Zo = (double)z0 + (double)zl0;
        const bool finite = isfinite(X1) && isfinite(Y1) && isfinite(Z1) && isfinite((double)vx) &&
                            isfinite((double)vy) && isfinite((double)vz);
        if (!finite) {
            cls = ST_NUMERIC;
        } else if (Z1 >= a.z_det || Z1 < 0.0) {
            const double zp = Z1 >= a.z_det ? a.z_det : 0.0;
            const double fr = (Z1 != Zo) ? (zp - Zo) / (Z1 - Zo) : 1.0;
            const double xc = X0 + fr * (X1 - X0), yc = Y0 + fr * (Y1 - Y0);
            rcross = sqrt(xc * xc + yc * yc);
            tcross = a.t0 + fr * a.dt;
            cls = (Z1 >= a.z_det && rcross <= a.r_det) ? ST_TRANSMITTED : ST_AXIAL;
        } else if (r1 > a.R) {
            cls = ST_RADIAL;
        } else {
            const int32_t ii = (int32_t)floor(r1 * a.inv_dr + 0.5), jj = (int32_t)floor(Z1 * a.inv_dz + 0.5);
            if (ii < a.nr && jj < a.nz && a.hit[(int64_t)jj * a.nr + ii]) {
                cls = ST_ELECTRODE;
                in = ii;
                jn = jj;
            }
        }
        }

        // internal energy: read now unless the pack is in the Langevin window,
        // whose branch leaves it unchanged (then it is read only if the pack
        // turns out to need it, and not written back)
        T e = (T)0, el = (T)0;
        bool have_e = false;
        const auto read_e = [&]() {
            if (!have_e) {
                e = a.p.e[s];
                if constexpr (P::kTwo) el = a.p.el[s];
                have_e = true;
            }
        };
        if (!(a.langevin_on && (!(a.lv_z_hi > a.lv_z_lo) || (Z1 >= a.lv_z_lo && Z1 < a.lv_z_hi)))) read_e();

        // the position is final: store it now so it is not held through the collision loop
        a.p.x[s] = x1;
        a.p.y[s] = y1;
        a.p.z[s] = z1;
        if constexpr (P::kTwo) {
            a.p.xl[s] = xl;
            a.p.yl[s] = yl;
            a.p.zl[s] = zl;
        }
        bool lang = false;
        if (cls == ST_ACTIVE && a.collisions_on) {
            // ---- collisions with the gas at the new position ----
            if (g.gas) {
                const T ag = P::sqrt_(P::div((T)kB * g.tg, (T)a.mg));
                const T abar = ag * (T)1.5957691216057308;  // sqrt(8/pi)
                const T rx = vx - g.ux, ry = vy - g.uy, rz = vz - g.uz;
                const T sv = P::sqrt_(rx * rx + ry * ry + rz * rz);
                const T lam = g.ngs * (sv + abar);
                lang = takes_langevin(a, Z1, lam);
                if constexpr (!P::kTwo) {
                    if (!lang) id = a.p.id[s];
                }
                if (lang) {
                    langevin_relax(a, sp, P::kTwo ? id : a.p.id[s], k0, k1, g, vx, vy, vz);
                    ++pc.lang;
                } else {
                    read_e();
                    collide_explicit(a, sp, id, k0, k1, g, ag, abar, sv, lam, vx, vy, vz, e, el, pc);
                }
            }
        }
        if (cls == ST_ACTIVE) {
            // ---- Eq. 7: hazard with the post-collision effective temperature ----
            // (not accumulated in an aggregated Langevin step, which leaves the
            // internal energy as it was)
            if (!lang) {
                read_e();
                accumulate_hazard(a, sp, s, e, el);
                a.p.e[s] = e;
                if constexpr (P::kTwo) a.p.el[s] = el;
            }
        } else {
            read_e();
            record_exit(a, s, cls, in, jn, X1, Y1, Z1, (double)vx, (double)vy, (double)vz, tcross, rcross,
                        (double)e + (double)el, (double)a.p.h[s], sp);
            a.p.status[s] = cls;
        }
        a.p.vx[s] = vx;
        a.p.vy[s] = vy;
        a.p.vz[s] = vz;
    }
    n.cand = pc.cand;
    n.acc = pc.acc;
    n.cap = pc.cap;
    n.clamp = pc.clamp;
    n.lang = pc.lang;
    n.exch = pc.exch;
}

// Block-aggregated counters: wavefront sums, then (blocks of several
// wavefronts) LDS, then one atomic per counter and block into the block's
// replica (every thread of the block calls this; all of a block's threads
// belong to one query).  The 0/1
// counters are counted from the wavefront's ballot (scalar unit); the others
// are summed across lanes by DPP, skipped where the whole wavefront holds
// zero (a Langevin step draws no candidates).
__device__ __forceinline__ void flush_counts(const TallyPtrs &t, const StepCount &n) {
    const auto sum = [](uint32_t x) -> uint64_t { return __ballot(x != 0u) ? wave_total_u32(x) : 0u; };
    const uint64_t v[HOT_N] = {(uint64_t)__popcll(__ballot(n.act != 0u)),
                               sum(n.cand),
                               sum(n.acc),
                               (uint64_t)__popcll(__ballot(n.cap != 0u)),
                               sum(n.clamp),
                               (uint64_t)__popcll(__ballot(n.lang != 0u)),
                               sum(n.exch)};
    unsigned long long *rep = t.hot + (int64_t)(blockIdx.x & (kHotRep - 1)) * kHotStride;
    if (blockDim.x == 64) {  // a block of one wavefront adds its sums straight into its replica
        if (threadIdx.x == 0) {
#pragma unroll
            for (int k = 0; k < HOT_N; ++k)
                if (v[k]) atomicAdd(&rep[k], (unsigned long long)v[k]);
        }
        return;
    }
    __shared__ unsigned long long red[HOT_N];
    if (threadIdx.x < HOT_N) red[threadIdx.x] = 0ull;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < HOT_N; ++k)
            if (v[k]) atomicAdd(&red[k], (unsigned long long)v[k]);
    }
    __syncthreads();
    if (threadIdx.x < HOT_N && red[threadIdx.x]) atomicAdd(&rep[threadIdx.x], red[threadIdx.x]);
}

// Waves per SIMD the step kernel is compiled for (its register budget):
// the FP64 form holds its loop state in register pairs and runs three waves
// in 143 registers (three measured 3 % faster than two and 2 % faster than
// four, which spill); the FP32 form with BF16
// tables fits five.  Neither spills.
template <class P, class Tab>
constexpr int step_waves() {
    return P::kTwo ? (sizeof(Tab) == 8 ? 5 : 4) : 3;
}

template <class P, class Tab, bool kOneSpecies>
__global__ __launch_bounds__(256, (step_waves<P, Tab>())) void k_step(StepArgs<P, Tab> a) {
    if (a.dyn) {
        // the step's time, length and RF stage coefficients from the device
        // record; a zero length marks an adaptive run halted by a collapsed
        // step (every thread returns: no barrier is left waiting)
        if (!(a.dyn[1] > 0.0)) return;
        a.t0 = a.dyn[0];
        a.dt = a.dyn[1];
        a.c0 = a.dyn[2];
        a.ch = a.dyn[3];
        a.c1 = a.dyn[4];
    }
    P::prepare_tables(a.tables);
    StepCount n{0, 0, 0, 0, 0, 0, 0};
    step_one<P, Tab, kOneSpecies>(a, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, n, a.k0, a.k1);
    flush_counts(a.t, n);
}

// ---------------------------------------------------------------------------
// Adaptive step (Eq. 1): the per-pack limits at the start of a step (state at
// t0, RF coefficient c0), minimised over the block and added into one of
// kHotRep replica lines: word 0 holds the limit's bits (positive doubles
// order like their bit patterns), word 1 flags a pack on the Langevin
// branch.  Per pack: half a spacing over |v|; a tenth of the speed scale
// |v - u| + sqrt(kB T/m) over |qE/m| (the time to move half a spacing from
// rest when there is no speed scale); 0.1 / lambda on the explicit branch.
// ---------------------------------------------------------------------------
constexpr unsigned long long kInfBits = 0x7FF0000000000000ull;

template <class P, class Tab>
__global__ __launch_bounds__(256) void k_dt_limits(StepArgs<P, Tab> a, unsigned long long *rep) {
    using T = typename P::T;
    __shared__ double red[256];
    __shared__ int any_lang;
    if (threadIdx.x == 0) any_lang = 0;
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double lim = HUGE_VAL;
    if (s < a.n_slots && a.p.status[s] == ST_ACTIVE) {
        const Species sp = a.sp[a.p.tag[s]];
        const T x = a.p.x[s], y = a.p.y[s], z = a.p.z[s];
        double Z = (double)z;
        if constexpr (P::kTwo) Z += (double)a.p.zl[s];
        const T vx = a.p.vx[s], vy = a.p.vy[s], vz = a.p.vz[s];
        const T h = (T)(1.0 / fmax(a.inv_dr, a.inv_dz));
        const T vn = P::sqrt_(vx * vx + vy * vy + vz * vz);
        if (vn > (T)0) lim = fmin(lim, (double)((T)0.5 * P::div(h, vn)));
        T ex, ey, ez;
        efield(a, x, y, z, (T)(a.dyn ? a.dyn[6] : a.c0), ex, ey, ez);
        const T an = (T)fabs(sp.qm) * P::sqrt_(ex * ex + ey * ey + ez * ez);
        const T rr = P::sqrt_(x * x + y * y);
        const Cell<T> cl = locate<T>(rr, z, (T)a.inv_dr, (T)a.inv_dz, a.nr, a.nz);
        const Q4<T> g = gather4<T>(a.gtab, a.gsc, cl, a.nr);
        const T sr = rr > (T)0 ? P::div(g.a, rr) : (T)0;
        const T rx = vx - sr * x, ry = vy - sr * y, rz = vz - g.b, tg = g.d;
        const T sv = P::sqrt_(rx * rx + ry * ry + rz * rz);
        const T vth = tg > (T)0 ? P::sqrt_(P::div((T)kB * tg, (T)sp.m)) : (T)0;
        if (an > (T)0)
            lim = fmin(lim, (double)((sv + vth) > (T)0 ? (T)0.1 * P::div(sv + vth, an) : P::sqrt_(P::div(h, an))));
        const T ngs = tg > (T)0 ? P::div(g.c, (T)kB * tg) * (T)sp.ccs : (T)0;
        if (a.collisions_on && ngs > (T)0 && isfinite(ngs)) {
            const T abar = P::sqrt_(P::div((T)kB * tg, (T)a.mg)) * (T)1.5957691216057308;
            const T lam = ngs * (sv + abar);
            const bool in_window = !(a.lv_z_hi > a.lv_z_lo) || (Z >= a.lv_z_lo && Z < a.lv_z_hi);
            if (a.langevin_on && in_window && lam * (T)a.lv_dt_ref >= (T)a.lv_switch) atomicOr(&any_lang, 1);
            else if (lam > (T)0) lim = fmin(lim, (double)P::div((T)0.1, lam));
        }
    }
    red[threadIdx.x] = lim;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        unsigned long long *line = rep + (int64_t)(blockIdx.x & (kHotRep - 1)) * kHotStride;
        atomicMin(line, (unsigned long long)__double_as_longlong(red[0]));
        if (any_lang) atomicOr(line + 1, 1ull);
    }
}

// Replica lines -> out[0] (limit bits), out[1] (Langevin flag); the lines are
// reset for the next step.  One block of kHotRep threads.
static __global__ __launch_bounds__(kHotRep) void k_dt_reduce(unsigned long long *rep, unsigned long long *out) {
    __shared__ unsigned long long mn[kHotRep], fl[kHotRep];
    const int k = threadIdx.x;
    mn[k] = rep[(int64_t)k * kHotStride];
    fl[k] = rep[(int64_t)k * kHotStride + 1];
    rep[(int64_t)k * kHotStride] = kInfBits;
    rep[(int64_t)k * kHotStride + 1] = 0ull;
    __syncthreads();
    for (int w = kHotRep / 2; w > 0; w >>= 1) {
        if (k < w) {
            mn[k] = mn[k] < mn[k + w] ? mn[k] : mn[k + w];
            fl[k] |= fl[k + w];
        }
        __syncthreads();
    }
    if (k == 0) {
        out[0] = mn[0];
        out[1] = fl[0];
    }
}

// The adaptive step on the device (one block of kHotRep threads): the
// replica lines reduced as in k_dt_reduce, then
//   dt = min(dt_max, limit, rf_cap, lv_cap if a pack takes the Langevin
//            branch, t_pic - t0)
// (the caps are +inf where they do not apply), and the step record: this
// step's (t0, dt, c0, ch, c1) with c = V_RF cos(w2 t + phase) at t0, t0 +
// dt/2 and t0 + dt, then the next step's t0 = t0 + dt and c0.  A step below
// `collapse` halts the run: the record's length becomes zero (the step
// kernels return at once) and word 7 keeps 1 + the step index, the time
// staying at the collapsed step's start.
static __global__ __launch_bounds__(kHotRep) void k_dt_finish(unsigned long long *rep, double *rec, double dt_max,
                                                              double rf_cap, double lv_cap, double t_pic,
                                                              double collapse, double v_rf, double w2, double phase,
                                                              int64_t step) {
#pragma clang fp contract(off)
    __shared__ unsigned long long mn[kHotRep], fl[kHotRep];
    const int k = threadIdx.x;
    mn[k] = rep[(int64_t)k * kHotStride];
    fl[k] = rep[(int64_t)k * kHotStride + 1];
    rep[(int64_t)k * kHotStride] = kInfBits;
    rep[(int64_t)k * kHotStride + 1] = 0ull;
    __syncthreads();
    for (int w = kHotRep / 2; w > 0; w >>= 1) {
        if (k < w) {
            mn[k] = mn[k] < mn[k + w] ? mn[k] : mn[k + w];
            fl[k] |= fl[k + w];
        }
        __syncthreads();
    }
    if (k != 0) return;
    unsigned long long *halted = reinterpret_cast<unsigned long long *>(rec + 7);
    const double t0 = rec[5], c0 = rec[6];
    double d = fmin(dt_max, __longlong_as_double((long long)mn[0]));
    d = fmin(d, rf_cap);
    if (fl[0]) d = fmin(d, lv_cap);
    d = fmin(d, t_pic - t0);
    if (*halted || !(d > collapse)) {
        if (!*halted) *halted = (unsigned long long)step + 1ull;
        rec[1] = 0.0;
        return;
    }
    const double t1 = t0 + d;
    const double c1 = v_rf * cos(w2 * t1 + phase);
    rec[0] = t0;
    rec[1] = d;
    rec[2] = c0;
    rec[3] = v_rf * cos(w2 * (t0 + 0.5 * d) + phase);
    rec[4] = c1;
    rec[5] = t1;
    rec[6] = c1;
}

static __global__ __launch_bounds__(kHotRep) void k_dt_reset(unsigned long long *rep) {
    rep[(int64_t)threadIdx.x * kHotStride] = kInfBits;
    rep[(int64_t)threadIdx.x * kHotStride + 1] = 0ull;
}

// All resident queries of a server advance one step in one launch; each
// block belongs to one query (descriptors in device memory).
template <class P, class Tab>
__global__ __launch_bounds__(256, (step_waves<P, Tab>())) void k_step_multi(const StepArgs<P, Tab> *descs, const int32_t *prefix,
                                                    int32_t nq) {
    const int q = block_query(prefix, nq);
    const StepArgs<P, Tab> &a = descs[q];
    P::prepare_tables(a.tables);
    StepCount n{0, 0, 0, 0, 0, 0, 0};
    // the random key is the query's, the same for the whole block: scalar.
    // A query's packs all carry tag 0, but the one-species variant measured
    // slower here (serving throughput 1.90e9 -> 1.83e9 pack-steps/s), so the
    // record is read per pack as in a context with several species
    step_one<P, Tab, false>(a, (int64_t)(blockIdx.x - prefix[q]) * blockDim.x + threadIdx.x, n,
             __builtin_amdgcn_readfirstlane(a.k0), __builtin_amdgcn_readfirstlane(a.k1));
    flush_counts(a.t, n);
}

// ---------------------------------------------------------------------------
// CIC deposit: bilinear split of the int64 pack charge, exact per pack:
//   a = rint(Q (1-f)), b = Q - a, a0 = rint(a (1-g)), a1 = a - a0,
//   b0 = rint(b (1-g)), b1 = b - b0.
// ---------------------------------------------------------------------------
template <class T>
struct DepositArgs {
    PackPtrs<T> p;
    unsigned long long *q;     // the grid (when qrep is null: the blocks' sums go here)
    unsigned long long *qrep;  // nrep zeroed copies of the grid, or null
    int32_t *range;            // lowest and highest node written (with qrep)
    int64_t n_slots, nn;
    int64_t chunk;             // slots per sub-range (a multiple of the block size; see k_deposit)
    double inv_dr, inv_dz;
    int32_t nr, nz, nrep;
};

// Block-local aggregation: each block sums its packs' contributions in an
// LDS hash table (open addressing) keyed by the CIC cell, i.e. the cell's
// lower-left node: one compare-and-swap per insertion, the four quanta added
// to the entry's four slots (lower-left, upper-left, lower-right,
// upper-right), and one device atomic per nonzero slot at the flush.
//
// Each block takes one contiguous range of `chunk` slots (a multiple of the
// block size), so that sorted slots give each block a few cells that few
// other blocks share (when the ranges were dealt out in several pieces per
// block, the flushes of more blocks met on each cell and the deposit of
// sorted packs ran at half the speed).  A thread sums the quanta
// of its consecutive packs while they stay in one cell and inserts the sums
// when the cell changes; at the end, where the runs of a wavefront's 64
// lanes all lie in one cell, their sums are added across the wavefront in
// registers (DPP row shifts and row broadcasts, no LDS traffic) and one
// lane inserts them.  Once the slots are sorted by cell -- a cell then
// holds thousands of consecutive packs -- a block makes a handful of
// insertions; unsorted, about one per pack.  Packs of the source region concentrate
// in a few cells, so when the slots are not sorted the blocks' flushes meet
// on the same few hundred addresses: the caller may then give nrep zeroed
// copies of the grid, block b flushing into copy b mod nrep, and
// k_deposit_sum adds the copies over the node range the blocks wrote (and
// clears them for the next update).  Integer sums make the result
// independent of the order.
constexpr int kDepHash = 2048;
// Grid of the deposit: one block of 16 wavefronts per CU, each thread
// reading two packs per pass with their loads issued together.
constexpr int64_t kDepositBlocks = 256;
constexpr int kDepositThreads = 1024, kDepositUnroll = 2;
// Copies of the grid for the flush: 16, fewer on grids where 16 copies would
// pass 64 MiB.
constexpr int64_t kDepositRepBytes = 64ll << 20;
constexpr int32_t kDepositMaxCopies = 16;
inline int32_t deposit_copies(int64_t nn) {
    const int64_t r = kDepositRepBytes / (8 * nn);
    return (int32_t)(r >= kDepositMaxCopies ? kDepositMaxCopies : r < 1 ? 1 : r);
}
// Launch shape for n slots: blocks, and the slots of each block's range (a
// multiple of the block size).
inline void deposit_shape(int64_t n, unsigned *nb, int64_t *chunk) {
    const int64_t b = (n + kDepositThreads - 1) / kDepositThreads;
    *nb = (unsigned)(b < 1 ? 1 : (b > kDepositBlocks ? kDepositBlocks : b));
    const int64_t c = (n + *nb - 1) / *nb;
    *chunk = (c + kDepositThreads - 1) / kDepositThreads * kDepositThreads;
}

// One pack's cell and its four quanta (k = -1 when the position is not
// finite):
//   a = rint(Q (1-f)), b = Q - a, a0 = rint(a (1-g)), a1 = a - a0,
//   b0 = rint(b (1-g)), b1 = b - b0.
__device__ __forceinline__ void dep_split(double X, double Y, double Z, int64_t Q, double inv_dr, double inv_dz,
                                          int32_t nr, int32_t nz, int32_t &k, int64_t &a0, int64_t &a1,
                                          int64_t &b0, int64_t &b1) {
#pragma clang fp contract(off)
    k = -1;
    a0 = a1 = b0 = b1 = 0;
    if (!isfinite(X) || !isfinite(Y) || !isfinite(Z)) return;
    const double r = sqrt(X * X + Y * Y);
    const double ur = r * inv_dr, uz = Z * inv_dz;
    double fi = floor(ur), fj = floor(uz);
    if (fi > (double)(nr - 2)) fi = (double)(nr - 2);
    if (fj > (double)(nz - 2)) fj = (double)(nz - 2);
    if (fj < 0.0) fj = 0.0;
    double f = ur - fi, g = uz - fj;
    if (f > 1.0) f = 1.0;
    if (g > 1.0) g = 1.0;
    if (g < 0.0) g = 0.0;
    const int64_t qa = (int64_t)rint((double)Q * (1.0 - f)), qb = Q - qa;
    a0 = (int64_t)rint((double)qa * (1.0 - g));
    a1 = qa - a0;
    b0 = (int64_t)rint((double)qb * (1.0 - g));
    b1 = qb - b0;
    k = (int32_t)fj * nr + (int32_t)fi;
}

// Quanta of cell k into the block's table (or, when its probes find no
// room, straight into the grid or its copy).
__device__ __forceinline__ void dep_insert(int32_t *keys, unsigned long long *vals, unsigned long long *grid,
                                           int32_t k, int32_t nr, int64_t a0, int64_t a1, int64_t b0, int64_t b1) {
    uint32_t h = ((uint32_t)k * 2654435761u) >> (32 - 11);
    for (int probe = 0; probe < 8; ++probe) {
        const int32_t old = atomicCAS(&keys[h], -1, k);
        if (old == -1 || old == k) {
            unsigned long long *v = vals + 4 * h;
            if (a0) atomicAdd(&v[0], (unsigned long long)a0);
            if (a1) atomicAdd(&v[1], (unsigned long long)a1);
            if (b0) atomicAdd(&v[2], (unsigned long long)b0);
            if (b1) atomicAdd(&v[3], (unsigned long long)b1);
            return;
        }
        h = (h + 1) & (kDepHash - 1);
    }
    if (a0) atom_add(&grid[k], a0);
    if (a1) atom_add(&grid[k + nr], a1);
    if (b0) atom_add(&grid[k + 1], b0);
    if (b1) atom_add(&grid[k + nr + 1], b1);
}

// 64-bit DPP move of v (row_mask selects the rows that take the moved value;
// lanes whose source is outside the row, and rows not selected, read 0).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, kCtrl, kRowMask, 0xf, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), kCtrl, kRowMask, 0xf, true);
    return ((uint64_t)hi << 32) | lo;
}

// Sum of v over the 64 lanes of a wavefront whose lanes are all active: an
// inclusive scan within each row of 16 lanes (shifts 1, 2, 4, 8), then the
// row totals carried across rows (broadcasts of lanes 15 and 31), which
// leaves the total in lane 63.  Modulo 2^64, like the int64 grid.
__device__ __forceinline__ uint64_t wave_total_u64(uint64_t v) {
    v += dpp_u64<0x111, 0xf>(v);  // row_shr:1
    v += dpp_u64<0x112, 0xf>(v);  // row_shr:2
    v += dpp_u64<0x114, 0xf>(v);  // row_shr:4
    v += dpp_u64<0x118, 0xf>(v);  // row_shr:8
    v += dpp_u64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_u64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

template <class P>
__global__ __launch_bounds__(kDepositThreads) void k_deposit(DepositArgs<typename P::T> a) {
    using T = typename P::T;
    __shared__ int32_t keys[kDepHash];
    __shared__ unsigned long long vals[4 * kDepHash];
    __shared__ int32_t blo, bhi;
    for (int k = threadIdx.x; k < kDepHash; k += blockDim.x) {
        keys[k] = -1;
        vals[4 * k] = vals[4 * k + 1] = vals[4 * k + 2] = vals[4 * k + 3] = 0ull;
    }
    if (threadIdx.x == 0) {
        blo = INT32_MAX;
        bhi = -1;
    }
    __syncthreads();
    unsigned long long *dst = a.qrep ? a.qrep + (int64_t)(blockIdx.x % (unsigned)a.nrep) * a.nn : a.q;
    const int lane = threadIdx.x & 63;
    int32_t lo = INT32_MAX, hi = -1;
    // the block's range in rows of blockDim.x slots; every wavefront of the
    // block runs the same passes (its lanes stay together for the wavefront
    // sums at the end)
    const int64_t rows = a.chunk / blockDim.x, base = (int64_t)blockIdx.x * a.chunk;
    const int64_t npass = (rows + kDepositUnroll - 1) / kDepositUnroll;
    // the thread's run: consecutive packs of the thread in one cell are
    // summed in registers and inserted once, when the cell changes or at the
    // end (sorted slots: a cell holds thousands of consecutive packs)
    int32_t rk = -1;
    int64_t r0 = 0, r1 = 0, r2 = 0, r3 = 0;
    for (int64_t ps = 0; ps < npass; ++ps) {
        // the pass's reads first (a slot past the end reads nothing), then its packs
        int32_t st[kDepositUnroll];
        T x[kDepositUnroll], y[kDepositUnroll], z[kDepositUnroll], xl[kDepositUnroll], yl[kDepositUnroll],
            zl[kDepositUnroll];
        int64_t q[kDepositUnroll];
#pragma unroll
        for (int u = 0; u < kDepositUnroll; ++u) {
            const int64_t r = ps * kDepositUnroll + u;
            const int64_t s = base + r * blockDim.x + threadIdx.x;
            st[u] = -1;
            x[u] = y[u] = z[u] = xl[u] = yl[u] = zl[u] = (T)0;
            q[u] = 0;
            if (r < rows && s < a.n_slots) {
                st[u] = a.p.status[s];
                x[u] = a.p.x[s];
                y[u] = a.p.y[s];
                z[u] = a.p.z[s];
                if constexpr (P::kTwo) {
                    xl[u] = a.p.xl[s];
                    yl[u] = a.p.yl[s];
                    zl[u] = a.p.zl[s];
                }
                q[u] = a.p.q[s];
            }
        }
#pragma unroll
        for (int u = 0; u < kDepositUnroll; ++u) {
            if (st[u] != ST_ACTIVE) continue;
            double X = x[u], Y = y[u], Z = z[u];
            if constexpr (P::kTwo) {
                X += (double)xl[u];
                Y += (double)yl[u];
                Z += (double)zl[u];
            }
            int32_t k;
            int64_t a0, a1, c0, c1;
            dep_split(X, Y, Z, q[u], a.inv_dr, a.inv_dz, a.nr, a.nz, k, a0, a1, c0, c1);
            if (k < 0) continue;
            lo = min(lo, k);
            hi = max(hi, k + a.nr + 1);
            if (k != rk) {
                if (rk >= 0) dep_insert(keys, vals, dst, rk, a.nr, r0, r1, r2, r3);
                rk = k;
                r0 = r1 = r2 = r3 = 0;
            }
            r0 += a0;
            r1 += a1;
            r2 += c0;
            r3 += c1;
        }
    }
    // the runs left at the end: one insertion of the wavefront's sums when
    // all of its runs lie in one cell, else one per lane
    {
        const uint64_t act = __ballot(rk >= 0);
        if (act != 0ull) {
            const int lead = __builtin_ctzll(act);
            const int32_t kl = __builtin_amdgcn_readlane(rk, lead);
            if (__ballot(rk == kl || rk < 0) == ~0ull) {
                const uint64_t s00 = wave_total_u64((uint64_t)r0), s01 = wave_total_u64((uint64_t)r1),
                               s10 = wave_total_u64((uint64_t)r2), s11 = wave_total_u64((uint64_t)r3);
                if (lane == lead)
                    dep_insert(keys, vals, dst, kl, a.nr, (int64_t)s00, (int64_t)s01, (int64_t)s10, (int64_t)s11);
            } else if (rk >= 0) {
                dep_insert(keys, vals, dst, rk, a.nr, r0, r1, r2, r3);
            }
        }
    }
    if (a.range) {
        // lowest and highest node over the wavefront first: one LDS atomic per
        // wavefront instead of one per thread on the same two words
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lo = min(lo, __shfl_xor(lo, o, 64));
            hi = max(hi, __shfl_xor(hi, o, 64));
        }
        if (lane == 0 && hi >= 0) {
            atomicMin(&blo, lo);
            atomicMax(&bhi, hi);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kDepHash; k += blockDim.x)
        if (keys[k] >= 0) {
            const int64_t c = keys[k], off[4] = {0, a.nr, 1, a.nr + 1};
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (vals[4 * k + j] != 0ull) atomicAdd(&dst[c + off[j]], vals[4 * k + j]);
        }
    if (a.range && threadIdx.x == 0 && bhi >= 0) {
        atomicMin(&a.range[0], blo);
        atomicMax(&a.range[1], bhi);
    }
}

// The grid from the copies: q[n] = the sum of the copies' values at n for n
// in the range this deposit wrote (range; the copies are cleared there, after
// all of the thread's loads have been issued; nrep <= kDepositMaxCopies), 0
// elsewhere.  Only the nodes in the span of this range and of the previous
// deposit's (prev) are written -- the grid is zero outside the previous
// range already -- or every node when prev is null.  Grid-stride; the first
// thread also resets the range slot `next` for the deposit after this one.
static __global__ __launch_bounds__(256) void k_deposit_sum(unsigned long long *q, unsigned long long *qrep,
                                                            int32_t nrep, int64_t nn, const int32_t *range,
                                                            const int32_t *prev, int32_t *next) {
    int64_t n0 = 0, n1 = nn - 1;
    if (prev) {
        n0 = min((int64_t)range[0], (int64_t)prev[0]);
        n1 = max((int64_t)range[1], (int64_t)prev[1]);
        n1 = min(n1, nn - 1);
    }
    const int32_t lo = range[0], hi = range[1];
    for (int64_t n = n0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n <= n1;
         n += (int64_t)gridDim.x * blockDim.x) {
        unsigned long long v = 0ull;
        if (n >= lo && n <= hi) {
            unsigned long long w[kDepositMaxCopies];
#pragma unroll
            for (int32_t c = 0; c < kDepositMaxCopies; ++c) w[c] = c < nrep ? qrep[(int64_t)c * nn + n] : 0ull;
#pragma unroll
            for (int32_t c = 0; c < kDepositMaxCopies; ++c) v += w[c];
#pragma unroll
            for (int32_t c = 0; c < kDepositMaxCopies; ++c)
                if (c < nrep) qrep[(int64_t)c * nn + n] = 0ull;
        }
        q[n] = v;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        next[0] = INT32_MAX;
        next[1] = -1;
    }
}

// Blocks of the sum kernel: enough to cover a 1M-node grid in one sweep of
// 256-thread blocks, grid-stride beyond.
constexpr int64_t kDepositSumBlocks = 4096;

// E = -grad(phi) on nodes: central differences, one-sided at the outer
// edges, E_r = 0 on the axis.  clear (nullable): a charge grid zeroed on
// the way, for the next deposit that adds into it.
// E = -grad Phi at node n (central differences, one-sided at the ends, zero
// radial field on the axis).
__device__ __forceinline__ double2 sc_field_at(const double *phi, int64_t n, int32_t nr, int32_t nz, double dr,
                                              double dz) {
    const int32_t i = (int32_t)(n % nr), j = (int32_t)(n / nr);
    double vr, vz;
    if (i == 0) vr = 0.0;
    else if (i == nr - 1) vr = -(phi[n] - phi[n - 1]) / dr;
    else vr = -(phi[n + 1] - phi[n - 1]) / (2.0 * dr);
    if (j == 0) vz = -(phi[n + nr] - phi[n]) / dz;
    else if (j == nz - 1) vz = -(phi[n] - phi[n - nr]) / dz;
    else vz = -(phi[n + nr] - phi[n - nr]) / (2.0 * dz);
    return make_double2(vr, vz);
}

static __global__ __launch_bounds__(256) void k_bake(const double *phi, double2 *e, int32_t nr, int32_t nz, double dr,
                                                     double dz, unsigned long long *clear) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)nr * nz) return;
    if (clear) clear[n] = 0ull;
    e[n] = sc_field_at(phi, n, nr, nz, dr, dz);
}

// Folded static table: (E_DC + V_off E_OFF + E_SC, E_RF), converted to the
// table format with per-channel scales.
__device__ __forceinline__ void put4(double4 *t, int64_t n, double a, double b, double c, double d, const float *) {
    t[n] = make_double4(a, b, c, d);
}
__device__ __forceinline__ void put4(float4 *t, int64_t n, double a, double b, double c, double d, const float *) {
    t[n] = make_float4((float)a, (float)b, (float)c, (float)d);
}
__device__ __forceinline__ uint16_t f_to_bf16(float f) {
    // round to nearest even on the upper 16 bits
    const uint32_t u = __float_as_uint(f);
    const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}
__device__ __forceinline__ void put4(bf16x4 *t, int64_t n, double a, double b, double c, double d, const float *sc) {
    t[n] = bf16x4{f_to_bf16((float)(a / sc[0])), f_to_bf16((float)(b / sc[1])), f_to_bf16((float)(c / sc[2])),
                  f_to_bf16((float)(d / sc[3]))};
}

template <class Tab>
__global__ __launch_bounds__(256) void k_fold(Tab *etab, const double2 *edc, const double2 *eoff, const double2 *esc,
                                              const double2 *erf, double v_off, int64_t nn, float s0, float s1,
                                              float s2, float s3) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const double2 d = edc[n], o = eoff[n], c = esc[n], r = erf[n];
    const float sc[4] = {s0, s1, s2, s3};
    put4(etab, n, d.x + v_off * o.x + c.x, d.y + v_off * o.y + c.y, r.x, r.y, sc);
}

// k_bake and k_fold in one pass over the nodes (the space-charge update):
// the field of the new potential is written out and folded into the step's
// table at once.
template <class Tab>
__global__ __launch_bounds__(256) void k_bake_fold(const double *phi, double2 *e, int32_t nr, int32_t nz, double dr,
                                                   double dz, unsigned long long *clear, Tab *etab, const double2 *edc,
                                                   const double2 *eoff, const double2 *erf, double v_off, float s0,
                                                   float s1, float s2, float s3) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)nr * nz) return;
    if (clear) clear[n] = 0ull;
    const double2 c = sc_field_at(phi, n, nr, nz, dr, dz);
    e[n] = c;
    const double2 d = edc[n], o = eoff[n], r = erf[n];
    const float sc[4] = {s0, s1, s2, s3};
    put4(etab, n, d.x + v_off * o.x + c.x, d.y + v_off * o.y + c.y, r.x, r.y, sc);
}

template <class Tab>
__global__ __launch_bounds__(256) void k_gas(Tab *gtab, const double *ur, const double *uz, const double *p,
                                             const double *t, int64_t nn, float s0, float s1, float s2, float s3) {
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nn) return;
    const float sc[4] = {s0, s1, s2, s3};
    put4(gtab, n, ur[n], uz[n], p[n], t[n], sc);
}

// Electrode hit table: metal node, or a metal node within d_hit + h/2.
static __global__ __launch_bounds__(256) void k_hit(const uint8_t *mask, uint8_t *hit, int32_t nr, int32_t nz, double dr,
                                             double dz, double reach, int32_t wi, int32_t wj) {
#pragma clang fp contract(off)
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= (int64_t)nr * nz) return;
    const int32_t i = (int32_t)(n % nr), j = (int32_t)(n / nr);
    uint8_t h = mask[n];
    for (int32_t b = -wj; b <= wj && !h; ++b)
        for (int32_t a = -wi; a <= wi && !h; ++a) {
            const int32_t ii = i + a, jj = j + b;
            if (ii < 0 || jj < 0 || ii >= nr || jj >= nz) continue;
            if (!mask[(int64_t)jj * nr + ii]) continue;
            const double dx = a * dr, dy = b * dz;
            if (dx * dx + dy * dy <= reach * reach) h = 1;
        }
    hit[n] = h;
}

// Snapshot pack initialisation after a host write: charge from the ion
// charge and weight, status active.
template <class T>
__global__ __launch_bounds__(256) void k_init_written(PackPtrs<T> p, const Species *sp, const int32_t *charge,
                                                      int64_t n) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    p.q[s] = fx32((double)charge[p.tag[s]] * p.w[s]);
    p.status[s] = ST_ACTIVE;
}

// ---------------------------------------------------------------------------
// Read-time tallies: active count/weight and histograms (int64 atomics), and
// FP64 sums reduced per block in a fixed order (deterministic).
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void k_snapshot(PackPtrs<T> p, const Species *sp, int64_t n_slots,
                                                  unsigned long long *act, unsigned long long *hke,
                                                  unsigned long long *hte, double *partial) {
    __shared__ double red[3][256];
    __shared__ unsigned long long lke[MC_HIST_KE], lte[MC_HIST_TEFF], lact[2];
    for (int k = threadIdx.x; k < MC_HIST_KE; k += blockDim.x) lke[k] = 0ull;
    for (int k = threadIdx.x; k < MC_HIST_TEFF; k += blockDim.x) lte[k] = 0ull;
    if (threadIdx.x < 2) lact[threadIdx.x] = 0ull;
    __syncthreads();
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_slots; s += stride) {
#pragma clang fp contract(off)
        const Species S = sp[p.tag[s]];
        const double w = p.w[s];
        const double e = (double)p.e[s] + (p.el ? (double)p.el[s] : 0.0);
        if (p.status[s] == ST_ACTIVE) {
            const double vx = p.vx[s], vy = p.vy[s], vz = p.vz[s];
            const double ke = 0.5 * S.m * (vx * vx + vy * vy + vz * vz);
            const double te = e > 0.0 ? S.theta / log1p(S.skt / e) : 0.0;
            const int64_t wfx = fx32(w);
            atomicAdd(&lact[0], 1ull);
            atomicAdd(&lact[1], (unsigned long long)wfx);
            atomicAdd(&lke[hbin_ke(ke / kQe)], (unsigned long long)wfx);
            atomicAdd(&lte[hbin_teff(te)], (unsigned long long)wfx);
            a0 += w * ke;
            a1 += w * e;
        } else {
            a2 += w * (-expm1(-(double)p.h[s]));
        }
    }
    red[0][threadIdx.x] = a0;
    red[1][threadIdx.x] = a1;
    red[2][threadIdx.x] = a2;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
            red[2][threadIdx.x] += red[2][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[3 * (int64_t)blockIdx.x + 0] = red[0][0];
        partial[3 * (int64_t)blockIdx.x + 1] = red[1][0];
        partial[3 * (int64_t)blockIdx.x + 2] = red[2][0];
    }
    for (int k = threadIdx.x; k < MC_HIST_KE; k += blockDim.x)
        if (lke[k]) atomicAdd(&hke[k], lke[k]);
    for (int k = threadIdx.x; k < MC_HIST_TEFF; k += blockDim.x)
        if (lte[k]) atomicAdd(&hte[k], lte[k]);
    if (threadIdx.x < 2 && lact[threadIdx.x]) atomicAdd(&act[threadIdx.x], lact[threadIdx.x]);
}

// Sums of the blocks' partials (three channels) in a fixed order; `retired`
// (nullable) is added to the third: the survival-yield sum of terminal
// packs whose slots a sort has dropped.
static __global__ __launch_bounds__(256) void k_reduce_partials(const double *partial, int64_t nb, double *out,
                                                                const double *retired) {
    __shared__ double red[3][256];
    double a[3] = {0.0, 0.0, 0.0};
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x)
        for (int c = 0; c < 3; ++c) a[c] += partial[3 * b + c];
    for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = a[c];
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o)
            for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) out[c] = red[c][0];
        if (retired) out[2] += *retired;
    }
}

// Trajectory samples: active packs with id % stride == 0, one record each.
// Buffer slots are claimed once per block of kSampleThreads (wavefront
// ballots, their prefix in LDS, one device atomic): a claim per wavefront
// made the launch wait on some 16k same-address atomics at 1e6 packs
// (0.21 ms against the records' 0.02 ms of stores).  Launched with
// blockDim.x == kSampleThreads.
constexpr int kSampleThreads = 1024;

template <class T>
__global__ __launch_bounds__(kSampleThreads) void k_sample(PackPtrs<T> p, const Species *sp, int64_t n_slots,
                                                           int64_t step, int64_t stride, mc_sample_rec *out,
                                                           unsigned long long *count, int64_t cap,
                                                           const double *dyn = nullptr) {
#pragma clang fp contract(off)
    // an adaptive run halted on the device takes no further samples (the
    // record of the previous step has zero length)
    if (dyn && !(dyn[1] > 0.0) && reinterpret_cast<const unsigned long long *>(dyn)[7]) return;
    __shared__ unsigned int wave_base[kSampleThreads / 64];
    __shared__ unsigned long long block_base;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool take = false;
    if (s < n_slots && p.status[s] == ST_ACTIVE) take = p.id[s] % stride == 0;
    const uint64_t mask = __ballot(take);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) wave_base[wave] = (unsigned int)__popcll(mask);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int total = 0;
        for (int w = 0; w < kSampleThreads / 64; ++w) {  // exclusive prefix over the wavefronts
            const unsigned int c = wave_base[w];
            wave_base[w] = total;
            total += c;
        }
        block_base = total ? atomicAdd(count, (unsigned long long)total) : 0ull;
    }
    __syncthreads();
    if (!take) return;
    const unsigned long long slot = block_base + wave_base[wave] + __popcll(mask & ((1ull << lane) - 1ull));
    if ((int64_t)slot >= cap) return;
    const Species S = sp[p.tag[s]];
    double x = p.x[s], y = p.y[s], z = p.z[s], e = p.e[s];
    if constexpr (sizeof(T) == 4) {
        x += (double)p.xl[s];
        y += (double)p.yl[s];
        z += (double)p.zl[s];
        e += (double)p.el[s];
    }
    const double vx = p.vx[s], vy = p.vy[s], vz = p.vz[s];
    mc_sample_rec r;
    r.id = p.id[s];
    r.step = step;
    r.tag = p.tag[s];
    r.reserved = 0;
    r.x = x;
    r.y = y;
    r.z = z;
    r.vx = vx;
    r.vy = vy;
    r.vz = vz;
    r.ke_ev = 0.5 * S.m * (vx * vx + vy * vy + vz * vz) / kQe;
    r.t_eff = e > 0.0 ? S.theta / log1p(S.skt / e) : 0.0;
    r.h = p.h[s];
    r.w = p.w[s];
    out[slot] = r;
}

// Small utilities.
static __global__ __launch_bounds__(256) void k_zero_u64(unsigned long long *p, int64_t n) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) p[k] = 0ull;
}

}  // namespace mc

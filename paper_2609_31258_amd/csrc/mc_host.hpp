// mc_host.hpp -- host-side pieces shared by the single-simulation runtime and
// the serving runtime: per-species constants, the source accumulator (Eq. 5)
// and fixed-point conversion.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>

#include "../../include/mucite.h"
#include "mc_device.hpp"

namespace mc {

inline int64_t fx32_host(double v) { return (int64_t)std::llrint(std::ldexp(v, 32)); }

// Constants of one ion template (mass, q/m, Einstein s kB theta, initial
// internal energy U(T_eff0), activation rate constants).
inline Species make_species(const mc_ion *in) {
    Species S{};
    S.m = in->mass_da * kDa;
    S.qm = in->charge_z * kQe / S.m;
    S.ccs = in->ccs_m2;
    S.theta = in->theta_e;
    S.skt = (3.0 * in->n_atoms - 6.0) * kB * in->theta_e;
    S.e0 = in->t_eff0 > 0.0 ? S.skt / std::expm1(in->theta_e / in->t_eff0) : 0.0;
    S.n_atoms = in->n_atoms;
    S.act_kind = in->act_kind;
    const double R = kNA * kB;
    if (in->act_kind == 1) {
        S.act_a = kB / kH * std::exp(in->act_p2 / R);
        S.act_b = in->act_p1 / R;
    } else if (in->act_kind == 2) {
        S.act_a = in->act_p1;
        S.act_b = in->act_p2 * kQe / kB;
    }
    S.alpha = in->alpha;
    return S;
}

// Default internal-exchange probability: 4 mg ma / (mg + ma)^2, ma = m / N.
inline void species_alpha(Species &S, const mc_ion &in, double gas_mass_da) {
    const double mg = gas_mass_da * kDa, ma = S.m / in.n_atoms;
    S.alpha = in.alpha >= 0.0 ? in.alpha : 4.0 * mg * ma / ((mg + ma) * (mg + ma));
}

// Every field table present must be finite (a NaN or infinity would turn
// into non-finite packs at the first gather); gas pressure and temperature
// must not be negative.
inline bool valid_tables(const mc_field_tables *t, int64_t nn) {
    const double *all[] = {t->phi_dc, t->phi_off, t->phi_rf, t->gas_ur, t->gas_uz, t->gas_p, t->gas_t};
    for (const double *a : all) {
        if (!a) continue;
        for (int64_t k = 0; k < nn; ++k)
            if (!std::isfinite(a[k])) return false;
    }
    for (int64_t k = 0; k < nn; ++k)
        if (t->gas_p[k] < 0.0 || t->gas_t[k] < 0.0) return false;
    return true;
}

inline bool valid_ion(const mc_ion *ion) {
    return ion && ion->n_atoms >= 3 && ion->mass_da > 0 && ion->charge_z != 0 && ion->ccs_m2 >= 0 &&
           ion->theta_e > 0 && ion->act_kind >= 0 && ion->act_kind <= 2;
}

struct Src {
    mc_source in;
    double w;
    int64_t w_fx, q_fx, n_real_fx, acc_fx, emitted;
};

// Eq. 5: each step the accumulator receives N_real = I dt / (z e) real ions;
// a fixed-rate source splits them over its packs_per_step packs.  Redone for
// every step's dt under the adaptive step.
inline void source_dt(Src &S, int32_t charge_z, double dt) {
    const double z = (double)charge_z;
    const double n_real = S.in.current_a * dt / (z * kQe);
    S.w = S.in.kind == 1 ? n_real / (double)S.in.packs_per_step : S.in.weight;
    S.w_fx = fx32_host(S.w);
    S.q_fx = fx32_host(z * S.w);
    S.n_real_fx = fx32_host(n_real);
}

inline Src make_source(const mc_source &in, int32_t charge_z, double dt) {
    Src S{};
    S.in = in;
    source_dt(S, charge_z, dt);
    return S;
}

// Packs due at a step: fixed rate, or the Eq. 5 accumulator in integer units
// of 2^-32 real ions; capped by the source's total.
inline int64_t due(Src &S, int64_t step) {
    if (step < S.in.step_start || S.in.kind == 0) return 0;
    const int64_t left = S.in.n_total - S.emitted;
    if (left <= 0) return 0;
    int64_t k;
    if (S.in.kind == 1) {
        k = S.in.packs_per_step;
    } else {
        S.acc_fx += S.n_real_fx;
        k = S.w_fx > 0 ? S.acc_fx / S.w_fx : 0;
        S.acc_fx -= k * S.w_fx;
    }
    return std::min(k, left);
}

// RF coefficients c = V_RF cos(2 pi f t + phase) at t0, t0 + dt/2, t0 + dt (Eq. 4).
inline void rf_stages_at(const mc_operating &op, double t0, double dt, double c[3]) {
    const double w2 = 2.0 * kPi * op.f_rf;
    c[0] = op.v_rf * std::cos(w2 * t0 + op.phase_rf);
    c[1] = op.v_rf * std::cos(w2 * (t0 + 0.5 * dt) + op.phase_rf);
    c[2] = op.v_rf * std::cos(w2 * (t0 + dt) + op.phase_rf);
}

// The same for fixed steps: t0 = step dt.
inline void rf_stages(const mc_operating &op, int64_t step, double *t0, double c[3]) {
    *t0 = (double)step * op.dt;
    rf_stages_at(op, *t0, op.dt, c);
}

}  // namespace mc

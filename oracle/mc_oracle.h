/*
 * mc_oracle.h -- CPU FP64 oracle of the MuCITE ion-pack time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * reference that the HIP library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header, table or constant with
 * the HIP library: both are written separately from the paper.
 *
 * Everything is SI and FP64.  Tables are row-major [nz][nr]: element
 * j*nr + i is node (r_i = i*dr, z_j = j*dz).
 *
 * Parity status of each function is stated at its definition in
 * mc_oracle.c; the one part whose agreement with the paper cannot be pinned
 * (the internal-energy exchange of the impulsive-collision adapter, whose
 * equations the paper cites but does not print) is marked there
 * "parity unpinned".
 */
#ifndef MC_ORACLE_H
#define MC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_ACTIVE = 0, ORC_TRANSMITTED = 1, ORC_ELECTRODE = 2, ORC_RADIAL = 3, ORC_AXIAL = 4, ORC_NUMERIC = 5 };
enum { ORC_NCLASS = 6 };
enum { ORC_HIST_KE = 202, ORC_HIST_TEFF = 202, ORC_HIST_R = 102 };

typedef struct orc_ion {
    double mass_da;
    int32_t charge_z;
    double ccs_m2;
    int32_t n_atoms;
    double theta_e;   /* Einstein temperature [K] */
    double alpha;     /* internal-exchange probability, < 0 = default */
    double t_eff0;    /* initial effective temperature [K] */
    int32_t act_kind; /* 0 none, 1 Eyring(dH J/mol, dS J/mol/K), 2 Arrhenius(A 1/s, Ea eV) */
    double act_p1, act_p2;
} orc_ion;

typedef struct orc_source {
    int32_t kind;     /* 0 burst, 1 packs-per-step, 2 current accumulator (Eq. 5) */
    int32_t ion;
    double current_a;
    double weight;    /* burst/accumulator target weight */
    int64_t packs_per_step;
    int64_t n_total;
    double sigma_r, r_trunc, z_inj;
    int64_t step_start;
} orc_source;

typedef struct orc_operating {
    double dt, v_rf, f_rf, phase_rf, v_off, gas_mass_da;
    int32_t collisions_on, sc_on, sc_every;
    double z_det, r_det, d_hit, exit_bin_dt;
    int32_t n_exit_bins;
    /* hybrid Langevin branch: on, axial window [lv_z_lo, lv_z_hi) (no window
     * when lv_z_hi <= lv_z_lo), switch when lambda dt >= lv_switch */
    int32_t langevin_on;
    double lv_z_lo, lv_z_hi, lv_switch;
    int32_t sc_mask; /* space charge: Phi = 0 on the metal-mask nodes */
    /* snapshots: at the start of step n with n % sample_every == 0, every
     * active pack whose id is a multiple of sample_stride (0 = off) */
    int32_t sample_every, sample_stride;
    /* Eq. 1 adaptive step: off (0) = fixed dt; on (1) = dt is the largest step
     * and the space-charge update runs every sc_every * dt of simulated time;
     * lv_dt_max caps the step while any pack takes the Langevin branch
     * (0 = no cap) */
    int32_t adaptive;
    double lv_dt_max;
} orc_operating;

typedef struct orc_packs {
    int64_t n;
    double *x, *y, *z, *vx, *vy, *vz, *e_int, *h, *w;
    int64_t *id, *q;
    int32_t *tag, *status;
} orc_packs;

typedef struct orc_tallies {
    int64_t emitted_n, emitted_w;
    int64_t class_n[ORC_NCLASS], class_w[ORC_NCLASS];
    int64_t n_cand, n_coll, n_cap, n_clamp, exit_overflow, n_langevin;
    int64_t n_exchange; /* accepted collisions that exchanged internal energy */
    double sum_w_ke_active, sum_w_eint_active, sum_w_dissoc_terminal;
    int64_t *exit_bins; /* [n_exit_bins] */
    int64_t *loss_map;  /* [nz*nr] */
    int64_t *hist_ke, *hist_teff, *hist_r;   /* transmitted packs */
    int64_t *act_hist_ke, *act_hist_teff;    /* active packs at read time */
} orc_tallies;

typedef struct orc_exit {
    int64_t id, step;
    int32_t cls, inode, jnode, tag;
    double x, y, z, vx, vy, vz, t_cross, r_cross, ke_ev, t_eff, h, w;
} orc_exit;

/* One snapshot record: the pack's state at the start of step `step`. */
typedef struct orc_sample {
    int64_t id, step;
    int32_t tag, pad;
    double x, y, z, vx, vy, vz, ke_ev, t_eff, h, w;
} orc_sample;

typedef struct orc_probe {
    int64_t n_cand, n_acc;
    double sum_g, sum_g2;
} orc_probe;

typedef struct orc_sim orc_sim;

/* --- unit-level functions (pins) --- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_bake(const double *phi, int32_t nr, int32_t nz, double dr, double dz, double *er, double *ez);
double orc_gather(const double *tab, int32_t nr, int32_t nz, double dr, double dz, double r, double z);
double orc_einstein_u(double t, int32_t n_atoms, double theta);
double orc_einstein_t(double e, int32_t n_atoms, double theta);
double orc_rate(int32_t kind, double p1, double p2, double t);
void orc_dst1(const double *in, int32_t m, double *out);
void orc_poisson(int32_t nr, int32_t nz, double dr, double dz, const double *rho, double *phi);
/* The same equation with Phi = 0 on the metal-mask nodes (mask != 0), by
 * preconditioned conjugate gradients; returns iterations or -1. */
int32_t orc_poisson_masked(int32_t nr, int32_t nz, double dr, double dz, const double *rho, const uint8_t *mask,
                           double tol, int32_t max_iter, double *phi);
double orc_poisson_residual(int32_t nr, int32_t nz, double dr, double dz, const double *rho, const double *phi);
void orc_rho_from_charge(int32_t nr, int32_t nz, double dr, double dz, const int64_t *q, double *rho);
void orc_iict_update(double m, double mg, const double v[3], const double vgas[3], double e_int, double t_eff,
                     double alpha, const double u[5], double v_out[3], double vgas_out[3], double *e_int_out,
                     int32_t *clamped, int32_t *exchanged);
int32_t orc_collision_probe(double m_da, double ccs, double mg_da, double p, double t_gas, const double u[3],
                            const double v[3], double dt, int64_t n_steps, uint64_t seed, orc_probe *out);

/* --- simulation --- */
orc_sim *orc_create(uint64_t seed);
void orc_destroy(orc_sim *s);
int32_t orc_load_fields(orc_sim *s, int32_t nr, int32_t nz, double dr, double dz, const double *phi_dc,
                        const double *phi_off, const double *phi_rf, const double *gas_ur, const double *gas_uz,
                        const double *gas_p, const double *gas_t, const uint8_t *mask);
int32_t orc_define_ion(orc_sim *s, const orc_ion *ion);
int32_t orc_define_source(orc_sim *s, const orc_source *src);
int32_t orc_set_operating(orc_sim *s, const orc_operating *op);
int32_t orc_inject(orc_sim *s, int32_t src, int64_t n);
int32_t orc_step(orc_sim *s, int64_t n_steps);
int64_t orc_num_packs(const orc_sim *s);
int32_t orc_num_threads(void);
int64_t orc_current_step(const orc_sim *s);
/* Simulated time at the start of the current step, and the last step taken. */
double orc_current_time(const orc_sim *s);
double orc_last_dt(const orc_sim *s);
int32_t orc_read_packs(const orc_sim *s, orc_packs *out);
int32_t orc_write_packs(orc_sim *s, const orc_packs *in);
int32_t orc_read_tallies(const orc_sim *s, orc_tallies *out);
int64_t orc_read_exits(const orc_sim *s, orc_exit *buf, int64_t cap);
/* Snapshot records in (step, id) order; returns how many there are. */
int64_t orc_read_samples(const orc_sim *s, orc_sample *buf, int64_t cap);
int32_t orc_read_charge(const orc_sim *s, int64_t *q);
int32_t orc_read_sc(const orc_sim *s, double *phi, double *er, double *ez);
int32_t orc_read_hit(const orc_sim *s, uint8_t *hit);
int32_t orc_pic_update(orc_sim *s);
/* Hybrid Langevin branch: friction rate of the hard-sphere gas and the
 * exact relaxation of the velocity over dt (see mc_oracle.c). */
double orc_langevin_gamma(double m, double mg, double n_sigma, double t_gas);
void orc_langevin_relax(double m, double gamma, double t_gas, const double u[3], double dt, const double xi[3],
                        double v[3]);
/* CIC deposit only: refreshes the charge grid, leaves the potential alone. */
int32_t orc_deposit(orc_sim *s);

#ifdef __cplusplus
}
#endif
#endif

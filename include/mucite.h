/*
 * mucite.h -- C ABI of the MI355X (gfx950) ion-pack propagation library.
 *
 * The library advances weighted ion packs through baked axisymmetric DC, RF
 * and gas-flow fields with particle-in-cell space charge, stochastic
 * hard-sphere collisions with internal-energy exchange, dissociation
 * survival, and terminal classification -- the per-timestep path of the
 * MuCITE method (paper sections "Simulation scope and modular architecture"
 * through "Terminal events, snapshots, and reported observables", Eqs. 1-8).
 * Every step of the path runs in hand-written HIP kernels on one GPU.
 *
 * Conventions
 *  - Status: every call returns int32_t, MC_OK (0) or a negative MC_E* code.
 *    No C++ exception crosses this boundary.  mc_last_error() returns a
 *    ctx-owned NUL-terminated message, valid until the next call on that ctx.
 *  - Units: SI throughout (m, s, V, Pa, K, kg via Da, J).  Masses in Da,
 *    cross sections in m^2, activation enthalpy in J/mol, entropy in
 *    J/(mol K), Arrhenius energy in eV.
 *  - Grid: node (r_i = i*dr, z_j = j*dz), 0 <= i < nr, 0 <= j < nz.  Every
 *    table is row-major [nz][nr]: element j*nr + i.
 *  - Ownership: host arrays passed in are borrowed for the duration of the
 *    call and copied; host output buffers belong to the caller and must have
 *    the sizes stated at each call.  Device memory belongs to the ctx; it is
 *    obtained from the allocator callbacks in mc_options when given (so a
 *    framework's caching allocator can back it), otherwise from hipMalloc.
 *  - Streams: work is enqueued on the stream given in mc_options (a
 *    hipStream_t passed as void*), or on a stream the ctx creates.  mc_step,
 *    mc_inject and mc_pic_update are asynchronous; every mc_read_* call
 *    synchronises the stream first.  A ctx is not thread-safe.
 *  - Fixed point: pack weights and charges are int64 in units of 2^-32 real
 *    ions and 2^-32 elementary charges, so deposits and tallies are exact
 *    and independent of summation order.
 */
#ifndef MUCITE_H
#define MUCITE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MC_ABI_VERSION 6

enum {
    MC_OK = 0,
    MC_EINVAL = -1,     /* invalid argument */
    MC_ESTATE = -2,     /* call out of order (e.g. step before fields/operating point) */
    MC_ENOMEM = -3,     /* allocation failed or capacity exceeded */
    MC_EBUDGET = -4,    /* request exceeds the configured device-memory budget */
    MC_EDEVICE = -5,    /* HIP runtime error */
    MC_ENUMERIC = -6,   /* non-finite state detected (packs are counted, not dropped silently) */
    MC_EINTERNAL = -7
};

enum { MC_PREC_FP64 = 0, MC_PREC_FP32 = 1 };

/* Terminal classes ("Terminal events" section): transmitted through the
 * detector plane within the detector radius, electrode hit, radial loss,
 * axial domain exit; numeric marks a pack whose state became non-finite. */
enum { MC_ACTIVE = 0, MC_TRANSMITTED = 1, MC_ELECTRODE = 2, MC_RADIAL = 3, MC_AXIAL = 4, MC_NUMERIC = 5 };
enum { MC_NCLASS = 6 };

/* Histogram layouts (index 0 = underflow, last = overflow):
 *   KE      200 log10 bins over [1e-3, 1e3] eV            -> MC_HIST_KE entries
 *   T_eff   200 linear bins over [0, 5000] K              -> MC_HIST_TEFF entries
 *   r_exit  100 linear bins over [0, r_det] (transmitted) -> MC_HIST_R entries */
enum { MC_HIST_KE = 202, MC_HIST_TEFF = 202, MC_HIST_R = 102 };

typedef void *(*mc_alloc_fn)(size_t bytes, void *stream, void *user);
typedef void (*mc_free_fn)(void *ptr, void *stream, void *user);

typedef struct mc_options {
    int32_t precision;       /* MC_PREC_FP64, or MC_PREC_FP32 (FP32 state and math, BF16 tables) */
    int32_t device;          /* HIP device ordinal */
    uint64_t seed;           /* key of the counter-based random streams */
    int64_t pack_capacity;   /* maximum number of pack slots (> 0) */
    int64_t exit_capacity;   /* exit-record buffer size; 0 = pack_capacity */
    int64_t hbm_budget;      /* device bytes this ctx may allocate; 0 = unlimited */
    void *stream;            /* hipStream_t to enqueue on; NULL = ctx-owned stream */
    mc_alloc_fn alloc;       /* optional device allocator (both or neither) */
    mc_free_fn free;
    void *alloc_user;
    int32_t timing;          /* non-zero: record HIP events around every kernel (mc_read_timing) */
    int32_t fp32_tables;     /* FP32 form only: FP32 field tables instead of BF16 with per-table scale */
    int64_t sample_capacity; /* trajectory-sample buffer size in records (0 = none; see mc_read_samples) */
} mc_options;

typedef struct mc_grid {
    int32_t nr, nz;          /* nodes (>= 3 each) */
    double dr, dz;           /* spacings [m] */
} mc_grid;

/* Field tables on the node grid (host FP64 arrays of nr*nz, row-major [nz][nr]).
 * phi_dc: DC potential [V]; phi_off: DC-offset basis [V/V] (nullable);
 * phi_rf: RF basis potential for +/-1 V on the RF electrodes [V/V] (Eq. 4,
 * V_ref = 1 V; nullable); gas_ur, gas_uz [m/s], gas_p [Pa], gas_t [K]
 * (gas_ur, gas_uz nullable = 0); mask: 1 on metal nodes (nullable = none).
 * E = -grad(phi) is baked on the device by second-order central differences
 * (one-sided at the outer edges, E_r = 0 on the axis). */
typedef struct mc_field_tables {
    const double *phi_dc, *phi_off, *phi_rf;
    const double *gas_ur, *gas_uz, *gas_p, *gas_t;
    const uint8_t *mask;
} mc_field_tables;

/* Ion template ("Simulation scope and modular architecture": the ion is
 * described by its mass, charge, collision cross section, atom count, heat
 * capacity and, optionally, its activation parameters).  Heat capacity:
 * Einstein model, s = 3N-6 oscillators at theta_e.  alpha < 0 selects the
 * default internal-exchange probability 4 mg ma / (mg + ma)^2, ma = m /
 * n_atoms (the head-on elastic transfer share; "Particle transport,
 * collisions, and effective internal temperature"). */
typedef struct mc_ion {
    double mass_da;
    int32_t charge_z;        /* non-zero */
    double ccs_m2;
    int32_t n_atoms;         /* >= 3 */
    double theta_e;          /* [K] */
    double alpha;
    double t_eff0;           /* initial effective temperature [K] */
    int32_t act_kind;        /* 0 none, 1 Eyring (p1 = dH J/mol, p2 = dS J/mol/K), 2 Arrhenius (p1 = A 1/s, p2 = Ea eV) */
    double act_p1, act_p2;
} mc_ion;

/* Source definition ("Simulation scope and modular architecture" and
 * "Continuous current Gaussian source": current, transverse profile,
 * injection plane and initial velocities are given apart from the ion).
 * kind 0: burst, packs only via mc_inject, weight = weight;
 * kind 1: packs_per_step packs every step from step_start, weight
 *         I dt / (z e packs_per_step) so the packs carry the current;
 * kind 2: Eq. 5 accumulator: N_real = I dt / (z e) per step, a pack of
 *         weight `weight` emitted each time the accumulator reaches it.
 * Emission stops after n_total packs.  Radial profile: Gaussian of width
 * sigma_r truncated at r_trunc; injection plane z_inj; velocity: local gas
 * flow plus the ion's Maxwellian at the local gas temperature. */
typedef struct mc_source {
    int32_t kind;
    int32_t ion;             /* id from mc_define_ion */
    double current_a;
    double weight;
    int64_t packs_per_step;
    int64_t n_total;
    double sigma_r, r_trunc, z_inj;
    int64_t step_start;
} mc_source;

/* Operating point.  dt: fixed step [s]; RF: V_RF cos(2 pi f t + phase) (Eq. 4);
 * v_off scales the DC-offset basis; collisions_on enables the collision
 * step; sc_on/sc_every: deposit + Poisson + field every sc_every steps;
 * z_det/r_det: detector plane and radius; d_hit: electrode hit distance;
 * exit current (Eq. 8) is binned in n_exit_bins bins of exit_bin_dt.
 *
 * Hybrid Langevin branch (collision section; Ermak-Buckholz): with
 * langevin_on, a pack whose post-push z lies in [lv_z_lo, lv_z_hi) (any z
 * when lv_z_hi <= lv_z_lo) and whose candidate rate lambda = n sigma (s +
 * abar) satisfies lambda dt >= lv_switch (the paper's switch is 0.05) skips
 * the explicit events of the step: its velocity relaxes toward the local
 * gas velocity by the exact Ornstein-Uhlenbeck update over dt with the
 * hard-sphere friction rate gamma = (16/3)(n sigma/m) sqrt(mu kB T/(2 pi)),
 * and its internal energy and hazard are left unchanged for that step.
 * lv_switch must be >= 0 when the branch is on (MC_EINVAL otherwise).
 *
 * sc_mask: the space-charge potential also vanishes on the metal-mask nodes
 * (the space-charge section: zero perturbation potential on the mask,
 * whose potentials the static field already holds).  Imposed by a
 * capacitance-matrix correction built at the first such update (one solve
 * per interior mask node, at most 2048 of them, else MC_EINVAL) and then
 * applied with one extra solve per update.
 *
 * sample_every/sample_stride: time-resolved snapshots (the paper's
 * ion-distribution snapshots).  At the start of every step n with
 * n % sample_every == 0 (before the space-charge update and emission), each
 * active pack whose id is a multiple of sample_stride is recorded
 * (mc_sample_rec) into the buffer sized by mc_options.sample_capacity.
 * 0 turns sampling off; both must be >= 0.  The serving runtime takes them
 * per query as well (see mc_query).
 *
 * adaptive: the global step of Eq. 1, dt_n = min(0.05 t_RF, 0.1 tau_coll,
 * dt_acc, dt_CFL, dt_L, dt_rem), evaluated on the device at the start of
 * every step over the active packs (tau_coll = 1/lambda of the packs on the
 * explicit branch; dt_acc = 0.1 (|v-u| + sqrt(kB T/m))/|qE/m|, or
 * sqrt(min(dr,dz)/|qE/m|) for a pack with no speed scale; dt_CFL =
 * min(dr,dz)/(2|v|); dt_L = lv_dt_max (> 0) while any pack takes the
 * Langevin branch; dt_rem = time to the next space-charge update).  dt is
 * then the largest step, the space-charge update runs every sc_every * dt
 * of simulated time, sources emit per step with that step's dt (Eq. 5), and
 * the Langevin switch always compares with dt.  The lengths stay on the
 * device (see mc_step).  A step that collapses below 1e-9 dt fails with
 * MC_ENUMERIC.  The serving runtime runs it per query (see
 * mc_query).
 *
 * sort_every: at the start of every step n with n % sort_every == 0 (before
 * the snapshots, the space-charge update and emission) the active packs are
 * reordered by (species, lower-left node of their CIC cell) and the slots
 * of terminal packs are dropped, so mc_read_packs then returns the active
 * packs only and freed slots take new packs.  Slot order changes no pack's
 * state and no integer tally (random streams are keyed by pack id and step);
 * only the FP64 sums over the active population (sum_w_*_active) may change
 * in their last bits, being reduced in slot order.  Sorting groups packs of
 * like collision rate and place, for the step's wavefronts, the field
 * gathers and the deposit (which then adds straight into the grid instead of
 * grid copies).  0 = never; needs pack_capacity <= 2^28 and at most 2^32 - 2
 * (species x nodes) keys (MC_EINVAL from mc_step otherwise).  The serving
 * runtime ignores it. */
typedef struct mc_operating {
    double dt, v_rf, f_rf, phase_rf, v_off, gas_mass_da;
    int32_t collisions_on, sc_on, sc_every;
    double z_det, r_det, d_hit, exit_bin_dt;
    int32_t n_exit_bins;
    int32_t langevin_on;
    double lv_z_lo, lv_z_hi, lv_switch;
    int32_t sc_mask;
    int32_t sample_every, sample_stride;
    int32_t adaptive;
    double lv_dt_max;
    int32_t sort_every;
} mc_operating;

/* Pack population (host arrays of length n) for snapshot read/write.
 * Read: all slots in slot order, terminal packs included; every pointer may
 * be NULL to skip that field; n on input = buffer length.  Write: replaces
 * the population by n active packs (x..w, id and tag required; q and
 * status ignored -- q is recomputed from the ion charge and w). */
typedef struct mc_packs {
    int64_t n;
    double *x, *y, *z, *vx, *vy, *vz, *e_int, *h, *w;
    int64_t *id, *q;
    int32_t *tag, *status;
} mc_packs;

/* Tallies.  Scalars are filled by mc_read_tallies; each array pointer, when
 * non-NULL, must hold: exit_bins[n_exit_bins], loss_map[nz*nr],
 * hist_ke[MC_HIST_KE], hist_teff[MC_HIST_TEFF], hist_r[MC_HIST_R],
 * act_hist_ke[MC_HIST_KE], act_hist_teff[MC_HIST_TEFF].
 * class_n/class_w: packs and int64 weights per class (MC_ACTIVE = the
 * current active population); exit bins, loss map and hist_* collect the
 * weights of transmitted (hist_*, exit_bins) and electrode (loss_map) packs;
 * act_hist_* histogram the active population at read time.
 * n_cand/n_coll: collision candidates and accepted collisions; n_cap: pack
 * steps that hit the candidate cap; n_clamp: internal-energy clamps;
 * pack_steps: sum over steps of the active packs advanced; n_langevin:
 * pack steps taken by the hybrid Langevin branch; n_exchange: accepted
 * collisions that exchanged energy with the internal modes.
 * sum_w_*: FP64 sums, reduced in a fixed order (run-to-run identical). */
typedef struct mc_tallies {
    int64_t emitted_n, emitted_w;
    int64_t class_n[MC_NCLASS], class_w[MC_NCLASS];
    int64_t n_cand, n_coll, n_cap, n_clamp, pack_steps, exit_overflow, exit_dropped, n_langevin, n_exchange;
    double sum_w_ke_active, sum_w_eint_active, sum_w_dissoc_terminal;
    int64_t *exit_bins, *loss_map, *hist_ke, *hist_teff, *hist_r, *act_hist_ke, *act_hist_teff;
} mc_tallies;

/* One terminal event.  inode/jnode: nearest node for electrode hits, else -1;
 * t_cross/r_cross: plane-crossing time and radius for axial/transmitted exits. */
typedef struct mc_exit_rec {
    int64_t id, step;
    int32_t cls, inode, jnode, tag;
    double x, y, z, vx, vy, vz, t_cross, r_cross, ke_ev, t_eff, h, w;
} mc_exit_rec;

/* One trajectory sample (state at the start of step `step`, t = step dt). */
typedef struct mc_sample_rec {
    int64_t id, step;
    int32_t tag, reserved;
    double x, y, z, vx, vy, vz, ke_ev, t_eff, h, w;
} mc_sample_rec;

typedef struct mc_info {
    int64_t step, n_slots, capacity, exit_capacity, device_bytes;
    int32_t nr, nz, n_exit_bins, precision, n_ions, n_sources;
    double time;             /* simulated time at the start of the next step [s] */
    double last_dt;          /* length of the last step [s] */
} mc_info;

/* Per-kernel timing from HIP events (requires mc_options.timing). */
enum { MC_K_EMIT = 0, MC_K_STEP = 1, MC_K_DEPOSIT = 2, MC_K_POISSON = 3, MC_K_FIELD = 4, MC_K_TALLY = 5, MC_K_SORT = 6,
       MC_NKERNEL = 7 };
typedef struct mc_timing {
    double ms[MC_NKERNEL];
    int64_t launches[MC_NKERNEL];
    int64_t pack_steps;      /* sum over step launches of the slots scanned */
} mc_timing;

typedef struct mc_ctx mc_ctx;

/* Buffer layout of the tallies ("Terminal events, snapshots, and reported
 * observables"; Eq. 8 for the exit-current bins).  Filled by
 * mc_get_tally_layout from the context's grid and operating point, so a
 * caller can size the arrays of mc_tallies and the record buffers before
 * reading.  Every histogram has an underflow entry (index 0) and an
 * overflow entry (last); bin k (1 <= k <= bins) covers
 * [lo + (k-1) w, lo + k w) with w = (hi - lo) / bins, in log10(KE / eV) for
 * the kinetic-energy histogram and linearly for the others. */
typedef struct mc_tally_layout {
    int32_t n_classes;       /* MC_NCLASS: entries of class_n / class_w */
    int32_t n_exit_bins;     /* entries of exit_bins (Eq. 8) */
    double exit_bin_dt;      /* width of an exit-current bin [s]; bin b covers [b, b+1) exit_bin_dt */
    int32_t nr, nz;          /* loss_map holds nz*nr int64, row-major [nz][nr] */
    int64_t loss_map_len;
    int32_t hist_ke_len;     /* MC_HIST_KE entries: ke_bins + 2 */
    int32_t ke_bins;
    double ke_log10_lo, ke_log10_hi; /* log10 of the KE range in eV */
    int32_t hist_teff_len;   /* MC_HIST_TEFF entries: teff_bins + 2 */
    int32_t teff_bins;
    double teff_lo, teff_hi; /* [K] */
    int32_t hist_r_len;      /* MC_HIST_R entries: r_bins + 2 */
    int32_t r_bins;
    double r_lo, r_hi;       /* exit radius range [m]: 0 .. r_det */
    int64_t exit_capacity;   /* exit records kept (mc_read_exits) */
    int64_t sample_capacity; /* trajectory samples kept (mc_read_samples) */
    int64_t charge_grid_len; /* int64 entries of mc_read_charge: nz*nr */
} mc_tally_layout;

/* ABI version of the library (MC_ABI_VERSION of the header it was built from). */
int32_t mc_abi_version(void);

/* Create a context on options->device: the simulation of the paper's
 * "Simulation scope and modular architecture" (one run = fields, ion
 * templates, sources, operating point).  *out receives the handle.
 * Errors: MC_EINVAL (bad options), MC_EDEVICE. */
int32_t mc_create(const mc_options *options, mc_ctx **out);
/* Release all device memory and the ctx-owned stream.  NULL is a no-op. */
void mc_destroy(mc_ctx *ctx);
/* Message of the last failed call on ctx (ctx-owned; valid until the next call). */
const char *mc_last_error(const mc_ctx *ctx);

/* Load and bake the field tables ("Coordinate system, static fields, and RF
 * convention", Eqs. 2-4: E = -grad(phi) on the nodes; "Gas field and
 * electrode mask coupling": gas velocity, pressure, temperature and the
 * electrode mask).  May be called once per ctx.  The host arrays are copied.
 * Errors: MC_EINVAL (also for a non-finite table value or a negative gas
 * pressure or temperature; the ctx then keeps no fields), MC_ESTATE,
 * MC_ENOMEM, MC_EBUDGET. */
int32_t mc_load_fields(mc_ctx *ctx, const mc_grid *grid, const mc_field_tables *tables);
/* Define an ion template ("Simulation scope and modular architecture"; heat
 * capacity and activation as in "Particle transport, collisions, and
 * effective internal temperature" and Eq. 7); *ion_id receives its index
 * (the species tag of its packs).  Errors: MC_EINVAL (n_atoms < 3, charge 0,
 * mass <= 0), MC_ENOMEM (more than 64 templates). */
int32_t mc_define_ion(mc_ctx *ctx, const mc_ion *ion, int32_t *ion_id);
/* Set the operating point (time step, Eq. 1 when adaptive; RF of Eq. 4;
 * collision, Langevin and space-charge switches; detector and hit distance
 * of "Terminal events, snapshots, and reported observables"); requires
 * fields.  Rebuilds the electrode hit table and the folded static field.
 * Must precede mc_define_source.  Errors: MC_EINVAL, MC_ESTATE. */
int32_t mc_set_operating(mc_ctx *ctx, const mc_operating *op);
/* Define a source ("Continuous current Gaussian source", Eq. 5); *src_id
 * receives its index.  Pack ids of source s are (s << 32) | k for its k-th
 * pack; they key the random streams.  Errors: MC_EINVAL, MC_ESTATE. */
int32_t mc_define_source(mc_ctx *ctx, const mc_source *src, int32_t *src_id);
/* Emit n packs from source src_id now, at the current step (a burst; the
 * source's transverse profile and velocities of "Continuous current
 * Gaussian source").  Asynchronous.  Errors: MC_EINVAL, MC_ESTATE, MC_ENOMEM
 * (pack capacity exceeded). */
int32_t mc_inject(mc_ctx *ctx, int32_t src_id, int64_t n);
/* Advance n_steps steps of the operator-split cycle of "Simulation scope and
 * modular architecture".  Each step: space-charge update when sc_on and it
 * is due ("Axisymmetric PIC space charge update"); emission of due packs
 * (Eq. 5); then for every active pack the RK4 push in the field of Eqs. 3-4,
 * terminal classification ("Terminal events, snapshots, and reported
 * observables"), collisions (Eq. 6 and the internal-energy exchange) or the
 * hybrid Langevin relaxation, and the dissociation hazard (Eq. 7).
 * Asynchronous with a fixed step.  With the adaptive step (Eq. 1) each
 * step's length is found on the device and the step kernels read it there;
 * the call reads the step record back once per stretch of steps before a
 * space-charge update could fall due, and at its end (while a source still
 * emits, whose Eq. 5 counts need each length on the host, once per step).
 * Errors: MC_ESTATE, MC_ENOMEM (capacity), MC_ENUMERIC (adaptive step
 * collapsed; the step counter and time stay at the collapsed step),
 * MC_EDEVICE. */
int32_t mc_step(mc_ctx *ctx, int64_t n_steps);
/* Space-charge update now ("Axisymmetric PIC space charge update": CIC
 * deposit, cylindrical Poisson solve, E = -grad(Phi) folded into the static
 * field) from the current packs.  Asynchronous. */
int32_t mc_pic_update(mc_ctx *ctx);
/* Wait for the ctx stream. */
int32_t mc_synchronize(mc_ctx *ctx);
/* Step counter, simulated time, last step length, capacities and sizes. */
int32_t mc_get_info(const mc_ctx *ctx, mc_info *info);
/* Layout of the tally arrays and record buffers (see mc_tally_layout);
 * requires an operating point (MC_ESTATE otherwise). */
int32_t mc_get_tally_layout(const mc_ctx *ctx, mc_tally_layout *out);

/* Reported observables ("Terminal events, snapshots, and reported
 * observables"; exit current of Eq. 8; survival yield of Eq. 7): class
 * counts and weights, exit-current bins, loss map, histograms, FP64 energy
 * and survival sums; array sizes from mc_get_tally_layout.  Synchronises. */
int32_t mc_read_tallies(mc_ctx *ctx, mc_tallies *out);
/* Terminal events ("Terminal events, snapshots, and reported observables"):
 * copy up to cap exit records (sorted by pack id) into buf; *n receives the
 * total number recorded (may exceed cap).  Synchronises. */
int32_t mc_read_exits(mc_ctx *ctx, mc_exit_rec *buf, int64_t cap, int64_t *n);
/* Trajectory snapshots ("Terminal events, snapshots, and reported
 * observables"): copy up to cap samples, sorted by (step, id), into buf; *n
 * receives the number taken (may exceed the buffer: the rest were dropped). */
int32_t mc_read_samples(mc_ctx *ctx, mc_sample_rec *buf, int64_t cap, int64_t *n);
/* Pack population ("Simulation scope and modular architecture": the packs'
 * state) into host arrays (see mc_packs).  Synchronises. */
int32_t mc_read_packs(mc_ctx *ctx, mc_packs *out);
/* Replace the pack population by n active packs (snapshot restart; see
 * mc_packs).  Errors: MC_EINVAL (non-finite values, unknown tag), MC_ENOMEM. */
int32_t mc_write_packs(mc_ctx *ctx, const mc_packs *in);
/* Checkpoint and resume.  mc_save_state writes the context's dynamic state
 * (pack slots, tallies, exit records and samples taken, space-charge field,
 * step, time, source accumulators) to the file `path`; mc_load_state reads
 * it into a context whose fields, ions, sources, operating point, seed and
 * precision were set up exactly as when it was saved (checked against a
 * fingerprint: MC_EINVAL on a mismatch, a truncated file or a capacity too
 * small).  Stepping on after a load continues the saved run bit for bit.
 * Both synchronise the stream. */
int32_t mc_save_state(mc_ctx *ctx, const char *path);
int32_t mc_load_state(mc_ctx *ctx, const char *path);
/* int64 charge grid of the last CIC deposit ("Axisymmetric PIC space charge
 * update"), nz*nr, units of 2^-32 e. */
int32_t mc_read_charge(mc_ctx *ctx, int64_t *q);
/* Space-charge potential and field of the last update ("Axisymmetric PIC
 * space charge update"; nz*nr each; each pointer nullable). */
int32_t mc_read_sc(mc_ctx *ctx, double *phi, double *er, double *ez);
/* Electrode hit table ("Gas field and electrode mask coupling": a node is a
 * hit node when metal lies within the hit distance; nz*nr bytes). */
int32_t mc_read_hit(mc_ctx *ctx, uint8_t *hit);
/* Per-kernel HIP-event times (mc_options.timing) and their reset. */
int32_t mc_read_timing(mc_ctx *ctx, mc_timing *out);
int32_t mc_reset_timing(mc_ctx *ctx);
/* Per-kernel events on (on != 0) or off for the launches that follow; the
 * times gathered so far are kept.  The events add a marker to the stream on
 * both sides of every launch, which lengthens short steps: a caller may time
 * the kernels over one stretch of steps and the whole step without events
 * over another.  MC_EINVAL on a null context. */
int32_t mc_set_timing(mc_ctx *ctx, int32_t on);

/* ------------------------------------------------------------------------- */
/* Stand-alone CIC deposit on caller-owned device arrays.                     */
/* ------------------------------------------------------------------------- */
/* Packs for the stand-alone deposit: device arrays of length n (device
 * memory of the current HIP device; the caller keeps ownership).  Positions
 * in m (r = sqrt(x^2 + y^2)), charges in units of 2^-32 e; packs whose
 * status is not MC_ACTIVE are skipped, as are packs with a non-finite
 * position.  With n == 0 the pointers may be NULL. */
typedef struct mc_cic_packs {
    int64_t n;
    const double *x, *y, *z;
    const int64_t *q;
    const int32_t *status;
} mc_cic_packs;

/* Cloud-in-cell deposit of the packs' charges onto the node grid, the
 * deposit step of "Axisymmetric PIC space charge update" exactly as a
 * simulation's space-charge update does it: each pack's int64 charge is
 * split bilinearly in (r, z) onto the four nodes of its cell, the split
 * rounded so the four parts sum to the charge exactly (cell index clamped
 * to the grid).  q_out: device int64 array of grid->nz * grid->nr, row-major
 * [nz][nr], overwritten with the deposited charge (2^-32 e); the result does
 * not depend on the order of the packs.  Enqueued on `stream` (a
 * hipStream_t; NULL = the default stream); the call allocates its scratch
 * (copies of the grid for the blocks' flushes) with hipMalloc, waits for
 * the stream and frees it.  Errors: MC_EINVAL (NULL pointers, grid < 3 x 3
 * or non-positive spacing, n < 0), MC_ENOMEM, MC_EDEVICE. */
int32_t mc_deposit_cic(const mc_cic_packs *packs, const mc_grid *grid, int64_t *q_out, void *stream);

/* The deposit of mc_deposit_cic for callers that cannot allocate device
 * memory -- code being recorded into a HIP graph, tight serving loops,
 * harnesses that forbid hipMalloc: no allocation and no host
 * synchronisation (asynchronous on `stream`).  Its scratch is a fixed
 * library-owned device array of 8 MiB + 16 B per GPU, held until the
 * process ends, so the grid may hold at most 1 048 576 nodes (MC_EINVAL
 * beyond; 16 grid copies up to 65 536 nodes, fewer above).  Every call on a
 * GPU uses that GPU's one array and leaves it cleared for the next:
 * concurrent calls on one GPU (overlapping on different streams) race and
 * must be serialised by the caller.  Results are bit-identical to
 * mc_deposit_cic.  Errors: MC_EINVAL, MC_EDEVICE. */
int32_t mc_deposit_cic_noalloc(const mc_cic_packs *packs, const mc_grid *grid, int64_t *q_out, void *stream);

/* ------------------------------------------------------------------------- */
/* Serving: continuous batching of design queries over shared field tables.   */
/*                                                                           */
/* A server owns one field set (grid, potentials, gas, mask, hit distance and */
/* gas species shared by all queries) and a device pool of hbm_budget bytes.  */
/* Each query is a complete simulation (its own ion, source, operating point, */
/* seed, step count): its packs, space-charge grids, folded field table and   */
/* tallies stay resident in one pool block from admission to completion.     */
/* A worker thread admits pending queries in arrival order while their block  */
/* fits in the pool and fewer than max_resident are resident, advances every  */
/* resident query by one step per co-step (one launch of the step kernel for  */
/* all of them; emission likewise; space-charge updates per query), and      */
/* retires finished queries into host results.  A query's arithmetic does   */
/* not depend on which others share its launches: its result is the same     */
/* alone and in any mix.  submit/poll/wait/stats are thread-safe.            */
/* ------------------------------------------------------------------------- */
typedef struct mc_server_options {
    int32_t precision;       /* MC_PREC_FP64 or MC_PREC_FP32 */
    int32_t device;
    int64_t hbm_budget;      /* bytes of the query pool (> 0) */
    int32_t max_resident;    /* queries co-stepped at once, 1..4096 */
    int32_t steps_per_sync;  /* co-steps enqueued between host synchronisations, >= 1 */
    void *stream;            /* hipStream_t, NULL = server-owned */
    mc_alloc_fn alloc;       /* optional allocator for the pool and shared tables */
    mc_free_fn free;
    void *alloc_user;
    int32_t fp32_tables;     /* FP32 form: FP32 instead of BF16 field tables */
    int32_t reserved;
    double d_hit;            /* electrode hit distance shared by all queries [m] */
    double gas_mass_da;      /* gas molecule mass shared by all queries [Da] */
} mc_server_options;

/* A design query.  source.ion is ignored (the query's own ion); op.d_hit and
 * op.gas_mass_da are ignored (the server's).  kind 0 sources emit n_total
 * packs at the query's first step.  exit_capacity: exit records kept (0 = none);
 * sample_capacity: trajectory samples kept (0 = none), taken on the schedule of
 * op.sample_every / op.sample_stride as in a single run.  op.adaptive selects
 * the Eq. 1 step as in mc_step: each co-step then reduces the query's step
 * limits and reads them back (one synchronisation per co-step for all adaptive
 * queries); a query whose step collapses fails with MC_ENUMERIC alone. */
typedef struct mc_query {
    mc_ion ion;
    mc_source source;
    mc_operating op;
    int64_t n_steps;
    uint64_t seed;
    int64_t exit_capacity;
    int64_t sample_capacity;
} mc_query;

enum { MC_Q_PENDING = 0, MC_Q_RUNNING = 1, MC_Q_DONE = 2, MC_Q_FAILED = 3 };

/* Result of a query.  Before polling, set the tally array pointers you want
 * (sizes as for mc_read_tallies with the query's n_exit_bins) or NULL, and
 * the exit-record and sample buffers with their lengths in records (or NULL).
 * Once the query is done, n_exits / n_samples give the records it kept (at
 * most its capacities) and the first min(n, length) of them, in the order the
 * device appended them, are copied into the buffers.  Times are seconds on the
 * server clock (0 at creation). */
typedef struct mc_query_result {
    int32_t state, error;
    double t_submit, t_admit, t_done;
    int64_t device_bytes;
    mc_tallies tallies;
    mc_exit_rec *exits;        /* in: buffer or NULL */
    int64_t exits_len;         /* in: its length in records */
    int64_t n_exits;           /* out */
    mc_sample_rec *samples;    /* in: buffer or NULL */
    int64_t samples_len;       /* in */
    int64_t n_samples;         /* out */
} mc_query_result;

typedef struct mc_server_stats {
    int64_t submitted, admitted, completed, failed, resident, pending;
    int64_t pool_bytes, pool_in_use, pool_peak, shared_bytes;
    int64_t co_steps, pack_steps, max_resident_seen;
    double busy_s, wall_s;
} mc_server_stats;

typedef struct mc_server mc_server;

/* Create a server over one field set, baked as in mc_load_fields
 * ("Coordinate system, static fields, and RF convention"; "Gas field and
 * electrode mask coupling").  Each query it runs is one simulation of the
 * method with its own operating conditions, ion and current -- the paper's
 * simulation-guided design use ("Simulation scope and modular
 * architecture").  Errors: MC_EINVAL, MC_ENOMEM, MC_EBUDGET, MC_EDEVICE. */
int32_t mc_server_create(const mc_server_options *options, const mc_grid *grid, const mc_field_tables *tables,
                         mc_server **out);
/* Stop the worker (resident and pending queries are abandoned) and free everything. */
void mc_server_destroy(mc_server *server);
/* Message of the server's last failed call (server-owned). */
const char *mc_server_last_error(const mc_server *server);
/* Queue a query (one run of the step of mc_step with the query's own ion,
 * source and operating point); *qid receives its id.  Thread-safe.
 * Errors: MC_EINVAL (invalid query), MC_EBUDGET (its memory exceeds the pool). */
int32_t mc_server_submit(mc_server *server, const mc_query *query, uint64_t *qid);
/* Copy the query's state and, once done, its result (the observables of
 * mc_read_tallies plus its exit records and samples).  Thread-safe.
 * MC_EINVAL for an unknown id. */
int32_t mc_server_poll(mc_server *server, uint64_t qid, mc_query_result *out);
/* Block until the query is done (or failed) or timeout_s passes, then poll. */
int32_t mc_server_wait(mc_server *server, uint64_t qid, double timeout_s, mc_query_result *out);
/* Forget a finished query's host result. */
int32_t mc_server_release(mc_server *server, uint64_t qid);
/* Admission, pool and throughput counters of the server. */
int32_t mc_server_get_stats(mc_server *server, mc_server_stats *out);

#ifdef __cplusplus
}
#endif
#endif

// mc_runtime.hip -- host runtime and C ABI of the ion-pack library (gfx950).
//
// One context = one simulation on one GPU: baked field tables, ion species,
// sources, an operating point, a structure-of-arrays pack store, int64
// tallies and an exit-record buffer.  Every per-step operation is a kernel
// from mc_kernels.hpp enqueued on the context stream; the host only keeps
// integer bookkeeping (step counter, slot count, the Eq. 5 emission
// accumulators) and computes the three RF stage coefficients per step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "mc_host.hpp"
#include "mc_kernels.hpp"
#include "mc_poisson.hpp"
#include "mc_sort.hpp"

using namespace mc;

namespace {

constexpr int kBlock = 256;
// blocks of the step kernel: one wavefront each.  Blocks of one wavefront
// leave the smallest last, partly filled round of blocks at the end of a
// launch (the 1e6-pack step took 1.2-2 % less time than with blocks of
// four wavefronts); each block still loads the FP64 step's LDS tables and
// adds its counters once.
constexpr int kStepBlock = 64;
// blocks of the grid-stride aggregation kernels (deposit, snapshot): a few
// per CU, so each block's LDS table absorbs many packs
constexpr int64_t kAggBlocks = 1024;

struct EvPair {
    hipEvent_t a, b;
    int kind;
};

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

struct mc_ctx {
    mc_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    int64_t device_bytes = 0;
    std::vector<std::pair<void *, size_t>> allocs;

    bool has_fields = false, has_op = false;
    int32_t nr = 0, nz = 0;
    double dr = 0, dz = 0, inv_dr = 0, inv_dz = 0, R = 0;

    double2 *e_dc = nullptr, *e_off = nullptr, *e_rf = nullptr, *e_sc = nullptr;
    StepTables *tables = nullptr;  // the FP64 step's logarithm and turn tables
    double *phi_sc = nullptr;
    void *etab = nullptr, *gtab = nullptr;
    float esc[4] = {1, 1, 1, 1}, gsc[4] = {1, 1, 1, 1};
    uint8_t *mask = nullptr, *hit = nullptr;

    unsigned long long *qgrid = nullptr;
    unsigned long long *qrep = nullptr;  // the deposit's copies of the grid (nrep of them, kept zeroed)
    // with sorted slots the deposit flushes straight into a zeroed grid: the
    // other of two grids, cleared by the field bake of the update after it
    unsigned long long *qnext = nullptr;
    int32_t nrep = 1, dep_slot = 0;
    int32_t *dep_range = nullptr;        // three (lowest, highest) node slots, rotating by update
    bool dep_full = true;                // the next sum writes every node (the grid may hold charge anywhere)
    double *sine = nullptr, *tcp = nullptr, *tinv = nullptr;
    void *bh = nullptr;
    Bluestein blu;
    PoissonGrid pg;
    // metal-mask correction (built at the first masked space-charge update)
    std::vector<int32_t> mask_nodes;
    MaskCap mcap;
    double *rhs = nullptr, *phi_tmp = nullptr;
    // adaptive step (Eq. 1)
    unsigned long long *dt_rep = nullptr, *dt_out = nullptr;
    double *dt_rec = nullptr;   // the step record kept on the device (k_dt_finish)
    bool dt_rec_valid = false;  // its next-step time matches t
    double t = 0.0, t_next_pic = 0.0, last_dt = 0.0;
    // trajectory samples
    mc_sample_rec *samples = nullptr;
    unsigned long long *sample_count = nullptr;
    int64_t sample_cap = 0;

    std::vector<mc_ion> ions;
    std::vector<Species> sp_host;
    std::vector<int32_t> charge_host;
    Species *sp_dev = nullptr;
    int32_t *charge_dev = nullptr;

    std::vector<Src> srcs;
    mc_operating op{};

    int64_t cap = 0, n_slots = 0;
    PackPtrs<double> p64{};
    PackPtrs<float> p32{};
    // sorting of the slots (sort_every): the second set of pack arrays the
    // sorted packs are gathered into, and the radix sort's work arrays
    PackPtrs<double> p64b{};
    PackPtrs<float> p32b{};
    uint32_t *skey[2] = {nullptr, nullptr}, *sidx[2] = {nullptr, nullptr}, *shist = nullptr, *stot = nullptr;
    unsigned long long *sactive = nullptr;
    double *retired = nullptr;  // survival-yield sum of the terminal packs whose slots sorts dropped

    unsigned long long *tal = nullptr;  // cnt | exit_bins | loss_map | hist_ke | hist_teff | hist_r
    TallyPtrs tp{};
    int64_t tal_len = 0;
    unsigned long long *snap = nullptr;  // act[2] | act_hist_ke | act_hist_teff
    double *partial = nullptr, *sums = nullptr;
    int64_t partial_len = 0;

    int64_t emitted_n = 0, emitted_w = 0;
    int64_t step = 0;

    std::vector<EvPair> ev_used;
    std::vector<hipEvent_t> ev_pool;
    double t_ms[MC_NKERNEL] = {0};
    int64_t t_launch[MC_NKERNEL] = {0};

    bool fp32() const { return opt.precision == MC_PREC_FP32; }
    bool bf16() const { return fp32() && !opt.fp32_tables; }
};

// ---------------------------------------------------------------------------
// Errors, allocation, timing.
// ---------------------------------------------------------------------------
static int32_t fail(mc_ctx *c, int32_t code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(expr)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(ctx, MC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define LAUNCHCHK()                                                                            \
    do {                                                                                       \
        hipError_t e_ = hipGetLastError();                                                     \
        if (e_ != hipSuccess) return fail(ctx, MC_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e_)); \
    } while (0)

static int32_t dalloc(mc_ctx *ctx, void **out, size_t bytes) {
    *out = nullptr;
    if (bytes == 0) bytes = 256;
    bytes = (bytes + 255) & ~(size_t)255;
    if (ctx->opt.hbm_budget > 0 && ctx->device_bytes + (int64_t)bytes > ctx->opt.hbm_budget)
        return fail(ctx, MC_EBUDGET, "device-memory budget exceeded (" + std::to_string(ctx->device_bytes + bytes) +
                                         " > " + std::to_string(ctx->opt.hbm_budget) + " bytes)");
    void *p = nullptr;
    if (ctx->opt.alloc) {
        p = ctx->opt.alloc(bytes, ctx->stream, ctx->opt.alloc_user);
        if (!p) return fail(ctx, MC_ENOMEM, "allocator callback returned NULL for " + std::to_string(bytes) + " bytes");
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) return fail(ctx, MC_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    ctx->allocs.emplace_back(p, bytes);
    ctx->device_bytes += (int64_t)bytes;
    *out = p;
    return MC_OK;
}

template <class T>
static int32_t dalloc_t(mc_ctx *ctx, T **out, size_t n) {
    void *p = nullptr;
    int32_t rc = dalloc(ctx, &p, n * sizeof(T));
    *out = static_cast<T *>(p);
    return rc;
}

static void dfree_all(mc_ctx *ctx) {
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (auto &a : ctx->allocs) {
        if (ctx->opt.free) ctx->opt.free(a.first, ctx->stream, ctx->opt.alloc_user);
        else (void)hipFree(a.first);
    }
    ctx->allocs.clear();
    ctx->device_bytes = 0;
}

// Timing events come from a pool that is refilled in batches (creating an
// event inside a stretch of steps would stall the host between launches);
// read_timing and reset_timing return the used ones to it.
constexpr int kEventBatch = 1024;
static void ev_fill(mc_ctx *ctx, int n) {
    for (int k = 0; k < n; ++k) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) break;
        ctx->ev_pool.push_back(e);
    }
}
static hipEvent_t ev_get(mc_ctx *ctx) {
    if (ctx->ev_pool.empty()) ev_fill(ctx, kEventBatch);
    if (ctx->ev_pool.empty()) return nullptr;
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
}

struct Timer {
    mc_ctx *ctx;
    int kind;
    hipEvent_t a = nullptr;
    Timer(mc_ctx *c, int k) : ctx(c), kind(k) {
        if (ctx->opt.timing) {
            a = ev_get(ctx);
            if (a) (void)hipEventRecord(a, ctx->stream);
        }
    }
    ~Timer() {
        if (a) {
            hipEvent_t b = ev_get(ctx);
            if (!b) return;
            (void)hipEventRecord(b, ctx->stream);
            ctx->ev_used.push_back(EvPair{a, b, kind});
        }
    }
};

static void resolve_timing(mc_ctx *ctx) {
    for (auto &p : ctx->ev_used) {
        float ms = 0.f;
        (void)hipEventSynchronize(p.b);
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) ctx->t_ms[p.kind] += ms;
        ctx->t_launch[p.kind]++;
        ctx->ev_pool.push_back(p.a);
        ctx->ev_pool.push_back(p.b);
    }
    ctx->ev_used.clear();
}

// ---------------------------------------------------------------------------
// Device views.
// ---------------------------------------------------------------------------
static TallyPtrs tally_ptrs(mc_ctx *ctx) { return ctx->tp; }

template <class Tab>
static const Tab *etab_as(mc_ctx *ctx) { return static_cast<const Tab *>(ctx->etab); }
template <class Tab>
static const Tab *gtab_as(mc_ctx *ctx) { return static_cast<const Tab *>(ctx->gtab); }

static int32_t upload_species(mc_ctx *ctx) {
    const size_t n = ctx->sp_host.size();
    if (n == 0) return MC_OK;
    HIPCHK(hipMemcpyAsync(ctx->sp_dev, ctx->sp_host.data(), n * sizeof(Species), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->charge_dev, ctx->charge_host.data(), n * sizeof(int32_t), hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MC_OK;
}

// One set of pack arrays of the context's capacity.
static int32_t alloc_packs(mc_ctx *ctx, PackPtrs<float> &p) {
    int32_t rc = MC_OK;
    const int64_t cap = ctx->cap;
    float **fl[] = {&p.x, &p.y, &p.z, &p.xl, &p.yl, &p.zl, &p.vx, &p.vy, &p.vz, &p.e, &p.el, &p.h};
    for (auto f : fl)
        if (!rc) rc = dalloc_t(ctx, f, cap);
    if (!rc) rc = dalloc_t(ctx, &p.w, cap);
    if (!rc) rc = dalloc_t(ctx, &p.id, cap);
    if (!rc) rc = dalloc_t(ctx, &p.q, cap);
    if (!rc) rc = dalloc_t(ctx, &p.tag, cap);
    if (!rc) rc = dalloc_t(ctx, &p.status, cap);
    return rc;
}
static int32_t alloc_packs(mc_ctx *ctx, PackPtrs<double> &p) {
    int32_t rc = MC_OK;
    const int64_t cap = ctx->cap;
    double **fl[] = {&p.x, &p.y, &p.z, &p.vx, &p.vy, &p.vz, &p.e, &p.h, &p.w};
    for (auto f : fl)
        if (!rc) rc = dalloc_t(ctx, f, cap);
    if (!rc) rc = dalloc_t(ctx, &p.id, cap);
    if (!rc) rc = dalloc_t(ctx, &p.q, cap);
    if (!rc) rc = dalloc_t(ctx, &p.tag, cap);
    if (!rc) rc = dalloc_t(ctx, &p.status, cap);
    return rc;
}

static void ctx_alpha(mc_ctx *ctx, size_t k) { species_alpha(ctx->sp_host[k], ctx->ions[k], ctx->op.gas_mass_da); }

// ---------------------------------------------------------------------------
// Kernels launches.
// ---------------------------------------------------------------------------
template <class Tab>
static int32_t fold_table(mc_ctx *ctx) {
    const int64_t nn = (int64_t)ctx->nr * ctx->nz;
    k_fold<Tab><<<grid_for(nn), kBlock, 0, ctx->stream>>>(static_cast<Tab *>(ctx->etab), ctx->e_dc, ctx->e_off,
                                                           ctx->e_sc, ctx->e_rf, ctx->op.v_off, nn, ctx->esc[0],
                                                           ctx->esc[1], ctx->esc[2], ctx->esc[3]);
    LAUNCHCHK();
    return MC_OK;
}

static int32_t fold(mc_ctx *ctx) {
    if (!ctx->fp32()) return fold_table<double4>(ctx);
    if (ctx->bf16()) return fold_table<bf16x4>(ctx);
    return fold_table<float4>(ctx);
}

// The field of the new space-charge potential and the step's table from it,
// in one kernel (clear: the other charge grid of a direct deposit, or null).
template <class Tab>
static int32_t bake_fold_table(mc_ctx *ctx, unsigned long long *clear) {
    const int64_t nn = (int64_t)ctx->nr * ctx->nz;
    k_bake_fold<Tab><<<grid_for(nn), kBlock, 0, ctx->stream>>>(ctx->phi_sc, ctx->e_sc, ctx->nr, ctx->nz, ctx->dr,
                                                                ctx->dz, clear, static_cast<Tab *>(ctx->etab),
                                                                ctx->e_dc, ctx->e_off, ctx->e_rf, ctx->op.v_off,
                                                                ctx->esc[0], ctx->esc[1], ctx->esc[2], ctx->esc[3]);
    LAUNCHCHK();
    return MC_OK;
}

static int32_t bake_fold(mc_ctx *ctx, unsigned long long *clear) {
    if (!ctx->fp32()) return bake_fold_table<double4>(ctx, clear);
    if (ctx->bf16()) return bake_fold_table<bf16x4>(ctx, clear);
    return bake_fold_table<float4>(ctx, clear);
}

template <class P, class Tab>
static int32_t launch_emit(mc_ctx *ctx, int si, int64_t count, PackPtrs<typename P::T> p) {
    Src &S = ctx->srcs[si];
    EmitArgs<P, Tab> a{};
    a.p = p;
    a.gtab = gtab_as<Tab>(ctx);
    std::memcpy(a.gsc, ctx->gsc, sizeof(a.gsc));
    a.sp = ctx->sp_dev;
    a.slot0 = ctx->n_slots;
    a.count = count;
    a.id0 = ((int64_t)si << 32) | S.emitted;
    a.step = ctx->step;
    a.sigma_r = S.in.sigma_r;
    a.r_trunc = S.in.r_trunc;
    a.z_inj = S.in.z_inj;
    a.w = S.w;
    a.q = S.q_fx;
    a.inv_dr = ctx->inv_dr;
    a.inv_dz = ctx->inv_dz;
    a.nr = ctx->nr;
    a.nz = ctx->nz;
    a.ion = S.in.ion;
    a.k0 = (uint32_t)ctx->opt.seed;
    a.k1 = (uint32_t)(ctx->opt.seed >> 32);
    Timer t(ctx, MC_K_EMIT);
    k_emit<P, Tab><<<grid_for(count), kBlock, 0, ctx->stream>>>(a);
    LAUNCHCHK();
    return MC_OK;
}

static int32_t emit(mc_ctx *ctx, int si, int64_t count) {
    if (count <= 0) return MC_OK;
    if (ctx->n_slots + count > ctx->cap)
        return fail(ctx, MC_ENOMEM, "pack capacity exceeded (" + std::to_string(ctx->n_slots + count) + " > " +
                                        std::to_string(ctx->cap) + ")");
    int32_t rc;
    if (!ctx->fp32()) rc = launch_emit<P64, double4>(ctx, si, count, ctx->p64);
    else if (ctx->bf16()) rc = launch_emit<P32, bf16x4>(ctx, si, count, ctx->p32);
    else rc = launch_emit<P32, float4>(ctx, si, count, ctx->p32);
    if (rc) return rc;
    Src &S = ctx->srcs[si];
    ctx->n_slots += count;
    S.emitted += count;
    ctx->emitted_n += count;
    ctx->emitted_w += count * S.w_fx;
    return MC_OK;
}

template <class P, class Tab>
static StepArgs<P, Tab> step_args(mc_ctx *ctx, PackPtrs<typename P::T> p, double t0, double dt) {
    StepArgs<P, Tab> a{};
    a.p = p;
    a.etab = etab_as<Tab>(ctx);
    a.gtab = gtab_as<Tab>(ctx);
    std::memcpy(a.esc, ctx->esc, sizeof(a.esc));
    std::memcpy(a.gsc, ctx->gsc, sizeof(a.gsc));
    a.hit = ctx->hit;
    a.sp = ctx->sp_dev;
    a.t = tally_ptrs(ctx);
    a.tables = ctx->tables;
    a.n_slots = ctx->n_slots;
    a.step = ctx->step;
    const mc_operating &op = ctx->op;
    a.dt = dt;
    a.t0 = t0;
    double c[3];
    rf_stages_at(op, t0, dt, c);
    a.c0 = c[0];
    a.ch = c[1];
    a.c1 = c[2];
    a.z_det = op.z_det;
    a.r_det = op.r_det;
    a.R = ctx->R;
    a.inv_dr = ctx->inv_dr;
    a.inv_dz = ctx->inv_dz;
    a.mg = op.gas_mass_da * kDa;
    a.exit_bin_dt = op.exit_bin_dt;
    a.nr = ctx->nr;
    a.nz = ctx->nz;
    a.n_exit_bins = op.n_exit_bins;
    a.collisions_on = op.collisions_on;
    a.langevin_on = op.langevin_on;
    a.lv_z_lo = op.lv_z_lo;
    a.lv_z_hi = op.lv_z_hi;
    a.lv_switch = op.lv_switch;
    a.lv_dt_ref = op.dt;
    a.k0 = (uint32_t)ctx->opt.seed;
    a.k1 = (uint32_t)(ctx->opt.seed >> 32);
    return a;
}

template <class P, class Tab>
static int32_t launch_step(mc_ctx *ctx, PackPtrs<typename P::T> p, double t0, double dt, const double *dyn) {
    if (ctx->n_slots == 0) return MC_OK;
    StepArgs<P, Tab> a = step_args<P, Tab>(ctx, p, t0, dt);
    a.dyn = dyn;
    Timer t(ctx, MC_K_STEP);
    const unsigned nb = (unsigned)((ctx->n_slots + kStepBlock - 1) / kStepBlock);
    // one species defined: every pack carries tag 0 (tags are checked
    // against the species on write, and sources name a defined species)
    if (ctx->ions.size() == 1)
        k_step<P, Tab, true><<<nb, kStepBlock, 0, ctx->stream>>>(a);
    else
        k_step<P, Tab, false><<<nb, kStepBlock, 0, ctx->stream>>>(a);
    LAUNCHCHK();
    return MC_OK;
}

static int32_t step_once(mc_ctx *ctx, double t0, double dt, const double *dyn = nullptr) {
    if (!ctx->fp32()) return launch_step<P64, double4>(ctx, ctx->p64, t0, dt, dyn);
    if (ctx->bf16()) return launch_step<P32, bf16x4>(ctx, ctx->p32, t0, dt, dyn);
    return launch_step<P32, float4>(ctx, ctx->p32, t0, dt, dyn);
}

// Eq. 1 limits over the active packs at t0: returns the smallest per-pack
// limit (+inf with no packs) and whether a pack takes the Langevin branch.
template <class P, class Tab>
static int32_t pack_limits_t(mc_ctx *ctx, PackPtrs<typename P::T> p, double t0, double *lim, bool *lang) {
    if (ctx->n_slots > 0) {
        const StepArgs<P, Tab> a = step_args<P, Tab>(ctx, p, t0, ctx->op.dt);
        k_dt_limits<P, Tab><<<grid_for(ctx->n_slots), kBlock, 0, ctx->stream>>>(a, ctx->dt_rep);
        LAUNCHCHK();
    }
    k_dt_reduce<<<1, kHotRep, 0, ctx->stream>>>(ctx->dt_rep, ctx->dt_out);
    LAUNCHCHK();
    unsigned long long h[2];
    HIPCHK(hipMemcpyAsync(h, ctx->dt_out, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    std::memcpy(lim, &h[0], sizeof(double));
    *lang = h[1] != 0;
    return MC_OK;
}

// The Eq. 1 limits of this step into the replica lines, with the RF
// coefficient of the step's start from the device record.
template <class P, class Tab>
static int32_t pack_limits_dev(mc_ctx *ctx, PackPtrs<typename P::T> p) {
    if (ctx->n_slots == 0) return MC_OK;
    StepArgs<P, Tab> a = step_args<P, Tab>(ctx, p, 0.0, ctx->op.dt);
    a.dyn = ctx->dt_rec;
    k_dt_limits<P, Tab><<<grid_for(ctx->n_slots), kBlock, 0, ctx->stream>>>(a, ctx->dt_rep);
    LAUNCHCHK();
    return MC_OK;
}

static int32_t adaptive_buffers(mc_ctx *ctx) {
    if (ctx->dt_rep) return MC_OK;
    int32_t rc = dalloc_t(ctx, &ctx->dt_rep, (size_t)kHotLen);
    if (!rc) rc = dalloc_t(ctx, &ctx->dt_out, 2);
    if (!rc) rc = dalloc_t(ctx, &ctx->dt_rec, 8);
    if (rc) return rc;
    k_dt_reset<<<1, kHotRep, 0, ctx->stream>>>(ctx->dt_rep);
    LAUNCHCHK();
    return MC_OK;
}

static int32_t adaptive_dt(mc_ctx *ctx, double t0, double *dt) {
    double lim = HUGE_VAL;
    bool lang = false;
    int32_t rc = adaptive_buffers(ctx);
    if (rc) return rc;
    if (!ctx->fp32()) rc = pack_limits_t<P64, double4>(ctx, ctx->p64, t0, &lim, &lang);
    else if (ctx->bf16()) rc = pack_limits_t<P32, bf16x4>(ctx, ctx->p32, t0, &lim, &lang);
    else rc = pack_limits_t<P32, float4>(ctx, ctx->p32, t0, &lim, &lang);
    if (rc) return rc;
    const mc_operating &op = ctx->op;
    double d = std::min(op.dt, lim);
    if (op.v_rf != 0.0 && op.f_rf > 0.0) d = std::min(d, 0.05 / op.f_rf);
    if (lang && op.lv_dt_max > 0.0) d = std::min(d, op.lv_dt_max);
    if (op.sc_on) d = std::min(d, ctx->t_next_pic - t0);
    if (!(d > 1e-9 * op.dt)) return fail(ctx, MC_ENUMERIC, "adaptive step collapsed to " + std::to_string(d) + " s");
    *dt = d;
    return MC_OK;
}

// Capacitance matrix of the metal-mask nodes: one FP64 solve per node, once
// per grid (at the first space-charge update that asks for the mask
// condition).  The matrix is always built and inverted in FP64, also for the
// FP32 form: its inverse maps the potential on the mask to induced charges,
// and single-precision columns would lose digits to its conditioning.
static int32_t mask_setup(mc_ctx *ctx) {
    const int32_t M = (int32_t)ctx->mask_nodes.size();
    if (M > kMaxMaskNodes)
        return fail(ctx, MC_EINVAL, "the metal mask has " + std::to_string(M) +
                                        " interior nodes; the correction holds at most " + std::to_string(kMaxMaskNodes));
    const int64_t nn = (int64_t)ctx->nr * ctx->nz;
    const int32_t m = ctx->nz - 2, nu = ctx->nr - 1;
    int32_t rc = MC_OK;
    if (!ctx->rhs) rc = dalloc_t(ctx, &ctx->rhs, nn);
    if (!rc && !ctx->phi_tmp) rc = dalloc_t(ctx, &ctx->phi_tmp, nn);
    if (!rc && M > 0) rc = dalloc_t(ctx, &ctx->mcap.nodes, M);
    if (!rc && M > 0) rc = dalloc_t(ctx, &ctx->mcap.cinv, (size_t)M * M);
    if (rc) return rc;
    HIPCHK(hipMemsetAsync(ctx->rhs, 0, nn * sizeof(double), ctx->stream));
    PoissonGrid g64 = ctx->pg;
    double *bh64 = static_cast<double *>(ctx->bh);
    Bluestein b64;
    if (ctx->fp32()) {
        // FP64 transform tables and work array for the setup solves
        rc = dalloc_t(ctx, &bh64, (size_t)nu * m);
        const int32_t L = bluestein_length(m);
        const size_t cx = 2 * sizeof(double);
        if (!rc && bluestein_lds(L, cx) <= lds_per_block()) {
            b64.L = L;
            b64.lds = bluestein_lds(L, cx);
            rc = dalloc(ctx, &b64.chirp, (size_t)m * cx);
            if (!rc) rc = dalloc(ctx, &b64.tw, (size_t)std::max(L / 2, 1) * cx);
            if (!rc) rc = dalloc(ctx, &b64.fb, (size_t)L * cx);
            if (!rc && bluestein_prepare<double>(b64, m, ctx->stream) != hipSuccess) b64.L = 0;
        }
        if (rc) return rc;
        g64.blu = &b64;
    }
    const std::string err = mask_prepare<double>(g64, ctx->mcap, ctx->mask_nodes, bh64, ctx->rhs, ctx->phi_tmp,
                                                 ctx->stream);
    if (!err.empty()) return fail(ctx, MC_EDEVICE, err);
    return MC_OK;
}

// ---------------------------------------------------------------------------
// Sorting of the slots by (species, cell) with the terminal slots dropped
// (mc_sort.hpp).  The work arrays and the second set of pack arrays are
// allocated at the first sort.  One host read of the active count per sort.
// ---------------------------------------------------------------------------
static int32_t sort_buffers(mc_ctx *ctx) {
    if (ctx->sactive) return MC_OK;
    if (ctx->cap > kSortMaxSlots) return fail(ctx, MC_EINVAL, "sorting needs pack_capacity <= 2^28");
    int32_t rc = ctx->fp32() ? alloc_packs(ctx, ctx->p32b) : alloc_packs(ctx, ctx->p64b);
    const int64_t tiles = (ctx->cap + kSortTile - 1) / kSortTile;
    for (int k = 0; k < 2 && !rc; ++k) {
        rc = dalloc_t(ctx, &ctx->skey[k], ctx->cap);
        if (!rc) rc = dalloc_t(ctx, &ctx->sidx[k], ctx->cap);
    }
    if (!rc) rc = dalloc_t(ctx, &ctx->shist, (size_t)kRadixBins * tiles);
    if (!rc) rc = dalloc_t(ctx, &ctx->stot, (size_t)(kRadixBins * tiles + kSortTile - 1) / kSortTile);
    if (!rc) rc = dalloc_t(ctx, &ctx->sactive, 1);
    if (rc) ctx->sactive = nullptr;
    return rc;
}

template <class T>
static int32_t sort_packs_t(mc_ctx *ctx, PackPtrs<T> &p, PackPtrs<T> &alt) {
    const int64_t n = ctx->n_slots;
    const int64_t nn = (int64_t)ctx->nr * ctx->nz, n_keys = (int64_t)ctx->ions.size() * nn;
    if (n_keys >= (int64_t)0xFFFFFFFF) return fail(ctx, MC_EINVAL, "too many (species x node) keys to sort");
    int32_t rc = sort_buffers(ctx);
    if (rc) return rc;
    const int passes = sort_passes(n_keys);
    const uint32_t dead = passes == 4 ? 0xFFFFFFFFu : (uint32_t)((1ull << (8 * passes)) - 1);
    const int64_t tiles = (n + kSortTile - 1) / kSortTile, hlen = kRadixBins * tiles;
    const unsigned scan_blocks = (unsigned)((hlen + kSortTile - 1) / kSortTile);
    {
        Timer t(ctx, MC_K_SORT);
        k_sort_keys<T><<<grid_for(n), kBlock, 0, ctx->stream>>>(p, n, ctx->nr, ctx->nz, ctx->inv_dr, ctx->inv_dz, nn,
                                                                dead, ctx->skey[0], ctx->sidx[0], ctx->partial);
        LAUNCHCHK();
        k_retire<<<1, kBlock, 0, ctx->stream>>>(ctx->partial, (int64_t)grid_for(n), ctx->sactive, ctx->retired);
        LAUNCHCHK();
        int cur = 0;
        for (int pass = 0; pass < passes; ++pass) {
            const int32_t shift = 8 * pass;
            k_radix_count<<<(unsigned)tiles, kSortThreads, 0, ctx->stream>>>(ctx->skey[cur], n, shift, ctx->shist,
                                                                             tiles);
            LAUNCHCHK();
            k_scan_tiles<<<scan_blocks, kSortThreads, 0, ctx->stream>>>(ctx->shist, hlen, ctx->stot);
            LAUNCHCHK();
            k_scan_totals<<<1, kSortThreads, 0, ctx->stream>>>(ctx->stot, scan_blocks);
            LAUNCHCHK();
            k_radix_scatter<<<(unsigned)tiles, kSortThreads, 0, ctx->stream>>>(
                ctx->skey[cur], ctx->sidx[cur], ctx->skey[1 - cur], ctx->sidx[1 - cur], n, shift, ctx->shist,
                ctx->stot, tiles);
            LAUNCHCHK();
            cur = 1 - cur;
        }
        k_sort_permute<T><<<grid_for(n), kBlock, 0, ctx->stream>>>(p, alt, ctx->sidx[cur], n, ctx->sactive);
        LAUNCHCHK();
    }
    unsigned long long active = 0;
    HIPCHK(hipMemcpyAsync(&active, ctx->sactive, sizeof(active), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    std::swap(p, alt);
    ctx->n_slots = (int64_t)active;
    return MC_OK;
}

// The sort at the start of step `step` when one is due (every sort_every
// steps, counted from step 0).
static int32_t sort_if_due(mc_ctx *ctx) {
    if (!(ctx->op.sort_every > 0 && ctx->step % ctx->op.sort_every == 0 && ctx->n_slots > 0)) return MC_OK;
    return ctx->fp32() ? sort_packs_t(ctx, ctx->p32, ctx->p32b) : sort_packs_t(ctx, ctx->p64, ctx->p64b);
}

// Grid buffer the deposit adds into directly (sorted slots): allocated and
// zeroed once, and from then on cleared by the field bake of the update
// after the deposit that used it.
static int32_t direct_grid(mc_ctx *ctx) {
    if (ctx->qnext) return MC_OK;
    const int64_t nn = (int64_t)ctx->nr * ctx->nz;
    int32_t rc = dalloc_t(ctx, &ctx->qnext, nn);
    if (rc) return rc;
    HIPCHK(hipMemsetAsync(ctx->qnext, 0, nn * sizeof(unsigned long long), ctx->stream));
    return MC_OK;
}

template <class P, class D>
static int32_t pic_update_t(mc_ctx *ctx, PackPtrs<typename P::T> p) {
    const int64_t nn = (int64_t)ctx->nr * ctx->nz;
    // sorted slots: one deposit kernel adding straight into the zeroed grid
    const bool direct = ctx->op.sort_every > 0;
    if (direct) {
        int32_t rc = direct_grid(ctx);
        if (rc) return rc;
        Timer t(ctx, MC_K_DEPOSIT);
        if (ctx->n_slots > 0) {
            DepositArgs<typename P::T> a{};
            a.p = p;
            a.q = ctx->qnext;
            a.n_slots = ctx->n_slots;
            a.nn = nn;
            a.inv_dr = ctx->inv_dr;
            a.inv_dz = ctx->inv_dz;
            a.nr = ctx->nr;
            a.nz = ctx->nz;
            unsigned nb;
            deposit_shape(ctx->n_slots, &nb, &a.chunk);
            k_deposit<P><<<nb, kDepositThreads, 0, ctx->stream>>>(a);
            LAUNCHCHK();
        }
        std::swap(ctx->qgrid, ctx->qnext);  // qnext now holds the previous deposit: cleared below
        ctx->dep_full = true;               // a later sum over copies must write every node
    } else {
        Timer t(ctx, MC_K_DEPOSIT);
        // slots: this deposit's range, the previous deposit's, and the next one's
        int32_t *range = ctx->dep_range + 2 * ctx->dep_slot, *prev = ctx->dep_range + 2 * ((ctx->dep_slot + 2) % 3),
                *next = ctx->dep_range + 2 * ((ctx->dep_slot + 1) % 3);
        if (ctx->n_slots > 0) {
            DepositArgs<typename P::T> a{};
            a.p = p;
            a.q = ctx->qgrid;
            a.qrep = ctx->qrep;
            a.range = range;
            a.n_slots = ctx->n_slots;
            a.nn = nn;
            a.inv_dr = ctx->inv_dr;
            a.inv_dz = ctx->inv_dz;
            a.nr = ctx->nr;
            a.nz = ctx->nz;
            a.nrep = ctx->nrep;
            unsigned nb;
            deposit_shape(ctx->n_slots, &nb, &a.chunk);
            k_deposit<P><<<nb, kDepositThreads, 0, ctx->stream>>>(a);
            LAUNCHCHK();
        }
        // the grid from the copies: the nodes of this deposit's range and the
        // previous one's are written, the rest of the grid is zero already
        const unsigned sb = (unsigned)std::min<int64_t>(grid_for(nn), kDepositSumBlocks);
        k_deposit_sum<<<sb, kBlock, 0, ctx->stream>>>(ctx->qgrid, ctx->qrep, ctx->nrep, nn, range,
                                                      ctx->dep_full ? nullptr : prev, next);
        LAUNCHCHK();
        ctx->dep_slot = (ctx->dep_slot + 1) % 3;
        ctx->dep_full = false;
    }
    if (ctx->op.sc_mask && !ctx->mcap.ready) {
        const int32_t rc = mask_setup(ctx);
        if (rc) return rc;
    }
    {
        Timer t(ctx, MC_K_POISSON);
        D *bh = static_cast<D *>(ctx->bh);
        HIPCHK(poisson_solve<D>(ctx->pg, ctx->qgrid, nullptr, bh, ctx->phi_sc, false, ctx->stream));
        if (ctx->op.sc_mask) HIPCHK(mask_correct<D>(ctx->pg, ctx->mcap, bh, ctx->rhs, ctx->phi_sc, ctx->stream));
    }
    {
        Timer t(ctx, MC_K_FIELD);
        const int32_t rc = bake_fold(ctx, direct ? ctx->qnext : nullptr);
        if (rc) return rc;
    }
    return MC_OK;
}

static int32_t pic_update(mc_ctx *ctx) {
    if (!ctx->fp32()) return pic_update_t<P64, double>(ctx, ctx->p64);
    return pic_update_t<P32, float>(ctx, ctx->p32);
}

template <class T>
static int32_t snapshot_t(mc_ctx *ctx, PackPtrs<T> p) {
    const int64_t ns = 2 + MC_HIST_KE + MC_HIST_TEFF;
    Timer t(ctx, MC_K_TALLY);
    k_zero_u64<<<grid_for(ns), kBlock, 0, ctx->stream>>>(ctx->snap, ns);
    LAUNCHCHK();
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>((ctx->n_slots + kBlock - 1) / kBlock, kAggBlocks));
    if (ctx->n_slots > 0) {
        k_snapshot<T><<<(unsigned)nb, kBlock, 0, ctx->stream>>>(p, ctx->sp_dev, ctx->n_slots, ctx->snap,
                                                               ctx->snap + 2, ctx->snap + 2 + MC_HIST_KE, ctx->partial);
        LAUNCHCHK();
    }
    // with no slots the sums are zero, save the terminal packs a sort retired
    k_reduce_partials<<<1, kBlock, 0, ctx->stream>>>(ctx->partial, ctx->n_slots > 0 ? nb : 0, ctx->sums,
                                                     ctx->retired);
    LAUNCHCHK();
    return MC_OK;
}

// ---------------------------------------------------------------------------
// ABI.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Checkpoint and resume.  The file holds the dynamic state of a context: a
// header (configuration fingerprint, step, time, emission counters), each
// source's accumulator, then the device arrays -- pack slots, the tally
// block (counters, exit bins, loss map, histograms), the exit records taken,
// the space-charge field, potential and charge grid, and the samples.  The
// configuration itself (fields, ions, sources, operating point) is the
// caller's to set up identically before mc_load_state; the fingerprint is
// checked so that a mismatch fails instead of resuming a different run.
// ---------------------------------------------------------------------------
namespace {

struct CkptHeader {
    char magic[8];
    int32_t abi, precision, nr, nz, n_ions, n_srcs, n_exit_bins, fp32_tables;
    int64_t cap, n_slots, step, emitted_n, emitted_w, tal_len, n_exits, n_samples;
    double t, t_next_pic, last_dt;
    uint64_t seed;
};
constexpr char kCkptMagic[8] = {'M', 'U', 'C', 'K', 'P', 'T', '0', '1'};

struct Blob {
    void *dev;
    size_t bytes;
};

// The device arrays of a checkpoint, in file order.
std::vector<Blob> ckpt_blobs(mc_ctx *ctx, int64_t n_slots, int64_t n_exits, int64_t n_samples) {
    std::vector<Blob> v;
    const size_t n = (size_t)n_slots, nn = (size_t)ctx->nr * ctx->nz;
    if (!ctx->fp32()) {
        const PackPtrs<double> &p = ctx->p64;
        for (double *a : {p.x, p.y, p.z, p.vx, p.vy, p.vz, p.e, p.h, p.w}) v.push_back({a, n * 8});
        v.push_back({p.id, n * 8});
        v.push_back({p.q, n * 8});
        v.push_back({p.tag, n * 4});
        v.push_back({p.status, n * 4});
    } else {
        const PackPtrs<float> &p = ctx->p32;
        for (float *a : {p.x, p.y, p.z, p.xl, p.yl, p.zl, p.vx, p.vy, p.vz, p.e, p.el, p.h}) v.push_back({a, n * 4});
        v.push_back({p.w, n * 8});
        v.push_back({p.id, n * 8});
        v.push_back({p.q, n * 8});
        v.push_back({p.tag, n * 4});
        v.push_back({p.status, n * 4});
    }
    v.push_back({ctx->tal, (size_t)ctx->tal_len * 8});
    v.push_back({ctx->tp.exits, (size_t)n_exits * sizeof(mc_exit_rec)});
    v.push_back({ctx->e_sc, nn * sizeof(double2)});
    v.push_back({ctx->phi_sc, nn * 8});
    v.push_back({ctx->qgrid, nn * 8});
    v.push_back({ctx->samples, (size_t)n_samples * sizeof(mc_sample_rec)});
    v.push_back({ctx->sample_count, 8});
    v.push_back({ctx->retired, 8});
    return v;
}

CkptHeader ckpt_header(const mc_ctx *ctx) {
    CkptHeader h{};
    std::memcpy(h.magic, kCkptMagic, 8);
    h.abi = MC_ABI_VERSION;
    h.precision = ctx->opt.precision;
    h.nr = ctx->nr;
    h.nz = ctx->nz;
    h.n_ions = (int32_t)ctx->ions.size();
    h.n_srcs = (int32_t)ctx->srcs.size();
    h.n_exit_bins = ctx->op.n_exit_bins;
    h.fp32_tables = ctx->opt.fp32_tables;
    h.cap = ctx->cap;
    h.n_slots = ctx->n_slots;
    h.step = ctx->step;
    h.emitted_n = ctx->emitted_n;
    h.emitted_w = ctx->emitted_w;
    h.tal_len = ctx->tal_len;
    h.t = ctx->t;
    h.t_next_pic = ctx->t_next_pic;
    h.last_dt = ctx->last_dt;
    h.seed = ctx->opt.seed;
    return h;
}

}  // namespace

extern "C" {

int32_t mc_abi_version(void) { return MC_ABI_VERSION; }

const char *mc_last_error(const mc_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int32_t mc_create(const mc_options *o, mc_ctx **out) {
    if (!o || !out) return MC_EINVAL;
    *out = nullptr;
    if (o->pack_capacity <= 0 || (o->precision != MC_PREC_FP64 && o->precision != MC_PREC_FP32) ||
        (!o->alloc) != (!o->free) || o->sample_capacity < 0)
        return MC_EINVAL;
    mc_ctx *ctx = new (std::nothrow) mc_ctx();
    if (!ctx) return MC_ENOMEM;
    ctx->opt = *o;
    hipError_t e = hipSetDevice(o->device);
    if (e != hipSuccess) {
        delete ctx;
        return MC_EDEVICE;
    }
    if (o->stream) {
        ctx->stream = static_cast<hipStream_t>(o->stream);
    } else {
        e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
        if (e != hipSuccess) {
            delete ctx;
            return MC_EDEVICE;
        }
        ctx->own_stream = true;
    }
    ctx->cap = o->pack_capacity;
    const int64_t cap = ctx->cap;
    int32_t rc = ctx->fp32() ? alloc_packs(ctx, ctx->p32) : alloc_packs(ctx, ctx->p64);
    const int64_t ecap = o->exit_capacity > 0 ? o->exit_capacity : cap;
    ctx->tp.exit_cap = ecap;
    if (!rc) rc = dalloc_t(ctx, &ctx->tp.exits, ecap);
    if (!rc) rc = dalloc_t(ctx, &ctx->sp_dev, 64);
    if (!rc) rc = dalloc_t(ctx, &ctx->charge_dev, 64);
    ctx->partial_len = (cap + kBlock - 1) / kBlock;
    if (!rc) rc = dalloc_t(ctx, &ctx->partial, 3 * ctx->partial_len);
    if (!rc) rc = dalloc_t(ctx, &ctx->sums, 4);
    if (!rc) rc = dalloc_t(ctx, &ctx->retired, 1);
    if (!rc && hipMemsetAsync(ctx->retired, 0, sizeof(double), ctx->stream) != hipSuccess)
        rc = fail(ctx, MC_EDEVICE, "clearing the retired sum");
    if (!rc) rc = dalloc_t(ctx, &ctx->snap, 2 + MC_HIST_KE + MC_HIST_TEFF);
    ctx->sample_cap = o->sample_capacity;
    if (!rc && ctx->sample_cap > 0) rc = dalloc_t(ctx, &ctx->samples, ctx->sample_cap);
    if (!rc) rc = dalloc_t(ctx, &ctx->sample_count, 1);
    if (!rc && hipMemsetAsync(ctx->sample_count, 0, sizeof(unsigned long long), ctx->stream) != hipSuccess)
        rc = fail(ctx, MC_EDEVICE, "clearing the sample counter");
    if (!rc) rc = dalloc_t(ctx, &ctx->tables, 1);
    if (!rc) {
        StepTables host;
        step_tables_fill(&host);
        if (hipMemcpyAsync(ctx->tables, &host, sizeof(host), hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
            hipStreamSynchronize(ctx->stream) != hipSuccess)
            rc = fail(ctx, MC_EDEVICE, "uploading the step tables");
    }
    if (rc) {
        std::string msg = ctx->err;
        mc_destroy(ctx);
        std::fprintf(stderr, "mc_create: %s\n", msg.c_str());
        return rc;
    }
    *out = ctx;
    return MC_OK;
}

void mc_destroy(mc_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->opt.device);
    dfree_all(ctx);
    for (auto &p : ctx->ev_used) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

static double absmax(const double *a, int64_t n) {
    double m = 0.0;
    if (!a) return 0.0;
    for (int64_t k = 0; k < n; ++k) m = std::max(m, std::fabs(a[k]));
    return m;
}

static float scale_of(double m) { return m > 0.0 ? (float)m : 1.0f; }

int32_t mc_load_fields(mc_ctx *ctx, const mc_grid *g, const mc_field_tables *t) {
    if (!ctx) return MC_EINVAL;
    if (!g || !t || !t->phi_dc || !t->gas_p || !t->gas_t) return fail(ctx, MC_EINVAL, "missing grid or tables");
    if (g->nr < 3 || g->nz < 3 || !(g->dr > 0) || !(g->dz > 0)) return fail(ctx, MC_EINVAL, "bad grid");
    if (ctx->has_fields) return fail(ctx, MC_ESTATE, "fields already loaded");
    if (!valid_tables(t, (int64_t)g->nr * g->nz))
        return fail(ctx, MC_EINVAL, "field table with a non-finite value or a negative pressure or temperature");
    HIPCHK(hipSetDevice(ctx->opt.device));
    ctx->nr = g->nr;
    ctx->nz = g->nz;
    ctx->dr = g->dr;
    ctx->dz = g->dz;
    ctx->inv_dr = 1.0 / g->dr;
    ctx->inv_dz = 1.0 / g->dz;
    ctx->R = (g->nr - 1) * g->dr;
    const int64_t nn = (int64_t)g->nr * g->nz;
    const int32_t m = g->nz - 2, nu = g->nr - 1;
    int32_t rc = MC_OK;
    double *tmp = nullptr;
    if (!rc) rc = dalloc_t(ctx, &ctx->e_dc, nn);
    if (!rc) rc = dalloc_t(ctx, &ctx->e_off, nn);
    if (!rc) rc = dalloc_t(ctx, &ctx->e_rf, nn);
    if (!rc) rc = dalloc_t(ctx, &ctx->e_sc, nn);
    if (!rc) rc = dalloc_t(ctx, &ctx->phi_sc, nn);
    if (!rc) rc = dalloc_t(ctx, &ctx->mask, nn);
    if (!rc) rc = dalloc_t(ctx, &ctx->hit, nn);
    if (!rc) rc = dalloc_t(ctx, &ctx->qgrid, nn);
    ctx->nrep = deposit_copies(nn);
    if (!rc) rc = dalloc_t(ctx, &ctx->qrep, (size_t)ctx->nrep * nn);
    if (!rc) rc = dalloc_t(ctx, &ctx->dep_range, 6);
    if (!rc) rc = dalloc_t(ctx, &ctx->sine, 2 * (int64_t)(g->nz - 1));
    if (!rc) rc = dalloc_t(ctx, &ctx->tcp, (int64_t)nu * m);
    if (!rc) rc = dalloc_t(ctx, &ctx->tinv, (int64_t)nu * m);
    if (!rc) rc = dalloc(ctx, &ctx->bh, (size_t)nu * m * (ctx->fp32() ? sizeof(float) : sizeof(double)));
    const size_t node_bytes = !ctx->fp32() ? sizeof(double4) : (ctx->bf16() ? sizeof(bf16x4) : sizeof(float4));
    if (!rc) rc = dalloc(ctx, &ctx->etab, nn * node_bytes);
    if (!rc) rc = dalloc(ctx, &ctx->gtab, nn * node_bytes);
    // tallies: counters, exit bins (allocated at set_operating), loss map, histograms
    if (!rc) rc = dalloc_t(ctx, &tmp, 4 * nn);  // staging for the raw tables, released below
    if (rc) return rc;
    HIPCHK(hipMemsetAsync(ctx->e_sc, 0, nn * sizeof(double2), ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->phi_sc, 0, nn * sizeof(double), ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->e_off, 0, nn * sizeof(double2), ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->e_rf, 0, nn * sizeof(double2), ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->qgrid, 0, nn * sizeof(unsigned long long), ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->qrep, 0, (size_t)ctx->nrep * nn * sizeof(unsigned long long), ctx->stream));
    {
        static const int32_t empty[6] = {INT32_MAX, -1, INT32_MAX, -1, INT32_MAX, -1};
        HIPCHK(hipMemcpyAsync(ctx->dep_range, empty, sizeof(empty), hipMemcpyHostToDevice, ctx->stream));
        ctx->dep_slot = 0;
        ctx->dep_full = true;
    }
    // bake E = -grad(phi) for the three potentials
    const double *phis[3] = {t->phi_dc, t->phi_off, t->phi_rf};
    double2 *outs[3] = {ctx->e_dc, ctx->e_off, ctx->e_rf};
    for (int k = 0; k < 3; ++k) {
        if (!phis[k]) continue;
        HIPCHK(hipMemcpyAsync(tmp, phis[k], nn * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        k_bake<<<grid_for(nn), kBlock, 0, ctx->stream>>>(tmp, outs[k], g->nr, g->nz, g->dr, g->dz, nullptr);
        LAUNCHCHK();
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    // gas table (u_r, u_z, p, T)
    const double *gas[4] = {t->gas_ur, t->gas_uz, t->gas_p, t->gas_t};
    for (int k = 0; k < 4; ++k) {
        if (gas[k]) HIPCHK(hipMemcpyAsync(tmp + k * nn, gas[k], nn * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        else HIPCHK(hipMemsetAsync(tmp + k * nn, 0, nn * sizeof(double), ctx->stream));
        ctx->gsc[k] = scale_of(absmax(gas[k], nn));
    }
    if (!ctx->fp32())
        k_gas<double4><<<grid_for(nn), kBlock, 0, ctx->stream>>>(static_cast<double4 *>(ctx->gtab), tmp, tmp + nn,
                                                                  tmp + 2 * nn, tmp + 3 * nn, nn, 1, 1, 1, 1);
    else if (ctx->bf16())
        k_gas<bf16x4><<<grid_for(nn), kBlock, 0, ctx->stream>>>(static_cast<bf16x4 *>(ctx->gtab), tmp, tmp + nn,
                                                                 tmp + 2 * nn, tmp + 3 * nn, nn, ctx->gsc[0],
                                                                 ctx->gsc[1], ctx->gsc[2], ctx->gsc[3]);
    else
        k_gas<float4><<<grid_for(nn), kBlock, 0, ctx->stream>>>(static_cast<float4 *>(ctx->gtab), tmp, tmp + nn,
                                                                 tmp + 2 * nn, tmp + 3 * nn, nn, 1, 1, 1, 1);
    LAUNCHCHK();
    if (!ctx->bf16()) std::fill(ctx->gsc, ctx->gsc + 4, 1.0f);
    if (t->mask) HIPCHK(hipMemcpyAsync(ctx->mask, t->mask, nn, hipMemcpyHostToDevice, ctx->stream));
    else HIPCHK(hipMemsetAsync(ctx->mask, 0, nn, ctx->stream));
    k_sine_table<<<grid_for(2 * (g->nz - 1)), kBlock, 0, ctx->stream>>>(ctx->sine, g->nz);
    LAUNCHCHK();
    k_thomas_coef<<<grid_for(m), kBlock, 0, ctx->stream>>>(ctx->tcp, ctx->tinv, g->nr, g->nz, g->dr, g->dz);
    LAUNCHCHK();
    // chirp z sine transform tables when the FFT length fits in LDS
    {
        Bluestein &B = ctx->blu;
        const size_t cx = ctx->fp32() ? 2 * sizeof(float) : 2 * sizeof(double);
        const int32_t L = bluestein_length(m);
        if (bluestein_lds(L, cx) <= lds_per_block()) {
            B.L = L;
            B.lds = bluestein_lds(L, cx);
            int32_t rc2 = dalloc(ctx, &B.chirp, (size_t)m * cx);
            if (!rc2) rc2 = dalloc(ctx, &B.tw, (size_t)std::max(L / 2, 1) * cx);
            if (!rc2) rc2 = dalloc(ctx, &B.fb, (size_t)L * cx);
            if (rc2) return rc2;
            const hipError_t e = ctx->fp32() ? bluestein_prepare<float>(B, m, ctx->stream)
                                             : bluestein_prepare<double>(B, m, ctx->stream);
            if (e != hipSuccess) B.L = 0;  // fall back to the direct sine sums
        }
    }
    ctx->pg.nr = g->nr;
    ctx->pg.nz = g->nz;
    ctx->pg.dr = g->dr;
    ctx->pg.dz = g->dz;
    ctx->pg.sine = ctx->sine;
    ctx->pg.tcp = ctx->tcp;
    ctx->pg.tinv = ctx->tinv;
    ctx->pg.blu = &ctx->blu;
    ctx->mask_nodes = mask_unknowns(t->mask, g->nr, g->nz);
    HIPCHK(hipStreamSynchronize(ctx->stream));
    // the staging buffer is returned at once
    for (size_t k = 0; k < ctx->allocs.size(); ++k)
        if (ctx->allocs[k].first == tmp) {
            if (ctx->opt.free) ctx->opt.free(tmp, ctx->stream, ctx->opt.alloc_user);
            else HIPCHK(hipFree(tmp));
            ctx->device_bytes -= (int64_t)ctx->allocs[k].second;
            ctx->allocs.erase(ctx->allocs.begin() + k);
            break;
        }
    // E-table scales for the BF16 form: the largest magnitude of each static channel
    if (ctx->bf16()) {
        std::vector<double2> h(nn);
        double mx[4] = {0, 0, 0, 0};
        HIPCHK(hipMemcpy(h.data(), ctx->e_dc, nn * sizeof(double2), hipMemcpyDeviceToHost));
        for (auto &v : h) { mx[0] = std::max(mx[0], std::fabs(v.x)); mx[1] = std::max(mx[1], std::fabs(v.y)); }
        HIPCHK(hipMemcpy(h.data(), ctx->e_rf, nn * sizeof(double2), hipMemcpyDeviceToHost));
        for (auto &v : h) { mx[2] = std::max(mx[2], std::fabs(v.x)); mx[3] = std::max(mx[3], std::fabs(v.y)); }
        for (int k = 0; k < 4; ++k) ctx->esc[k] = scale_of(mx[k]);
    }
    ctx->has_fields = true;
    return MC_OK;
}

int32_t mc_define_ion(mc_ctx *ctx, const mc_ion *ion, int32_t *ion_id) {
    if (!ctx) return MC_EINVAL;
    if (!valid_ion(ion)) return fail(ctx, MC_EINVAL, "invalid ion template");
    if (ctx->ions.size() >= 64) return fail(ctx, MC_ENOMEM, "at most 64 ion templates");
    ctx->ions.push_back(*ion);
    ctx->sp_host.push_back(make_species(ion));
    ctx->charge_host.push_back(ion->charge_z);
    if (ctx->has_op) ctx_alpha(ctx, ctx->ions.size() - 1);
    if (ion_id) *ion_id = (int32_t)ctx->ions.size() - 1;
    return upload_species(ctx);
}

int32_t mc_set_operating(mc_ctx *ctx, const mc_operating *op) {
    if (!ctx) return MC_EINVAL;
    if (!op || !(op->dt > 0) || op->sc_every < 1 || op->n_exit_bins < 1 || !(op->exit_bin_dt > 0) ||
        !(op->gas_mass_da > 0) || !(op->r_det > 0) || !(op->d_hit >= 0) ||
        (op->langevin_on && !(op->lv_switch >= 0)) || op->sample_every < 0 || op->sample_stride < 0 ||
        !(op->lv_dt_max >= 0) || op->sort_every < 0)
        return fail(ctx, MC_EINVAL, "invalid operating point");
    if (!ctx->has_fields) return fail(ctx, MC_ESTATE, "load fields first");
    HIPCHK(hipSetDevice(ctx->opt.device));
    const bool first = !ctx->has_op;
    if (!first && op->n_exit_bins != ctx->op.n_exit_bins)
        return fail(ctx, MC_ESTATE, "the number of exit bins is fixed by the first operating point");
    ctx->op = *op;
    ctx->dt_rec_valid = false;  // RF and step settings may have changed
    ctx->has_op = true;
    for (size_t k = 0; k < ctx->ions.size(); ++k) ctx_alpha(ctx, k);
    int32_t rc = upload_species(ctx);
    if (rc) return rc;
    const int64_t nn = (int64_t)ctx->nr * ctx->nz;
    if (first) {
        const int64_t base = TC_N + op->n_exit_bins + nn + MC_HIST_KE + MC_HIST_TEFF + MC_HIST_R;
        ctx->tal_len = hot_offset(base) + kHotLen;
        rc = dalloc_t(ctx, &ctx->tal, ctx->tal_len);
        if (rc) return rc;
        HIPCHK(hipMemsetAsync(ctx->tal, 0, ctx->tal_len * sizeof(unsigned long long), ctx->stream));
        unsigned long long *p = ctx->tal;
        ctx->tp.cnt = p;
        p += TC_N;
        ctx->tp.exit_bins = p;
        p += op->n_exit_bins;
        ctx->tp.loss_map = p;
        p += nn;
        ctx->tp.hist_ke = p;
        p += MC_HIST_KE;
        ctx->tp.hist_teff = p;
        p += MC_HIST_TEFF;
        ctx->tp.hist_r = p;
        ctx->tp.hot = ctx->tal + hot_offset(base);
    }
    const double reach = op->d_hit + 0.5 * std::min(ctx->dr, ctx->dz);
    const int32_t wi = (int32_t)std::ceil(reach / ctx->dr), wj = (int32_t)std::ceil(reach / ctx->dz);
    k_hit<<<grid_for(nn), kBlock, 0, ctx->stream>>>(ctx->mask, ctx->hit, ctx->nr, ctx->nz, ctx->dr, ctx->dz, reach, wi,
                                                    wj);
    LAUNCHCHK();
    rc = fold(ctx);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MC_OK;
}

int32_t mc_define_source(mc_ctx *ctx, const mc_source *src, int32_t *src_id) {
    if (!ctx) return MC_EINVAL;
    if (!ctx->has_op) return fail(ctx, MC_ESTATE, "set the operating point first");
    if (!src || src->ion < 0 || src->ion >= (int32_t)ctx->ions.size() || src->kind < 0 || src->kind > 2 ||
        !(src->sigma_r > 0) || !(src->r_trunc > 0) || src->n_total < 0 ||
        (src->kind == 1 && src->packs_per_step <= 0) || (src->kind != 1 && !(src->weight > 0)))
        return fail(ctx, MC_EINVAL, "invalid source");
    if (ctx->srcs.size() >= 1024) return fail(ctx, MC_ENOMEM, "too many sources");
    ctx->srcs.push_back(make_source(*src, ctx->ions[src->ion].charge_z, ctx->op.dt));
    if (src_id) *src_id = (int32_t)ctx->srcs.size() - 1;
    return MC_OK;
}

int32_t mc_inject(mc_ctx *ctx, int32_t src_id, int64_t n) {
    if (!ctx) return MC_EINVAL;
    if (src_id < 0 || src_id >= (int32_t)ctx->srcs.size() || n < 0) return fail(ctx, MC_EINVAL, "invalid inject");
    HIPCHK(hipSetDevice(ctx->opt.device));
    return emit(ctx, src_id, n);
}

// Trajectory samples at the start of the current step when it is one of the
// sampled steps (dyn: the device step record of an adaptive run, whose
// halted state stops sampling).
static int32_t sample_if_due(mc_ctx *ctx, const double *dyn) {
    if (!(ctx->op.sample_every > 0 && ctx->op.sample_stride > 0 && ctx->step % ctx->op.sample_every == 0 &&
          ctx->n_slots > 0))
        return MC_OK;
    const unsigned sgrid = (unsigned)((ctx->n_slots + kSampleThreads - 1) / kSampleThreads);
    if (ctx->fp32())
        k_sample<float><<<sgrid, kSampleThreads, 0, ctx->stream>>>(ctx->p32, ctx->sp_dev, ctx->n_slots, ctx->step,
                                                                   ctx->op.sample_stride, ctx->samples,
                                                                   ctx->sample_count, ctx->sample_cap, dyn);
    else
        k_sample<double><<<sgrid, kSampleThreads, 0, ctx->stream>>>(ctx->p64, ctx->sp_dev, ctx->n_slots, ctx->step,
                                                                    ctx->op.sample_stride, ctx->samples,
                                                                    ctx->sample_count, ctx->sample_cap, dyn);
    LAUNCHCHK();
    return MC_OK;
}

// Whether no source emits any more (emission needs each step's length on
// the host: Eq. 5 counts and weights).
static bool sources_idle(const mc_ctx *ctx) {
    for (const Src &S : ctx->srcs)
        if (S.in.kind != 0 && S.emitted < S.in.n_total) return false;
    return true;
}

// Adaptive steps with the step length kept on the device: up to max_steps
// steps, as many as can run before a space-charge update could fall due
// (the time grows by at most dt_max per step), then one read of the step
// record.  *done receives the steps taken.
static int32_t adaptive_batch(mc_ctx *ctx, int64_t max_steps, int64_t *done) {
    *done = 0;
    int32_t rc = adaptive_buffers(ctx);
    if (rc) return rc;
    const mc_operating &op = ctx->op;
    if (!ctx->dt_rec_valid) {
        double init[8] = {ctx->t, 0.0, 0.0, 0.0, 0.0, ctx->t, 0.0, 0.0};
        double c[3];
        rf_stages_at(op, ctx->t, 0.0, c);
        init[6] = c[0];
        HIPCHK(hipMemcpyAsync(ctx->dt_rec, init, sizeof(init), hipMemcpyHostToDevice, ctx->stream));
        ctx->dt_rec_valid = true;
    }
    const double tol = 1e-6 * op.dt, t0 = ctx->t;
    int64_t k = max_steps;
    if (op.sort_every > 0) {
        // the stretch ends before the next sorted step
        rc = sort_if_due(ctx);
        if (rc) return rc;
        k = std::min<int64_t>(k, op.sort_every - ctx->step % op.sort_every);
    }
    for (int64_t j = 0; j < k; ++j) {
        rc = sample_if_due(ctx, ctx->dt_rec);
        if (rc) return rc;
        if (j == 0 && op.sc_on) {
            if (t0 >= ctx->t_next_pic - tol) {
                rc = pic_update(ctx);
                if (rc) return rc;
                const double period = op.sc_every * op.dt;
                while (ctx->t_next_pic <= t0 + tol) ctx->t_next_pic += period;
            }
            // the first step whose start could reach the next update's time
            const double room = ctx->t_next_pic - tol - t0;
            k = std::min<int64_t>(k, std::max<int64_t>(1, (int64_t)std::ceil(room / op.dt)));
        }
        if (!ctx->fp32()) rc = pack_limits_dev<P64, double4>(ctx, ctx->p64);
        else if (ctx->bf16()) rc = pack_limits_dev<P32, bf16x4>(ctx, ctx->p32);
        else rc = pack_limits_dev<P32, float4>(ctx, ctx->p32);
        if (rc) return rc;
        const double inf = HUGE_VAL;
        k_dt_finish<<<1, kHotRep, 0, ctx->stream>>>(
            ctx->dt_rep, ctx->dt_rec, op.dt, (op.v_rf != 0.0 && op.f_rf > 0.0) ? 0.05 / op.f_rf : inf,
            op.lv_dt_max > 0.0 ? op.lv_dt_max : inf, op.sc_on ? ctx->t_next_pic : inf, 1e-9 * op.dt, op.v_rf,
            2.0 * kPi * op.f_rf, op.phase_rf, ctx->step);
        LAUNCHCHK();
        rc = step_once(ctx, 0.0, op.dt, ctx->dt_rec);
        if (rc) return rc;
        ctx->step++;
        ++*done;
    }
    double rec[8];
    HIPCHK(hipMemcpyAsync(rec, ctx->dt_rec, sizeof(rec), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    uint64_t halted;
    std::memcpy(&halted, &rec[7], sizeof(halted));
    ctx->t = rec[5];
    if (halted) {
        ctx->step = (int64_t)halted - 1;
        return fail(ctx, MC_ENUMERIC, "adaptive step collapsed below 1e-9 dt at step " + std::to_string(ctx->step));
    }
    ctx->last_dt = rec[1];
    return MC_OK;
}

int32_t mc_step(mc_ctx *ctx, int64_t n_steps) {
    if (!ctx) return MC_EINVAL;
    if (!ctx->has_fields || !ctx->has_op) return fail(ctx, MC_ESTATE, "fields and operating point required");
    if (n_steps < 0) return fail(ctx, MC_EINVAL, "negative step count");
    HIPCHK(hipSetDevice(ctx->opt.device));
    for (int64_t it = 0; it < n_steps;) {
        int32_t rc;
        if (ctx->op.adaptive && sources_idle(ctx)) {
            int64_t done = 0;
            rc = adaptive_batch(ctx, n_steps - it, &done);
            if (rc) return rc;
            it += done;
            continue;
        }
        ctx->dt_rec_valid = false;  // the host advances the time below
        rc = sort_if_due(ctx);
        if (rc) return rc;
        rc = sample_if_due(ctx, nullptr);
        if (rc) return rc;
        double t0 = (double)ctx->step * ctx->op.dt, dt = ctx->op.dt;
        if (ctx->op.adaptive) {
            t0 = ctx->t;
            const double tol = 1e-6 * ctx->op.dt;
            if (ctx->op.sc_on && t0 >= ctx->t_next_pic - tol) {
                rc = pic_update(ctx);
                if (rc) return rc;
                const double period = ctx->op.sc_every * ctx->op.dt;
                while (ctx->t_next_pic <= t0 + tol) ctx->t_next_pic += period;
            }
            rc = adaptive_dt(ctx, t0, &dt);
            if (rc) return rc;
            for (auto &S : ctx->srcs) source_dt(S, ctx->ions[S.in.ion].charge_z, dt);
        } else if (ctx->op.sc_on && ctx->step % ctx->op.sc_every == 0) {
            rc = pic_update(ctx);
            if (rc) return rc;
        }
        for (size_t si = 0; si < ctx->srcs.size(); ++si) {
            rc = emit(ctx, (int)si, due(ctx->srcs[si], ctx->step));
            if (rc) return rc;
        }
        rc = step_once(ctx, t0, dt);
        if (rc) return rc;
        ctx->last_dt = dt;
        ctx->t = ctx->op.adaptive ? t0 + dt : (double)(ctx->step + 1) * ctx->op.dt;
        ctx->step++;
        ++it;
    }
    return MC_OK;
}

int32_t mc_pic_update(mc_ctx *ctx) {
    if (!ctx) return MC_EINVAL;
    if (!ctx->has_fields || !ctx->has_op) return fail(ctx, MC_ESTATE, "fields and operating point required");
    HIPCHK(hipSetDevice(ctx->opt.device));
    return pic_update(ctx);
}

int32_t mc_synchronize(mc_ctx *ctx) {
    if (!ctx) return MC_EINVAL;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MC_OK;
}

int32_t mc_get_info(const mc_ctx *ctx, mc_info *info) {
    if (!ctx || !info) return MC_EINVAL;
    info->step = ctx->step;
    info->n_slots = ctx->n_slots;
    info->capacity = ctx->cap;
    info->exit_capacity = ctx->tp.exit_cap;
    info->device_bytes = ctx->device_bytes;
    info->nr = ctx->nr;
    info->nz = ctx->nz;
    info->n_exit_bins = ctx->has_op ? ctx->op.n_exit_bins : 0;
    info->precision = ctx->opt.precision;
    info->time = ctx->t;
    info->last_dt = ctx->last_dt;
    info->n_ions = (int32_t)ctx->ions.size();
    info->n_sources = (int32_t)ctx->srcs.size();
    return MC_OK;
}

int32_t mc_get_tally_layout(const mc_ctx *ctx, mc_tally_layout *out) {
    if (!ctx || !out) return MC_EINVAL;
    if (!ctx->has_op) return MC_ESTATE;
    mc_tally_layout L{};
    L.n_classes = MC_NCLASS;
    L.n_exit_bins = ctx->op.n_exit_bins;
    L.exit_bin_dt = ctx->op.exit_bin_dt;
    L.nr = ctx->nr;
    L.nz = ctx->nz;
    L.loss_map_len = (int64_t)ctx->nr * ctx->nz;
    L.hist_ke_len = MC_HIST_KE;
    L.ke_bins = kKeBins;
    L.ke_log10_lo = kKeLog10Lo;
    L.ke_log10_hi = kKeLog10Hi;
    L.hist_teff_len = MC_HIST_TEFF;
    L.teff_bins = kTeffBins;
    L.teff_lo = kTeffLo;
    L.teff_hi = kTeffHi;
    L.hist_r_len = MC_HIST_R;
    L.r_bins = kRBins;
    L.r_lo = 0.0;
    L.r_hi = ctx->op.r_det;
    L.exit_capacity = ctx->tp.exit_cap;
    L.sample_capacity = ctx->sample_cap;
    L.charge_grid_len = (int64_t)ctx->nr * ctx->nz;
    *out = L;
    return MC_OK;
}

int32_t mc_read_tallies(mc_ctx *ctx, mc_tallies *out) {
    if (!ctx || !out) return MC_EINVAL;
    if (!ctx->has_op) return fail(ctx, MC_ESTATE, "no operating point");
    HIPCHK(hipSetDevice(ctx->opt.device));
    int32_t rc = ctx->fp32() ? snapshot_t<float>(ctx, ctx->p32) : snapshot_t<double>(ctx, ctx->p64);
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    std::vector<unsigned long long> cnt(TC_N), hot(kHotLen), snap(2 + MC_HIST_KE + MC_HIST_TEFF);
    double sums[3];
    HIPCHK(hipMemcpy(cnt.data(), ctx->tp.cnt, TC_N * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(hot.data(), ctx->tp.hot, kHotLen * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    fold_hot(hot.data(), cnt.data());
    HIPCHK(hipMemcpy(snap.data(), ctx->snap, snap.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(sums, ctx->sums, 3 * sizeof(double), hipMemcpyDeviceToHost));
    out->emitted_n = ctx->emitted_n;
    out->emitted_w = ctx->emitted_w;
    for (int c = 0; c < MC_NCLASS; ++c) {
        out->class_n[c] = (int64_t)cnt[TC_CLASS_N + c];
        out->class_w[c] = (int64_t)cnt[TC_CLASS_W + c];
    }
    out->class_n[MC_ACTIVE] = (int64_t)snap[0];
    out->class_w[MC_ACTIVE] = (int64_t)snap[1];
    out->n_cand = (int64_t)cnt[TC_CAND];
    out->n_coll = (int64_t)cnt[TC_COLL];
    out->n_cap = (int64_t)cnt[TC_CAP];
    out->n_clamp = (int64_t)cnt[TC_CLAMP];
    out->pack_steps = (int64_t)cnt[TC_PACKSTEPS];
    out->exit_overflow = (int64_t)cnt[TC_EXOVER];
    out->exit_dropped = (int64_t)cnt[TC_EXDROP];
    out->n_langevin = (int64_t)cnt[TC_LANG];
    out->n_exchange = (int64_t)cnt[TC_EXCH];
    out->sum_w_ke_active = sums[0];
    out->sum_w_eint_active = sums[1];
    out->sum_w_dissoc_terminal = sums[2];
    const int64_t nn = (int64_t)ctx->nr * ctx->nz;
    if (out->exit_bins)
        HIPCHK(hipMemcpy(out->exit_bins, ctx->tp.exit_bins, ctx->op.n_exit_bins * sizeof(int64_t), hipMemcpyDeviceToHost));
    if (out->loss_map) HIPCHK(hipMemcpy(out->loss_map, ctx->tp.loss_map, nn * sizeof(int64_t), hipMemcpyDeviceToHost));
    if (out->hist_ke) HIPCHK(hipMemcpy(out->hist_ke, ctx->tp.hist_ke, MC_HIST_KE * 8, hipMemcpyDeviceToHost));
    if (out->hist_teff) HIPCHK(hipMemcpy(out->hist_teff, ctx->tp.hist_teff, MC_HIST_TEFF * 8, hipMemcpyDeviceToHost));
    if (out->hist_r) HIPCHK(hipMemcpy(out->hist_r, ctx->tp.hist_r, MC_HIST_R * 8, hipMemcpyDeviceToHost));
    if (out->act_hist_ke) std::memcpy(out->act_hist_ke, snap.data() + 2, MC_HIST_KE * 8);
    if (out->act_hist_teff) std::memcpy(out->act_hist_teff, snap.data() + 2 + MC_HIST_KE, MC_HIST_TEFF * 8);
    return MC_OK;
}

int32_t mc_read_samples(mc_ctx *ctx, mc_sample_rec *buf, int64_t cap, int64_t *n) {
    if (!ctx || !n || cap < 0) return MC_EINVAL;
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    unsigned long long count = 0;
    HIPCHK(hipMemcpy(&count, ctx->sample_count, sizeof(count), hipMemcpyDeviceToHost));
    *n = (int64_t)count;
    if (!buf || cap == 0) return MC_OK;
    const int64_t have = std::min<int64_t>((int64_t)count, ctx->sample_cap);
    std::vector<mc_sample_rec> all(have);
    if (have > 0) HIPCHK(hipMemcpy(all.data(), ctx->samples, have * sizeof(mc_sample_rec), hipMemcpyDeviceToHost));
    std::sort(all.begin(), all.end(), [](const mc_sample_rec &a, const mc_sample_rec &b) {
        return a.step != b.step ? a.step < b.step : a.id < b.id;
    });
    std::memcpy(buf, all.data(), std::min(have, cap) * sizeof(mc_sample_rec));
    return MC_OK;
}

int32_t mc_read_exits(mc_ctx *ctx, mc_exit_rec *buf, int64_t cap, int64_t *n) {
    if (!ctx || !n || cap < 0) return MC_EINVAL;
    if (!ctx->has_op) return fail(ctx, MC_ESTATE, "no operating point");
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    unsigned long long count = 0;
    HIPCHK(hipMemcpy(&count, ctx->tp.cnt + TC_EXCOUNT, sizeof(count), hipMemcpyDeviceToHost));
    *n = (int64_t)count;
    if (!buf || cap == 0) return MC_OK;
    const int64_t have = std::min<int64_t>((int64_t)count, ctx->tp.exit_cap);
    std::vector<mc_exit_rec> all(have);
    if (have > 0) HIPCHK(hipMemcpy(all.data(), ctx->tp.exits, have * sizeof(mc_exit_rec), hipMemcpyDeviceToHost));
    std::sort(all.begin(), all.end(), [](const mc_exit_rec &a, const mc_exit_rec &b) { return a.id < b.id; });
    std::memcpy(buf, all.data(), std::min(have, cap) * sizeof(mc_exit_rec));
    return MC_OK;
}

int32_t mc_read_packs(mc_ctx *ctx, mc_packs *o) {
    if (!ctx || !o) return MC_EINVAL;
    if (o->n < ctx->n_slots) return fail(ctx, MC_EINVAL, "buffer shorter than the slot count");
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const int64_t n = ctx->n_slots;
    o->n = n;
    if (n == 0) return MC_OK;
    auto cp = [&](void *dst, const void *src, size_t b) -> hipError_t {
        return dst ? hipMemcpy(dst, src, b, hipMemcpyDeviceToHost) : hipSuccess;
    };
    if (!ctx->fp32()) {
        const PackPtrs<double> &p = ctx->p64;
        double *dsts[] = {o->x, o->y, o->z, o->vx, o->vy, o->vz, o->e_int, o->h, o->w};
        double *srcs[] = {p.x, p.y, p.z, p.vx, p.vy, p.vz, p.e, p.h, p.w};
        for (int k = 0; k < 9; ++k) HIPCHK(cp(dsts[k], srcs[k], n * sizeof(double)));
        HIPCHK(cp(o->id, p.id, n * 8));
        HIPCHK(cp(o->q, p.q, n * 8));
        HIPCHK(cp(o->tag, p.tag, n * 4));
        HIPCHK(cp(o->status, p.status, n * 4));
    } else {
        const PackPtrs<float> &p = ctx->p32;
        std::vector<float> hi(n), lo(n);
        double *dsts[] = {o->x, o->y, o->z, o->e_int};
        float *shi[] = {p.x, p.y, p.z, p.e}, *slo[] = {p.xl, p.yl, p.zl, p.el};
        for (int k = 0; k < 4; ++k) {
            if (!dsts[k]) continue;
            HIPCHK(hipMemcpy(hi.data(), shi[k], n * 4, hipMemcpyDeviceToHost));
            HIPCHK(hipMemcpy(lo.data(), slo[k], n * 4, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < n; ++i) dsts[k][i] = (double)hi[i] + (double)lo[i];
        }
        double *d1[] = {o->vx, o->vy, o->vz, o->h};
        float *s1[] = {p.vx, p.vy, p.vz, p.h};
        for (int k = 0; k < 4; ++k) {
            if (!d1[k]) continue;
            HIPCHK(hipMemcpy(hi.data(), s1[k], n * 4, hipMemcpyDeviceToHost));
            for (int64_t i = 0; i < n; ++i) d1[k][i] = (double)hi[i];
        }
        HIPCHK(cp(o->w, p.w, n * 8));
        HIPCHK(cp(o->id, p.id, n * 8));
        HIPCHK(cp(o->q, p.q, n * 8));
        HIPCHK(cp(o->tag, p.tag, n * 4));
        HIPCHK(cp(o->status, p.status, n * 4));
    }
    return MC_OK;
}

int32_t mc_write_packs(mc_ctx *ctx, const mc_packs *in) {
    if (!ctx || !in) return MC_EINVAL;
    if (in->n < 0 || in->n > ctx->cap) return fail(ctx, MC_ENOMEM, "snapshot larger than the pack capacity");
    if (!in->x || !in->y || !in->z || !in->vx || !in->vy || !in->vz || !in->e_int || !in->h || !in->w || !in->id ||
        !in->tag)
        return fail(ctx, MC_EINVAL, "snapshot field missing");
    for (int64_t k = 0; k < in->n; ++k) {
        if (in->tag[k] < 0 || in->tag[k] >= (int32_t)ctx->ions.size()) return fail(ctx, MC_EINVAL, "bad ion tag");
        if (!std::isfinite(in->x[k]) || !std::isfinite(in->y[k]) || !std::isfinite(in->z[k]) ||
            !std::isfinite(in->vx[k]) || !std::isfinite(in->vy[k]) || !std::isfinite(in->vz[k]) ||
            !std::isfinite(in->e_int[k]) || !std::isfinite(in->w[k]) || !std::isfinite(in->h[k]))
            return fail(ctx, MC_EINVAL, "non-finite snapshot state");
    }
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const int64_t n = in->n;
    if (n > 0) {
        if (!ctx->fp32()) {
            const PackPtrs<double> &p = ctx->p64;
            const double *s[] = {in->x, in->y, in->z, in->vx, in->vy, in->vz, in->e_int, in->h, in->w};
            double *d[] = {p.x, p.y, p.z, p.vx, p.vy, p.vz, p.e, p.h, p.w};
            for (int k = 0; k < 9; ++k) HIPCHK(hipMemcpy(d[k], s[k], n * 8, hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(p.id, in->id, n * 8, hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(p.tag, in->tag, n * 4, hipMemcpyHostToDevice));
            k_init_written<double><<<grid_for(n), kBlock, 0, ctx->stream>>>(p, ctx->sp_dev, ctx->charge_dev, n);
        } else {
            const PackPtrs<float> &p = ctx->p32;
            std::vector<float> hi(n), lo(n);
            const double *s2[] = {in->x, in->y, in->z, in->e_int};
            float *dh[] = {p.x, p.y, p.z, p.e}, *dl[] = {p.xl, p.yl, p.zl, p.el};
            for (int k = 0; k < 4; ++k) {
                for (int64_t i = 0; i < n; ++i) {
                    hi[i] = (float)s2[k][i];
                    lo[i] = (float)(s2[k][i] - (double)hi[i]);
                }
                HIPCHK(hipMemcpy(dh[k], hi.data(), n * 4, hipMemcpyHostToDevice));
                HIPCHK(hipMemcpy(dl[k], lo.data(), n * 4, hipMemcpyHostToDevice));
            }
            const double *s1[] = {in->vx, in->vy, in->vz, in->h};
            float *d1[] = {p.vx, p.vy, p.vz, p.h};
            for (int k = 0; k < 4; ++k) {
                for (int64_t i = 0; i < n; ++i) hi[i] = (float)s1[k][i];
                HIPCHK(hipMemcpy(d1[k], hi.data(), n * 4, hipMemcpyHostToDevice));
            }
            HIPCHK(hipMemcpy(p.w, in->w, n * 8, hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(p.id, in->id, n * 8, hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(p.tag, in->tag, n * 4, hipMemcpyHostToDevice));
            k_init_written<float><<<grid_for(n), kBlock, 0, ctx->stream>>>(p, ctx->sp_dev, ctx->charge_dev, n);
        }
        LAUNCHCHK();
    }
    ctx->n_slots = n;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MC_OK;
}


int32_t mc_save_state(mc_ctx *ctx, const char *path) {
    if (!ctx || !path) return MC_EINVAL;
    if (!ctx->has_fields || !ctx->has_op) return fail(ctx, MC_ESTATE, "fields and operating point required");
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    CkptHeader h = ckpt_header(ctx);
    unsigned long long ne = 0, ns = 0;
    HIPCHK(hipMemcpy(&ne, ctx->tp.cnt + TC_EXCOUNT, 8, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(&ns, ctx->sample_count, 8, hipMemcpyDeviceToHost));
    h.n_exits = std::min<int64_t>((int64_t)ne, ctx->tp.exit_cap);
    h.n_samples = std::min<int64_t>((int64_t)ns, ctx->sample_cap);
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(ctx, MC_EINVAL, std::string("cannot write ") + path);
    bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1;
    for (const Src &S : ctx->srcs) {
        const int64_t st[2] = {S.acc_fx, S.emitted};
        ok = ok && std::fwrite(st, sizeof(st), 1, f) == 1;
    }
    std::vector<char> buf;
    for (const Blob &b : ckpt_blobs(ctx, h.n_slots, h.n_exits, h.n_samples)) {
        const int64_t nb = (int64_t)b.bytes;
        ok = ok && std::fwrite(&nb, 8, 1, f) == 1;
        if (!ok || nb == 0) continue;
        buf.resize(b.bytes);
        if (hipMemcpy(buf.data(), b.dev, b.bytes, hipMemcpyDeviceToHost) != hipSuccess) {
            std::fclose(f);
            return fail(ctx, MC_EDEVICE, "reading device state");
        }
        ok = std::fwrite(buf.data(), 1, b.bytes, f) == b.bytes;
    }
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) return fail(ctx, MC_EINVAL, std::string("short write to ") + path);
    return MC_OK;
}

int32_t mc_load_state(mc_ctx *ctx, const char *path) {
    if (!ctx || !path) return MC_EINVAL;
    if (!ctx->has_fields || !ctx->has_op) return fail(ctx, MC_ESTATE, "fields and operating point required");
    HIPCHK(hipSetDevice(ctx->opt.device));
    ctx->dep_full = true;  // the restored charge grid may hold charge anywhere
    ctx->dt_rec_valid = false;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(ctx, MC_EINVAL, std::string("cannot read ") + path);
    CkptHeader h{};
    const CkptHeader want = ckpt_header(ctx);
    bool ok = std::fread(&h, sizeof(h), 1, f) == 1;
    std::string why;
    if (!ok || std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.abi != MC_ABI_VERSION) why = "not a checkpoint of this library";
    else if (h.precision != want.precision || h.nr != want.nr || h.nz != want.nz || h.n_ions != want.n_ions ||
             h.n_srcs != want.n_srcs || h.n_exit_bins != want.n_exit_bins || h.fp32_tables != want.fp32_tables ||
             h.tal_len != want.tal_len || h.seed != want.seed)
        why = "checkpoint of a different configuration";
    else if (h.n_slots < 0 || h.n_slots > ctx->cap || h.n_exits < 0 || h.n_exits > ctx->tp.exit_cap ||
             h.n_samples < 0 || h.n_samples > ctx->sample_cap)
        why = "checkpoint larger than this context's capacities";
    std::vector<int64_t> src_state(2 * h.n_srcs);
    if (why.empty() && h.n_srcs > 0) ok = std::fread(src_state.data(), 16, h.n_srcs, f) == (size_t)h.n_srcs;
    std::vector<char> buf;
    if (why.empty()) {
        for (const Blob &b : ckpt_blobs(ctx, h.n_slots, h.n_exits, h.n_samples)) {
            int64_t nb = -1;
            ok = ok && std::fread(&nb, 8, 1, f) == 1 && nb == (int64_t)b.bytes;
            if (!ok) break;
            if (nb == 0) continue;
            buf.resize(b.bytes);
            ok = std::fread(buf.data(), 1, b.bytes, f) == b.bytes;
            if (!ok) break;
            if (hipMemcpy(b.dev, buf.data(), b.bytes, hipMemcpyHostToDevice) != hipSuccess) {
                std::fclose(f);
                return fail(ctx, MC_EDEVICE, "writing device state");
            }
        }
        if (!ok) why = "truncated or inconsistent checkpoint";
    }
    std::fclose(f);
    if (!why.empty()) return fail(ctx, MC_EINVAL, why + ": " + path);
    for (size_t k = 0; k < ctx->srcs.size(); ++k) {
        ctx->srcs[k].acc_fx = src_state[2 * k];
        ctx->srcs[k].emitted = src_state[2 * k + 1];
    }
    ctx->n_slots = h.n_slots;
    ctx->step = h.step;
    ctx->emitted_n = h.emitted_n;
    ctx->emitted_w = h.emitted_w;
    ctx->t = h.t;
    ctx->t_next_pic = h.t_next_pic;
    ctx->last_dt = h.last_dt;
    const int32_t rc = fold(ctx);  // static field plus the restored space-charge field
    if (rc) return rc;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return MC_OK;
}

int32_t mc_read_charge(mc_ctx *ctx, int64_t *q) {
    if (!ctx || !q) return MC_EINVAL;
    if (!ctx->has_fields) return fail(ctx, MC_ESTATE, "no fields");
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipMemcpy(q, ctx->qgrid, (int64_t)ctx->nr * ctx->nz * 8, hipMemcpyDeviceToHost));
    return MC_OK;
}

int32_t mc_read_sc(mc_ctx *ctx, double *phi, double *er, double *ez) {
    if (!ctx) return MC_EINVAL;
    if (!ctx->has_fields) return fail(ctx, MC_ESTATE, "no fields");
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const int64_t nn = (int64_t)ctx->nr * ctx->nz;
    if (phi) HIPCHK(hipMemcpy(phi, ctx->phi_sc, nn * 8, hipMemcpyDeviceToHost));
    if (er || ez) {
        std::vector<double2> e(nn);
        HIPCHK(hipMemcpy(e.data(), ctx->e_sc, nn * sizeof(double2), hipMemcpyDeviceToHost));
        for (int64_t k = 0; k < nn; ++k) {
            if (er) er[k] = e[k].x;
            if (ez) ez[k] = e[k].y;
        }
    }
    return MC_OK;
}

int32_t mc_read_hit(mc_ctx *ctx, uint8_t *hit) {
    if (!ctx || !hit) return MC_EINVAL;
    if (!ctx->has_op) return fail(ctx, MC_ESTATE, "no operating point");
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipMemcpy(hit, ctx->hit, (int64_t)ctx->nr * ctx->nz, hipMemcpyDeviceToHost));
    return MC_OK;
}

int32_t mc_read_timing(mc_ctx *ctx, mc_timing *out) {
    if (!ctx || !out) return MC_EINVAL;
    HIPCHK(hipSetDevice(ctx->opt.device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    resolve_timing(ctx);
    for (int k = 0; k < MC_NKERNEL; ++k) {
        out->ms[k] = ctx->t_ms[k];
        out->launches[k] = ctx->t_launch[k];
    }
    std::vector<unsigned long long> cnt(TC_N, 0ull), hot(kHotLen);
    if (ctx->tp.hot) {
        HIPCHK(hipMemcpy(hot.data(), ctx->tp.hot, kHotLen * sizeof(unsigned long long), hipMemcpyDeviceToHost));
        fold_hot(hot.data(), cnt.data());
    }
    out->pack_steps = (int64_t)cnt[TC_PACKSTEPS];
    return MC_OK;
}

int32_t mc_reset_timing(mc_ctx *ctx) {
    if (!ctx) return MC_EINVAL;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    resolve_timing(ctx);
    for (int k = 0; k < MC_NKERNEL; ++k) {
        ctx->t_ms[k] = 0;
        ctx->t_launch[k] = 0;
    }
    // events for the stretch that follows (a timed window of steps)
    if (ctx->opt.timing && ctx->ev_pool.size() < 4 * (size_t)kEventBatch)
        ev_fill(ctx, 4 * kEventBatch - (int)ctx->ev_pool.size());
    return MC_OK;
}

int32_t mc_set_timing(mc_ctx *ctx, int32_t on) {
    if (!ctx) return MC_EINVAL;
    HIPCHK(hipSetDevice(ctx->opt.device));
    ctx->opt.timing = on ? 1 : 0;
    if (ctx->opt.timing && ctx->ev_pool.size() < 4 * (size_t)kEventBatch)
        ev_fill(ctx, 4 * kEventBatch - (int)ctx->ev_pool.size());
    return MC_OK;
}

}  // extern "C"

// mc_server.hip -- serving runtime: continuous batching of design queries.
//
// One worker thread per server runs rounds of: admit (FIFO, pool permitting)
// -> steps_per_sync co-steps -> synchronise -> retire finished queries.  A
// co-step advances every resident query by one step: per-query space-charge
// updates where due, one multi-query emission launch, one multi-query step
// launch.  Launch descriptors go through a ring of pinned host buffers and
// device buffers, each guarded by an event, so the host never overwrites a
// descriptor the GPU has not read yet.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mc_host.hpp"
#include "mc_kernels.hpp"
#include "mc_poisson.hpp"
#include "mc_pool.hpp"

using namespace mc;

namespace {

constexpr int kBlk = 256;
constexpr int kRing = 8;
constexpr int64_t kAggMax = 1024;

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlk - 1) / kBlk); }
// blocks of the co-step's step kernel: one wavefront each, as in a single
// context (the smallest last, partly filled round of blocks)
constexpr int kStepBlk = 64;

struct Query {
    uint64_t id = 0;
    mc_query q{};
    int32_t state = MC_Q_PENDING, err = MC_OK;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int64_t bytes = 0, pool_off = -1;
    Species sp{};
    Src src{};
    int64_t n_slots = 0, step = 0, emitted_n = 0, emitted_w = 0, partial_len = 0;
    // device views into the query's pool block
    PackPtrs<double> p64{};
    PackPtrs<float> p32{};
    void *etab = nullptr, *bh = nullptr;
    double2 *e_sc = nullptr;
    double *phi = nullptr, *partial = nullptr, *sums = nullptr, *rhs = nullptr;
    unsigned long long *qgrid = nullptr, *tal = nullptr, *snap = nullptr;
    int64_t tal_len = 0;
    mc_sample_rec *samples = nullptr;
    unsigned long long *scount = nullptr;
    // adaptive step (Eq. 1): simulated time, time of the next space-charge
    // update, this step's length, the limit reduction's replicated lines
    double t = 0.0, t_next_pic = 0.0, dt_now = 0.0;
    unsigned long long *dt_rep = nullptr, *dt_out = nullptr;
    int32_t fail_code = MC_OK;  // set when the query stops on its own error (its step collapsed)
    TallyPtrs tp{};
    Species *sp_dev = nullptr;
    int32_t *charge_dev = nullptr;
    // host result
    mc_tallies r{};
    std::vector<int64_t> r_bins, r_loss, r_hke, r_hte, r_hr, r_ahke, r_ahte;
    std::vector<mc_exit_rec> r_exits;
    std::vector<mc_sample_rec> r_samples;
};

}  // namespace

struct mc_server {
    mc_server_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    int32_t nr = 0, nz = 0;
    double dr = 0, dz = 0, inv_dr = 0, inv_dz = 0, R = 0;
    double2 *e_dc = nullptr, *e_off = nullptr, *e_rf = nullptr, *e_zero = nullptr;
    void *gtab = nullptr;
    float gsc[4] = {1, 1, 1, 1}, esc[4] = {1, 1, 1, 1};
    uint8_t *hit = nullptr;
    StepTables *tables = nullptr;  // the FP64 step's logarithm and turn tables
    double *sine = nullptr, *tcp = nullptr, *tinv = nullptr;
    Bluestein blu;
    PoissonGrid pg;
    std::vector<int32_t> mask_nodes;  // metal-mask nodes among the Poisson unknowns
    MaskCap cap;                      // their capacitance correction, built at first use
    std::vector<std::pair<void *, size_t>> allocs;
    int64_t shared_bytes = 0;
    char *pool_base = nullptr;
    Pool pool;
    char *h_ring = nullptr, *d_ring = nullptr;
    unsigned long long *h_dt = nullptr;  // pinned: step limits of the adaptive queries, two words each
    hipEvent_t ring_ev[kRing] = {};
    bool ring_used[kRing] = {};
    size_t ring_slot = 0;
    int ring_pos = 0;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    std::deque<Query *> pending;
    std::vector<Query *> resident;
    std::unordered_map<uint64_t, Query *> all;
    uint64_t next_id = 1;
    bool stop = false, dead = false;
    std::thread worker;
    mc_server_stats st{};
    std::chrono::steady_clock::time_point t0;
    double busy_since = -1;

    bool fp32() const { return opt.precision == MC_PREC_FP32; }
    bool bf16() const { return fp32() && !opt.fp32_tables; }
    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    size_t node_bytes() const { return !fp32() ? sizeof(double4) : (bf16() ? sizeof(bf16x4) : sizeof(float4)); }
};

// ---------------------------------------------------------------------------
// Allocation of shared tables (outside the pool) and the pool itself.
// ---------------------------------------------------------------------------
static int32_t sfail(mc_server *S, int32_t code, const std::string &m) {
    S->err = m;
    return code;
}

#define SCHK(expr)                                                                                        \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess) return sfail(S, MC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

static int32_t salloc(mc_server *S, void **out, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    void *p = nullptr;
    if (S->opt.alloc) {
        p = S->opt.alloc(bytes, S->stream, S->opt.alloc_user);
        if (!p) return sfail(S, MC_ENOMEM, "allocator callback failed");
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        return sfail(S, MC_ENOMEM, "hipMalloc failed for " + std::to_string(bytes) + " bytes");
    }
    S->allocs.emplace_back(p, bytes);
    *out = p;
    return MC_OK;
}

template <class T>
static int32_t salloc_t(mc_server *S, T **out, size_t n) {
    void *p = nullptr;
    int32_t rc = salloc(S, &p, n * sizeof(T));
    *out = static_cast<T *>(p);
    return rc;
}

// ---------------------------------------------------------------------------
// Per-query memory: one pool block holding every array of the query.
// ---------------------------------------------------------------------------
struct Layout {
    int64_t off = 0;
    int64_t take(int64_t bytes) {
        const int64_t o = off;
        off += Pool::round_up(bytes);
        return o;
    }
};

template <class F>
static int64_t query_layout(const mc_server *S, const Query &Q, F &&place) {
    Layout L;
    const int64_t cap = std::max<int64_t>(Q.q.source.n_total, 1);
    const int64_t nn = (int64_t)S->nr * S->nz;
    const int32_t m = S->nz - 2, nu = S->nr - 1;
    const bool sc = Q.q.op.sc_on != 0;
    const int64_t fsz = S->fp32() ? 4 : 8;
    const int nfloat = S->fp32() ? 12 : 8;
    for (int k = 0; k < nfloat; ++k) place("f", k, L.take(cap * fsz));
    place("w", 0, L.take(cap * 8));
    place("id", 0, L.take(cap * 8));
    place("q", 0, L.take(cap * 8));
    place("tag", 0, L.take(cap * 4));
    place("status", 0, L.take(cap * 4));
    place("etab", 0, L.take(nn * (int64_t)S->node_bytes()));
    if (sc) {
        place("esc", 0, L.take(nn * 16));
        place("phi", 0, L.take(nn * 8));
        place("qgrid", 0, L.take(nn * 8));
        place("bh", 0, L.take((int64_t)nu * m * fsz));
        if (Q.q.op.sc_mask) place("rhs", 0, L.take(nn * 8));
    }
    const int64_t tal_len = hot_offset(TC_N + Q.q.op.n_exit_bins + nn + MC_HIST_KE + MC_HIST_TEFF + MC_HIST_R) + kHotLen;
    place("tal", tal_len, L.take(tal_len * 8));
    place("snap", 0, L.take((2 + MC_HIST_KE + MC_HIST_TEFF) * 8));
    const int64_t pl = std::max<int64_t>(1, std::min<int64_t>(blocks_for(cap), kAggMax));
    place("partial", pl, L.take(3 * pl * 8));
    place("sums", 0, L.take(4 * 8));
    place("sp", 0, L.take(sizeof(Species)));
    place("charge", 0, L.take(4));
    place("exits", 0, L.take(std::max<int64_t>(Q.q.exit_capacity, 0) * (int64_t)sizeof(mc_exit_rec)));
    place("samples", 0, L.take(std::max<int64_t>(Q.q.sample_capacity, 0) * (int64_t)sizeof(mc_sample_rec)));
    place("scount", 0, L.take(8));
    if (Q.q.op.adaptive) {
        place("dtrep", 0, L.take(kHotLen * 8));
        place("dtout", 0, L.take(16));
    }
    return L.off;
}

static void bind_query(mc_server *S, Query &Q) {
    char *base = S->pool_base + Q.pool_off;
    float *f32[12] = {};
    double *f64[8] = {};
    query_layout(S, Q, [&](const char *what, int64_t k, int64_t off) {
        char *p = base + off;
        const std::string w(what);
        if (w == "f") {
            if (S->fp32()) f32[k] = (float *)p;
            else f64[k] = (double *)p;
        } else if (w == "w") {
            Q.p64.w = Q.p32.w = (double *)p;
        } else if (w == "id") {
            Q.p64.id = Q.p32.id = (int64_t *)p;
        } else if (w == "q") {
            Q.p64.q = Q.p32.q = (int64_t *)p;
        } else if (w == "tag") {
            Q.p64.tag = Q.p32.tag = (int32_t *)p;
        } else if (w == "status") {
            Q.p64.status = Q.p32.status = (int32_t *)p;
        } else if (w == "etab") {
            Q.etab = p;
        } else if (w == "esc") {
            Q.e_sc = (double2 *)p;
        } else if (w == "phi") {
            Q.phi = (double *)p;
        } else if (w == "qgrid") {
            Q.qgrid = (unsigned long long *)p;
        } else if (w == "bh") {
            Q.bh = p;
        } else if (w == "rhs") {
            Q.rhs = (double *)p;
        } else if (w == "tal") {
            Q.tal = (unsigned long long *)p;
            Q.tal_len = k;
        } else if (w == "snap") {
            Q.snap = (unsigned long long *)p;
        } else if (w == "partial") {
            Q.partial = (double *)p;
            Q.partial_len = k;
        } else if (w == "sums") {
            Q.sums = (double *)p;
        } else if (w == "sp") {
            Q.sp_dev = (Species *)p;
        } else if (w == "charge") {
            Q.charge_dev = (int32_t *)p;
        } else if (w == "exits") {
            Q.tp.exits = (mc_exit_rec *)p;
        } else if (w == "samples") {
            Q.samples = (mc_sample_rec *)p;
        } else if (w == "scount") {
            Q.scount = (unsigned long long *)p;
        } else if (w == "dtrep") {
            Q.dt_rep = (unsigned long long *)p;
        } else if (w == "dtout") {
            Q.dt_out = (unsigned long long *)p;
        }
    });
    if (S->fp32()) {
        PackPtrs<float> &P = Q.p32;
        float **dst[12] = {&P.x, &P.y, &P.z, &P.xl, &P.yl, &P.zl, &P.vx, &P.vy, &P.vz, &P.e, &P.el, &P.h};
        for (int k = 0; k < 12; ++k) *dst[k] = f32[k];
    } else {
        PackPtrs<double> &P = Q.p64;
        double **dst[8] = {&P.x, &P.y, &P.z, &P.vx, &P.vy, &P.vz, &P.e, &P.h};
        for (int k = 0; k < 8; ++k) *dst[k] = f64[k];
    }
    if (!Q.e_sc) Q.e_sc = S->e_zero;
    const int64_t nn = (int64_t)S->nr * S->nz;
    unsigned long long *p = Q.tal;
    Q.tp.cnt = p;
    p += TC_N;
    Q.tp.exit_bins = p;
    p += Q.q.op.n_exit_bins;
    Q.tp.loss_map = p;
    p += nn;
    Q.tp.hist_ke = p;
    p += MC_HIST_KE;
    Q.tp.hist_teff = p;
    p += MC_HIST_TEFF;
    Q.tp.hist_r = p;
    Q.tp.hot = Q.tal + (Q.tal_len - kHotLen);
    Q.tp.exit_cap = std::max<int64_t>(Q.q.exit_capacity, 0);
}

// ---------------------------------------------------------------------------
// Kernel launches for one query / one co-step.
// ---------------------------------------------------------------------------
template <class Tab>
static int32_t fold_query(mc_server *S, Query &Q) {
    const int64_t nn = (int64_t)S->nr * S->nz;
    k_fold<Tab><<<blocks_for(nn), kBlk, 0, S->stream>>>(static_cast<Tab *>(Q.etab), S->e_dc, S->e_off, Q.e_sc, S->e_rf,
                                                        Q.q.op.v_off, nn, S->esc[0], S->esc[1], S->esc[2], S->esc[3]);
    SCHK(hipGetLastError());
    return MC_OK;
}

template <class P, class Tab>
static int32_t admit_query(mc_server *S, Query &Q) {
    bind_query(S, Q);
    k_zero_u64<<<blocks_for(Q.tal_len), kBlk, 0, S->stream>>>(Q.tal, Q.tal_len);
    k_zero_u64<<<1, kBlk, 0, S->stream>>>(Q.scount, 1);
    if (Q.dt_rep) k_dt_reset<<<1, kHotRep, 0, S->stream>>>(Q.dt_rep);
    SCHK(hipGetLastError());
    const int64_t nn = (int64_t)S->nr * S->nz;
    if (Q.q.op.sc_on) {
        k_zero_u64<<<blocks_for(2 * nn), kBlk, 0, S->stream>>>((unsigned long long *)Q.e_sc, 2 * nn);
        k_zero_u64<<<blocks_for(nn), kBlk, 0, S->stream>>>((unsigned long long *)Q.phi, nn);
        if (Q.rhs) k_zero_u64<<<blocks_for(nn), kBlk, 0, S->stream>>>((unsigned long long *)Q.rhs, nn);
        SCHK(hipGetLastError());
    }
    SCHK(hipMemcpyAsync(Q.sp_dev, &Q.sp, sizeof(Species), hipMemcpyHostToDevice, S->stream));
    SCHK(hipMemcpyAsync(Q.charge_dev, &Q.q.ion.charge_z, sizeof(int32_t), hipMemcpyHostToDevice, S->stream));
    int32_t rc = fold_query<Tab>(S, Q);
    if (rc) return rc;
    // host copies above come from Query fields that stay alive while resident
    return MC_OK;
}

template <class P, class Tab, class D>
static int32_t pic_query(mc_server *S, Query &Q, PackPtrs<typename P::T> p) {
    const int64_t nn = (int64_t)S->nr * S->nz;
    k_zero_u64<<<blocks_for(nn), kBlk, 0, S->stream>>>(Q.qgrid, nn);
    if (Q.n_slots > 0) {
        DepositArgs<typename P::T> a{};
        a.p = p;
        a.q = Q.qgrid;
        a.n_slots = Q.n_slots;
        a.inv_dr = S->inv_dr;
        a.inv_dz = S->inv_dz;
        a.nr = S->nr;
        a.nz = S->nz;
        unsigned nb;
        deposit_shape(Q.n_slots, &nb, &a.chunk);
        k_deposit<P><<<nb, kDepositThreads, 0, S->stream>>>(a);
    }
    D *bh = static_cast<D *>(Q.bh);
    SCHK(poisson_solve<D>(S->pg, Q.qgrid, nullptr, bh, Q.phi, false, S->stream));
    if (Q.q.op.sc_mask) {
        if (!S->cap.ready) {
            // first masked query: the capacitance matrix, using this query's
            // work arrays (its potential is recomputed right after)
            // (always in FP64: the inverse capacitance matrix needs the digits)
            const int32_t M = (int32_t)S->mask_nodes.size();
            const int32_t m = S->nz - 2, nu = S->nr - 1;
            if (M > kMaxMaskNodes) return sfail(S, MC_EINVAL, "too many metal-mask nodes for the correction");
            if (M > 0 && (salloc_t(S, &S->cap.nodes, M) || salloc_t(S, &S->cap.cinv, (size_t)M * M)))
                return MC_ENOMEM;
            PoissonGrid g64 = S->pg;
            double *bh64 = reinterpret_cast<double *>(bh);
            Bluestein b64;
            if (S->fp32()) {
                const int32_t L = bluestein_length(m);
                const size_t cx = 2 * sizeof(double);
                if (salloc_t(S, &bh64, (size_t)nu * m)) return MC_ENOMEM;
                if (bluestein_lds(L, cx) <= lds_per_block()) {
                    b64.L = L;
                    b64.lds = bluestein_lds(L, cx);
                    if (salloc(S, &b64.chirp, (size_t)m * cx) || salloc(S, &b64.tw, (size_t)std::max(L / 2, 1) * cx) ||
                        salloc(S, &b64.fb, (size_t)L * cx))
                        return MC_ENOMEM;
                    if (bluestein_prepare<double>(b64, m, S->stream) != hipSuccess) b64.L = 0;
                }
                g64.blu = &b64;
            }
            const std::string err = mask_prepare<double>(g64, S->cap, S->mask_nodes, bh64, Q.rhs, Q.phi, S->stream);
            if (!err.empty()) return sfail(S, MC_EDEVICE, err);
            SCHK(poisson_solve<D>(S->pg, Q.qgrid, nullptr, bh, Q.phi, false, S->stream));
        }
        SCHK(mask_correct<D>(S->pg, S->cap, bh, Q.rhs, Q.phi, S->stream));
    }
    // the field of the new potential folded into the query's table in one pass
    k_bake_fold<Tab><<<blocks_for(nn), kBlk, 0, S->stream>>>(Q.phi, Q.e_sc, S->nr, S->nz, S->dr, S->dz, nullptr,
                                                             static_cast<Tab *>(Q.etab), S->e_dc, S->e_off, S->e_rf,
                                                             Q.q.op.v_off, S->esc[0], S->esc[1], S->esc[2], S->esc[3]);
    SCHK(hipGetLastError());
    return MC_OK;
}

template <class P, class Tab>
static PackPtrs<typename P::T> packs_of(Query &Q) {
    if constexpr (P::kTwo) return Q.p32;
    else return Q.p64;
}

// The step kernel's arguments for one query, a step of length dt from t0.
template <class P, class Tab>
static StepArgs<P, Tab> query_step_args(mc_server *S, Query &Q, double t0, double dt) {
    StepArgs<P, Tab> a{};
    a.p = packs_of<P, Tab>(Q);
    a.etab = static_cast<const Tab *>(Q.etab);
    a.gtab = static_cast<const Tab *>(S->gtab);
    std::memcpy(a.esc, S->esc, sizeof(a.esc));
    std::memcpy(a.gsc, S->gsc, sizeof(a.gsc));
    a.hit = S->hit;
    a.sp = Q.sp_dev;
    a.t = Q.tp;
    a.tables = S->tables;
    a.n_slots = Q.n_slots;
    a.step = Q.step;
    const mc_operating &op = Q.q.op;
    a.dt = dt;
    a.t0 = t0;
    double c[3];
    rf_stages_at(op, t0, dt, c);
    a.c0 = c[0];
    a.ch = c[1];
    a.c1 = c[2];
    a.z_det = op.z_det;
    a.r_det = op.r_det;
    a.R = S->R;
    a.inv_dr = S->inv_dr;
    a.inv_dz = S->inv_dz;
    a.mg = S->opt.gas_mass_da * kDa;
    a.exit_bin_dt = op.exit_bin_dt;
    a.nr = S->nr;
    a.nz = S->nz;
    a.n_exit_bins = op.n_exit_bins;
    a.collisions_on = op.collisions_on;
    a.langevin_on = op.langevin_on;
    a.lv_z_lo = op.lv_z_lo;
    a.lv_z_hi = op.lv_z_hi;
    a.lv_switch = op.lv_switch;
    a.lv_dt_ref = op.dt;
    a.k0 = (uint32_t)Q.q.seed;
    a.k1 = (uint32_t)(Q.q.seed >> 32);
    return a;
}

// Trajectory samples at the start of the query's step (before the
// space-charge update and emission), on the query's schedule.
template <class P, class Tab>
static int32_t sample_query(mc_server *S, Query &Q) {
    const mc_operating &qo = Q.q.op;
    if (qo.sample_every > 0 && qo.sample_stride > 0 && Q.step % qo.sample_every == 0 && Q.n_slots > 0 &&
        Q.q.sample_capacity > 0) {
        k_sample<typename P::T><<<(unsigned)((Q.n_slots + kSampleThreads - 1) / kSampleThreads), kSampleThreads, 0,
                                  S->stream>>>(
            packs_of<P, Tab>(Q), Q.sp_dev, Q.n_slots, Q.step, qo.sample_stride, Q.samples, Q.scount,
            Q.q.sample_capacity);
        SCHK(hipGetLastError());
    }
    return MC_OK;
}

// Adaptive queries (Eq. 1): their samples and the space-charge updates due by
// simulated time, then the per-pack limit reductions of all of them, and one
// synchronisation for their limits; a query whose step collapses stops with
// MC_ENUMERIC (the others go on).
template <class P, class Tab>
static int32_t adaptive_steps(mc_server *S, std::vector<Query *> &act) {
    int na = 0;
    for (Query *Qp : act) {
        Query &Q = *Qp;
        if (!Q.q.op.adaptive) continue;
        const mc_operating &op = Q.q.op;
        int32_t rc = sample_query<P, Tab>(S, Q);
        if (rc) return rc;
        const double tol = 1e-6 * op.dt;
        if (op.sc_on && Q.t >= Q.t_next_pic - tol) {
            rc = pic_query<P, Tab, typename P::T>(S, Q, packs_of<P, Tab>(Q));
            if (rc) return rc;
            const double period = op.sc_every * op.dt;
            while (Q.t_next_pic <= Q.t + tol) Q.t_next_pic += period;
        }
        if (Q.n_slots > 0) {
            const StepArgs<P, Tab> a = query_step_args<P, Tab>(S, Q, Q.t, op.dt);
            k_dt_limits<P, Tab><<<blocks_for(Q.n_slots), kBlk, 0, S->stream>>>(a, Q.dt_rep);
        }
        k_dt_reduce<<<1, kHotRep, 0, S->stream>>>(Q.dt_rep, Q.dt_out);
        SCHK(hipGetLastError());
        SCHK(hipMemcpyAsync(S->h_dt + 2 * na, Q.dt_out, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                            S->stream));
        ++na;
    }
    if (na == 0) return MC_OK;
    SCHK(hipStreamSynchronize(S->stream));
    int k = 0;
    for (Query *Qp : act) {
        Query &Q = *Qp;
        if (!Q.q.op.adaptive) continue;
        const mc_operating &op = Q.q.op;
        double lim;
        std::memcpy(&lim, &S->h_dt[2 * k], sizeof(double));
        const bool lang = S->h_dt[2 * k + 1] != 0ull;
        ++k;
        double d = std::min(op.dt, lim);
        if (op.v_rf != 0.0 && op.f_rf > 0.0) d = std::min(d, 0.05 / op.f_rf);
        if (lang && op.lv_dt_max > 0.0) d = std::min(d, op.lv_dt_max);
        if (op.sc_on) d = std::min(d, Q.t_next_pic - Q.t);
        if (!(d > 1e-9 * op.dt)) {
            Q.fail_code = MC_ENUMERIC;
            continue;
        }
        Q.dt_now = d;
        source_dt(Q.src, Q.q.ion.charge_z, d);
    }
    return MC_OK;
}

template <class P, class Tab>
static int32_t co_step(mc_server *S, std::vector<Query *> &act) {
    using D = typename P::T;
    const int32_t maxres = S->opt.max_resident;
    // ring slot: wait until the GPU has consumed its previous contents
    const int slot = S->ring_pos;
    S->ring_pos = (S->ring_pos + 1) % kRing;
    if (S->ring_used[slot]) SCHK(hipEventSynchronize(S->ring_ev[slot]));
    char *h = S->h_ring + slot * S->ring_slot;
    char *d = S->d_ring + slot * S->ring_slot;
    const size_t pre = (size_t)Pool::round_up(2 * (maxres + 1) * sizeof(int32_t));
    int32_t *pe = (int32_t *)h, *ps = pe + (maxres + 1);
    EmitArgs<P, Tab> *ed = (EmitArgs<P, Tab> *)(h + pre);
    StepArgs<P, Tab> *sd = (StepArgs<P, Tab> *)(h + pre + maxres * sizeof(EmitArgs<P, Tab>));
    int ne = 0, ns = 0, be = 0, bs = 0;
    int32_t rc0 = adaptive_steps<P, Tab>(S, act);
    if (rc0) return rc0;
    for (Query *Qp : act) {
        Query &Q = *Qp;
        if (Q.fail_code) continue;
        if (!Q.q.op.adaptive) {
            int32_t rc = sample_query<P, Tab>(S, Q);
            if (rc) return rc;
        }
        if (!Q.q.op.adaptive && Q.q.op.sc_on && Q.step % Q.q.op.sc_every == 0) {
            int32_t rc = pic_query<P, Tab, D>(S, Q, packs_of<P, Tab>(Q));
            if (rc) return rc;
        }
        int64_t cnt = (Q.src.in.kind == 0) ? (Q.step == 0 ? Q.src.in.n_total : 0) : due(Q.src, Q.step);
        cnt = std::min(cnt, Q.src.in.n_total - Q.src.emitted);
        if (cnt > 0) {
            EmitArgs<P, Tab> a{};
            a.p = packs_of<P, Tab>(Q);
            a.gtab = static_cast<const Tab *>(S->gtab);
            std::memcpy(a.gsc, S->gsc, sizeof(a.gsc));
            a.sp = Q.sp_dev;
            a.slot0 = Q.n_slots;
            a.count = cnt;
            a.id0 = Q.src.emitted;
            a.step = Q.step;
            a.sigma_r = Q.src.in.sigma_r;
            a.r_trunc = Q.src.in.r_trunc;
            a.z_inj = Q.src.in.z_inj;
            a.w = Q.src.w;
            a.q = Q.src.q_fx;
            a.inv_dr = S->inv_dr;
            a.inv_dz = S->inv_dz;
            a.nr = S->nr;
            a.nz = S->nz;
            a.ion = 0;
            a.k0 = (uint32_t)Q.q.seed;
            a.k1 = (uint32_t)(Q.q.seed >> 32);
            pe[ne] = be;
            ed[ne++] = a;
            be += (int)blocks_for(cnt);
            Q.n_slots += cnt;
            Q.src.emitted += cnt;
            Q.emitted_n += cnt;
            Q.emitted_w += cnt * Q.src.w_fx;
        }
        if (Q.n_slots > 0) {
            const StepArgs<P, Tab> a = Q.q.op.adaptive ? query_step_args<P, Tab>(S, Q, Q.t, Q.dt_now)
                                                       : query_step_args<P, Tab>(S, Q, (double)Q.step * Q.q.op.dt,
                                                                                 Q.q.op.dt);
            ps[ns] = bs;
            sd[ns++] = a;
            bs += (int)((Q.n_slots + kStepBlk - 1) / kStepBlk);
        }
        if (Q.q.op.adaptive) Q.t += Q.dt_now;
        Q.step++;
    }
    pe[ne] = be;
    ps[ns] = bs;
    const size_t used = pre + maxres * sizeof(EmitArgs<P, Tab>) + ns * sizeof(StepArgs<P, Tab>);
    SCHK(hipMemcpyAsync(d, h, used, hipMemcpyHostToDevice, S->stream));
    const int32_t *dpe = (const int32_t *)d, *dps = dpe + (maxres + 1);
    if (ne > 0) {
        k_emit_multi<P, Tab><<<be, kBlk, 0, S->stream>>>((const EmitArgs<P, Tab> *)(d + pre), dpe, ne);
        SCHK(hipGetLastError());
    }
    if (ns > 0) {
        k_step_multi<P, Tab><<<bs, kStepBlk, 0, S->stream>>>(
            (const StepArgs<P, Tab> *)(d + pre + maxres * sizeof(EmitArgs<P, Tab>)), dps, ns);
        SCHK(hipGetLastError());
    }
    SCHK(hipEventRecord(S->ring_ev[slot], S->stream));
    S->ring_used[slot] = true;
    S->st.co_steps++;
    return MC_OK;
}

template <class T>
static int32_t retire_query(mc_server *S, Query &Q, PackPtrs<T> p) {
    const int64_t ns = 2 + MC_HIST_KE + MC_HIST_TEFF;
    k_zero_u64<<<blocks_for(ns), kBlk, 0, S->stream>>>(Q.snap, ns);
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(blocks_for(Q.n_slots), Q.partial_len));
    if (Q.n_slots > 0) {
        k_snapshot<T><<<(unsigned)nb, kBlk, 0, S->stream>>>(p, Q.sp_dev, Q.n_slots, Q.snap, Q.snap + 2,
                                                           Q.snap + 2 + MC_HIST_KE, Q.partial);
        k_reduce_partials<<<1, kBlk, 0, S->stream>>>(Q.partial, nb, Q.sums, nullptr);
    } else {
        k_zero_u64<<<1, kBlk, 0, S->stream>>>((unsigned long long *)Q.sums, 4);
    }
    SCHK(hipGetLastError());
    std::vector<unsigned long long> tal(Q.tal_len), snap(ns);
    double sums[4];
    unsigned long long nsamp = 0;
    SCHK(hipMemcpyAsync(tal.data(), Q.tal, Q.tal_len * 8, hipMemcpyDeviceToHost, S->stream));
    SCHK(hipMemcpyAsync(snap.data(), Q.snap, ns * 8, hipMemcpyDeviceToHost, S->stream));
    SCHK(hipMemcpyAsync(sums, Q.sums, 4 * 8, hipMemcpyDeviceToHost, S->stream));
    SCHK(hipMemcpyAsync(&nsamp, Q.scount, 8, hipMemcpyDeviceToHost, S->stream));
    SCHK(hipStreamSynchronize(S->stream));
    // exit records and samples the query kept (appends beyond the capacity were counted, not stored)
    const int64_t nex = std::min<int64_t>((int64_t)tal[TC_EXCOUNT], Q.tp.exit_cap);
    Q.r_exits.resize((size_t)std::max<int64_t>(nex, 0));
    if (nex > 0)
        SCHK(hipMemcpyAsync(Q.r_exits.data(), Q.tp.exits, nex * sizeof(mc_exit_rec), hipMemcpyDeviceToHost,
                            S->stream));
    const int64_t nsm = std::min<int64_t>((int64_t)nsamp, std::max<int64_t>(Q.q.sample_capacity, 0));
    Q.r_samples.resize((size_t)std::max<int64_t>(nsm, 0));
    if (nsm > 0)
        SCHK(hipMemcpyAsync(Q.r_samples.data(), Q.samples, nsm * sizeof(mc_sample_rec), hipMemcpyDeviceToHost,
                            S->stream));
    if (nex > 0 || nsm > 0) SCHK(hipStreamSynchronize(S->stream));
    fold_hot(tal.data() + (Q.tal_len - kHotLen), tal.data());
    mc_tallies &r = Q.r;
    r.emitted_n = Q.emitted_n;
    r.emitted_w = Q.emitted_w;
    for (int c = 0; c < MC_NCLASS; ++c) {
        r.class_n[c] = (int64_t)tal[TC_CLASS_N + c];
        r.class_w[c] = (int64_t)tal[TC_CLASS_W + c];
    }
    r.class_n[MC_ACTIVE] = (int64_t)snap[0];
    r.class_w[MC_ACTIVE] = (int64_t)snap[1];
    r.n_cand = (int64_t)tal[TC_CAND];
    r.n_coll = (int64_t)tal[TC_COLL];
    r.n_cap = (int64_t)tal[TC_CAP];
    r.n_clamp = (int64_t)tal[TC_CLAMP];
    r.pack_steps = (int64_t)tal[TC_PACKSTEPS];
    r.exit_overflow = (int64_t)tal[TC_EXOVER];
    r.exit_dropped = (int64_t)tal[TC_EXDROP];
    r.n_langevin = (int64_t)tal[TC_LANG];
    r.n_exchange = (int64_t)tal[TC_EXCH];
    r.sum_w_ke_active = sums[0];
    r.sum_w_eint_active = sums[1];
    r.sum_w_dissoc_terminal = sums[2];
    const int64_t nn = (int64_t)S->nr * S->nz;
    const unsigned long long *b = tal.data() + TC_N;
    Q.r_bins.assign(b, b + Q.q.op.n_exit_bins);
    b += Q.q.op.n_exit_bins;
    Q.r_loss.assign(b, b + nn);
    b += nn;
    Q.r_hke.assign(b, b + MC_HIST_KE);
    b += MC_HIST_KE;
    Q.r_hte.assign(b, b + MC_HIST_TEFF);
    b += MC_HIST_TEFF;
    Q.r_hr.assign(b, b + MC_HIST_R);
    Q.r_ahke.assign(snap.begin() + 2, snap.begin() + 2 + MC_HIST_KE);
    Q.r_ahte.assign(snap.begin() + 2 + MC_HIST_KE, snap.end());
    return MC_OK;
}

// ---------------------------------------------------------------------------
// Worker.
// ---------------------------------------------------------------------------
static void fail_all(mc_server *S, int32_t code) {
    std::lock_guard<std::mutex> lk(S->mu);
    for (Query *Q : S->resident) {
        Q->state = MC_Q_FAILED;
        Q->err = code;
        Q->t_done = S->now();
        S->st.failed++;
    }
    for (Query *Q : S->pending) {
        Q->state = MC_Q_FAILED;
        Q->err = code;
        Q->t_done = S->now();
        S->st.failed++;
    }
    S->resident.clear();
    S->pending.clear();
    S->dead = true;
    S->cv_done.notify_all();
}

template <class P, class Tab>
static int32_t worker_round(mc_server *S) {
    std::vector<Query *> admitted;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv.wait(lk, [&] { return S->stop || !S->pending.empty() || !S->resident.empty(); });
        if (S->stop) return MC_OK;
        while (!S->pending.empty() && (int32_t)S->resident.size() < S->opt.max_resident) {
            Query *Q = S->pending.front();
            const int64_t off = S->pool.alloc(Q->bytes);
            if (off < 0) break;  // first in line does not fit yet: keep arrival order
            Q->pool_off = off;
            Q->state = MC_Q_RUNNING;
            Q->t_admit = S->now();
            S->pending.pop_front();
            S->resident.push_back(Q);
            S->st.admitted++;
            admitted.push_back(Q);
        }
        S->st.max_resident_seen = std::max<int64_t>(S->st.max_resident_seen, (int64_t)S->resident.size());
        if (S->busy_since < 0 && !S->resident.empty()) S->busy_since = S->now();
    }
    for (Query *Q : admitted) {
        int32_t rc = admit_query<P, Tab>(S, *Q);
        if (rc) return rc;
    }
    std::vector<Query *> act;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        act = S->resident;
    }
    for (int k = 0; k < S->opt.steps_per_sync; ++k) {
        std::vector<Query *> live;
        for (Query *Q : act)
            if (Q->step < Q->q.n_steps && !Q->fail_code) live.push_back(Q);
        if (live.empty()) break;
        int32_t rc = co_step<P, Tab>(S, live);
        if (rc) return rc;
    }
    SCHK(hipStreamSynchronize(S->stream));
    for (Query *Q : act) {
        if (Q->step < Q->q.n_steps && !Q->fail_code) continue;
        if (!Q->fail_code) {
            int32_t rc;
            if constexpr (P::kTwo) rc = retire_query<float>(S, *Q, Q->p32);
            else rc = retire_query<double>(S, *Q, Q->p64);
            if (rc) return rc;
        }
        std::lock_guard<std::mutex> lk(S->mu);
        S->pool.release(Q->pool_off);
        Q->pool_off = -1;
        Q->t_done = S->now();
        if (Q->fail_code) {
            Q->state = MC_Q_FAILED;
            Q->err = Q->fail_code;
            S->st.failed++;
        } else {
            Q->state = MC_Q_DONE;
            S->st.completed++;
            S->st.pack_steps += Q->r.pack_steps;
        }
        S->resident.erase(std::find(S->resident.begin(), S->resident.end(), Q));
        if (S->resident.empty() && S->busy_since >= 0) {
            S->st.busy_s += S->now() - S->busy_since;
            S->busy_since = -1;
        }
        S->cv_done.notify_all();
    }
    return MC_OK;
}

template <class P, class Tab>
static void worker_main(mc_server *S) {
    if (hipSetDevice(S->opt.device) != hipSuccess) {
        fail_all(S, MC_EDEVICE);
        return;
    }
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->stop) return;
        }
        const int32_t rc = worker_round<P, Tab>(S);
        if (rc) {
            fail_all(S, rc);
            return;
        }
    }
}

// ---------------------------------------------------------------------------
// ABI.
// ---------------------------------------------------------------------------
extern "C" {

const char *mc_server_last_error(const mc_server *S) { return S ? S->err.c_str() : "null server"; }

static double absmax_h(const double *a, int64_t n) {
    double m = 0.0;
    if (!a) return 0.0;
    for (int64_t k = 0; k < n; ++k) m = std::max(m, std::fabs(a[k]));
    return m;
}

int32_t mc_server_create(const mc_server_options *o, const mc_grid *g, const mc_field_tables *t, mc_server **out) {
    if (!o || !g || !t || !out || !t->phi_dc || !t->gas_p || !t->gas_t) return MC_EINVAL;
    *out = nullptr;
    if (o->hbm_budget <= 0 || o->max_resident < 1 || o->max_resident > 4096 || o->steps_per_sync < 1 ||
        (o->precision != MC_PREC_FP64 && o->precision != MC_PREC_FP32) || (!o->alloc) != (!o->free) ||
        !(o->gas_mass_da > 0) || !(o->d_hit >= 0) || g->nr < 3 || g->nz < 3 || !(g->dr > 0) || !(g->dz > 0))
        return MC_EINVAL;
    if (!valid_tables(t, (int64_t)g->nr * g->nz)) return MC_EINVAL;
    mc_server *S = new (std::nothrow) mc_server();
    if (!S) return MC_ENOMEM;
    S->opt = *o;
    S->t0 = std::chrono::steady_clock::now();
    auto bail = [&](int32_t rc) {
        std::fprintf(stderr, "mc_server_create: %s\n", S->err.c_str());
        mc_server_destroy(S);
        return rc;
    };
    if (hipSetDevice(o->device) != hipSuccess) return bail(sfail(S, MC_EDEVICE, "hipSetDevice"));
    if (o->stream) {
        S->stream = static_cast<hipStream_t>(o->stream);
    } else {
        if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess)
            return bail(sfail(S, MC_EDEVICE, "stream"));
        S->own_stream = true;
    }
    S->nr = g->nr;
    S->nz = g->nz;
    S->dr = g->dr;
    S->dz = g->dz;
    S->inv_dr = 1.0 / g->dr;
    S->inv_dz = 1.0 / g->dz;
    S->R = (g->nr - 1) * g->dr;
    const int64_t nn = (int64_t)g->nr * g->nz;
    const int32_t m = g->nz - 2, nu = g->nr - 1;
    double *tmp = nullptr;
    uint8_t *mask = nullptr;
    int32_t rc = MC_OK;
    if (!rc) rc = salloc_t(S, &S->e_dc, nn);
    if (!rc) rc = salloc_t(S, &S->e_off, nn);
    if (!rc) rc = salloc_t(S, &S->e_rf, nn);
    if (!rc) rc = salloc_t(S, &S->e_zero, nn);
    if (!rc) rc = salloc(S, &S->gtab, nn * S->node_bytes());
    if (!rc) rc = salloc_t(S, &S->hit, nn);
    if (!rc) rc = salloc_t(S, &mask, nn);
    if (!rc) rc = salloc_t(S, &S->sine, 2 * (int64_t)(g->nz - 1));
    if (!rc) rc = salloc_t(S, &S->tcp, (int64_t)nu * m);
    if (!rc) rc = salloc_t(S, &S->tinv, (int64_t)nu * m);
    if (!rc) rc = salloc_t(S, &tmp, 4 * nn);
    if (!rc) rc = salloc_t(S, &S->tables, 1);
    if (rc) return bail(rc);
    for (auto &a : S->allocs) S->shared_bytes += (int64_t)a.second;
#define SC2(expr) do { if ((expr) != hipSuccess) return bail(sfail(S, MC_EDEVICE, #expr)); } while (0)
    SC2(hipMemsetAsync(S->e_off, 0, nn * sizeof(double2), S->stream));
    SC2(hipMemsetAsync(S->e_rf, 0, nn * sizeof(double2), S->stream));
    SC2(hipMemsetAsync(S->e_zero, 0, nn * sizeof(double2), S->stream));
    const double *phis[3] = {t->phi_dc, t->phi_off, t->phi_rf};
    double2 *outs[3] = {S->e_dc, S->e_off, S->e_rf};
    for (int k = 0; k < 3; ++k) {
        if (!phis[k]) continue;
        SC2(hipMemcpyAsync(tmp, phis[k], nn * sizeof(double), hipMemcpyHostToDevice, S->stream));
        k_bake<<<blocks_for(nn), kBlk, 0, S->stream>>>(tmp, outs[k], g->nr, g->nz, g->dr, g->dz, nullptr);
        SC2(hipStreamSynchronize(S->stream));
    }
    const double *gas[4] = {t->gas_ur, t->gas_uz, t->gas_p, t->gas_t};
    for (int k = 0; k < 4; ++k) {
        if (gas[k]) SC2(hipMemcpyAsync(tmp + k * nn, gas[k], nn * 8, hipMemcpyHostToDevice, S->stream));
        else SC2(hipMemsetAsync(tmp + k * nn, 0, nn * 8, S->stream));
        S->gsc[k] = absmax_h(gas[k], nn) > 0 ? (float)absmax_h(gas[k], nn) : 1.0f;
    }
    if (!S->fp32())
        k_gas<double4><<<blocks_for(nn), kBlk, 0, S->stream>>>((double4 *)S->gtab, tmp, tmp + nn, tmp + 2 * nn,
                                                                tmp + 3 * nn, nn, 1, 1, 1, 1);
    else if (S->bf16())
        k_gas<bf16x4><<<blocks_for(nn), kBlk, 0, S->stream>>>((bf16x4 *)S->gtab, tmp, tmp + nn, tmp + 2 * nn,
                                                               tmp + 3 * nn, nn, S->gsc[0], S->gsc[1], S->gsc[2],
                                                               S->gsc[3]);
    else
        k_gas<float4><<<blocks_for(nn), kBlk, 0, S->stream>>>((float4 *)S->gtab, tmp, tmp + nn, tmp + 2 * nn,
                                                               tmp + 3 * nn, nn, 1, 1, 1, 1);
    if (!S->bf16()) std::fill(S->gsc, S->gsc + 4, 1.0f);
    StepTables tables_host;
    step_tables_fill(&tables_host);
    SC2(hipMemcpyAsync(S->tables, &tables_host, sizeof(tables_host), hipMemcpyHostToDevice, S->stream));
    if (t->mask) SC2(hipMemcpyAsync(mask, t->mask, nn, hipMemcpyHostToDevice, S->stream));
    else SC2(hipMemsetAsync(mask, 0, nn, S->stream));
    const double reach = o->d_hit + 0.5 * std::min(g->dr, g->dz);
    k_hit<<<blocks_for(nn), kBlk, 0, S->stream>>>(mask, S->hit, g->nr, g->nz, g->dr, g->dz, reach,
                                                 (int32_t)std::ceil(reach / g->dr), (int32_t)std::ceil(reach / g->dz));
    k_sine_table<<<blocks_for(2 * (g->nz - 1)), kBlk, 0, S->stream>>>(S->sine, g->nz);
    k_thomas_coef<<<blocks_for(m), kBlk, 0, S->stream>>>(S->tcp, S->tinv, g->nr, g->nz, g->dr, g->dz);
    SC2(hipGetLastError());
    {
        Bluestein &B = S->blu;
        const size_t cx = S->fp32() ? 2 * sizeof(float) : 2 * sizeof(double);
        const int32_t L = bluestein_length(m);
        if (bluestein_lds(L, cx) <= lds_per_block()) {
            B.L = L;
            B.lds = bluestein_lds(L, cx);
            if (salloc(S, &B.chirp, (size_t)m * cx) || salloc(S, &B.tw, (size_t)std::max(L / 2, 1) * cx) ||
                salloc(S, &B.fb, (size_t)L * cx))
                return bail(MC_ENOMEM);
            const hipError_t e = S->fp32() ? bluestein_prepare<float>(B, m, S->stream)
                                           : bluestein_prepare<double>(B, m, S->stream);
            if (e != hipSuccess) B.L = 0;
        }
    }
    S->pg.nr = g->nr;
    S->pg.nz = g->nz;
    S->pg.dr = g->dr;
    S->pg.dz = g->dz;
    S->pg.sine = S->sine;
    S->pg.tcp = S->tcp;
    S->pg.tinv = S->tinv;
    S->pg.blu = &S->blu;
    S->mask_nodes = mask_unknowns(t->mask, g->nr, g->nz);
    SC2(hipStreamSynchronize(S->stream));
    if (S->bf16()) {
        std::vector<double2> h(nn);
        double mx[4] = {0, 0, 0, 0};
        SC2(hipMemcpy(h.data(), S->e_dc, nn * sizeof(double2), hipMemcpyDeviceToHost));
        for (auto &v : h) { mx[0] = std::max(mx[0], std::fabs(v.x)); mx[1] = std::max(mx[1], std::fabs(v.y)); }
        SC2(hipMemcpy(h.data(), S->e_rf, nn * sizeof(double2), hipMemcpyDeviceToHost));
        for (auto &v : h) { mx[2] = std::max(mx[2], std::fabs(v.x)); mx[3] = std::max(mx[3], std::fabs(v.y)); }
        for (int k = 0; k < 4; ++k) S->esc[k] = mx[k] > 0 ? (float)mx[k] : 1.0f;
    }
    // descriptor ring (pinned host + device)
    const size_t emit_sz = S->fp32() ? (S->bf16() ? sizeof(EmitArgs<P32, bf16x4>) : sizeof(EmitArgs<P32, float4>))
                                     : sizeof(EmitArgs<P64, double4>);
    const size_t step_sz = S->fp32() ? (S->bf16() ? sizeof(StepArgs<P32, bf16x4>) : sizeof(StepArgs<P32, float4>))
                                     : sizeof(StepArgs<P64, double4>);
    S->ring_slot = (size_t)Pool::round_up((int64_t)(Pool::round_up(2 * (o->max_resident + 1) * sizeof(int32_t)) +
                                                    o->max_resident * (emit_sz + step_sz)));
    if (hipHostMalloc((void **)&S->h_ring, kRing * S->ring_slot, hipHostMallocDefault) != hipSuccess)
        return bail(sfail(S, MC_ENOMEM, "pinned descriptor ring"));
    if (hipHostMalloc((void **)&S->h_dt, 2 * (size_t)o->max_resident * sizeof(unsigned long long),
                      hipHostMallocDefault) != hipSuccess)
        return bail(sfail(S, MC_ENOMEM, "pinned step-limit buffer"));
    if (salloc(S, (void **)&S->d_ring, kRing * S->ring_slot)) return bail(MC_ENOMEM);
    for (int k = 0; k < kRing; ++k) SC2(hipEventCreateWithFlags(&S->ring_ev[k], hipEventDisableTiming));
    // the query pool
    if (salloc(S, (void **)&S->pool_base, (size_t)o->hbm_budget)) return bail(MC_ENOMEM);
    S->pool.reset(o->hbm_budget);
#undef SC2
    if (!S->fp32()) S->worker = std::thread(worker_main<P64, double4>, S);
    else if (S->bf16()) S->worker = std::thread(worker_main<P32, bf16x4>, S);
    else S->worker = std::thread(worker_main<P32, float4>, S);
    *out = S;
    return MC_OK;
}

void mc_server_destroy(mc_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    (void)hipSetDevice(S->opt.device);
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    for (auto &a : S->allocs) {
        if (S->opt.free) S->opt.free(a.first, S->stream, S->opt.alloc_user);
        else (void)hipFree(a.first);
    }
    for (int k = 0; k < kRing; ++k)
        if (S->ring_ev[k]) (void)hipEventDestroy(S->ring_ev[k]);
    if (S->h_ring) (void)hipHostFree(S->h_ring);
    if (S->h_dt) (void)hipHostFree(S->h_dt);
    if (S->own_stream && S->stream) (void)hipStreamDestroy(S->stream);
    for (auto &kv : S->all) delete kv.second;
    delete S;
}

static bool valid_query(const mc_server *S, const mc_query *q) {
    if (!q || !valid_ion(&q->ion) || q->n_steps < 0) return false;
    const mc_operating &op = q->op;
    if (!(op.dt > 0) || op.sc_every < 1 || op.n_exit_bins < 1 || !(op.exit_bin_dt > 0) || !(op.r_det > 0)) return false;
    if (op.langevin_on && !(op.lv_switch >= 0)) return false;
    if (!(op.lv_dt_max >= 0)) return false;
    if (op.sample_every < 0 || op.sample_stride < 0 || q->sample_capacity < 0) return false;
    const mc_source &s = q->source;
    if (s.kind < 0 || s.kind > 2 || !(s.sigma_r > 0) || !(s.r_trunc > 0) || s.n_total < 0) return false;
    if ((s.kind == 1 && s.packs_per_step <= 0) || (s.kind != 1 && !(s.weight > 0))) return false;
    return q->exit_capacity >= 0;
}

int32_t mc_server_submit(mc_server *S, const mc_query *q, uint64_t *qid) {
    if (!S || !qid) return MC_EINVAL;
    if (!valid_query(S, q)) return sfail(S, MC_EINVAL, "invalid query");
    Query *Q = new (std::nothrow) Query();
    if (!Q) return MC_ENOMEM;
    Q->q = *q;
    Q->q.op.gas_mass_da = S->opt.gas_mass_da;
    Q->q.op.d_hit = S->opt.d_hit;
    Q->sp = make_species(&Q->q.ion);
    species_alpha(Q->sp, Q->q.ion, S->opt.gas_mass_da);
    Q->src = make_source(Q->q.source, Q->q.ion.charge_z, Q->q.op.dt);
    Q->bytes = query_layout(S, *Q, [](const char *, int64_t, int64_t) {});
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->dead) {
        delete Q;
        return sfail(S, MC_EDEVICE, "server stopped after a device error: " + S->err);
    }
    if (Q->bytes > S->pool.size()) {
        const std::string m = "query needs " + std::to_string(Q->bytes) + " bytes, pool has " +
                              std::to_string(S->pool.size());
        delete Q;
        return sfail(S, MC_EBUDGET, m);
    }
    Q->id = S->next_id++;
    Q->t_submit = S->now();
    S->all[Q->id] = Q;
    S->pending.push_back(Q);
    S->st.submitted++;
    *qid = Q->id;
    S->cv.notify_all();
    return MC_OK;
}

static void copy_arr(int64_t *dst, const std::vector<int64_t> &v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(int64_t));
}

static int32_t poll_locked(mc_server *S, uint64_t qid, mc_query_result *out) {
    auto it = S->all.find(qid);
    if (it == S->all.end()) return sfail(S, MC_EINVAL, "unknown query id");
    Query &Q = *it->second;
    if (!out) return MC_OK;
    out->state = Q.state;
    out->error = Q.err;
    out->t_submit = Q.t_submit;
    out->t_admit = Q.t_admit;
    out->t_done = Q.t_done;
    out->device_bytes = Q.bytes;
    if (Q.state == MC_Q_DONE) {
        mc_tallies &o = out->tallies;
        int64_t *ptrs[7] = {o.exit_bins, o.loss_map, o.hist_ke, o.hist_teff, o.hist_r, o.act_hist_ke, o.act_hist_teff};
        o = Q.r;
        o.exit_bins = ptrs[0];
        o.loss_map = ptrs[1];
        o.hist_ke = ptrs[2];
        o.hist_teff = ptrs[3];
        o.hist_r = ptrs[4];
        o.act_hist_ke = ptrs[5];
        o.act_hist_teff = ptrs[6];
        copy_arr(o.exit_bins, Q.r_bins);
        copy_arr(o.loss_map, Q.r_loss);
        copy_arr(o.hist_ke, Q.r_hke);
        copy_arr(o.hist_teff, Q.r_hte);
        copy_arr(o.hist_r, Q.r_hr);
        copy_arr(o.act_hist_ke, Q.r_ahke);
        copy_arr(o.act_hist_teff, Q.r_ahte);
        out->n_exits = (int64_t)Q.r_exits.size();
        if (out->exits && out->exits_len > 0)
            std::memcpy(out->exits, Q.r_exits.data(),
                        (size_t)std::min<int64_t>(out->n_exits, out->exits_len) * sizeof(mc_exit_rec));
        out->n_samples = (int64_t)Q.r_samples.size();
        if (out->samples && out->samples_len > 0)
            std::memcpy(out->samples, Q.r_samples.data(),
                        (size_t)std::min<int64_t>(out->n_samples, out->samples_len) * sizeof(mc_sample_rec));
    } else {
        out->n_exits = 0;
        out->n_samples = 0;
    }
    return MC_OK;
}

int32_t mc_server_poll(mc_server *S, uint64_t qid, mc_query_result *out) {
    if (!S) return MC_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    return poll_locked(S, qid, out);
}

int32_t mc_server_wait(mc_server *S, uint64_t qid, double timeout_s, mc_query_result *out) {
    if (!S) return MC_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(qid);
    if (it == S->all.end()) return sfail(S, MC_EINVAL, "unknown query id");
    Query *Q = it->second;
    S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                        [&] { return Q->state == MC_Q_DONE || Q->state == MC_Q_FAILED; });
    return poll_locked(S, qid, out);
}

int32_t mc_server_release(mc_server *S, uint64_t qid) {
    if (!S) return MC_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(qid);
    if (it == S->all.end()) return sfail(S, MC_EINVAL, "unknown query id");
    if (it->second->state != MC_Q_DONE && it->second->state != MC_Q_FAILED)
        return sfail(S, MC_ESTATE, "query not finished");
    delete it->second;
    S->all.erase(it);
    return MC_OK;
}

int32_t mc_server_get_stats(mc_server *S, mc_server_stats *out) {
    if (!S || !out) return MC_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->resident = (int64_t)S->resident.size();
    out->pending = (int64_t)S->pending.size();
    out->pool_bytes = S->pool.size();
    out->pool_in_use = S->pool.in_use();
    out->pool_peak = S->pool.peak();
    out->shared_bytes = S->shared_bytes;
    out->wall_s = S->now();
    if (S->busy_since >= 0) out->busy_s += S->now() - S->busy_since;
    return MC_OK;
}

}  // extern "C"

// Autotuner of the plan's tile shapes: atoms per cluster tile and work-item
// length of the Vlocal kernel, and the brick shape of the bigcell-stationary
// rho/force kernels, each chosen by timing its own stage on the caller's
// device (paper: parameters tuned by short timed trials before the
// production run, "Device Performance Optimization").
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <mutex>
#include <vector>

#include "gint.h"
#include "gint_internal.h"

hipError_t gint_launch_fill(double *p, long long n, double v, hipStream_t s);

namespace {

// candidates in trial order (0 = the plan's default): (cluster_atoms,
// max_bigcells_per_item) of Vlocal, and bricks in bigcells along a1, a2, a3.
// Mixed-precision plans with rho and force on bricks take clusters of up to
// eight atoms (the eight-wave Vlocal kernel), the others up to four.
constexpr int kCand[][2] = {{4, 0}, {3, 0}, {4, 32}, {2, 0}, {4, 128}, {3, 32}, {4, 8}, {2, 32}};
constexpr int kCandWide[][2] = {{4, 0}, {8, 0}, {3, 0}, {6, 0}, {4, 128}, {8, 32}, {4, 32}, {2, 0}};
static_assert(sizeof(kCand) == sizeof(kCandWide), "one cluster candidate per trial in both lists");
constexpr int kBrick[][3] = {{0, 0, 0}, {1, 1, 1}, {2, 2, 1}, {2, 2, 4}, {1, 1, 2}, {2, 2, 2}, {4, 4, 2}, {4, 4, 4}};
constexpr int kNCand = (int)(sizeof(kCand) / sizeof(kCand[0]));
static_assert(kNCand <= GINT_TUNE_MAX, "candidate list longer than the report");
static_assert(sizeof(kBrick) / sizeof(kBrick[0]) == (size_t)kNCand, "one brick candidate per trial");

struct Buffers {
    double *v = nullptr, *d = nullptr, *h = nullptr, *rho = nullptr, *f = nullptr, *sig = nullptr;
    ~Buffers() {
        double *all[] = {v, d, h, rho, f, sig};
        for (double *p : all)
            if (p) (void)hipFree(p);
    }
};

// Shape class of a tuning request: the device, the form, and the sizes of
// the workload (two requests with equal keys get the same choice).
struct TuneKey {
    int device, precision, decomposition, n_sys;
    long long natom, nblk;
    int grid0[3];
    double cell0[9];
    bool operator==(const TuneKey &o) const {
        return device == o.device && precision == o.precision && decomposition == o.decomposition &&
               n_sys == o.n_sys && natom == o.natom && nblk == o.nblk &&
               std::memcmp(grid0, o.grid0, sizeof(grid0)) == 0 && std::memcmp(cell0, o.cell0, sizeof(cell0)) == 0;
    }
};

struct TuneEntry {
    TuneKey key;
    gint_options opt;
    gint_tune_report rep;
};

std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune_cache;

TuneKey tune_key(const gint_system *sys, int n_sys, const gint_options *opt) {
    TuneKey k;
    std::memset(&k, 0, sizeof(k));
    if (hipGetDevice(&k.device) != hipSuccess) k.device = -1;
    k.precision = opt->precision;
    k.decomposition = opt->decomposition;
    k.n_sys = n_sys;
    for (int i = 0; i < n_sys; ++i) {
        k.natom += sys[i].natom;
        k.nblk += sys[i].nblk;
    }
    for (int d = 0; d < 3; ++d) k.grid0[d] = sys[0].grid[d];
    for (int d = 0; d < 9; ++d) k.cell0[d] = sys[0].cell[d];
    return k;
}

int step(gint_plan *p, Buffers &b, hipStream_t s) {
    int rc = gint_vlocal(p, b.v, b.h, s);
    if (rc == GINT_OK) rc = gint_rho(p, b.d, b.rho, nullptr, s);
    if (rc == GINT_OK) rc = gint_force_stress(p, b.v, b.d, b.f, b.sig, nullptr, s);
    return rc;
}

// One timed step: Vlocal between e0 and e1, rho + force/stress between e1 and e2.
int timed_step(gint_plan *p, Buffers &b, hipStream_t s, hipEvent_t ev[3], float *vl_ms, float *rf_ms) {
    hipError_t e = hipEventRecord(ev[0], s);
    int rc = e == hipSuccess ? gint_vlocal(p, b.v, b.h, s) : GINT_EHIP;
    if (rc == GINT_OK && (e = hipEventRecord(ev[1], s)) != hipSuccess) rc = GINT_EHIP;
    if (rc == GINT_OK) rc = gint_rho(p, b.d, b.rho, nullptr, s);
    if (rc == GINT_OK) rc = gint_force_stress(p, b.v, b.d, b.f, b.sig, nullptr, s);
    if (rc == GINT_OK && (e = hipEventRecord(ev[2], s)) != hipSuccess) rc = GINT_EHIP;
    if (rc == GINT_OK && (e = hipEventSynchronize(ev[2])) != hipSuccess) rc = GINT_EHIP;
    if (rc == GINT_OK && ((e = hipEventElapsedTime(vl_ms, ev[0], ev[1])) != hipSuccess ||
                          (e = hipEventElapsedTime(rf_ms, ev[1], ev[2])) != hipSuccess))
        rc = GINT_EHIP;
    return rc;
}

}  // namespace

extern "C" int gint_autotune(const gint_system *sys, int n_sys, gint_options *opt, double budget_seconds,
                             void *stream, gint_tune_report *report) {
    if (!sys || n_sys < 1 || !opt || !report || !(budget_seconds >= 0.0)) return GINT_EINVAL;
    const TuneKey key = tune_key(sys, n_sys, opt);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const TuneEntry &e : g_tune_cache)
            if (e.key == key) {
                opt->cluster_atoms = e.opt.cluster_atoms;
                opt->max_bigcells_per_item = e.opt.max_bigcells_per_item;
                for (int k = 0; k < 3; ++k) opt->brick[k] = e.opt.brick[k];
                *report = e.rep;
                report->cached = 1;
                return GINT_OK;
            }
    }
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    gint_tune_report rep{};
    rep.best = -1;
    Buffers b;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    for (hipEvent_t &x : ev)
        if (hipEventCreate(&x) != hipSuccess) {
            for (hipEvent_t y : ev)
                if (y) (void)hipEventDestroy(y);
            return GINT_EHIP;
        }
    rep.best_brick = -1;
    const bool wide = opt->precision != GINT_FP64 &&
                      (opt->decomposition == GINT_DECOMP_DEFAULT || opt->decomposition == GINT_DECOMP_BIGCELL_RHO_FORCE);
    const int(*cand)[2] = wide ? kCandWide : kCand;
    int rc = GINT_OK;
    for (int c = 0; c < kNCand; ++c) {
        const double elapsed = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (c > 0 && elapsed >= budget_seconds) break;
        gint_options o = *opt;
        o.cluster_atoms = cand[c][0];
        o.max_bigcells_per_item = cand[c][1];
        for (int k = 0; k < 3; ++k) o.brick[k] = kBrick[c][k];
        gint_plan *p = nullptr;
        rc = gint_plan_create(&p, sys, n_sys, &o, stream);
        if (rc != GINT_OK) break;
        gint_sizes q{};
        gint_plan_query(p, &q);
        if (!b.v) {
            hipError_t e = hipSuccess;
            if (e == hipSuccess) e = hipMalloc(&b.v, sizeof(double) * (size_t)q.ngrid);
            if (e == hipSuccess) e = hipMalloc(&b.rho, sizeof(double) * (size_t)q.ngrid);
            if (e == hipSuccess) e = hipMalloc(&b.d, sizeof(double) * (size_t)(q.nnz > 0 ? q.nnz : 1));
            if (e == hipSuccess) e = hipMalloc(&b.h, sizeof(double) * (size_t)(q.nnz > 0 ? q.nnz : 1));
            if (e == hipSuccess) e = hipMalloc(&b.f, sizeof(double) * 3 * (size_t)q.natom);
            if (e == hipSuccess) e = hipMalloc(&b.sig, sizeof(double) * 9 * (size_t)n_sys);
            if (e == hipSuccess) e = gint_launch_fill(b.v, q.ngrid, 0.1, s);
            if (e == hipSuccess) e = gint_launch_fill(b.d, q.nnz, 0.01, s);
            if (e != hipSuccess) {
                gint_plan_destroy(p);
                rc = GINT_ENOMEM;
                break;
            }
        }
        rc = step(p, b, s);   // untimed: first launches load the code objects
        float vl = 0.f, rf = 0.f;
        if (rc == GINT_OK) rc = timed_step(p, b, s, ev, &vl, &rf);
        gint_plan_destroy(p);
        if (rc != GINT_OK) break;
        const int t = rep.ntrials;
        rep.cluster_atoms[t] = o.cluster_atoms;
        rep.max_bigcells_per_item[t] = o.max_bigcells_per_item;
        for (int k = 0; k < 3; ++k) rep.brick[t][k] = q.decomposition != GINT_DECOMP_CLUSTER_PAIRS ? q.brick[k] : 0;
        rep.vlocal_ms[t] = vl;
        rep.rho_force_ms[t] = rf;
        rep.step_ms[t] = (double)vl + (double)rf;
        if (rep.best < 0 || vl < rep.vlocal_ms[rep.best]) rep.best = t;
        if (rep.best_brick < 0 || rf < rep.rho_force_ms[rep.best_brick]) rep.best_brick = t;
        ++rep.ntrials;
    }
    for (hipEvent_t x : ev) (void)hipEventDestroy(x);
    if (rc != GINT_OK) return rc;
    opt->cluster_atoms = rep.cluster_atoms[rep.best];
    opt->max_bigcells_per_item = rep.max_bigcells_per_item[rep.best];
    for (int k = 0; k < 3; ++k) opt->brick[k] = rep.brick[rep.best_brick][k];
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    rep.cached = 0;
    *report = rep;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache.push_back(TuneEntry{key, *opt, rep});
    }
    return GINT_OK;
}

extern "C" void gint_autotune_forget(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache.clear();
}

// Autotuner of the plan's tile shape: atoms per cluster tile and work-item
// length, chosen by timing one full pass (Vlocal + rho + force/stress) of
// each candidate on the caller's device (paper: parameters tuned by short
// timed trials before the production run, "Device Performance Optimization").
#include <hip/hip_runtime.h>

#include <chrono>

#include "gint.h"
#include "gint_internal.h"

hipError_t gint_launch_fill(double *p, long long n, double v, hipStream_t s);

namespace {

// candidate (cluster_atoms, max_bigcells_per_item) in trial order; 0 = plan default
constexpr int kCand[][2] = {{4, 0}, {3, 0}, {4, 32}, {2, 0}, {4, 128}, {3, 32}, {4, 8}, {2, 32}};
constexpr int kNCand = (int)(sizeof(kCand) / sizeof(kCand[0]));
static_assert(kNCand <= GINT_TUNE_MAX, "candidate list longer than the report");

struct Buffers {
    double *v = nullptr, *d = nullptr, *h = nullptr, *rho = nullptr, *f = nullptr, *sig = nullptr;
    ~Buffers() {
        double *all[] = {v, d, h, rho, f, sig};
        for (double *p : all)
            if (p) (void)hipFree(p);
    }
};

int step(gint_plan *p, Buffers &b, hipStream_t s) {
    int rc = gint_vlocal(p, b.v, b.h, s);
    if (rc == GINT_OK) rc = gint_rho(p, b.d, b.rho, nullptr, s);
    if (rc == GINT_OK) rc = gint_force_stress(p, b.v, b.d, b.f, b.sig, nullptr, s);
    return rc;
}

}  // namespace

extern "C" int gint_autotune(const gint_system *sys, int n_sys, gint_options *opt, double budget_seconds,
                             void *stream, gint_tune_report *report) {
    if (!sys || n_sys < 1 || !opt || !report || !(budget_seconds >= 0.0)) return GINT_EINVAL;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    gint_tune_report rep{};
    rep.best = -1;
    Buffers b;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return GINT_EHIP;
    }
    int rc = GINT_OK;
    for (int c = 0; c < kNCand; ++c) {
        const double elapsed = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (c > 0 && elapsed >= budget_seconds) break;
        gint_options o = *opt;
        o.cluster_atoms = kCand[c][0];
        o.max_bigcells_per_item = kCand[c][1];
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
            rc = step(p, b, s);   // untimed: first launches load the code objects
            if (rc != GINT_OK) {
                gint_plan_destroy(p);
                break;
            }
        }
        hipError_t e = hipEventRecord(e0, s);
        if (e == hipSuccess) rc = step(p, b, s);
        if (e == hipSuccess && rc == GINT_OK) e = hipEventRecord(e1, s);
        if (e == hipSuccess && rc == GINT_OK) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess && rc == GINT_OK) e = hipEventElapsedTime(&ms, e0, e1);
        gint_plan_destroy(p);
        if (rc != GINT_OK) break;
        if (e != hipSuccess) {
            rc = GINT_EHIP;
            break;
        }
        rep.cluster_atoms[rep.ntrials] = o.cluster_atoms;
        rep.max_bigcells_per_item[rep.ntrials] = o.max_bigcells_per_item;
        rep.step_ms[rep.ntrials] = ms;
        if (rep.best < 0 || ms < rep.step_ms[rep.best]) rep.best = rep.ntrials;
        ++rep.ntrials;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != GINT_OK) return rc;
    opt->cluster_atoms = rep.cluster_atoms[rep.best];
    opt->max_bigcells_per_item = rep.max_bigcells_per_item[rep.best];
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *report = rep;
    return GINT_OK;
}

// C ABI of the grid-integration library: plan lifetime, validation and
// launch sequencing.  All device work is enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <new>

#include "gint.h"
#include "gint_internal.h"
#include "gint_plan.hpp"

hipError_t gint_launch_fill(double *p, long long n, double v, hipStream_t s);
hipError_t gint_launch_vlocal(const GDev &P, const double *V, double *H, hipStream_t s);
hipError_t gint_launch_rho(const GDev &P, const double *D, double *rho, hipStream_t s);
hipError_t gint_launch_force(const GDev &P, const double *V, const double *D, double *F, double *ZE, hipStream_t s);
hipError_t gint_launch_work(const GDev &P, double *W, hipStream_t s);
hipError_t gint_launch_sum(const double *x, long long n, double scale, double *part, int nparts, double *out,
                           hipStream_t s);
hipError_t gint_launch_finish_stress(const double *ZE, double inv_omega, double *stress, double *energy,
                                     hipStream_t s);

namespace {

thread_local int g_last_hip = 0;
constexpr int kParts = 1024;

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct gint_plan {
    int device = 0;
    GDev canon{};      // canonical items (vlocal, rho, work)
    GDev ordered{};    // canonical + swapped items (force)
    DevBuf species, atoms, tab, pairs, bigcells, items_canon, items_ordered, ws;
    double *ZE = nullptr;      // [10]: Z (9) and E
    double *part = nullptr;    // [kParts]
    gint_sizes sizes{};
};

namespace {

int hip_fail(hipError_t e) {
    g_last_hip = (int)e;
    return GINT_EHIP;
}

template <class T>
int upload(DevBuf &b, const std::vector<T> &v, size_t &total) {
    b.bytes = v.size() * sizeof(T);
    if (b.bytes == 0) b.bytes = sizeof(T);
    hipError_t e = hipMalloc(&b.p, b.bytes);
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        b.p = nullptr;
        return GINT_ENOMEM;
    }
    total += b.bytes;
    if (!v.empty()) {
        e = hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e);
    }
    return GINT_OK;
}

void release(gint_plan *p) {
    DevBuf *bufs[] = {&p->species, &p->atoms, &p->tab, &p->pairs, &p->bigcells, &p->items_canon, &p->items_ordered,
                      &p->ws};
    for (DevBuf *b : bufs)
        if (b->p) {
            (void)hipFree(b->p);
            b->p = nullptr;
        }
}

}  // namespace

extern "C" {

int gint_plan_create(gint_plan **out, const gint_system *sys, int n_sys, const gint_options *opt, void *stream) {
    (void)stream;
    if (!out || !sys) return GINT_EINVAL;
    if (n_sys != 1) return n_sys < 1 ? GINT_EINVAL : GINT_EUNSUPPORTED;
    if (opt && opt->precision != GINT_FP64) return GINT_EUNSUPPORTED;
    const auto t0 = std::chrono::steady_clock::now();
    HostPlan hp;
    int rc;
    try {
        rc = gint_build_host_plan(sys, opt, hp);
    } catch (const std::bad_alloc &) {
        return GINT_ENOMEM;
    } catch (...) {
        return GINT_EINVAL;
    }
    if (rc != GINT_OK) return rc;
    if (hp.items_canon.size() > 0x7fffffffu || hp.items_ordered.size() > 0x7fffffffu) return GINT_ENOMEM;

    gint_plan *p = new (std::nothrow) gint_plan();
    if (!p) return GINT_ENOMEM;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e);
    }
    size_t total = 0;
    std::vector<double> wsinit(10 + kParts, 0.0);
    if ((rc = upload(p->species, hp.species, total)) || (rc = upload(p->atoms, hp.atoms, total)) ||
        (rc = upload(p->tab, hp.tab, total)) || (rc = upload(p->pairs, hp.pairs, total)) ||
        (rc = upload(p->bigcells, hp.bigcells, total)) || (rc = upload(p->items_canon, hp.items_canon, total)) ||
        (rc = upload(p->items_ordered, hp.items_ordered, total)) || (rc = upload(p->ws, wsinit, total))) {
        release(p);
        delete p;
        return rc;
    }
    p->ZE = (double *)p->ws.p;
    p->part = p->ZE + 10;

    GDev d{};
    d.species = (const GSpecies *)p->species.p;
    d.atoms = (const GAtom *)p->atoms.p;
    d.tab = (const double *)p->tab.p;
    d.pairs = (const GPair *)p->pairs.p;
    d.bigcells = (const GBig *)p->bigcells.p;
    d.natom = hp.natom;
    for (int i = 0; i < 3; ++i) {
        d.N[i] = hp.N[i];
        for (int k = 0; k < 3; ++k) d.e[i][k] = hp.e[i][k];
    }
    d.w = hp.w;
    p->canon = d;
    p->canon.items = (const GItem *)p->items_canon.p;
    p->canon.nitems = (int)hp.items_canon.size();
    p->ordered = d;
    p->ordered.items = (const GItem *)p->items_ordered.p;
    p->ordered.nitems = (int)hp.items_ordered.size();

    gint_sizes &s = p->sizes;
    s.ngrid = hp.ngrid;
    s.nnz = hp.nnz;
    s.natom = hp.natom;
    s.ncluster = hp.ncluster;
    s.npairs = hp.ncanon;
    s.nitems = (int64_t)hp.items_canon.size();
    s.nbigcells = (int64_t)hp.bigcells.size();
    s.work_units = 0.0;
    s.volume = hp.omega;
    s.device_bytes = (int64_t)total;
    s.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = p;
    return GINT_OK;
}

int gint_vlocal(gint_plan *p, const double *v_loc, double *h_vals, void *stream) {
    if (!p || !v_loc || !h_vals) return GINT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = gint_launch_fill(h_vals, p->sizes.nnz, 0.0, s);
    if (e != hipSuccess) return hip_fail(e);
    e = gint_launch_vlocal(p->canon, v_loc, h_vals, s);
    if (e != hipSuccess) return hip_fail(e);
    return GINT_OK;
}

int gint_rho(gint_plan *p, const double *d_vals, double *rho, double *n_elec, void *stream) {
    if (!p || !d_vals || !rho) return GINT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = gint_launch_fill(rho, p->sizes.ngrid, 0.0, s);
    if (e != hipSuccess) return hip_fail(e);
    e = gint_launch_rho(p->canon, d_vals, rho, s);
    if (e != hipSuccess) return hip_fail(e);
    if (n_elec) {
        e = gint_launch_sum(rho, p->sizes.ngrid, p->canon.w, p->part, kParts, n_elec, s);
        if (e != hipSuccess) return hip_fail(e);
    }
    return GINT_OK;
}

int gint_force_stress(gint_plan *p, const double *v_loc, const double *d_vals, double *force, double *stress,
                      double *energy, void *stream) {
    if (!p || !v_loc || !d_vals || !force || !stress) return GINT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = gint_launch_fill(force, 3LL * p->sizes.natom, 0.0, s);
    if (e == hipSuccess) e = gint_launch_fill(p->ZE, 10, 0.0, s);
    if (e == hipSuccess) e = gint_launch_force(p->ordered, v_loc, d_vals, force, p->ZE, s);
    if (e == hipSuccess) e = gint_launch_finish_stress(p->ZE, 1.0 / p->sizes.volume, stress, energy, s);
    if (e != hipSuccess) return hip_fail(e);
    return GINT_OK;
}

// W = sum_g n_orb(g)^2, the unit of work of the throughput metric.
int gint_work_units(gint_plan *p, double *w_out, void *stream) {
    if (!p || !w_out) return GINT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = gint_launch_fill(w_out, 1, 0.0, s);
    if (e == hipSuccess) e = gint_launch_work(p->canon, w_out, s);
    if (e != hipSuccess) return hip_fail(e);
    return GINT_OK;
}

int gint_plan_query(const gint_plan *p, gint_sizes *out) {
    if (!p || !out) return GINT_EINVAL;
    *out = p->sizes;
    return GINT_OK;
}

void gint_plan_destroy(gint_plan *p) {
    if (!p) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p->device);
    release(p);
    (void)hipSetDevice(cur);
    delete p;
}

const char *gint_strerror(int code) {
    switch (code) {
        case GINT_OK: return "success";
        case GINT_EINVAL: return "invalid argument";
        case GINT_EPATTERN: return "block pattern misses an overlapping pair or is not transpose-closed";
        case GINT_ENOMEM: return "out of memory";
        case GINT_EHIP: return "HIP runtime error";
        case GINT_EUNSUPPORTED: return "unsupported (l > 2, > 16 orbitals per atom, or precision)";
        default: return "unknown error";
    }
}

int gint_last_hip_error(void) { return g_last_hip; }

}  // extern "C"

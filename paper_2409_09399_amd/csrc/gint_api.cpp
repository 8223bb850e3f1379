// C ABI of the grid-integration library: plan lifetime, validation and
// launch sequencing.  All device work is enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "gint.h"
#include "gint_internal.h"
#include "gint_plan.hpp"
#include "gint_plan_impl.h"

#include "gint_launch.h"

namespace {
thread_local int g_last_hip = 0;
}  // namespace

void gint_record_hip_error(int e) { g_last_hip = e; }

namespace {

int hip_fail(hipError_t e) {
    g_last_hip = (int)e;
    return GINT_EHIP;
}

// The plan's device must be current (its descriptors live there).  Checked
// before anything is enqueued.
int check_device(const gint_plan *p);

template <class T, class A>
int upload(DevBuf &b, const std::vector<T, A> &v, size_t &total) {
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
    DevBuf *bufs[] = {&p->species, &p->atoms, &p->tab, &p->tab32, &p->pairs, &p->pairs8, &p->bigcells, &p->items_canon,
                      &p->items_ordered, &p->sys, &p->ws, &p->blocks, &p->bricks, &p->uatoms, &p->ptab, &p->d16};
    for (DevBuf *b : bufs)
        if (b->p) {
            (void)hipFree(b->p);
            b->p = nullptr;
        }
}

int check_device(const gint_plan *p) {
    int cur = 0;
    const hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e);
    return cur == p->device ? GINT_OK : GINT_EINVAL;
}

template <class T, class A>
size_t upload_bytes(const std::vector<T, A> &v) {
    return v.empty() ? sizeof(T) : v.size() * sizeof(T);
}

}  // namespace

// The orbital scale of the 16-bit operands (a power of two with
// phi_max * phi_scale in [2^12, 2^13)) and the plan-wide channel layout.
void gint_plan_scales(const HostPlan &hp, GDev &d) {
    int e = 0;
    if (hp.phi_max > 0.0 && std::isfinite(hp.phi_max)) (void)std::frexp(hp.phi_max, &e);
    int k = hp.phi_max > 0.0 ? 13 - e : 0;
    k = k < -60 ? -60 : (k > 60 ? 60 : k);
    d.phi_scale = std::ldexp(1.0, k);
    d.shape_all = hp.species.empty() ? GINT_SHAPE_ANY : hp.species[0].shape;
    for (const GSpecies &g : hp.species)
        if (g.shape != d.shape_all) d.shape_all = GINT_SHAPE_ANY;
}

extern "C" {

int gint_plan_create(gint_plan **out, const gint_system *sys, int n_sys, const gint_options *opt, void *stream) {
    (void)stream;
    if (!out || !sys || n_sys < 1) return GINT_EINVAL;
    const int prec = opt ? opt->precision : GINT_FP64;
    if (prec != GINT_FP64 && prec != GINT_MIXED_FP16X3 && prec != GINT_MIXED_BF16X3) return GINT_EUNSUPPORTED;
    const int decomp = opt ? opt->decomposition : GINT_DECOMP_DEFAULT;
    if (decomp < GINT_DECOMP_DEFAULT || decomp > GINT_DECOMP_BIGCELL_RHO_FORCE) return GINT_EINVAL;
    if ((decomp == GINT_DECOMP_BIGCELL || decomp == GINT_DECOMP_BIGCELL_RHO_FORCE) && prec == GINT_FP64)
        return GINT_EUNSUPPORTED;
    const bool bc = prec != GINT_FP64 && decomp != GINT_DECOMP_CLUSTER_PAIRS;
    // the default keeps Vlocal on cluster pairs: on the bilayers its brick
    // form is slower (it stages each chunk pair's images once per bigcell)
    const bool bc_vlocal = bc && decomp == GINT_DECOMP_BIGCELL;
    const auto t0 = std::chrono::steady_clock::now();
    HostPlan hp;
    int rc;
    try {
        rc = gint_build_host_plan(sys, n_sys, opt, bc, hp);
    } catch (const std::bad_alloc &) {
        return GINT_ENOMEM;
    } catch (...) {
        return GINT_EINVAL;
    }
    if (rc != GINT_OK) return rc;
    if (hp.items_canon.size() > 0x7fffffffu || hp.items_ordered.size() > 0x7fffffffu) return GINT_ENOMEM;
    // workspace: [0, 4) work counters (eight ints: one queue per XCD for the
    // brick kernels, the first for the others), [4] max |V|, [5] max |D|,
    // then ZE, then partial sums
    std::vector<double> wsinit(6 + (size_t)n_sys * (10 + kParts), 0.0);
    const size_t d16_bytes = bc ? hp.blocks.size() * (size_t)1024 : 0;
    if (bc && hp.blocks.size() > 0x7fffffffu) return GINT_ENOMEM;
    if (opt && opt->device_mib_cap > 0) {
        size_t need = upload_bytes(hp.species) + upload_bytes(hp.atoms) + upload_bytes(hp.tab) +
                      upload_bytes(hp.tab32) + upload_bytes(hp.pairs) + upload_bytes(hp.pairs8) + upload_bytes(hp.bigcells) +
                      upload_bytes(hp.items_canon) + upload_bytes(hp.items_ordered) + upload_bytes(hp.sys) +
                      upload_bytes(wsinit);
        if (bc)
            need += upload_bytes(hp.bricks) + upload_bytes(hp.uatoms) + upload_bytes(hp.ptab) +
                    upload_bytes(hp.blocks) + d16_bytes;
        if (need > ((size_t)opt->device_mib_cap << 20)) return GINT_ENOMEM;
    }

    gint_plan *p = new (std::nothrow) gint_plan();
    if (!p) return GINT_ENOMEM;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e);
    }
    size_t total = 0;
    if ((rc = upload(p->species, hp.species, total)) || (rc = upload(p->atoms, hp.atoms, total)) ||
        (rc = upload(p->tab, hp.tab, total)) || (rc = upload(p->tab32, hp.tab32, total)) ||
        (rc = upload(p->pairs, hp.pairs, total)) || (rc = upload(p->pairs8, hp.pairs8, total)) ||
        (rc = upload(p->bigcells, hp.bigcells, total)) || (rc = upload(p->items_canon, hp.items_canon, total)) ||
        (rc = upload(p->items_ordered, hp.items_ordered, total)) || (rc = upload(p->sys, hp.sys, total)) ||
        (rc = upload(p->ws, wsinit, total))) {
        release(p);
        delete p;
        return rc;
    }
    if (bc) {
        if ((rc = upload(p->bricks, hp.bricks, total)) || (rc = upload(p->uatoms, hp.uatoms, total)) ||
            (rc = upload(p->ptab, hp.ptab, total)) || (rc = upload(p->blocks, hp.blocks, total))) {
            release(p);
            delete p;
            return rc;
        }
        p->d16.bytes = d16_bytes > 0 ? d16_bytes : 1024;
        e = hipMalloc(&p->d16.p, p->d16.bytes);
        if (e != hipSuccess) {
            g_last_hip = (int)e;
            p->d16.p = nullptr;
            release(p);
            delete p;
            return GINT_ENOMEM;
        }
        total += p->d16.bytes;
    }
    p->bc = bc;
    p->bc_vlocal = bc_vlocal;
    p->n_sys = n_sys;
    p->sys_host = hp.sys;
    p->atom_norb.resize(hp.atoms.size());
    for (size_t a = 0; a < hp.atoms.size(); ++a) p->atom_norb[a] = hp.atoms[a].norb;
    p->blocks_host = std::move(hp.blocks);
    // resident-block counts of the persistent kernels, queried once here so
    // that no launch (eager or captured) needs a device query
    gint_prime_grids_fp64();   // k_work serves every precision form
    if (prec != GINT_FP64) gint_prime_grids_mx(prec);
    if (bc) gint_prime_grids_bc(prec);
    p->counter = (int *)p->ws.p;
    p->ZE = (double *)p->ws.p + 6;
    p->part = p->ZE + 10 * n_sys;

    GDev d{};
    d.species = (const GSpecies *)p->species.p;
    d.atoms = (const GAtom *)p->atoms.p;
    d.tab = (const double *)p->tab.p;
    d.tab32 = (const float *)p->tab32.p;
    d.pairs = hp.pairs8.empty() ? (const GPair *)p->pairs.p : nullptr;
    d.pairs8 = hp.pairs8.empty() ? nullptr : (const GPair8 *)p->pairs8.p;
    d.bigcells = (const GBig *)p->bigcells.p;
    d.sys = (const GSys *)p->sys.p;
    d.counter = p->counter;
    d.nsys = n_sys;
    d.natom = hp.natom;
    for (int i = 0; i < 3; ++i) {
        d.N[i] = hp.N[i];
        for (int k = 0; k < 3; ++k) d.e[i][k] = hp.e[i][k];
    }
    d.w = hp.w;
    gint_plan_scales(hp, d);
    d.vmax = (const double *)p->ws.p + 4;
    d.dmax = (const double *)p->ws.p + 5;
    if (bc) {
        d.bricks = (const GBrick *)p->bricks.p;
        d.uatoms = (const GUAtom *)p->uatoms.p;
        d.ptab = (const int *)p->ptab.p;
        d.d16 = (const unsigned short *)p->d16.p;
        d.nbricks = (int)hp.bricks.size();
        d.nblocks = (int)p->blocks_host.size();   // (hp.blocks has been moved into the plan)
    }
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
    s.precision = prec;
    s.n_sys = n_sys;
    s.decomposition = !bc ? GINT_DECOMP_CLUSTER_PAIRS : (bc_vlocal ? GINT_DECOMP_BIGCELL : GINT_DECOMP_BIGCELL_RHO_FORCE);
    s.nbricks = (int64_t)hp.bricks.size();
    s.brick_images = (int64_t)hp.uatoms.size();
    for (int k = 0; k < 3; ++k) s.brick[k] = hp.brick[k];
    p->precision = prec;
    s.build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = p;
    return GINT_OK;
}

int gint_vlocal(gint_plan *p, const double *v_loc, double *h_vals, void *stream) {
    if (!p || !v_loc || !h_vals) return GINT_EINVAL;
    if (const int rc = check_device(p)) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = gint_launch_fill(h_vals, p->sizes.nnz, 0.0, s);
    if (e != hipSuccess) return hip_fail(e);
    if (p->precision == GINT_FP64) {
        e = gint_launch_vlocal(p->canon, v_loc, h_vals, s);
    } else if (p->bc_vlocal) {
        e = gint_launch_fill(const_cast<double *>(p->canon.vmax), 1, 0.0, s);
        if (e == hipSuccess) e = gint_launch_absmax(v_loc, p->sizes.ngrid, const_cast<double *>(p->canon.vmax), s);
        if (e == hipSuccess)
            e = gint_launch_vlocal_bc(p->canon, p->precision, (const GBlk *)p->blocks.p, v_loc, h_vals, s);
    } else {
        e = gint_launch_vlocal_mx(p->canon, p->precision, v_loc, p->sizes.ngrid, h_vals, s);
    }
    if (e != hipSuccess) return hip_fail(e);
    return GINT_OK;
}

int gint_rho(gint_plan *p, const double *d_vals, double *rho, double *n_elec, void *stream) {
    if (!p || !d_vals || !rho) return GINT_EINVAL;
    if (const int rc = check_device(p)) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = gint_launch_fill(rho, p->sizes.ngrid, 0.0, s);
    if (e != hipSuccess) return hip_fail(e);
    e = p->precision == GINT_FP64
            ? gint_launch_rho(p->canon, d_vals, rho, s)
            : (p->bc ? gint_launch_rho_bc(p->canon, p->precision, (const GBlk *)p->blocks.p, p->sizes.nnz, d_vals,
                                          rho, s)
                     : gint_launch_rho_mx(p->canon, p->precision, d_vals, rho, s));
    if (e != hipSuccess) return hip_fail(e);
    if (n_elec) {
        e = gint_launch_seg_sum(p->canon, rho, nullptr, p->part, kParts, n_elec, s);
        if (e != hipSuccess) return hip_fail(e);
    }
    return GINT_OK;
}

namespace {

// force/stress (and rho when given) in one pass over the ordered pairs
int force_pass(gint_plan *p, const double *v_loc, const double *d_vals, double *rho, double *n_elec,
               double *force, double *stress, double *energy, hipStream_t s) {
    if (const int rc = check_device(p)) return rc;
    hipError_t e = gint_launch_fill(force, 3LL * p->sizes.natom, 0.0, s);
    if (e == hipSuccess) e = gint_launch_fill(p->ZE, 10LL * p->n_sys, 0.0, s);
    if (e == hipSuccess && rho) e = gint_launch_fill(rho, p->sizes.ngrid, 0.0, s);
    if (e == hipSuccess) {
        if (p->precision == GINT_FP64)
            e = gint_launch_force(p->ordered, v_loc, d_vals, force, p->ZE, rho, s);
        else if (p->bc)
            e = gint_launch_force_bc(p->ordered, p->precision, (const GBlk *)p->blocks.p, p->sizes.nnz, v_loc,
                                     d_vals, force, p->ZE, rho, s);
        else
            e = gint_launch_force_mx(p->ordered, p->precision, v_loc, d_vals, force, p->ZE, rho, s);
    }
    if (e == hipSuccess) e = gint_launch_finish_stress(p->ordered, p->ZE, stress, energy, s);
    if (e == hipSuccess && rho && n_elec) e = gint_launch_seg_sum(p->canon, rho, nullptr, p->part, kParts, n_elec, s);
    if (e != hipSuccess) return hip_fail(e);
    return GINT_OK;
}

}  // namespace

int gint_force_stress(gint_plan *p, const double *v_loc, const double *d_vals, double *force, double *stress,
                      double *energy, void *stream) {
    if (!p || !v_loc || !d_vals || !force || !stress) return GINT_EINVAL;
    return force_pass(p, v_loc, d_vals, nullptr, nullptr, force, stress, energy, (hipStream_t)stream);
}

int gint_rho_force_stress(gint_plan *p, const double *v_loc, const double *d_vals, double *rho, double *n_elec,
                          double *force, double *stress, double *energy, void *stream) {
    if (!p || !v_loc || !d_vals || !rho || !force || !stress) return GINT_EINVAL;
    return force_pass(p, v_loc, d_vals, rho, n_elec, force, stress, energy, (hipStream_t)stream);
}

// Largest |D_IJR[mu,nu] - D_JI(-R)[nu,mu]| per system.
int gint_check_symmetry(gint_plan *p, const double *d_vals, double *max_asym, void *stream) {
    if (!p || !d_vals || !max_asym) return GINT_EINVAL;
    if (const int rc = check_device(p)) return rc;
    hipStream_t s = (hipStream_t)stream;
    if (!p->blocks.p && !p->blocks_host.empty()) {
        size_t total = 0;
        const int rc = upload(p->blocks, p->blocks_host, total);
        if (rc != GINT_OK) {
            if (p->blocks.p) (void)hipFree(p->blocks.p);
            p->blocks.p = nullptr;
            return rc;
        }
    }
    hipError_t e = gint_launch_fill(max_asym, p->n_sys, 0.0, s);
    if (e == hipSuccess)
        e = gint_launch_dsym_check((const GBlk *)p->blocks.p, (long long)p->blocks_host.size(), d_vals, max_asym, s);
    if (e != hipSuccess) return hip_fail(e);
    return GINT_OK;
}

// E = w sum_g V_g rho_g per system (two-pass device reduction).
int gint_energy(gint_plan *p, const double *v_loc, const double *rho, double *energy, void *stream) {
    if (!p || !v_loc || !rho || !energy) return GINT_EINVAL;
    if (const int rc = check_device(p)) return rc;
    const hipError_t e = gint_launch_seg_sum(p->canon, v_loc, rho, p->part, kParts, energy, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);
    return GINT_OK;
}

// E as gint_energy, with the partial sums in the library's static device
// scratch instead of the plan's workspace: no allocation, no plan state
// written.
int gint_energy_noalloc(gint_plan *p, const double *v_loc, const double *rho, double *energy, void *stream) {
    if (!p || !v_loc || !rho || !energy) return GINT_EINVAL;
    if (const int rc = check_device(p)) return rc;
    const size_t need = (size_t)p->n_sys * kParts * sizeof(double);
    void *scr = nullptr;
    size_t cap = 0;
    hipError_t e = gint_static_scratch(&scr, &cap);
    if (e != hipSuccess) return hip_fail(e);
    if (need > cap) return GINT_ENOMEM;
    e = gint_launch_seg_sum(p->canon, v_loc, rho, (double *)scr, kParts, energy, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);
    return GINT_OK;
}

// W = sum_g n_orb(g)^2, the unit of work of the throughput metric.
int gint_work_units(gint_plan *p, double *w_out, void *stream) {
    if (!p || !w_out) return GINT_EINVAL;
    if (const int rc = check_device(p)) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = gint_launch_fill(w_out, p->n_sys, 0.0, s);
    if (e == hipSuccess) e = gint_launch_work(p->canon, w_out, s);
    if (e != hipSuccess) return hip_fail(e);
    return GINT_OK;
}

struct gint_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
};

int gint_graph_create(gint_graph **out, gint_plan *p, const double *v_loc, const double *d_vals, double *h_vals,
                      double *rho, double *n_elec, double *force, double *stress, double *energy) {
    if (!out || !p) return GINT_EINVAL;
    if ((h_vals || force) && !v_loc) return GINT_EINVAL;
    if ((rho || force) && !d_vals) return GINT_EINVAL;
    if (!!force != !!stress) return GINT_EINVAL;
    if (!rho && n_elec) return GINT_EINVAL;
    if (!h_vals && !rho && !force) return GINT_EINVAL;
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e);
    if (cur != p->device) return GINT_EINVAL;
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e);
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_fail(e);
    }
    int rc = GINT_OK;
    if (h_vals) rc = gint_vlocal(p, v_loc, h_vals, cs);
    if (rc == GINT_OK && rho) rc = gint_rho(p, d_vals, rho, n_elec, cs);
    if (rc == GINT_OK && force) rc = gint_force_stress(p, v_loc, d_vals, force, stress, energy, cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    if (rc != GINT_OK || e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc != GINT_OK ? rc : hip_fail(e);
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e);
    }
    gint_graph *g = new (std::nothrow) gint_graph();
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return GINT_ENOMEM;
    }
    g->graph = graph;
    g->exec = exec;
    g->device = cur;
    *out = g;
    return GINT_OK;
}

int gint_graph_launch(gint_graph *g, void *stream) {
    if (!g) return GINT_EINVAL;
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e);
    return GINT_OK;
}

void gint_graph_destroy(gint_graph *g) {
    if (!g) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(g->device);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    (void)hipSetDevice(cur);
    delete g;
}

int gint_plan_query(const gint_plan *p, gint_sizes *out) {
    if (!p || !out) return GINT_EINVAL;
    *out = p->sizes;
    return GINT_OK;
}

int gint_plan_query_system(const gint_plan *p, int i, gint_system_sizes *out) {
    if (!p || !out || i < 0 || i >= p->n_sys) return GINT_EINVAL;
    const GSys &S = p->sys_host[i];
    const long long nnz_end = i + 1 < p->n_sys ? p->sys_host[i + 1].nnz_off : p->sizes.nnz;
    out->g_off = S.g_off;
    out->ngrid = (int64_t)S.N[0] * S.N[1] * S.N[2];
    out->nnz_off = S.nnz_off;
    out->nnz = nnz_end - S.nnz_off;
    out->atom_off = S.atom_off;
    out->natom = S.natom;
    for (int k = 0; k < 3; ++k) out->grid[k] = S.N[k];
    out->volume = S.volume;
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

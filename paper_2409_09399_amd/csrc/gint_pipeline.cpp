// Streaming pipeline (include/gint_pipeline.h): the plans of a system's grid
// slabs are built on a host thread, copied from pinned staging buffers on a
// copy stream, and computed on the caller's stream, with two descriptor
// slots on the device so that slab k+1's copy overlaps slab k's kernels.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "gint.h"
#include "gint_internal.h"
#include "gint_launch.h"
#include "gint_pipeline.h"
#include "gint_plan.hpp"
#include "gint_plan_impl.h"

namespace {

using Clock = std::chrono::steady_clock;

double seconds_since(Clock::time_point t0) { return std::chrono::duration<double>(Clock::now() - t0).count(); }

// A private copy of one gint_system (the builder thread reads it after the
// caller's arrays may be gone).
struct SysCopy {
    gint_system sys{};
    std::vector<double> pos;
    std::vector<int> species;
    std::vector<gint_species> sps;
    std::vector<std::vector<int>> chan_l;
    std::vector<std::vector<double>> f, fp;
    std::vector<int> bi, bj, br;
    std::vector<int64_t> boff;
};

// Copies the arrays the plan builder reads; their contents are validated by
// the builder itself.  false when a needed array is missing.
bool copy_system(const gint_system &s, SysCopy &c) {
    if (s.natom < 1 || !s.pos || !s.species || s.nspecies < 1 || !s.species_list || s.nblk < 0) return false;
    if (s.nblk > 0 && (!s.blk_i || !s.blk_j || !s.blk_r || !s.blk_off)) return false;
    c.sys = s;
    c.pos.assign(s.pos, s.pos + 3 * (size_t)s.natom);
    c.species.assign(s.species, s.species + s.natom);
    c.sps.assign(s.species_list, s.species_list + s.nspecies);
    c.chan_l.resize(s.nspecies);
    c.f.resize(s.nspecies);
    c.fp.resize(s.nspecies);
    for (int k = 0; k < s.nspecies; ++k) {
        const gint_species &sp = s.species_list[k];
        if (sp.nchan < 1 || sp.nknots < 1 || !sp.chan_l || !sp.f || !sp.fp) return false;
        const size_t n = (size_t)sp.nchan * sp.nknots;
        c.chan_l[k].assign(sp.chan_l, sp.chan_l + sp.nchan);
        c.f[k].assign(sp.f, sp.f + n);
        c.fp[k].assign(sp.fp, sp.fp + n);
        c.sps[k].chan_l = c.chan_l[k].data();
        c.sps[k].f = c.f[k].data();
        c.sps[k].fp = c.fp[k].data();
    }
    c.bi.assign(s.blk_i, s.blk_i + s.nblk);
    c.bj.assign(s.blk_j, s.blk_j + s.nblk);
    c.br.assign(s.blk_r, s.blk_r + 3 * (size_t)s.nblk);
    c.boff.assign(s.blk_off, s.blk_off + s.nblk);
    c.sys.pos = c.pos.data();
    c.sys.species = c.species.data();
    c.sys.species_list = c.sps.data();
    c.sys.blk_i = c.bi.data();
    c.sys.blk_j = c.bj.data();
    c.sys.blk_r = c.br.data();
    c.sys.blk_off = c.boff.data();
    return true;
}

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Offsets of a slab's descriptor arrays in its packed buffer.
struct Packed {
    size_t pairs = 0, pairs8 = 0, bigcells = 0, items_canon = 0, items_ordered = 0, bricks = 0, uatoms = 0, ptab = 0;
    size_t bytes = 0;
};

template <class T, class A>
size_t place(size_t &at, const std::vector<T, A> &v) {
    const size_t o = at;
    at = align_up(at + v.size() * sizeof(T));
    return o;
}

Packed layout(const HostPlan &hp) {
    Packed L;
    size_t at = 0;
    L.pairs = place(at, hp.pairs);
    L.pairs8 = place(at, hp.pairs8);
    L.bigcells = place(at, hp.bigcells);
    L.items_canon = place(at, hp.items_canon);
    L.items_ordered = place(at, hp.items_ordered);
    L.bricks = place(at, hp.bricks);
    L.uatoms = place(at, hp.uatoms);
    L.ptab = place(at, hp.ptab);
    L.bytes = at > 0 ? at : kAlign;
    return L;
}

template <class T, class A>
void put(char *dst, size_t off, const std::vector<T, A> &v) {
    if (!v.empty()) std::memcpy(dst + off, v.data(), v.size() * sizeof(T));
}

void pack(const HostPlan &hp, const Packed &L, char *dst) {
    put(dst, L.pairs, hp.pairs);
    put(dst, L.pairs8, hp.pairs8);
    put(dst, L.bigcells, hp.bigcells);
    put(dst, L.items_canon, hp.items_canon);
    put(dst, L.items_ordered, hp.items_ordered);
    put(dst, L.bricks, hp.bricks);
    put(dst, L.uatoms, hp.uatoms);
    put(dst, L.ptab, hp.ptab);
}

// One of the two device descriptor buffers with its pinned staging copy.
// copied: the last copy out of `pin` has finished; done: the last kernels
// reading `dev` have finished.
struct Slot {
    char *dev = nullptr;
    size_t cap = 0;
    char *pin = nullptr;
    size_t pincap = 0;
    hipEvent_t copied = nullptr, done = nullptr;
    bool used = false;
};

int hip_rc(hipError_t e) {
    if (e == hipSuccess) return GINT_OK;
    gint_record_hip_error((int)e);
    return e == hipErrorOutOfMemory ? GINT_ENOMEM : GINT_EHIP;
}

}  // namespace

struct gint_pipeline {
    int device = 0;
    int prec = GINT_FP64;
    int n_slabs = 1;
    bool bc = false, bc_vlocal = false;
    gint_options opt{};
    SysCopy sc;
    GintSlabShared *shared_idx = nullptr;   // pattern indexes, built by slab 0's build
    // slab plans on the host, built in order by the builder thread
    std::vector<std::unique_ptr<HostPlan>> host;
    std::mutex mu;
    std::condition_variable cv;
    int built = 0;
    int build_rc = GINT_OK;
    bool stop = false;
    std::thread builder;
    // device data shared by every slab: tables, atoms, systems, pattern
    // blocks, D operand copy, workspace
    char *shared = nullptr;
    unsigned short *d16 = nullptr;
    double *ws = nullptr;
    GDev base{};
    const GBlk *blocks = nullptr;
    long long nnz = 0, ngrid = 0;
    int natom = 0;
    double *ZE = nullptr, *part = nullptr;
    Slot slot[2];
    hipStream_t copy = nullptr;
    gint_pipeline_stats st{};
    std::vector<size_t> slab_bytes;
};

namespace {

void build_all(gint_pipeline *p) {
    for (int k = 0; k < p->n_slabs; ++k) {
        {
            std::lock_guard<std::mutex> lk(p->mu);
            if (p->stop) return;
        }
        std::unique_ptr<HostPlan> hp(new (std::nothrow) HostPlan());
        int rc = hp ? GINT_OK : GINT_ENOMEM;
        const auto t0 = Clock::now();
        if (rc == GINT_OK) {
            GintSlab slab;
            slab.count = p->n_slabs;
            slab.index = k;
            slab.shared = p->shared_idx;
            try {
                rc = gint_build_host_plan(&p->sc.sys, 1, &p->opt, p->bc, *hp, &slab);
            } catch (const std::bad_alloc &) {
                rc = GINT_ENOMEM;
            } catch (...) {
                rc = GINT_EINVAL;
            }
        }
        const double dt = seconds_since(t0);
        std::lock_guard<std::mutex> lk(p->mu);
        p->st.build_seconds += dt;
        if (rc != GINT_OK) {
            p->build_rc = rc;
            p->cv.notify_all();
            return;
        }
        p->host[k] = std::move(hp);
        p->built = k + 1;
        p->st.slabs_built = k + 1;
        p->cv.notify_all();
    }
}

const HostPlan *wait_slab(gint_pipeline *p, int k, int &rc) {
    const auto t0 = Clock::now();
    std::unique_lock<std::mutex> lk(p->mu);
    p->cv.wait(lk, [&] { return p->built > k || p->build_rc != GINT_OK; });
    p->st.wait_seconds += seconds_since(t0);
    if (p->built <= k) {
        rc = p->build_rc;
        return nullptr;
    }
    rc = GINT_OK;
    return p->host[k].get();
}

// Tables, atoms, system record and pattern blocks of slab 0's plan (the same
// for every slab), the D operand copy and the workspace, in one allocation.
int upload_shared(gint_pipeline *p, const HostPlan &hp) {
    size_t at = 0;
    const size_t o_species = place(at, hp.species), o_atoms = place(at, hp.atoms), o_tab = place(at, hp.tab),
                 o_tab32 = place(at, hp.tab32), o_sys = place(at, hp.sys), o_blocks = place(at, hp.blocks);
    const size_t o_d16 = at;
    at = align_up(at + (p->bc ? hp.blocks.size() * (size_t)1024 : 0));
    const size_t nws = 6 + 10 + kParts;
    const size_t o_ws = at;
    at = align_up(at + nws * sizeof(double));
    // the host image covers the tables, atoms, systems and blocks; the D copy
    // is written on the device each step before it is read, and only the
    // workspace needs zeros
    std::vector<char> img(o_d16, 0);
    put(img.data(), o_species, hp.species);
    put(img.data(), o_atoms, hp.atoms);
    put(img.data(), o_tab, hp.tab);
    put(img.data(), o_tab32, hp.tab32);
    put(img.data(), o_sys, hp.sys);
    put(img.data(), o_blocks, hp.blocks);
    const std::vector<double> ws0(nws, 0.0);
    hipError_t e = hipMalloc(&p->shared, at);
    if (e != hipSuccess) {
        p->shared = nullptr;
        return hip_rc(e);
    }
    e = hipMemcpy(p->shared, img.data(), o_d16, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(p->shared + o_ws, ws0.data(), nws * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_rc(e);
    p->st.shared_device_bytes = (int64_t)at;
    char *b = p->shared;
    p->ws = (double *)(b + o_ws);
    p->ZE = p->ws + 6;
    p->part = p->ZE + 10;
    p->d16 = p->bc ? (unsigned short *)(b + o_d16) : nullptr;
    p->blocks = (const GBlk *)(b + o_blocks);
    p->nnz = hp.nnz;
    p->ngrid = hp.ngrid;
    p->natom = hp.natom;
    GDev &d = p->base;
    d = GDev{};
    d.species = (const GSpecies *)(b + o_species);
    d.atoms = (const GAtom *)(b + o_atoms);
    d.tab = (const double *)(b + o_tab);
    d.tab32 = (const float *)(b + o_tab32);
    d.sys = (const GSys *)(b + o_sys);
    d.counter = (int *)p->ws;
    d.nsys = 1;
    d.natom = hp.natom;
    for (int i = 0; i < 3; ++i) {
        d.N[i] = hp.N[i];
        for (int k = 0; k < 3; ++k) d.e[i][k] = hp.e[i][k];
    }
    d.w = hp.w;
    gint_plan_scales(hp, d);
    d.vmax = p->ws + 4;
    d.dmax = p->ws + 5;
    d.d16 = p->d16;
    d.nblocks = (int)hp.blocks.size();
    return GINT_OK;
}

// The slab's two kernel views (canonical and ordered items) over its
// descriptors at `dev`.
void slab_views(const gint_pipeline *p, const HostPlan &hp, const Packed &L, char *dev, GDev &canon, GDev &ordered) {
    GDev d = p->base;
    d.pairs = hp.pairs8.empty() ? (const GPair *)(dev + L.pairs) : nullptr;
    d.pairs8 = hp.pairs8.empty() ? nullptr : (const GPair8 *)(dev + L.pairs8);
    d.bigcells = (const GBig *)(dev + L.bigcells);
    if (p->bc) {
        d.bricks = (const GBrick *)(dev + L.bricks);
        d.uatoms = (const GUAtom *)(dev + L.uatoms);
        d.ptab = (const int *)(dev + L.ptab);
        d.nbricks = (int)hp.bricks.size();
    }
    canon = d;
    canon.items = (const GItem *)(dev + L.items_canon);
    canon.nitems = (int)hp.items_canon.size();
    ordered = d;
    ordered.items = (const GItem *)(dev + L.items_ordered);
    ordered.nitems = (int)hp.items_ordered.size();
}

// What every slab of a step shares, once per step: max |V| (the mixed
// Vlocal's operand scale) and, with bricks, max |D| and the 16-bit D copy.
hipError_t prepare_step(gint_pipeline *p, const double *v, const double *d, hipStream_t s) {
    if (p->prec == GINT_FP64) return hipSuccess;
    hipError_t e = gint_launch_vmax(p->base, v, p->ngrid, s);
    if (e == hipSuccess && p->bc) e = gint_launch_d16(p->base, p->prec, p->blocks, p->nnz, d, s);
    return e;
}

// The slab's share of Vlocal, rho and force/stress (accumulated into the
// outputs the step has cleared; prepare_step has run on the stream).
hipError_t run_slab(gint_pipeline *p, const GDev &canon, const GDev &ordered, const double *v, const double *d,
                    double *h, double *rho, double *force, hipStream_t s) {
    hipError_t e;
    if (p->prec == GINT_FP64) {
        e = gint_launch_vlocal(canon, v, h, s);
        if (e == hipSuccess) e = gint_launch_rho(canon, d, rho, s);
        if (e == hipSuccess) e = gint_launch_force(ordered, v, d, force, p->ZE, nullptr, s);
        return e;
    }
    e = p->bc_vlocal ? gint_launch_vlocal_bc(canon, p->prec, p->blocks, v, h, s)
                     : gint_launch_vlocal_mx_prepared(canon, p->prec, v, h, s);
    if (e != hipSuccess) return e;
    e = p->bc ? gint_launch_rho_bc_prepared(canon, p->prec, rho, s) : gint_launch_rho_mx(canon, p->prec, d, rho, s);
    if (e != hipSuccess) return e;
    return p->bc ? gint_launch_force_bc_prepared(ordered, p->prec, v, force, p->ZE, nullptr, s)
                 : gint_launch_force_mx(ordered, p->prec, v, d, force, p->ZE, nullptr, s);
}

void release(gint_pipeline *p) {
    {
        std::lock_guard<std::mutex> lk(p->mu);
        p->stop = true;
    }
    if (p->builder.joinable()) p->builder.join();
    for (Slot &sl : p->slot) {
        if (sl.used && sl.done) (void)hipEventSynchronize(sl.done);
        if (sl.used && sl.copied) (void)hipEventSynchronize(sl.copied);
    }
    for (Slot &sl : p->slot) {
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.pin) (void)hipHostFree(sl.pin);
        if (sl.copied) (void)hipEventDestroy(sl.copied);
        if (sl.done) (void)hipEventDestroy(sl.done);
    }
    if (p->copy) (void)hipStreamDestroy(p->copy);
    if (p->shared) (void)hipFree(p->shared);
    gint_slab_shared_free(p->shared_idx);
    p->shared_idx = nullptr;
}

}  // namespace

extern "C" {

int gint_pipeline_create(gint_pipeline **out, const gint_system *sys, const gint_options *opt, int n_slabs) {
    if (!out || !sys || n_slabs < 1 || n_slabs > 4096) return GINT_EINVAL;
    *out = nullptr;
    const int prec = opt ? opt->precision : GINT_FP64;
    if (prec != GINT_FP64 && prec != GINT_MIXED_FP16X3 && prec != GINT_MIXED_BF16X3) return GINT_EUNSUPPORTED;
    const int decomp = opt ? opt->decomposition : GINT_DECOMP_DEFAULT;
    if (decomp < GINT_DECOMP_DEFAULT || decomp > GINT_DECOMP_BIGCELL_RHO_FORCE) return GINT_EINVAL;
    if ((decomp == GINT_DECOMP_BIGCELL || decomp == GINT_DECOMP_BIGCELL_RHO_FORCE) && prec == GINT_FP64)
        return GINT_EUNSUPPORTED;
    gint_pipeline *p = new (std::nothrow) gint_pipeline();
    if (!p) return GINT_ENOMEM;
    p->prec = prec;
    p->n_slabs = n_slabs;
    p->bc = prec != GINT_FP64 && decomp != GINT_DECOMP_CLUSTER_PAIRS;
    p->bc_vlocal = p->bc && decomp == GINT_DECOMP_BIGCELL;
    if (opt) p->opt = *opt;
    p->opt.precision = prec;
    p->st.n_slabs = n_slabs;
    try {
        if (!copy_system(*sys, p->sc)) {
            delete p;
            return GINT_EINVAL;
        }
        p->host.resize(n_slabs);
        p->slab_bytes.assign(n_slabs, 0);
        p->shared_idx = gint_slab_shared_new();
    } catch (const std::bad_alloc &) {
        delete p;
        return GINT_ENOMEM;
    }
    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->copy, hipStreamNonBlocking);
    for (Slot &sl : p->slot) {
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.copied, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        release(p);
        delete p;
        return hip_rc(e);
    }
    // resident-block counts of the persistent kernels, queried here so that
    // no step needs a device query
    gint_prime_grids_fp64();
    if (prec != GINT_FP64) gint_prime_grids_mx(prec);
    if (p->bc) gint_prime_grids_bc(prec);
    try {
        p->builder = std::thread(build_all, p);
    } catch (...) {
        release(p);
        delete p;
        return GINT_ENOMEM;
    }
    *out = p;
    return GINT_OK;
}

namespace {

int step_impl(gint_pipeline *p, const double *v_loc, const double *d_vals, double *h_vals, double *rho,
              double *n_elec, double *force, double *stress, double *energy, void *stream) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_rc(e);
    if (cur != p->device) return GINT_EINVAL;
    const auto t_call = Clock::now();
    hipStream_t s = (hipStream_t)stream;
    int rc = GINT_OK;
    const HostPlan *h0 = wait_slab(p, 0, rc);
    if (!h0) return rc;
    if (!p->shared && (rc = upload_shared(p, *h0)) != GINT_OK) return rc;
    e = gint_launch_fill(h_vals, p->nnz, 0.0, s);
    if (e == hipSuccess) e = gint_launch_fill(rho, p->ngrid, 0.0, s);
    if (e == hipSuccess) e = gint_launch_fill(force, 3LL * p->natom, 0.0, s);
    if (e == hipSuccess) e = gint_launch_fill(p->ZE, 10, 0.0, s);
    if (e == hipSuccess) e = prepare_step(p, v_loc, d_vals, s);
    if (e != hipSuccess) return hip_rc(e);
    long long copied = 0;
    for (int k = 0; k < p->n_slabs; ++k) {
        const HostPlan *hp = wait_slab(p, k, rc);
        if (!hp) return rc;
        Slot &sl = p->slot[k & 1];
        const Packed L = layout(*hp);
        p->slab_bytes[k] = L.bytes;
        // the staging buffer is free once its previous copy has finished
        if (sl.used && (e = hipEventSynchronize(sl.copied)) != hipSuccess) return hip_rc(e);
        if (sl.pincap < L.bytes) {
            if (sl.pin) (void)hipHostFree(sl.pin);
            sl.pin = nullptr;
            sl.pincap = 0;
            if ((e = hipHostMalloc((void **)&sl.pin, L.bytes, hipHostMallocDefault)) != hipSuccess) {
                sl.pin = nullptr;
                return hip_rc(e);
            }
            sl.pincap = L.bytes;
        }
        pack(*hp, L, sl.pin);
        if (sl.cap < L.bytes) {
            // growth (first steps only): the slot's kernels must be done with it
            if (sl.used && (e = hipEventSynchronize(sl.done)) != hipSuccess) return hip_rc(e);
            if (sl.dev) (void)hipFree(sl.dev);
            sl.dev = nullptr;
            sl.cap = 0;
            if ((e = hipMalloc((void **)&sl.dev, L.bytes)) != hipSuccess) {
                sl.dev = nullptr;
                return hip_rc(e);
            }
            sl.cap = L.bytes;
            p->st.slot_device_bytes = (int64_t)(p->slot[0].cap + p->slot[1].cap);
        }
        if (sl.used && (e = hipStreamWaitEvent(p->copy, sl.done, 0)) != hipSuccess) return hip_rc(e);
        if ((e = hipMemcpyAsync(sl.dev, sl.pin, L.bytes, hipMemcpyHostToDevice, p->copy)) != hipSuccess ||
            (e = hipEventRecord(sl.copied, p->copy)) != hipSuccess || (e = hipStreamWaitEvent(s, sl.copied, 0)) != hipSuccess)
            return hip_rc(e);
        GDev canon, ordered;
        slab_views(p, *hp, L, sl.dev, canon, ordered);
        if ((e = run_slab(p, canon, ordered, v_loc, d_vals, h_vals, rho, force, s)) != hipSuccess) return hip_rc(e);
        if ((e = hipEventRecord(sl.done, s)) != hipSuccess) return hip_rc(e);
        sl.used = true;
        copied += (long long)L.bytes;
    }
    e = gint_launch_finish_stress(p->base, p->ZE, stress, energy, s);
    if (e == hipSuccess && n_elec) e = gint_launch_seg_sum(p->base, rho, nullptr, p->part, kParts, n_elec, s);
    if (e != hipSuccess) return hip_rc(e);
    std::lock_guard<std::mutex> lk(p->mu);
    p->st.steps += 1;
    p->st.copied_bytes = copied;
    size_t all = 0, largest = 0;
    for (size_t b : p->slab_bytes) {
        all += b;
        largest = b > largest ? b : largest;
    }
    p->st.all_slabs_bytes = (int64_t)all;
    p->st.largest_slab_bytes = (int64_t)largest;
    if (p->st.steps == 1) p->st.first_step_seconds = seconds_since(t_call);
    return GINT_OK;
}

}  // namespace

int gint_pipeline_step(gint_pipeline *p, const double *v_loc, const double *d_vals, double *h_vals, double *rho,
                       double *n_elec, double *force, double *stress, double *energy, void *stream) {
    if (!p || !v_loc || !d_vals || !h_vals || !rho || !force || !stress) return GINT_EINVAL;
    try {
        return step_impl(p, v_loc, d_vals, h_vals, rho, n_elec, force, stress, energy, stream);
    } catch (const std::bad_alloc &) {
        return GINT_ENOMEM;
    } catch (...) {
        return GINT_EINVAL;
    }
}

int gint_pipeline_query(const gint_pipeline *p, gint_pipeline_stats *out) {
    if (!p || !out) return GINT_EINVAL;
    std::lock_guard<std::mutex> lk(const_cast<gint_pipeline *>(p)->mu);
    *out = p->st;
    return GINT_OK;
}

void gint_pipeline_destroy(gint_pipeline *p) {
    if (!p) return;
    release(p);
    delete p;
}

}  // extern "C"

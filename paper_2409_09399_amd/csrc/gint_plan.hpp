// Host-side plan builder: sub-task division and descriptor generation
// (paper: "Computational Collaboration Between Host and Device" — grid
// batches plus their neighbouring atoms, with the GEMM descriptors stored
// contiguously by integer index).
#pragma once
#include <memory>
#include <new>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "gint.h"
#include "gint_internal.h"

// An allocator whose resize leaves trivially constructible elements
// uninitialised: the plan's largest arrays are written in full by worker
// threads right after they are sized, so their pages are first touched (and
// zeroed by the OS) in parallel rather than by one thread.
template <class T>
struct NoInitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = NoInitAlloc<U>;
    };
    NoInitAlloc() = default;
    template <class U>
    NoInitAlloc(const NoInitAlloc<U> &) noexcept {}
    template <class U>
    void construct(U *p) noexcept(std::is_nothrow_default_constructible<U>::value) {
        ::new ((void *)p) U;
    }
    template <class U, class... A>
    void construct(U *p, A &&...a) {
        ::new ((void *)p) U(std::forward<A>(a)...);
    }
};
template <class T>
using BigVec = std::vector<T, NoInitAlloc<T>>;

struct HostPlan {
    std::vector<GSpecies> species;
    std::vector<GAtom> atoms;
    std::vector<double> tab;
    std::vector<float> tab32;
    std::vector<GPair> pairs;        // clusters of <= 4 atoms: [0, ncanon) canonical, then swapped copies
    std::vector<GPair8> pairs8;      // clusters of 5..8 atoms (canonical only; instead of pairs)
    BigVec<GBig> bigcells;
    std::vector<GItem> items_canon;  // canonical pairs, longest first
    std::vector<GItem> items_ordered;// canonical + swapped, longest first (only the canonical ones with pairs8)
    std::vector<GSys> sys;           // one per system
    std::vector<GBlk> blocks;        // pattern blocks with their transposes (symmetry check, D16 conversion)
    std::vector<GBrick> bricks;      // bigcell-stationary bricks (rho and force), empty unless built
    std::vector<GUAtom> uatoms;      // their atom-image unions
    BigVec<int> ptab;                // their pair tables (block indices, -1 = none)
    int brick[3] = {0, 0, 0};        // bigcells per brick along a1, a2, a3
    int ncanon = 0;
    int ncluster = 0;
    int natom = 0;
    int N[3] = {0, 0, 0};
    double cell[9] = {0};
    double e[3][3] = {{0}};
    double omega = 0.0;
    double w = 0.0;
    double phi_max = 0.0;            // bound on |phi| over every species (mixed-precision scaling)
    long long nnz = 0;
    long long ngrid = 0;
    int cluster_atoms = GINT_CL;
    std::string error;
};

// One slab of a grid cut along a1: the bigcells and bricks whose origin has
// wrapped a1 index n0 with floor(n0 * count / N1) == index.  The slabs of a
// count partition every pair's bigcells and every brick, so the per-slab
// plans together do the work of the whole plan.
struct GintSlabShared;   // the pattern indexes of a system, built by its first slab's build and reused
GintSlabShared *gint_slab_shared_new();
void gint_slab_shared_free(GintSlabShared *s);

struct GintSlab {
    int count = 1;
    int index = 0;
    // optional: with it, the builds of one system's slabs (in any order, one
    // at a time) validate and index the pattern once; the later builds leave
    // hp.blocks empty (the first one's plan carries them)
    GintSlabShared *shared = nullptr;
    bool has(int n0_wrapped, int N0) const {
        return count <= 1 || (int)((long long)n0_wrapped * count / N0) == index;
    }
};

// Builds the plan of n_sys systems (their work items merged into one queue).
// With bricks set, also the bigcell-stationary bricks of every system.  With
// a slab of count > 1 (one system only), only that slab's bigcells and
// bricks, and every work item is marked as sharing its blocks (the other
// slabs add to the same H blocks).
// Returns GINT_OK or a negative gint error code (hp.error holds a message).
int gint_build_host_plan(const gint_system *sys, int n_sys, const gint_options *opt, bool bricks, HostPlan &hp,
                         const GintSlab *slab = nullptr);

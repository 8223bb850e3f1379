// The plan object behind the C ABI's opaque gint_plan, shared by the
// source files that implement entry points on it.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "gint.h"
#include "gint_internal.h"

constexpr int kParts = 256;   // partial sums per system of the two-pass grid reductions

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct gint_plan {
    int device = 0;
    GDev canon{};      // canonical items (vlocal, rho, work)
    GDev ordered{};    // canonical + swapped items (force)
    DevBuf species, atoms, tab, tab32, pairs, pairs8, bigcells, items_canon, items_ordered, sys, ws;
    DevBuf bricks, uatoms, ptab, d16;   // bigcell-stationary path (rho and force)
    bool bc = false;                    // rho and force run over bricks
    bool bc_vlocal = false;             // and Vlocal too
    int precision = GINT_FP64;
    int n_sys = 1;
    int *counter = nullptr;    // work counter of the persistent launches
    double *ZE = nullptr;      // [n_sys][10]: Z (9) and E
    double *part = nullptr;    // [n_sys][kParts]
    std::vector<GSys> sys_host;
    std::vector<GBlk> blocks_host;   // pattern blocks (on the device from creation with bricks, else
                                     // uploaded by the first symmetry check)
    std::vector<int> atom_norb;      // orbitals of each atom (packed over systems)
    DevBuf blocks;
    gint_sizes sizes{};
};

// Records e as the value gint_last_hip_error() reports.
void gint_record_hip_error(int e);

struct HostPlan;
// The orbital scale of the mixed forms' 16-bit operands and the plan-wide
// channel layout, from a host plan, into d.
void gint_plan_scales(const HostPlan &hp, GDev &d);

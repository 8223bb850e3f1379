// Host-side plan builder: sub-task division and descriptor generation
// (paper: "Computational Collaboration Between Host and Device" — grid
// batches plus their neighbouring atoms, with the GEMM descriptors stored
// contiguously by integer index).
#pragma once
#include <string>
#include <vector>

#include "gint.h"
#include "gint_internal.h"

struct HostPlan {
    std::vector<GSpecies> species;
    std::vector<GAtom> atoms;
    std::vector<double> tab;
    std::vector<float> tab32;
    std::vector<GPair> pairs;        // clusters of <= 4 atoms: [0, ncanon) canonical, then swapped copies
    std::vector<GPair8> pairs8;      // clusters of 5..8 atoms (canonical only; instead of pairs)
    std::vector<GBig> bigcells;
    std::vector<GItem> items_canon;  // canonical pairs, longest first
    std::vector<GItem> items_ordered;// canonical + swapped, longest first (only the canonical ones with pairs8)
    std::vector<GSys> sys;           // one per system
    std::vector<GBlk> blocks;        // pattern blocks with their transposes (symmetry check, D16 conversion)
    std::vector<GBrick> bricks;      // bigcell-stationary bricks (rho and force), empty unless built
    std::vector<GUAtom> uatoms;      // their atom-image unions
    std::vector<int> ptab;           // their pair tables (block indices, -1 = none)
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

// Builds the plan of n_sys systems (their work items merged into one queue).
// With bricks set, also the bigcell-stationary bricks of every system.
// Returns GINT_OK or a negative gint error code (hp.error holds a message).
int gint_build_host_plan(const gint_system *sys, int n_sys, const gint_options *opt, bool bricks, HostPlan &hp);

// Internal layout shared by the plan builder (host C++) and the HIP kernels.
//
// Work decomposition.  Atoms are grouped into spatially compact clusters of
// at most CL atoms.  A cluster pair (A at image TA, B at image TB) owns the
// 16 x 16 orbital tiles of every atom pair (a in A, b in B); each atom takes
// one 16-wide orbital slot (13 orbitals of 2s2p1d padded to 16).  The region
// where the pair's orbitals overlap is covered by bigcells of 4x4x4 grid
// points on the unwrapped (infinite) grid; V and rho are indexed modulo the
// grid.  A work item is a run of bigcells of one pair and is processed by one
// workgroup, which keeps the pair's output tiles in registers across the
// whole run (output-stationary), so H needs one write per item instead of
// one read-modify-write per bigcell.
#pragma once
#include <stdint.h>

#define GINT_CL 4            // atoms per cluster of the four-wave cluster-pair kernels (max)
#define GINT_CL8 8           // atoms per cluster of the eight-wave mixed Vlocal (max)
#define GINT_ORB 16          // orbital slots per atom
#define GINT_MAXCHAN 8       // radial channels per species
#define GINT_BC 4            // bigcell edge in grid points
#define GINT_BCPTS 64        // points per bigcell
#define GINT_MAXSPECIES 16

struct GSpecies {
    double rcut;
    double rcut2;
    double dr;
    double inv_dr;
    int nknots;
    int nchan;
    int norb;
    int tab_off;                 // offset (doubles) of [knot][chan][f, f'] in the table array
    int shape;                   // channel layout the kernels have a fixed path for (GINT_SHAPE_*)
    int chan_l[GINT_MAXCHAN];
};

// Channel layouts (l of each channel, in order) with fixed evaluation paths:
// the double-zeta-polarised sets of second-row elements (2s2p1d) and of
// hydrogen (2s1p).  Any other layout takes the general path.
enum { GINT_SHAPE_ANY = 0, GINT_SHAPE_2S2P1D = 1, GINT_SHAPE_2S1P = 2 };

struct GAtom {
    double x, y, z;
    int species;
    int norb;
};

// One cluster pair of clusters of at most CL atoms.  hoff[i*CL+j] is the
// element offset of block (a_i -> b_j, R = TB - TA) or -1; hoff_t[i*CL+j]
// that of (b_j -> a_i, -R).  Clusters of four serve every cluster-pair
// kernel; clusters of eight serve the eight-wave mixed-precision Vlocal.
template <int CL>
struct GPairT {
    int a[CL];                   // atom ids, -1 = empty slot
    int b[CL];
    double shiftA[3];            // TA.h added to A-atom positions
    double shiftB[3];            // TB.h added to B-atom positions
    int self;                    // 1: A == B with TA == TB (tiles cover both orders)
    int sys;                     // system of a batched plan
    long long hoff[CL * CL];
    long long hoff_t[CL * CL];
};
typedef GPairT<GINT_CL> GPair;
typedef GPairT<GINT_CL8> GPair8;

struct GBig {
    int x, y, z;                 // origin point index of a bigcell (unwrapped)
    int w;                       // flat index of the wrapped origin when no point of the bigcell
                                 // wraps and the grid has < 2^31 points, else -1
};

// One (I, J, R) block of the sparse pattern with its transpose (J, I, -R),
// for the symmetry check of D.
struct GBlk {
    long long off, off_t;        // element offsets of the block and of its transpose
    int ni, nj;                  // orbitals of I and J (the block is ni x nj, row-major)
    int sys;                     // system of a batched plan
    int i, j;                    // atoms I and J (packed over the systems of a plan)
    int pad;
};

struct GItem {
    int pair;
    int bc_begin;
    int bc_count;
    int pad;                     // 1: the item covers its whole pair (H written with plain stores)
};

// Bigcell-stationary decomposition (rho and force).  The grid of each system
// is tiled by bricks of bigcells (4x4x4 points each); a brick lists every atom
// image whose orbitals reach one of its points (its "union") and, for every
// ordered pair (i, j) of those images, the index of the pattern block that
// couples them, (atom_i, atom_j, T_j - T_i), or -1 if the pattern has none
// (then the two never overlap at a grid point: the plan checks the pattern
// against every overlapping pair).  One workgroup owns a brick: it evaluates
// each orbital once per bigcell and writes each grid point's rho once.
#define GINT_UMAX 256        // atom images per brick (max)

struct GUAtom {
    double x, y, z;              // position of the image: tau + T.h
    int atom;                    // atom index (packed over the systems of a plan)
    int species;
};

struct GBrick {
    int o[3];                    // origin point (grid indices in [0, N), multiples of 4)
    int sys;                     // system of a batched plan
    int u_begin, u_count;        // union atom images [u_begin, u_begin + u_count)
    long long pt_off;            // pair table: u_count^2 block indices, row i (k side), column j
    int nb[3];                   // bigcells of the brick along each axis that start inside the grid
    int pad;
};

// Geometry of one system of a (possibly batched) plan and the offsets of its
// data in the packed grid arrays (V, rho) and per-system scalars.
struct GSys {
    int N[3];
    int natom;
    double e[3][3];              // grid step vectors e_i = a_i / N_i (rows)
    double w;                    // volume per grid point
    double volume;
    long long g_off;             // first grid point in packed V / rho
    long long nnz_off;           // first element in packed H / D
    int atom_off;                // first atom in packed F
    int pad;
};

// Everything a kernel needs, passed by value.
struct GDev {
    const GSpecies *species;
    const GAtom *atoms;
    const double *tab;           // interleaved radial tables
    const float *tab32;          // the same interpolant in FP32 by knot interval (mixed precision), times the
                                 // channel's harmonic constant K_l: [k][chan][c0, c1, c2, c3],
                                 // K_l p = c0 + c1 t + c2 t^2 + c3 t^3, at 2 tab_off
    const GPair *pairs;          // clusters of <= 4 atoms (null when the plan has clusters of 8)
    const GPair8 *pairs8;        // clusters of 5..8 atoms (null otherwise)
    const GBig *bigcells;
    const GItem *items;
    const GSys *sys;             // per-system geometry (one entry for a single system)
    int *counter;                // work counter of persistent launches (reset before each launch)
    int nitems;
    int nsys;
    int natom;
    int N[3];
    double e[3][3];              // grid step vectors e_i = a_i / N_i (rows)
    double w;                    // volume per grid point
    // mixed precision: orbitals enter the 16-bit MFMA operands multiplied by
    // phi_scale (a power of two with |phi| phi_scale <= 2^13), so that their
    // hi/lo splits stay clear of the FP16 subnormal range; vmax points to
    // max_g |V_g| of the current call (reduced on the device)
    double phi_scale;
    const double *vmax;
    int shape_all;               // GINT_SHAPE_* shared by every species of the plan, else GINT_SHAPE_ANY
    int pad_;
    // bigcell-stationary path (mixed-precision rho and force)
    const GBrick *bricks;
    const GUAtom *uatoms;
    const int *ptab;             // pair tables of the bricks
    const unsigned short *d16;   // per pattern block: D_sym * dscale as 16-bit hi [nu][mu] then lo [nu][mu] (1 KiB)
    const double *dmax;          // max |D| of the current call (reduced on the device)
    int nbricks;
    int nblocks;
};

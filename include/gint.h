/* gint.h — C ABI of the MI355X grid-integration ("Gint") library.
 *
 * The library evaluates the three real-space grid integrals of LCAO density
 * functional theory (paper: "Real-Space Grid Integrals", Eq. 1-5) on an AMD
 * Instinct MI355X (gfx950):
 *
 *   H_IJR[mu,nu] = sum_g w V_g sum_{T} phi_Imu(r_g - tau_I - T.h) phi_Jnu(r_g - tau_J - (T+R).h)   (Eq. 2)
 *   rho_g        = sum_{(I,T,mu),(J,T',nu)} D_(I,J,T'-T)[mu,nu] phi_Imu phi_Jnu                      (Eq. 3)
 *   F_K = -dE/dtau_K and Z = dE/d(strain) of E = sum_g w V_g rho_g (Pulay terms, Eq. 4-5)
 *
 * where g runs over the uniform grid r_g = sum_i (n_i/N_i) a_i of the periodic
 * cell, w = Omega/N_g is the volume per point (Eq. 2's dV), T runs over lattice
 * translations, and the orbitals are numerical atomic orbitals
 * phi_{c,m}(x) = p_c(|x|) S_{l_c m}(x) with p_c the cubic Hermite interpolant
 * of the tabulated radial function f_c and S_lm = r^l Y_lm the real solid
 * harmonics (orthonormal Y_lm, m = -l..l, sin-type for m < 0, l <= 2),
 * strictly zero for |x| >= rcut (paper: "Numerical Atomic Orbitals").
 *
 * Conventions shared by every entry point
 *  - Units: Bohr, Hartree.  All floating-point inputs and outputs are FP64.
 *  - Orbitals of an atom are ordered by channel (in the order given), then
 *    m = -l..l.  At most 16 orbitals per atom, l <= 2.
 *  - Block (I, J, R) couples atom I in cell 0 with atom J in cell R
 *    (R = T' - T, an integer triple); it is stored row-major n_I x n_J at
 *    element offset blk_off.  The pattern must be transpose-closed:
 *    (I,J,R) present <=> (J,I,-R) present.
 *  - D must satisfy D_JI(-R) = D_IJR^T up to round-off; the kernels use the
 *    symmetrised D_sym = (D_IJR + D_JI(-R)^T)/2 throughout.
 *  - Grid arrays (v_loc, rho) are FP64 [N1][N2][N3] in C order,
 *    g = (n1 N2 + n2) N3 + n3.
 *  - Device arrays are allocated and owned by the caller (e.g. through
 *    PyTorch) on the plan's device; the library only reads inputs and
 *    overwrites outputs.  Inputs are never modified.
 *  - Every call enqueues its work on `stream` (a hipStream_t, NULL = the
 *    default stream) and returns without synchronising.  Scalar outputs are
 *    device pointers so that no call forces a host round trip.
 *  - A plan is not thread-safe; separate plans are independent.
 *  - Errors: every function returns GINT_OK (0) or a negative code.  Every
 *    argument check (null pointers, the current device against the plan's)
 *    comes before any work is enqueued, so a call rejected with GINT_EINVAL
 *    leaves its outputs untouched and enqueues nothing.  A call runs as a
 *    few launches in order (clear the outputs, the persistent kernel, small
 *    reductions); if a launch itself fails (GINT_EHIP), launches already
 *    enqueued before it are not undone, so outputs may have been cleared.
 *    No exception, abort or exit crosses this interface.
 */
#ifndef GINT_H
#define GINT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GINT_OK = 0,
    GINT_EINVAL = -1,        /* bad shape, index, non-finite input, bad option */
    GINT_EPATTERN = -2,      /* an overlapping (I,J,R) is missing, or the pattern is not transpose-closed */
    GINT_ENOMEM = -3,        /* host or device allocation failed (or exceeded a workspace cap) */
    GINT_EHIP = -4,          /* a HIP runtime call failed; see gint_last_hip_error() */
    GINT_EUNSUPPORTED = -5   /* l > 2, more than 16 orbitals per atom, unavailable precision */
};

enum {
    GINT_FP64 = 0,           /* plain path: FP64 orbitals, FP64 MFMA contractions */
    GINT_MIXED_FP16X3 = 1,   /* FP32 orbitals; FP16 hi+lo split operands, 3 FP16 MFMA products,
                                FP32 accumulation per bigcell, FP64 across bigcells and for E, N_e */
    GINT_MIXED_BF16X3 = 2    /* as GINT_MIXED_FP16X3 with BF16 hi+lo splits (wider range, ~16 bits) */
};

typedef struct gint_plan gint_plan;

/* Radial basis of one species (host memory, read during gint_plan_create).
 * Knots r_k = k dr, k = 0..nknots-1, with (nknots-1) dr >= rcut.  f[c][k]
 * and fp[c][k] hold f_c(r_k) and f_c'(r_k) of channel c; the radial factor
 * of the orbital is R_c(r) = r^l f_c(r), interpolated by the cubic Hermite
 * polynomial on [r_k, r_k+1]; this is the reading of "tabulated cubic-spline
 * radial functions" used throughout (the interpolant's own derivative is used
 * for gradients, so forces are exact derivatives of the energy). */
typedef struct {
    double rcut;             /* strict cutoff: phi = 0 for r >= rcut */
    double dr;               /* knot spacing (> 0) */
    int nknots;              /* >= 2 */
    int nchan;               /* >= 1 */
    const int *chan_l;       /* [nchan], 0 <= l <= 2 */
    const double *f;         /* [nchan][nknots] */
    const double *fp;        /* [nchan][nknots] */
} gint_species;

/* One periodic system (host memory, read during gint_plan_create). */
typedef struct {
    double cell[9];          /* rows a1, a2, a3 (Bohr); Omega = |det| > 0 */
    int natom;               /* >= 1 */
    const double *pos;       /* [natom][3] Cartesian, used as given (never wrapped) */
    const int *species;      /* [natom], indices into species_list */
    int nspecies;
    const gint_species *species_list;
    int grid[3];             /* N1, N2, N3 >= 1 */
    int nblk;                /* number of (I, J, R) blocks */
    const int *blk_i;        /* [nblk] */
    const int *blk_j;        /* [nblk] */
    const int *blk_r;        /* [nblk][3] */
    const int64_t *blk_off;  /* [nblk] element offset of each block */
} gint_system;

/* Plan options; pass NULL for defaults. */
typedef struct {
    int precision;           /* GINT_FP64, GINT_MIXED_FP16X3 or GINT_MIXED_BF16X3 */
    int cluster_atoms;       /* atoms per cluster of the cluster-pair work items, 1..8 (0 = default 4).
                                Values above 4 select the eight-wave Vlocal kernel and are accepted
                                only for mixed-precision plans whose rho and force run on bricks
                                (GINT_DECOMP_DEFAULT, GINT_DECOMP_BIGCELL_RHO_FORCE); else GINT_EINVAL. */
    int max_bigcells_per_item; /* work-item length cap (0 = default) */
    int device_mib_cap;      /* device memory the plan may hold, in MiB (0 = no cap): a plan
                                that needs more fails with GINT_ENOMEM before any HIP call */
    int brick[3];            /* bigcell-stationary path: bigcells per brick along a1, a2, a3
                                (each 1..8; 0 = chosen by the plan) */
    int decomposition;       /* GINT_DECOMP_*: how rho and the force are divided into work */
} gint_options;

/* Work decomposition of the three integrals.  CLUSTER_PAIRS:
 * output-stationary cluster-pair items, every orbital evaluated once per
 * cluster pair that needs it.  BIGCELL: bigcell-stationary bricks (the
 * paper's grid batches, "Computational Collaboration Between Host and
 * Device"): rho and the force pass evaluate every orbital once per bigcell
 * and write rho once per point without atomics; Vlocal evaluates each
 * orbital once per bigcell and chunk pair of the brick's atom images and adds
 * each H block once per brick.  BIGCELL_RHO_FORCE: bricks for rho and the
 * force pass, cluster pairs for Vlocal.  The brick forms exist in the mixed
 * precisions.  DEFAULT: BIGCELL_RHO_FORCE for the mixed forms (measured
 * fastest), CLUSTER_PAIRS for FP64. */
enum { GINT_DECOMP_DEFAULT = 0, GINT_DECOMP_CLUSTER_PAIRS = 1, GINT_DECOMP_BIGCELL = 2,
       GINT_DECOMP_BIGCELL_RHO_FORCE = 3 };

/* Sizes of a plan (host struct filled by gint_plan_query). */
typedef struct {
    int64_t ngrid;           /* N1 N2 N3 */
    int64_t nnz;             /* length of h_vals / d_vals */
    int natom;
    int ncluster;
    int64_t npairs;          /* canonical cluster pairs */
    int64_t nitems;          /* work items of the canonical list */
    int64_t nbigcells;       /* bigcell visits summed over canonical pairs */
    double work_units;       /* W = sum_g n_orb(g)^2 (0 unless computed) */
    double volume;           /* Omega */
    int64_t device_bytes;    /* device memory held by the plan */
    int precision;           /* the plan's precision form */
    double build_seconds;    /* host time of gint_plan_create */
    int n_sys;               /* systems in the plan (packed buffers when > 1) */
    int decomposition;       /* the GINT_DECOMP_* in use (never DEFAULT) */
    int brick[3];            /* bigcells per brick (bigcell-stationary plans; of system 0) */
    int64_t nbricks;         /* bricks with at least one atom image (bigcell-stationary plans) */
    int64_t brick_images;    /* atom images summed over the bricks' unions */
} gint_sizes;

/* Where system i of a plan lives in the packed buffers (host struct filled by
 * gint_plan_query_system).  For a single-system plan every offset is 0. */
typedef struct {
    int64_t g_off;           /* first element of the system in v_loc / rho */
    int64_t ngrid;           /* its N1 N2 N3 */
    int64_t nnz_off;         /* first element in h_vals / d_vals */
    int64_t nnz;
    int atom_off;            /* first atom (row) in force */
    int natom;
    int grid[3];
    double volume;
} gint_system_sizes;

/* Build a plan for n_sys >= 1 systems: validates the inputs, groups atoms
 * into clusters, enumerates cluster-image pairs and the bigcells (4x4x4 grid
 * points) where their orbitals overlap, maps every overlapping atom pair to
 * its pattern block (paper: sub-task division and sub-task descriptors,
 * "Computational Collaboration Between Host and Device"), and uploads the
 * descriptors to the current device.  Synchronous.  With n_sys > 1 the
 * systems' work items form one queue served by one persistent launch per
 * call, and every data array is packed: system i occupies the slice given by
 * gint_plan_query_system (v_loc, rho: grid points; h_vals, d_vals: block
 * elements; force: atoms), and the scalar outputs n_elec, energy and
 * w_out hold n_sys values, stress n_sys 3x3 matrices.  Each system keeps its
 * own cell, grid, species and pattern.  On success *out owns device memory
 * until gint_plan_destroy. */
int gint_plan_create(gint_plan **out, const gint_system *sys, int n_sys,
                     const gint_options *opt, void *stream);

/* H_IJR (Eq. 2) for every block of the pattern.  v_loc: device f64[N_g].
 * h_vals: device f64[nnz], overwritten (blocks with no overlap become 0).
 * (N_g, nnz, natom below: the plan's totals over its systems.) */
int gint_vlocal(gint_plan *p, const double *v_loc, double *h_vals, void *stream);

/* rho_g (Eq. 3).  d_vals: device f64[nnz].  rho: device f64[N_g], overwritten.
 * n_elec: device f64[n_sys] receiving sum_g w rho_g per system, or NULL. */
int gint_rho(gint_plan *p, const double *d_vals, double *rho, double *n_elec, void *stream);

/* Grid Pulay force and stress (Eq. 4-5).  force: device f64[natom][3],
 * F_K = -dE/dtau_K.  stress: device f64[n_sys][3][3], sigma = -Z/Omega with
 * Z_ab = dE/d(eps_ab) at fixed w (unsymmetrised).  energy: device
 * f64[n_sys] receiving E = sum_g w V_g rho_g, or NULL.  All outputs
 * overwritten. */
int gint_force_stress(gint_plan *p, const double *v_loc, const double *d_vals,
                      double *force, double *stress, double *energy, void *stream);

/* rho (Eq. 3), the force and stress (Eq. 4-5) and E in one pass: the same
 * outputs as gint_rho followed by gint_force_stress, for callers that need
 * both (the per-point values phi_A . psi_A that E needs are the terms of rho,
 * so rho costs little on top of the force pass).  n_elec and energy may be
 * NULL; every other output is overwritten. */
int gint_rho_force_stress(gint_plan *p, const double *v_loc, const double *d_vals, double *rho,
                          double *n_elec, double *force, double *stress, double *energy, void *stream);

/* Symmetry check of D (a debug aid; the kernels assume D_JI(-R) = D_IJR^T
 * and use D_sym, see the conventions above).  max_asym: device f64[n_sys],
 * overwritten with max over the blocks of each system of
 * |D_IJR[mu,nu] - D_JI(-R)[nu,mu]| (0 for an exactly symmetric D; NaN if a
 * difference is NaN).  d_vals as for gint_rho.  The first call uploads the
 * plan's block table (one allocation and a synchronous copy, so it is not
 * for stream capture); later calls only enqueue two kernels on `stream`.
 * The plan's device must be current (else GINT_EINVAL). */
int gint_check_symmetry(gint_plan *p, const double *d_vals, double *max_asym, void *stream);

/* E = w sum_g V_g rho_g per system (the energy of Eq. 4-5 for a given rho),
 * reduced in FP64 on the device in a fixed order (deterministic).  v_loc,
 * rho: device f64[N_g] (packed as for gint_rho); energy: device f64[n_sys],
 * overwritten. */
int gint_energy(gint_plan *p, const double *v_loc, const double *rho, double *energy, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same E
 * as gint_energy, from the same two-pass reduction in the same order (equal
 * bit for bit), but its scratch (the partial sums, 256 doubles per system)
 * is a static device array of 1 MiB in the library, so the call allocates
 * nothing and writes no plan state.  Each GPU holds its own copy of that
 * array for the life of the process; its address is looked up once per
 * device on the first call made with that device current.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (several
 * streams or threads) race and must be serialised by the caller.  Plans with
 * n_sys > 512 (more partial sums than the array holds) are rejected with
 * GINT_ENOMEM before anything is enqueued.  Arguments as for gint_energy. */
int gint_energy_noalloc(gint_plan *p, const double *v_loc, const double *rho, double *energy,
                        void *stream);

/* W = sum_g n_orb(g)^2 (grid points x ordered orbital pairs within rcut),
 * the unit of work of the throughput metric, counted exactly from the plan's
 * neighbour lists.  w_out: device f64[n_sys], overwritten. */
int gint_work_units(gint_plan *p, double *w_out, void *stream);

/* One full step captured into a HIP graph (paper: device work launched with
 * few host interactions, "Computational Collaboration Between Host and
 * Device"; replay removes the per-call launch overhead, which dominates for
 * batches of small structures).  The graph enqueues, in this order,
 * gint_vlocal (if h_vals), gint_rho (if rho) and gint_force_stress (if
 * force; stress must then be given too) with exactly these device buffers;
 * it is captured on a private stream and nothing runs until
 * gint_graph_launch.  The buffers and the plan must outlive the graph.  A
 * replay overwrites the outputs like the eager calls.  Replays of graphs of
 * one plan share its workspace: they must be serialised (one stream, or
 * events), as eager calls on one plan must.  The graph is bound to the
 * plan's device (GINT_EINVAL if another device is current). */
typedef struct gint_graph gint_graph;
int gint_graph_create(gint_graph **out, gint_plan *p, const double *v_loc, const double *d_vals,
                      double *h_vals, double *rho, double *n_elec, double *force, double *stress,
                      double *energy);
/* Enqueue one replay on `stream` (NULL = default stream). */
int gint_graph_launch(gint_graph *g, void *stream);
void gint_graph_destroy(gint_graph *g);

/* Autotuner of the tile shapes (paper: short timed trials pick the kernel
 * parameters, "Device Performance Optimization").  Two independent choices:
 * the cluster tile of the Vlocal kernel (cluster_atoms,
 * max_bigcells_per_item) and, for the bigcell-stationary rho/force path, the
 * brick shape (bigcells per brick along a1, a2, a3).  Trial k builds a plan
 * with cluster candidate k and brick candidate k (fixed orders) and times,
 * with HIP events on `stream`, one Vlocal call and one rho + force/stress
 * pass on constant V and D in scratch buffers the tuner allocates and frees;
 * the Vlocal time scores the cluster candidate, the rho + force time the
 * brick candidate.  No new trial starts once budget_seconds of wall time
 * have passed (the first always runs).  On input opt->precision and
 * opt->decomposition select the form (FP64 plans have no brick choice); on
 * success opt->cluster_atoms, opt->max_bigcells_per_item and opt->brick hold
 * the fastest candidates and *report every trial.  Synchronous.
 * The choice is cached per process, keyed by the device, the form and the
 * workload's shape class (number of systems, total atoms, grid points and
 * pattern blocks, the first system's cell and grid): a later call for the
 * same key returns the stored choice and report (report->cached = 1)
 * without timing anything.  gint_autotune_forget() empties the cache. */
#define GINT_TUNE_MAX 16
typedef struct {
    int ntrials;                         /* trials timed */
    int best;                            /* trial with the fastest Vlocal (cluster choice) */
    int best_brick;                      /* trial with the fastest rho + force (brick choice) */
    int cluster_atoms[GINT_TUNE_MAX];
    int max_bigcells_per_item[GINT_TUNE_MAX];
    int brick[GINT_TUNE_MAX][3];         /* as resolved by the plan (0 when the plan has no bricks) */
    double vlocal_ms[GINT_TUNE_MAX];     /* one Vlocal call */
    double rho_force_ms[GINT_TUNE_MAX];  /* one rho + force/stress pass */
    double step_ms[GINT_TUNE_MAX];       /* their sum */
    double seconds;                      /* wall time of the search */
    int cached;                          /* 1: returned from the cache, no trial run by this call */
} gint_tune_report;
int gint_autotune(const gint_system *sys, int n_sys, gint_options *opt, double budget_seconds,
                  void *stream, gint_tune_report *report);
void gint_autotune_forget(void);

/* Totals of a plan.  GINT_EINVAL on NULL arguments. */
int gint_plan_query(const gint_plan *p, gint_sizes *out);
/* Offsets and sizes of system i (0 <= i < n_sys) in the packed buffers.
 * GINT_EINVAL if i is out of range. */
int gint_plan_query_system(const gint_plan *p, int i, gint_system_sizes *out);
void gint_plan_destroy(gint_plan *p);
const char *gint_strerror(int code);
/* Last HIP error code recorded by a failing call (0 if none). */
int gint_last_hip_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GINT_H */

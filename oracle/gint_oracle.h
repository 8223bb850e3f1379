/* FP64 CPU oracle for real-space grid integration ("Gint").
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * reference the HIP library is checked against.  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it; the product path
 * never does.  It shares no code with the HIP library.
 *
 * What it computes (paper: "Real-Space Grid Integrals", Eq. 1-5, with the
 * grid sum of Eq. 2):
 *   C(g)  = { (I, T, mu) : |r_g - tau_I - T.h| < rcut_I }           (neighbour set)
 *   H_IJR[mu,nu] = sum_g w V_g sum_{(I,T,mu),(J,T',nu) in C(g), T'-T=R} phi_Imu phi_Jnu   (Eq. 2)
 *   rho_g        = sum_{pairs in C(g)} D_(I,J,T'-T)[mu,nu] phi_Imu phi_Jnu              (Eq. 3)
 *   E = sum_g w V_g rho_g,  N_e = sum_g w rho_g
 *   F_K^a = 2 sum_g w V_g sum_{(K,T,mu)} d_a phi_Kmu(x) sum_{(J,T',nu)} Dsym_(K,J,T'-T)[mu,nu] phi_Jnu(x')  (Eq. 4, reading: F = -dE/dtau)
 *   Z_ab  = 2 sum_g w V_g sum_{(K,T,mu)} d_a phi_Kmu(x) x_b sum_{(J,T',nu)} Dsym phi_Jnu(x')               (Eq. 5, reading: strain derivative)
 * with x = r_g - tau_K - T.h, w = Omega / N_g, Dsym = (D_IJR + D_JI(-R)^T)/2.
 *
 * Orbitals: phi_{c,m}(x) = p_c(|x|) S_{l_c m}(x), real solid harmonics
 * S_lm = r^l Y_lm (orthonormal Y, m = -l..l, sin-type for m < 0), l <= 2.
 * p_c is either the analytic radial f_c(r) = exp(-a_c r^2) chi(r) or the
 * cubic Hermite interpolant of the tabulated f_c, f_c' (knots k*dr).
 *
 * The paper prints no values of H, rho, F or sigma, so nothing here is
 * compared with printed numbers.  Every routine is pinned by mathematics
 * instead, in the CPU test suite: closed-form Gaussian overlaps, forces and
 * strain derivatives; the trace and electron-count identities; brute-force
 * enumeration (which also fixes the work count W exactly); finite
 * differences; and the smooth cutoff against the six end conditions that
 * define the C2 quintic step.
 */
#ifndef GINT_ORACLE_H
#define GINT_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int natom;
    const double *cell;      /* [3][3], rows a1, a2, a3 (Bohr) */
    const double *pos;       /* [natom][3] Cartesian (Bohr), used as given */
    const int *species;      /* [natom] */
    int nspecies;
    const double *sp_rcut;   /* [nspecies] strict cutoff r < rcut */
    const double *sp_dr;     /* [nspecies] knot spacing */
    const double *sp_rs;     /* [nspecies] start of the smooth taper (analytic mode) */
    const int *sp_nknots;    /* [nspecies] */
    const int *sp_cutoff;    /* [nspecies] 1: taper active, 0: plain Gaussian (analytic mode) */
    const int *sp_chan_off;  /* [nspecies+1] channel ranges */
    const int *chan_l;       /* [nchan_total] */
    const double *chan_alpha;/* [nchan_total] Gaussian exponent (analytic mode) */
    const long *chan_tab_off;/* [nchan_total] offset of the channel's table */
    const double *tab_f;     /* knots of f */
    const double *tab_fp;    /* knots of f' */
    const int *grid;         /* N1, N2, N3 */
    int nblk;
    const int *blk_i, *blk_j;/* [nblk] */
    const int *blk_r;        /* [nblk][3] */
    const long *blk_off;     /* [nblk] offset of the row-major n_I x n_J block */
    int radial_mode;         /* 0: table (Hermite), 1: analytic */
} oracle_system;

enum { ORACLE_OK = 0, ORACLE_EINVAL = -1, ORACLE_EPATTERN = -2, ORACLE_ENOMEM = -3 };

/* Full sums; g_begin/g_end restrict the sum over grid points to a range of
 * flat indices (pass 0, -1 for all points).  Outputs are overwritten. */
int oracle_vlocal(const oracle_system *s, const double *v, double *h, long g_begin, long g_end);
int oracle_rho(const oracle_system *s, const double *d, double *rho, long g_begin, long g_end);
int oracle_force_stress(const oracle_system *s, const double *v, const double *d,
                        double *force, double *zstrain, double *energy,
                        long g_begin, long g_end);

/* Sampled outputs, each computed on its own. */
int oracle_rho_points(const oracle_system *s, const double *d, long npts, const long *gidx, double *out);
/* Magnitude scale of rho's terms at each point, sum |phi_Imu| |D_IJR[mu,nu]| |phi_Jnu|
 * over the same pairs as rho (>= |rho_g|): the bound of rounding-error
 * tests of reordered or reduced-precision evaluations of rho. */
int oracle_rho_abs(const oracle_system *s, const double *d, double *out, long g_begin, long g_end);
int oracle_rho_abs_points(const oracle_system *s, const double *d, long npts, const long *gidx, double *out);
int oracle_vlocal_blocks(const oracle_system *s, const double *v, int nsel, const int *blk, double *out);
int oracle_force_atoms(const oracle_system *s, const double *v, const double *d,
                       int nsel, const int *atoms, double *force, double *zstrain);

/* Orbital values and gradients of one species at displacements x. */
int oracle_orbitals(const oracle_system *s, int species, long n, const double *x,
                    double *phi, double *grad);
/* Radial function p_c(r), p_c'(r) of one channel. */
int oracle_radial(const oracle_system *s, int species, int chan, long n, const double *r,
                  double *p, double *dp);
/* Neighbour set C(g) of one grid point: atom, T, |x|; returns count or error. */
int oracle_neighbours(const oracle_system *s, long g, int cap, int *atom, int *T, double *x);
/* Sum over grid points of n_orb(g)^2 (the unit of work W) over a range. */
int oracle_work(const oracle_system *s, long g_begin, long g_end, double *w_out);
/* OpenMP threads the oracle uses. */
int oracle_num_threads(void);
/* Threads used by later calls (the OpenMP team size); n <= 0 is ignored. */
void oracle_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif

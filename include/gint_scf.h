/* gint_scf.h — one self-consistent-field step closed on the device, around
 * the grid integrals of gint.h.
 *
 * In a self-consistent LCAO calculation the grid integrals sit between two
 * dense steps (paper: "GPU Acceleration of Diagonalization", Eq. 6-8, and
 * the SCF flow of the Methods section): the Hamiltonian and overlap blocks
 * H_IJR, S_IJR are summed over lattice vectors into the matrices of a
 * k-point, the generalised eigenproblem H c_i = e_i S c_i is solved, and the
 * density matrix D = sum_i f_i c_i c_i^T is formed from the occupied
 * eigenvectors and handed back to the density integral.  This interface
 * does that at the Gamma point (k = 0):
 *
 *   H^G[I mu, J nu] = sum_R H_IJR[mu, nu],  S^G likewise           (Bloch sum at k = 0)
 *   H^G c_i = e_i S^G c_i,  c_i^T S^G c_j = delta_ij                 (rocSOLVER dsygvd)
 *   f_i: 2 per orbital by increasing e_i (aufbau; the last one partly
 *        filled if n_electrons is not even), or 2/(1 + exp((e_i - mu)/kT))
 *        with mu fixed by sum_i f_i = n_electrons (Fermi-Dirac, kT > 0)
 *   D_IJR[mu, nu] = sum_i f_i c_i[I mu] c_i[J nu]  for every block (I, J, R)
 *
 * The Gamma-point D is the same for every R (a Gamma-only calculation).
 * With D from here, gint_rho gives rho and N_e = sum_g w rho_g
 * = sum_i f_i (the S^G-orthonormality of the c_i).  The overlap S(R) is an
 * input: the grid estimate S = H[V = 1] (gint_vlocal with a constant
 * potential of 1) stands in for the two-centre overlap a full code
 * computes analytically.
 *
 * Orbital order of the dense matrices: atoms in order, each atom's orbitals
 * in the order of gint.h.  Conventions (streams, errors, device pointers)
 * as in gint.h.  Single-system plans only (GINT_EUNSUPPORTED otherwise).
 */
#ifndef GINT_SCF_H
#define GINT_SCF_H

#include "gint.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gint_scf gint_scf;

/* Dense work arrays for the plan's n = sum_I n_orb(I) orbitals (four n x n
 * FP64 matrices and a few vectors, on the plan's device) and a rocBLAS
 * handle.  Synchronous.  *n_orbitals (nullable) receives n. */
int gint_scf_create(gint_scf **out, gint_plan *p, int64_t *n_orbitals);

/* From H(R) and S(R) (device f64[nnz], the plan's pattern) to the
 * eigenvalues (device f64[n], increasing), the occupations (device f64[n])
 * and D(R) (device f64[nnz], overwritten on every block).  kT <= 0 selects
 * aufbau filling.  info (device int, nullable) receives rocSOLVER's status:
 * 0 on success; i <= n: the eigensolver did not converge; n + i: S^G is not
 * positive definite (its leading minor of order i).  Enqueued on `stream`;
 * the scf object must not be used on two streams at once. */
int gint_scf_solve(gint_scf *s, const double *h_vals, const double *s_vals, double n_electrons, double kT,
                   double *eigvals, double *occupations, double *d_vals, int *info, void *stream);

/* H^G of h_vals into dense (device f64[n * n], column-major; symmetric):
 * the Bloch sum at k = 0 on its own. */
int gint_scf_fold_gamma(gint_scf *s, const double *h_vals, double *dense, void *stream);

void gint_scf_destroy(gint_scf *s);

#ifdef __cplusplus
}
#endif
#endif /* GINT_SCF_H */

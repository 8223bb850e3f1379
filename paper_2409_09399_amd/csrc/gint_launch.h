// Kernel launchers of the grid-integration library (defined with their
// kernels), shared by the source files that sequence them.  Every launcher
// enqueues on `s` and returns the launch's HIP status.
#pragma once
#include <hip/hip_runtime.h>

#include "gint_internal.h"

hipError_t gint_launch_fill(double *p, long long n, double v, hipStream_t s);
hipError_t gint_launch_vlocal(const GDev &P, const double *V, double *H, hipStream_t s);
hipError_t gint_launch_rho(const GDev &P, const double *D, double *rho, hipStream_t s);
hipError_t gint_launch_force(const GDev &P, const double *V, const double *D, double *F, double *ZE, double *rho,
                             hipStream_t s);
hipError_t gint_launch_work(const GDev &P, double *W, hipStream_t s);
hipError_t gint_launch_dsym_check(const GBlk *blk, long long nblk, const double *D, double *out, hipStream_t s);
hipError_t gint_launch_seg_sum(const GDev &P, const double *x, const double *y, double *part, int nparts,
                               double *out, hipStream_t s);
hipError_t gint_launch_finish_stress(const GDev &P, const double *ZE, double *stress, double *energy,
                                     hipStream_t s);
hipError_t gint_static_scratch(void **ptr, size_t *bytes);
void gint_prime_grids_fp64();
void gint_prime_grids_mx(int prec);
// The mixed and brick launchers below that take V or D prepare their 16-bit
// operand scales (and, for the bricks, the 16-bit D copy) on each call; the
// _prepared forms skip that, for callers that ran gint_launch_vmax or
// gint_launch_d16 on the same arrays earlier on the stream.
hipError_t gint_launch_vmax(const GDev &P, const double *V, long long ngrid, hipStream_t s);
hipError_t gint_launch_d16(const GDev &P, int prec, const GBlk *blocks, long long nnz, const double *D,
                           hipStream_t s);
hipError_t gint_launch_vlocal_mx(const GDev &P, int prec, const double *V, long long ngrid, double *H,
                                 hipStream_t s);
hipError_t gint_launch_vlocal_mx_prepared(const GDev &P, int prec, const double *V, double *H, hipStream_t s);
hipError_t gint_launch_rho_mx(const GDev &P, int prec, const double *D, double *rho, hipStream_t s);
hipError_t gint_launch_force_mx(const GDev &P, int prec, const double *V, const double *D, double *F, double *ZE,
                                double *rho, hipStream_t s);
hipError_t gint_launch_rho_bc(const GDev &P, int prec, const GBlk *blocks, long long nnz, const double *D,
                              double *rho, hipStream_t s);
hipError_t gint_launch_force_bc(const GDev &P, int prec, const GBlk *blocks, long long nnz, const double *V,
                                const double *D, double *F, double *ZE, double *rho, hipStream_t s);
hipError_t gint_launch_rho_bc_prepared(const GDev &P, int prec, double *rho, hipStream_t s);
hipError_t gint_launch_force_bc_prepared(const GDev &P, int prec, const double *V, double *F, double *ZE, double *rho,
                                         hipStream_t s);
void gint_prime_grids_bc(int prec);
hipError_t gint_launch_vlocal_bc(const GDev &P, int prec, const GBlk *blocks, const double *V, double *H,
                                 hipStream_t s);
hipError_t gint_launch_absmax(const double *x, long long n, double *out, hipStream_t s);


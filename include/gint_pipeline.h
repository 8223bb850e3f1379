/* Streaming pipeline of the grid integrals (paper: "Computational
 * Collaboration Between Host and Device" — the host divides the grid into
 * sub-tasks and prepares their descriptors while the device computes the
 * earlier ones, with the transfers in between, a three-stage pipeline).
 *
 * A pipeline holds one system whose grid is cut into n_slabs slabs along a1
 * (a bigcell or brick belongs to the slab of its origin's a1 index).  A host
 * thread builds the plan of each slab in turn (the same construction as
 * gint_plan_create, restricted to the slab) and keeps it in host memory; a
 * step copies slab k+1's descriptors to the device, from pinned memory on a
 * copy stream of its own, while slab k's kernels run on the caller's
 * stream, and the first step also overlaps the host builds with both.  The
 * device holds the shared tables and at most two slabs' descriptors, so the
 * descriptors of a system may exceed what one plan could keep resident.
 *
 * One step computes what gint_vlocal, gint_rho (with N_e) and
 * gint_force_stress (with E) compute for the same system and options: H and
 * rho are cleared first, every slab adds its share (H through atomics, rho
 * once per point), and the reductions of N_e, E and the stress follow the
 * last slab.  Arrays and their layouts are those of include/gint.h for one
 * system.  Numerically the sums are regrouped over slabs, so results agree
 * with a single plan's to rounding.
 */
#ifndef GINT_PIPELINE_H
#define GINT_PIPELINE_H

#include <stdint.h>

#include "gint.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gint_pipeline gint_pipeline;

typedef struct {
    int n_slabs;
    int slabs_built;              /* host plans built so far (all of them after the first step) */
    int steps;                    /* steps run */
    double build_seconds;         /* host time of the slab builds (builder thread, summed) */
    double first_step_seconds;    /* wall time of the first step's call, builds included */
    double wait_seconds;          /* host time steps spent waiting for the builder */
    int64_t shared_device_bytes;  /* tables, pattern blocks, D operand copy, workspace */
    int64_t slot_device_bytes;    /* the two slabs' descriptor buffers together */
    int64_t largest_slab_bytes;   /* descriptors of the largest slab */
    int64_t all_slabs_bytes;      /* descriptors of every slab, summed (what one plan would hold) */
    int64_t copied_bytes;         /* descriptor bytes copied to the device by the last step */
} gint_pipeline_stats;

/* Deep-copies *sys (one system; its arrays may be freed after the call),
 * validates the options as gint_plan_create does, and starts the host
 * builder thread.  1 <= n_slabs <= 4096.  The device current at this call is
 * the pipeline's.  GINT_EINVAL / GINT_EUNSUPPORTED as gint_plan_create (plan
 * errors of a slab, e.g. GINT_EPATTERN, surface from the step that needs
 * it); GINT_ENOMEM; GINT_EHIP. */
int gint_pipeline_create(gint_pipeline **out, const gint_system *sys, const gint_options *opt, int n_slabs);

/* One step on `stream` (device pointers: v_loc, d_vals [nnz]; outputs h_vals
 * [nnz], rho [N_g], n_elec [1] (nullable), force [natom][3], stress [3][3],
 * energy [1] (nullable)).  The call returns once every slab is enqueued; it
 * blocks only on the builder and on the reuse of its two pinned staging
 * buffers.  Not thread-safe; one step at a time per pipeline.  Errors as the
 * entry points of gint.h; on a slab's plan error the outputs may have been
 * cleared and partly accumulated. */
int gint_pipeline_step(gint_pipeline *p, const double *v_loc, const double *d_vals, double *h_vals, double *rho,
                       double *n_elec, double *force, double *stress, double *energy, void *stream);

/* Counters and sizes of the pipeline.  GINT_EINVAL on NULL. */
int gint_pipeline_query(const gint_pipeline *p, gint_pipeline_stats *out);

/* Waits for the builder thread and for the pipeline's copies and kernels,
 * then frees everything.  NULL is a no-op. */
void gint_pipeline_destroy(gint_pipeline *p);

#ifdef __cplusplus
}
#endif

#endif

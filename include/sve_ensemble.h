/*
 * sve_ensemble.h -- many independent runs of the solver advanced together
 * (declarations of the solver itself in sve.h).
 *
 * Each member is a 2D grid with its own size, extent, Grass constant A_g
 * and exponent m_g (eq. "bedload Grass"), periodic boundaries, FP64
 * storage and its own CFL time step (sve_step's rule, per member).  One
 * step of the whole ensemble is one launch of a persistent work-queue
 * kernel: its wavefronts take tiles of any member from a device queue
 * (largest members first), so uneven member sizes share the GPU; several
 * steps are captured once in a HIP graph and replayed.  The tile height and
 * the scheduling mode come from sve_ens_autotune or sve_ens_set_schedule.
 *
 * Ownership: the library owns all member states (double-buffered) and
 * their control blocks; the host arrays given to sve_ens_create are copied.
 * Errors are per member and sticky: a member whose step fails keeps its
 * last good state and stops; other members go on; the step call returns
 * the first failing member's code.
 */
#ifndef SVE_ENSEMBLE_H
#define SVE_ENSEMBLE_H

#include "sve.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sve_member {
    int nx, ny;                 /* grid of this member                        */
    double Lx, Ly;              /* extent [m]                                 */
    double A_g, m_g;            /* Grass constant and exponent of this member */
    const double *h, *hu, *hv, *zb;   /* host arrays, nx*ny each, row-major  */
} sve_member;

typedef struct sve_ens sve_ens;

/* Scheduling modes of the ensemble kernel */
#define SVE_ENS_QUEUE 0   /* persistent wavefronts pull tiles from a queue  */
#define SVE_ENS_GRID  1   /* one wavefront per tile, hardware dispatch      */

/*
 * Create an ensemble of n members (n >= 1).  p: shared parameters (law must
 * be SVE_LAW_GRASS, reconstruction 0 and order 0 or 1; g is used; each
 * member's A_g and m_g replace p's).  stream: hipStream_t for all work (may be NULL).
 * Returns SVE_ERR_ARG for invalid members (size, h <= 0, m_g outside
 * [1, 4]) or parameters.
 */
int sve_ens_create(sve_ens **ens, int n, const sve_member *members,
                   const sve_params *p, void *stream);

/* Advance every member by nsteps CFL steps (replays a captured graph). */
int sve_ens_step(sve_ens *ens, int nsteps, double cfl);

/*
 * Reference schedule: the same steps, member after member, with the
 * single-grid kernel of sve_step and its default (automatic) tiling, one
 * launch per step per member.
 */
int sve_ens_step_sequential(sve_ens *ens, int nsteps, double cfl);

/* Copy member m's state (host arrays nx*ny, NULL to skip) and time. */
int sve_ens_get(sve_ens *ens, int m, double *h, double *hu, double *hv, double *zb,
                double *t, long long *nsteps);

/*
 * Time nprobe steps for each tile height in {8, 16, 32, 48, 64, 96, 128} and both modes
 * (member states are saved before and restored after) and keep the fastest;
 * *rows and *mode (may be NULL) receive the choice.
 */
int sve_ens_autotune(sve_ens *ens, int nprobe, double cfl, int *rows, int *mode);

/* Set the schedule directly (rows in {8, 16, 32, 48, 64, 96, 128}, mode SVE_ENS_*). */
int sve_ens_set_schedule(sve_ens *ens, int rows, int mode);

/* Milliseconds between HIP events around the last step call's launches. */
int sve_ens_last_elapsed_ms(sve_ens *ens, double *ms);

/* Release all buffers.  NULL is accepted. */
int sve_ens_destroy(sve_ens *ens);

#ifdef __cplusplus
}
#endif
#endif /* SVE_ENSEMBLE_H */

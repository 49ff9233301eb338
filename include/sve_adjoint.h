/*
 * sve_adjoint.h -- discrete adjoint of fixed-dt steps of the solver
 * (declarations of the solver itself in sve.h).
 *
 * The adjoint is the exact transpose of the linearisation of the library's
 * own fixed-dt step: one explicit step of the relaxation scheme (section
 * "Numerical method"), its interface solver and its lambda = 0 projection,
 * differentiated by hand in reverse mode.  Branches of the solver (maxima,
 * the fan state at x/t = 0) are taken as in the forward step.  Supported:
 * 2D grids, FP64 storage, the Grass law (eq. "bedload Grass", uniform or
 * per-cell A_g), periodic boundaries, no momentum friction, the paper's
 * first-order scheme (reconstruction = 0, order 0 or 1); other set-ups
 * return SVE_ERR_ARG.
 *
 * Memory: the forward keeps ceil(n/k) checkpoints of the state and the
 * backward one segment of k states (k = ceil(sqrt(n)) by default), 32 bytes
 * per cell each; all buffers are owned by the context and freed by
 * sve_destroy or by an sve_adj_forward with another segment layout (a
 * forward run with the same number of steps and checkpoint interval reuses
 * them).
 *
 * Device arrays below are caller-owned, on the context's device, read and
 * written on the context's stream; a "state array" is 4*nx*ny doubles
 * holding h, hu, hv, z_b one after the other (each row-major, k = j*nx+i).
 */
#ifndef SVE_ADJOINT_H
#define SVE_ADJOINT_H

#include "sve.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Advance the context by nsteps fixed-dt steps (as sve_step_fixed_dt) and
 * keep the state every `every` steps (every <= 0: ceil(sqrt(nsteps))).
 * Returns SVE_ERR_ARG for unsupported set-ups, SVE_ERR_HIP when the
 * checkpoints do not fit, or a step error.
 */
int sve_adj_forward(sve_ctx *ctx, int nsteps, double dt, int every);

/*
 * Gradient of a scalar L of the final state.  gT: state array with dL/dU at
 * the final time (input).  g0: state array receiving dL/dU at the time of
 * the sve_adj_forward call.  gAg: nx*ny doubles receiving dL/dA_g (the
 * per-cell Grass constant, or the cells' share of the scalar one), or NULL.
 * Recomputes each segment from its checkpoint.  SVE_ERR_STATE when no
 * forward run is recorded.  Synchronises the stream.
 */
int sve_adj_backward(sve_ctx *ctx, const double *gT, double *g0, double *gAg);

/*
 * One reverse step at the context's current state: lam_out = J^T lam_in for
 * the fixed-dt step of size dt, gAg (nx*ny doubles, may be NULL) =
 * (dU^{n+1}/dA_g)^T lam_in.  lam_in, lam_out: state arrays.  Synchronises
 * the stream.
 */
int sve_adj_step_vjp(sve_ctx *ctx, double dt, const double *lam_in, double *lam_out,
                     double *gAg);

/*
 * Tile height (rows per wavefront, 1..65536, or 0 for the automatic split
 * described at sve_set_tile_rows; default 0) of the reverse-step kernel of
 * this context.  Results do not depend on it.  SVE_ERR_ARG for other
 * values.
 */
int sve_adj_set_tile_rows(sve_ctx *ctx, int rows);

#ifdef __cplusplus
}
#endif
#endif /* SVE_ADJOINT_H */

/*
 * sve.h -- C ABI of the MI355X Saint-Venant--Exner relaxation solver.
 *
 * The library advances the coupled shallow-water / Exner system of the
 * paper (eq. "bedload system"; 2D form of section "2D dune evolution
 * cases") with the relaxation scheme of section "Numerical method": per
 * step, a lambda = 0 projection of the relaxation variables (eqs. "relaxh"
 * ... "relaxqs"), one homogeneous Riemann problem per interface with
 * celerities bounded as in eq. "ab", and the cell mean of the Riemann
 * solutions; 2D by the method of lines on a structured mesh (section
 * "Parallelization").  Bedload closures: Grass (eq. "bedload Grass") and the
 * threshold laws of eqs. "MPM" ... "Camenen" fed by the Darcy-Weisbach or
 * Manning/Strickler friction slope (section "Bedload modelling").
 *
 * Conventions
 *   Grid      nx x ny cells on [0, Lx] x [0, Ly]; dx = Lx/nx, dy = Ly/ny;
 *             cell centres x_i = (i + 1/2) dx.  1D runs use ny = 1 and
 *             hv = NULL (then Ly is ignored and only bc[0], bc[1] are used).
 *   Layout    every field is a row-major array of nx*ny doubles, index
 *             k = j*nx + i (x fastest): structure of arrays h, hu, hv, z_b.
 *   Units     SI (metres, seconds); g is taken from sve_params.
 *   Streams   all device work of a context runs on the hipStream_t given to
 *             its init call (NULL: the default stream).  Entry points that
 *             return host data synchronise that stream.
 *   Ownership the library owns every device buffer of a context (double-
 *             buffered state, per-cell A_g, control block); host arrays and
 *             caller device arrays passed in are copied and stay the
 *             caller's.  A context is not thread-safe; use one per stream.
 *   Errors    0 on success, a negative SVE_ERR_* code otherwise.  Step
 *             errors (positivity, ordering, non-finite state) are detected
 *             on the device and are sticky: the context keeps the last state
 *             that completed without error (and its time), and further steps
 *             return the same code until the context is re-initialised.
 */
#ifndef SVE_H
#define SVE_H

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define SVE_OK               0
#define SVE_ERR_ARG         (-1)  /* invalid argument (size, h <= 0, NaN, law) */
#define SVE_ERR_HIP         (-2)  /* HIP runtime failure (allocation, launch)  */
#define SVE_ERR_POSITIVITY  (-3)  /* an intermediate 1/h of a Riemann fan <= 0,
                                     or h <= 0 after an update                 */
#define SVE_ERR_ORDER       (-4)  /* bed-jump quadratic without admissible root */
#define SVE_ERR_NONFINITE   (-5)  /* non-finite value in the state              */
#define SVE_ERR_STATE       (-6)  /* call out of order (e.g. backward before
                                     forward) or context in an error state     */

/* ---- bedload laws (section "Bedload modelling") ------------------------- */
#define SVE_LAW_GRASS      0  /* q_b = A_g u |u|^(m_g - 1), eq. "bedload Grass" */
#define SVE_LAW_MPM        1  /* q* = 8 (tau* - tau*_cr)_+^(3/2), eq. "MPM"     */
#define SVE_LAW_FLVB       2  /* q* = 5.7 (tau* - tau*_cr)_+^(3/2), eq. "FLVB"  */
#define SVE_LAW_NIELSEN    3  /* q* = 12 sqrt(tau*) (tau* - tau*_cr)_+          */
#define SVE_LAW_RIBBERINK  4  /* q* = 11 (tau* - tau*_cr)_+^1.65                */
#define SVE_LAW_CAMENEN    5  /* q* = 12 tau*^1.5 exp(-4.5 tau*_cr / tau*)      */

/* ---- friction slope inside tau_b = rho g h S_f ------------------------- */
#define SVE_FRIC_STRICKLER 0  /* S_f = |U|^2 / (K_s^2 h^(4/3)), fric_coef = K_s */
#define SVE_FRIC_MANNING   1  /* S_f = n^2 |U|^2 / h^(4/3),     fric_coef = n   */
#define SVE_FRIC_DARCY     2  /* S_f = f |U|^2 / (8 g h),       fric_coef = f   */

/* ---- boundary conditions, order {west, east, south, north} -------------- */
#define SVE_BC_PERIODIC 0  /* wrap around                                      */
#define SVE_BC_FREE     1  /* ghost cell = copy of the adjacent cell            */
#define SVE_BC_INFLOW   2  /* ghost (h, hu, hv) = the sve_bc values, z_b copied */

/* ---- storage ----------------------------------------------------------- */
#define SVE_FP64 0  /* state stored and computed in double                    */
#define SVE_FP32 1  /* state stored as float, every operation in double       */

typedef struct sve_params {
    int    law;              /* SVE_LAW_*                                      */
    double g;                /* gravity [m/s^2]                                */
    double A_g;              /* Grass constant (used when no A_g field given)  */
    double m_g;              /* Grass exponent, 1 <= m_g <= 4                   */
    int    friction;         /* SVE_FRIC_* (threshold laws, momentum friction) */
    double fric_coef;        /* K_s, n or f                                    */
    double d_s;              /* mean grain diameter [m]                        */
    double s;                /* rho_s / rho                                    */
    double tau_cr;           /* critical Shields number (0.05 in the paper)    */
    int    momentum_friction;/* 0: eq. "bedload system" as printed; 1: adds
                                a semi-implicit -g h S_f momentum source       */
    int    reconstruction;   /* 0: the paper's scheme; 1: well-balanced variant
                                (hydrostatic reconstruction, see below)        */
    int    order;            /* 1 (or 0): the paper's first-order scheme;
                                2: second-order variant (see below)            */
} sve_params;

/*
 * Well-balanced variant (reconstruction = 1).  The paper's scheme is not
 * well balanced (section "Parallelization": a lake at rest over a varying
 * bed does not stay at rest) and well balancing is its stated future work
 * (section "Conclusions and perspectives").  The variant applies the
 * hydrostatic reconstruction of Audusse, Bouchut, Bristeau, Klein and
 * Perthame (2004), which the paper cites, with the relaxation solver as the
 * interface solver: at each interface z* = max(z_L, z_R) and
 * h* = max(0, h + z_b - z*) on each side (velocities kept); the relaxation
 * Riemann problem is solved between the projected reconstructed states on
 * the bed z*, and each cell's momentum flux gets g/2 (h^2 - h*^2).  A lake at
 * rest then stays at rest for every bedload law and exponent; on a flat bed
 * the variant is the paper's scheme.  Supported by sve_step and
 * sve_step_fixed_dt on the fused, split and 1D resident paths (the residual
 * path runs it as fused); the adjoint, the ensemble and
 * sve_step_dev_noalloc return SVE_ERR_ARG for it.
 *
 * Second-order variant (order = 2).  The paper finds its first-order
 * scheme very diffusive and names a higher order as future work (sections
 * "Parallelization" and "Conclusions and perspectives").  The variant is the
 * classical second-order extension: per cell and direction, minmod-limited
 * slopes of h, u, v and the free surface h + z_b give face states; each
 * interface solves the first-order problem (the relaxation Riemann problem,
 * or its hydrostatic reconstruction when reconstruction = 1) between the
 * two face states that meet there; the bed slope inside a cell adds
 * g (h_lo + h_hi)/2 (z_hi - z_lo) to the normal momentum's flux difference;
 * time stepping is Heun's method, U^{n+1} = (U^n + S(S(U^n)))/2 with the
 * Euler stage S(U) = U - dt D(U) (then the optional momentum friction) and
 * dt from the outer wave speeds of U^n's interface problems.  Two ghost
 * layers per side, filled by the boundary rules above.  A lake at rest
 * stays at rest (Grass m_g >= 3 and MPM with reconstruction = 0, every
 * closure with reconstruction = 1).  Supported by sve_step and
 * sve_step_fixed_dt in 1D and 2D, FP64 and FP32 storage, on its own pair of
 * kernels per step (sve_set_path accepts SVE_PATH_FUSED only, the tile
 * height of sve_set_tile_rows applies); the context then holds one more
 * FP64 buffer of 4 nx ny values (the first stage's rate).  An error of
 * either stage (an interface, a non-positive depth of U1 or of the new
 * state) fails that step with the rules of sve_step.  The adjoint, the
 * ensemble and sve_step_dev_noalloc return SVE_ERR_ARG for it.
 */

typedef struct sve_bc {
    int    kind;             /* SVE_BC_*                                       */
    double h, hu, hv;        /* Dirichlet values for SVE_BC_INFLOW             */
} sve_bc;

typedef struct sve_ctx sve_ctx;

/*
 * Create a context holding the initial state (host arrays).
 *   h, hu, zb  : nx*ny values each (required); hv: nx*ny values, or NULL for
 *                a 1D run (ny must then be 1).  h must be > 0 and finite.
 *   Ag_field   : nx*ny per-cell Grass constants, or NULL for p->A_g.
 *   bc         : 4 entries {W, E, S, N} (1D: the first 2 are used).
 *   storage    : SVE_FP64 or SVE_FP32.
 *   stream     : hipStream_t used for all work of this context (may be NULL).
 * The time is set to 0 and the first CFL time step is prepared on the device.
 * Returns SVE_ERR_ARG for invalid sizes, parameters or non-positive depth.
 */
int sve_init_state(sve_ctx **ctx, int nx, int ny, double Lx, double Ly,
                   const double *h, const double *hu, const double *hv,
                   const double *zb, const double *Ag_field,
                   const sve_params *p, const sve_bc bc[4], int storage,
                   void *stream);

/* Same as sve_init_state with device pointers (read on `stream`). */
int sve_init_state_dev(sve_ctx **ctx, int nx, int ny, double Lx, double Ly,
                       const double *h, const double *hu, const double *hv,
                       const double *zb, const double *Ag_field,
                       const sve_params *p, const sve_bc bc[4], int storage,
                       void *stream);

/*
 * Advance n explicit steps with the CFL time step
 *   dt = cfl / (S_x/dx + S_y/dy)     (1D: cfl dx / S_x),
 * S the largest outer relaxation wave speed max(|u_L - a/h_L|, |u_R + a/h_R|)
 * over the interfaces of each direction of the current state (the paper
 * states no time-step rule; this is the reading the library implements).
 * With t_end > 0, dt is clipped so that t stops exactly at t_end and later
 * steps leave the state unchanged.  The time step never returns to the host
 * between steps.  *t_out (may be NULL) receives the time reached.
 */
int sve_step(sve_ctx *ctx, int n, double cfl, double t_end, double *t_out);

/* Advance n steps with a fixed dt > 0 (no CFL reduction). */
int sve_step_fixed_dt(sve_ctx *ctx, int n, double dt);

/*
 * Copy the current state to host arrays (nx*ny doubles each; hv may be NULL;
 * any pointer may be NULL to skip it).  *t, *dt_last and *nsteps receive the
 * time, the last time step and the number of completed steps (each may be
 * NULL).  Synchronises the context's stream.
 */
int sve_get_state(sve_ctx *ctx, double *h, double *hu, double *hv, double *zb,
                  double *t, double *dt_last, long long *nsteps);

/* Same as sve_get_state with caller device pointers (written on the stream). */
int sve_get_state_dev(sve_ctx *ctx, double *h, double *hu, double *hv,
                      double *zb, double *t, double *dt_last,
                      long long *nsteps);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): n CFL
 * steps as sve_step, on a state held in caller device memory, with nothing
 * allocated by the library (no context, no hipMalloc/hipFree, no
 * allocating library routine).
 *   Scope     2D grids, FP64 state, uniform A_g (p->A_g), the paper's
 *             first-order scheme (reconstruction 0, order 0 or 1), the fused
 *             step kernel with the automatic tile split, i.e. the arithmetic
 *             of sve_step on a context created from the same arguments.
 *   State     h, hu, hv, zb: the initial state (nx*ny doubles each, layout as
 *             above, on the current device); they are also the second
 *             buffer of the steps and are overwritten when n >= 2.
 *             h_out .. zb_out: receive the state after the n steps.  The
 *             eight arrays must not overlap.
 *   Time      *t: the time of the initial state on entry, the time reached
 *             on return; t_end > 0 clips the last step as for sve_step.
 *             *dt_last (may be NULL) receives the last step's dt on success.
 *   Stream    all work runs on `stream` (NULL: the default stream); the call
 *             returns after synchronising it.
 *   Scratch   the steps' control block (wave-speed maxima, times, error
 *             word) lives in a fixed 4 KiB device array of the library, one
 *             per GPU, held until the process ends; it is independent of
 *             the grid size, so no grid is too large for it (grids beyond
 *             the kernels' nx*ny <= 2^31 - 1 are rejected).  Every call on a
 *             GPU uses that GPU's array and starts by resetting it: calls
 *             that overlap on one GPU (from several host threads or
 *             streams) race and must be serialised by the caller.
 *   Errors    SVE_ERR_ARG for invalid arguments, overlapping arrays or an
 *             input state that sve_init_state would refuse (non-finite,
 *             h <= 0); a step error returns its code, with the last state
 *             that completed in h_out .. zb_out and its time in *t.
 */
int sve_step_dev_noalloc(int nx, int ny, double Lx, double Ly, const sve_params *p,
                         const sve_bc bc[4], double *h, double *hu, double *hv,
                         double *zb, double *h_out, double *hu_out, double *hv_out,
                         double *zb_out, int n, double cfl, double t_end, double *t,
                         double *dt_last, void *stream);

/* Release every device buffer of the context.  NULL is accepted. */
int sve_destroy(sve_ctx *ctx);

/* Static description of an error code. */
const char *sve_strerror(int code);

/*
 * Path selection for tests and measurements (not needed in normal use).
 * The default is SVE_PATH_RESIDENT for 1D grids of up to 1536 cells, else
 * SVE_PATH_FUSED.
 *   SVE_PATH_FUSED   one kernel per step: update of step n and
 *                    the wave speeds of step n+1 in a single pass;
 *   SVE_PATH_SPLIT   two kernels per step (update, then wave speeds);
 *   SVE_PATH_RESIDENT (1D only, grids whose state and fluxes fit in one
 *                    workgroup's LDS: 56 bytes per cell, nx <= 2922 on
 *                    gfx950) one workgroup keeps the whole grid in LDS and
 *                    runs all n steps in one launch;
 *   SVE_PATH_RESIDUAL (2D CFL steps; 1D and fixed-dt steps run as FUSED)
 *                    one kernel per step that applies U - dt R of the
 *                    previous pass and solves the new state's interfaces
 *                    once, keeping the residual R (32 bytes per cell, FP64,
 *                    two buffers allocated on first use) for the next step.
 *                    An interface error of the state reached by a call's
 *                    last step is then found one step early; it is reported
 *                    by the next stepping call, as with the other paths.
 * Results agree across paths to rounding.
 */
#define SVE_PATH_FUSED    0
#define SVE_PATH_SPLIT    1
#define SVE_PATH_RESIDENT 2
#define SVE_PATH_RESIDUAL 3
int sve_set_path(sve_ctx *ctx, int path);

/*
 * Rows per tile of the fused 2D kernel: 1..65536, or 0 (the default) for an
 * automatic split.  Each wavefront owns 61 columns x about `rows` rows
 * (tile heights differ by at most one) and recomputes one row and one
 * column around them, so taller tiles cost less redundant work but give
 * fewer wavefronts.  The automatic split makes the tiles as short as keeps
 * every wavefront of a step resident on the device at once (two per SIMD),
 * with at least 8 rows each.  Results do not depend on it.  SVE_ERR_ARG for
 * values outside that range.
 */
int sve_set_tile_rows(sve_ctx *ctx, int rows);

/*
 * Overwrite one value of the device state (field 0..3 = h, hu, hv, z_b; k a
 * cell index).  Used to test the device-side error detection.
 */
int sve_debug_poke(sve_ctx *ctx, int field, long long k, double value);

/*
 * Time, in milliseconds, of the last sve_step / sve_step_fixed_dt call
 * between HIP events recorded on the context's stream around its launches.
 */
int sve_last_elapsed_ms(sve_ctx *ctx, double *ms);

#ifdef __cplusplus
}
#endif
#endif /* SVE_H */

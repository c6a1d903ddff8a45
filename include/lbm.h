/*
 * lbm.h -- C-ABI of the curved-space D3Q19 lattice Boltzmann library (liblbm.so)
 *
 * Method: the second-order curved-space lattice Boltzmann scheme of Flouris et
 * al., "Fluid structure interaction with curved space lattice Boltzmann"
 * (arXiv 1803.07822): Eq. (CE-LB) split into collision Eq. (collision) and
 * streaming Eq. (streaming), with the metric-dependent Hermite equilibrium
 * (Eq. expansion-equilibrium, App. B), the forcing of Eqs. (forcing2),
 * (forcing-A), (forcing-B), (forcing-C), the geometry of App. A computed with
 * the fourth-order lattice derivative of App. D, the re-projection of the
 * populations on a chart change (Sec. IV.B) and the node-exact wall force
 * (Sec. IV.A.2).
 *
 * Units and lattice: dx = dt = 1, c_s^2 = theta = 1/3.  D3Q19, population
 * order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = (+x+y,-x-y), (+x-y,-x+y),
 * (+x+z,-x-z), (+x-z,-x+z), (+y+z,-y-z), (+y-z,-y+z).
 *
 * Grid: nodes (i,j,k), x fastest.  Layers j = 0 and j = ny-1 are solid walls;
 * fluid layers are j = 1..ny-2 (H = ny-2 of them); x and z are periodic.  The
 * halfway walls sit half a cell outside the first and last fluid layer.
 *
 * Array layouts (all C order; "fluid" = [nz][H][nx]):
 *   chart          double [3][nz][ny][nx]  Cartesian node positions h(xi)
 *   displacement   double [nz][nx]         y-displacement of one wall
 *   wall velocity  double [nz][nx][3]      Cartesian
 *   populations    double [19][fluid]      f_l(x,t), Eq. (streaming)
 *   history        double [10][fluid]      A, B^x, B^y, B^z, C^xx, C^xy,
 *                                          C^xz, C^yy, C^yz, C^zz of F(x,t-1)
 *   geometry       double [28][fluid]      sqrt g, g^xx, g^xy, g^xz, g^yy,
 *                                          g^yz, g^zz, Gamma^i_jk (i = x,y,z;
 *                                          jk = xx,xy,xz,yy,yz,zz), F^x,F^y,F^z
 *   jacobian       double [9][fluid]       J[a][i] = d h^a / d xi^i
 *   rho            double [fluid];  u double [3][fluid]
 *
 * Ownership: every d_* pointer is device memory owned by the caller; it must
 * stay valid until the stream has passed the call.  The workspace (sized by
 * lbm_workspace_bytes) is caller-owned device memory that must outlive the
 * context.  The library never allocates device memory; it allocates only the
 * small host-side context.  Host pointers are marked h_*.
 *
 * Streams: all device work is enqueued on the hip stream given to lbm_create
 * (NULL = the null stream).  Calls return once the work is enqueued, except
 * the sync points (lbm_sync, lbm_moments, lbm_backward) and calls documented
 * as synchronising.
 *
 * Graph capture: lbm_step, lbm_step_force, lbm_couple, lbm_wall_force,
 * lbm_plate_force and the setters a time loop repeats (lbm_set_metric,
 * lbm_set_wall_displacement, lbm_set_wall_velocity,
 * lbm_set_plate_displacement, lbm_set_plate_velocity, lbm_set_body_force)
 * enqueue kernels and device-to-device copies only (no
 * memsets, no host waits), so a sequence of them may be captured on a
 * non-null context stream into a HIP graph and replayed.  The captured work
 * reads the argument pointers of the calls captured, and keeps the choices the
 * context made on the host while it was captured: which of two buffers each
 * call reads and writes (the populations alternate at every step, the chart
 * displacement at every re-projection), and which kernels serve the charts in
 * place (a chart built from wall and plate displacements moves the nodes along
 * y only and takes a cheaper path than a chart given whole).  Replay a
 * sequence that leaves the buffers as it found them (an even number of steps
 * and of re-projections), and do not switch between lbm_set_metric and the
 * displacement setters between its capture and its replays.
 *
 * Errors: every call returns LBM_OK or a negative code; lbm_last_error gives a
 * message.  LBM_EHIP and LBM_EUNSTABLE are sticky: once raised, every later
 * call on the context returns them.  The instability guard (a non-finite
 * population, density <= 0 or |u|^2 > 0.1 at any node) is raised by the
 * kernels and reported at the next sync point.  A context is not thread safe.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef struct {
  int nx, ny, nz; /* ny includes the two solid wall layers */
} lbm_grid;

enum { LBM_D3Q19 = 19 };
/* LBM_FP64: populations, history and geometry stored and computed in FP64.
 * LBM_FP32_DEV: populations stored as deviations f - w_l, history and
 * geometry as FP32 deviations (sqrt g - 1, g^ij - delta^ij, Gamma, F^i),
 * arithmetic in FP32; the geometry itself is computed in FP64. */
enum { LBM_FP64 = 0, LBM_FP32_DEV = 1 };
enum { LBM_WALL_YMIN = 0, LBM_WALL_YMAX = 1 };
enum { LBM_FORCE_STRESS = 0, LBM_FORCE_MEM = 1 };
enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,      /* bad argument */
  LBM_ENOMEM = -2,      /* workspace too small */
  LBM_EHIP = -3,        /* a HIP call failed (sticky) */
  LBM_ESTATE = -4,      /* call out of order */
  LBM_EUNSTABLE = -5,   /* instability guard tripped (sticky) */
  LBM_EUNSUPPORTED = -6 /* option not provided */
};

/* Bytes of device workspace a context needs.  adjoint_K > 0 reserves the
 * trajectory storage of lbm_forward_record/lbm_backward for K steps with a
 * checkpoint every ckpt_every steps (ckpt_every in 1..K).  Returns 0 for an
 * invalid grid (nx, nz >= 1, ny >= 4, nx*(ny-2)*nz < 2^28 fluid nodes) or
 * lattice. */
size_t lbm_workspace_bytes(const lbm_grid* h_grid, int lattice, int precision, int adjoint_K,
                           int ckpt_every);

/* Create a context.  tau > 1/2 is the BGK relaxation time (kinematic
 * viscosity (tau - 1/2)/3, App. C).  d_workspace: bytes >= lbm_workspace_bytes
 * of the same arguments (adjoint sizes from the last two of them are taken as
 * adjoint_K = ckpt_every = 0 unless set with lbm_reserve_adjoint).  The body
 * force is zero and the walls are at rest until set. */
int lbm_create(lbm_ctx** out, const lbm_grid* h_grid, int lattice, double tau, int precision,
               void* d_workspace, size_t bytes, void* hip_stream);

/* Declare the adjoint trajectory sizes the workspace was sized for (before
 * the first metric is set). */
int lbm_reserve_adjoint(lbm_ctx* ctx, int adjoint_K, int ckpt_every);

int lbm_destroy(lbm_ctx* ctx);

/* Cartesian body-force density F_ext (force per physical volume).  It enters
 * B^i of Eq. (forcing-B) as F^i = (J^{-1} F)^i.  Takes effect at the next
 * step (the history of the current state is not rewritten). */
int lbm_set_body_force(lbm_ctx* ctx, const double h_F_cart[3]);

/* Set the chart (node positions, wall layers included) and precompute the
 * geometry of App. A with the fourth-order derivative of App. D (FP64).  The
 * chart is continued three layers beyond each wall layer by the cubic through
 * the four nearest layers.  reproject != 0 carries the current state onto the
 * new chart (Sec. IV.B); it needs a state.  Enqueued on the context's stream
 * like the other setters (capture-safe, see above). */
int lbm_set_metric(lbm_ctx* ctx, const double* d_chart, int reproject);

/* Set the y-displacement d of one wall and rebuild the chart by the linear
 * blending of Sec. IV.A.1 (i):
 *   h = (xi_x, xi_y + (1 - eta/H) d_bot + (eta/H) d_top, xi_z), eta = xi_y - 1/2.
 * The other wall keeps its last displacement (initially 0).  Otherwise as
 * lbm_set_metric. */
int lbm_set_wall_displacement(lbm_ctx* ctx, int wall, const double* d_disp, int reproject);

/* Cartesian velocity of a wall ([nz][nx][3], NULL = at rest; Sec. IV.A.2:
 * the shell's velocity is transformed to the chart, Eq. (vector_transform),
 * and imposed on the fluid at the wall).  It enters the halfway bounce-back
 * as the moving-wall term and the momentum ghost of the lattice gradient, in
 * chart components J^{-1} v at the adjacent fluid node.  The velocity holds
 * until set again; EINVAL for a bad wall.  A NULL clears it with a kernel
 * (capture-safe). */
int lbm_set_wall_velocity(lbm_ctx* ctx, int wall, const double* d_vcart);

/* Initial state f = f_eq(rho, u) (Eq. expansion-equilibrium truncated at
 * second order, App. B) with u = J^{-1} u_cart; d_rho [fluid] (NULL = 1) and
 * d_ucart [3][fluid] (NULL = 0) are FP64 device arrays.  The forcing history
 * F(x, -1) is set to the forcing of this state (Eqs. forcing-A/B/C).  ESTATE
 * before a metric is set. */
int lbm_init_equilibrium(lbm_ctx* ctx, const double* d_rho, const double* d_ucart);

/* Set / read the populations f_l(x,t) (FP64, full values).  Setting recomputes
 * the forcing history from the given state, as lbm_init_equilibrium does. */
int lbm_set_populations(lbm_ctx* ctx, const double* d_f);
int lbm_get_populations(lbm_ctx* ctx, double* d_f);

/* Read the forcing history (coefficients of F(x,t-1)) and the precomputed
 * geometry (d_jac9 may be NULL). */
int lbm_get_history(lbm_ctx* ctx, double* d_coef);
int lbm_get_geometry(lbm_ctx* ctx, double* d_geo28, double* d_jac9);

/* Advance n >= 0 steps: collision, Eq. (collision), with the equilibrium of
 * Eq. (expansion-equilibrium) and the forcing of Eq. (forcing2); streaming,
 * Eq. (streaming), with halfway bounce-back at the walls (and the plate) and
 * the moving-wall term; update of the forcing history.  Asynchronous (the
 * instability guard is reported at the next sync point).  EINVAL for n < 0,
 * ESTATE before a state exists. */
int lbm_step(lbm_ctx* ctx, int n);

/* n >= 0 steps as lbm_step, each also giving the force of the fluid on `wall`
 * (LBM_FORCE_STRESS, as lbm_wall_force: the traction of Sec. IV.A.2 with T
 * from Eq. (fields3)) at the state it steps from: d_forces ([n][3] doubles,
 * device) receives the forces of the states t0 .. t0+n-1, t0 being the state
 * on entry; the force of the state left after the call comes from the next
 * call or from lbm_wall_force.  The fused step forms the traction from the
 * stress its collision computes, so the force costs no launch of its own;
 * grids with a plate or open ends, or with the two-pass step selected, run
 * lbm_wall_force and then the step, with the same result up to rounding.
 * EINVAL for n < 0, a bad wall or a NULL output (n > 0); ESTATE before a
 * state exists.  Capture-safe as lbm_step. */
int lbm_step_force(lbm_ctx* ctx, int n, int wall, double* d_forces);

/* rho = sqrt g sum f, u = (sqrt g sum f c)/rho (Eqs. fields1-2); u in chart
 * components, or Cartesian (J u) if cartesian != 0.  Either output may be
 * NULL.  Checks the instability guard (synchronising). */
int lbm_moments(lbm_ctx* ctx, double* d_rho, double* d_u, int cartesian);

/* Force of the fluid on a wall at the current state, per column (Sec. IV.A.2).
 * LBM_FORCE_STRESS: the node-exact traction sqrt g T^{i y} e_i at the fluid
 * layer next to the wall (sign flipped for the bottom wall), T from
 * Eq. (fields3), e_i = J[.][i].  LBM_FORCE_MEM (a diagnostic, wall at rest
 * only): the momentum exchange of the last step, the sum over the links into
 * the wall of 2 sqrt g J c_l f*_l with f*_l the post-collision population
 * that bounced (EUNSUPPORTED for a wall given a velocity).  d_total3: the sum
 * over columns (3 doubles, device).  d_per_node ([nz][nx][3] or NULL).
 * EINVAL for another method. */
int lbm_wall_force(lbm_ctx* ctx, int wall, int method, double* d_total3, double* d_per_node);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): lbm_wall_force
 * with the same arguments, result and error behaviour, bit for bit, whose
 * reduction scratch (3 doubles per 256 wall columns and a completion counter)
 * lives in a static device array of the library, one per GPU, instead of the
 * context's workspace.  The call allocates nothing and launches one kernel.
 * Limit: nx * nz <= LBM_NOALLOC_MAX_COLUMNS wall columns, else EINVAL.  Every
 * context on a GPU shares that GPU's array: calls that overlap in time on one
 * GPU (contexts on different streams, or threads) race and must be ordered
 * by the caller.  EHIP if the array's address could not be resolved when the
 * context was created. */
enum { LBM_NOALLOC_MAX_COLUMNS = 256 * 2048 };
int lbm_wall_force_noalloc(lbm_ctx* ctx, int wall, int method, double* d_total3, double* d_per_node);

/* One coupling interval with an external structural solver (Sec. IV.A: the
 * fluid receives the wall's position and velocity, the structure receives
 * the traction).  In order, on the context's stream:
 *   - d_disp != NULL: the wall's new displacement [nz][nx]; the state is
 *     re-projected onto the new chart (as lbm_set_wall_displacement with
 *     reproject = 1); NULL keeps the shape;
 *   - the wall's Cartesian velocity d_vcart [nz][nx][3] (NULL = at rest);
 *   - n steps;
 *   - the force of the fluid on the wall at the resulting state into
 *     d_total3 (3 doubles) and, if d_per_node != NULL, per column
 *     [nz][nx][3] (as lbm_wall_force with LBM_FORCE_STRESS).
 * Asynchronous.  EINVAL for a bad wall, n < 0 or d_total3 NULL; ESTATE
 * before a state exists; errors of the composed calls are returned as they
 * occur. */
int lbm_couple(lbm_ctx* ctx, int wall, const double* d_disp, const double* d_vcart, int n, double* d_total3,
               double* d_per_node);

/* Interior plate (Sec. IV.A.1 (ii), Sec. VI.A: the flag, here without its
 * structural model): a thin plate on the half row between fluid rows jp - 1
 * and jp (1 <= jp <= H - 1) over columns i0..i1 (0 <= i0 <= i1 <= nx - 1) and
 * every z.  A link between those two rows whose crossing point x (halfway
 * between its end columns) lies in [i0 - 1/2, i1 + 1/2] is cut: it bounces
 * back halfway, with the moving-plate term, on either face, and the lattice
 * gradient replaces a neighbour across the plate by the mirror ghost of the
 * node on its own side, as at the walls.  A plate over every column also
 * cuts the links through the periodic seam.  jp = 0 removes the plate.  Set
 * it before the state (ESTATE after lbm_init_equilibrium or
 * lbm_set_populations); EINVAL outside the ranges.  It resets the plate's
 * displacement and velocity to zero; with open ends (lbm_set_open_x) the plate
 * keeps 3 columns from each end.  The fused step then runs on 64x4 tiles
 * whatever lbm_set_tuning asked for; the adjoint (lbm_forward_record) is not
 * provided with a plate (EUNSUPPORTED). */
int lbm_set_plate(lbm_ctx* ctx, int jp, int i0, int i1);

/* The plate's cross-section displacement d_disp [nz][nx] (device, the
 * y-displacement of the half row the plate lies on, in every column: the
 * caller continues the plate's shape beyond its ends) builds the chart
 * (Sec. IV.A.1 (ii)): y_c = xi_y + (wall blend of lbm_set_wall_displacement)
 * + D(x, z) S(eta), with S the natural cubic spline through (0, 0),
 * (jp, 1), (H, 0) in eta = xi_y - 1/2 (C^2 across the plate, the walls held
 * in place).  NULL = zero.  reproject as in lbm_set_metric; near the plate
 * the re-projection interpolates from the node's own side only.  ESTATE
 * without a plate or, with reproject, without a state. */
int lbm_set_plate_displacement(lbm_ctx* ctx, const double* d_disp, int reproject);

/* Cartesian plate velocity per column, d_vcart [nz][nx][3] (device; columns
 * off the plate take the nearest plate column's, for the diagonal links at
 * its ends).  NULL = at rest.  ESTATE without a plate. */
int lbm_set_plate_velocity(lbm_ctx* ctx, const double* d_vcart);

/* Node-exact force of the fluid on the plate at the current state: per plate
 * column, the traction sqrt g T^{iy} e_i at the fluid node below the plate
 * minus that at the node above (the two faces' outward normals), as in
 * lbm_wall_force.  d_total3: the sum (3 doubles, device); d_per_column
 * [nz][nx][3] or NULL, zero outside i0..i1.  Asynchronous.  ESTATE without a
 * plate or a state; EINVAL for d_total3 NULL. */
int lbm_plate_force(lbm_ctx* ctx, double* d_total3, double* d_per_column);

/* Open ends in x (Sec. VI.A): x stops being periodic; column 0 is an inlet
 * with the Cartesian velocity d_uin [nz][H][3] (device) and column nx - 1 an
 * outlet.  The streamed values that would arrive from outside are
 * extrapolated linearly from the two next columns in (f - F/2, the part
 * carried by streaming); at the inlet the equilibrium difference
 * f^eq(rho_e, u_in) - f^eq(rho_e, u_e) at the extrapolated moments is added,
 * so the inlet takes the prescribed velocity with its density and
 * non-equilibrium part extrapolated.  The lattice gradient takes the end
 * column's own momentum beyond each end.  The geometry's x-derivatives stay
 * periodic, so the chart must join smoothly across the two ends (an
 * undeformed chart near both ends does).  A fused step is then followed by
 * two small launches that redo the two columns at each end (moments of the
 * three end columns, then the collision).  Those cost a few tens of
 * microseconds whatever the grid, so unless lbm_set_tuning asks for a
 * variant, grids below 2^20 fluid nodes run the two-pass step instead.  NULL
 * restores periodic x.
 * Before the state (ESTATE); EINVAL for nx < 4 or a plate closer than 3
 * columns to an end.  The adjoint is not provided with open ends. */
int lbm_set_open_x(lbm_ctx* ctx, const double* d_uin);

/* Run K steps from the current state and record the force on `wall` at
 * states 1..K into d_forces [K][3]; the initial state and a checkpoint every
 * ckpt_every steps are kept for lbm_backward.  K and ckpt_every must match
 * lbm_reserve_adjoint.  Needs the FP64 form, no interior plate and periodic
 * x.  Walls may move: the velocities set by lbm_set_wall_velocity hold over
 * the K steps. */
int lbm_forward_record(lbm_ctx* ctx, int K, int ckpt_every, int wall, int method, double* d_forces);

/* Reverse sweep of the last lbm_forward_record: given dL/dF [K][3], write
 * dL/d(top-wall displacement) [nz][nx], dL/d(chart) [3][nz][ny][nx] and dL/d
 * f0 [19][fluid] (each may be NULL).  The initial populations f0 are an
 * independent input (the history F(x,-1) is recomputed from f0 and the chart).
 * A moving wall's Cartesian velocity is a constant; its chart components
 * J^{-1} v depend on the chart and are differentiated.
 * ESTATE unless lbm_forward_record ran since the last call that changes the
 * state or the fields it stepped with (every lbm_set_* call except
 * lbm_set_tuning, lbm_init_equilibrium, lbm_step, lbm_reserve_adjoint).
 * The context's state stays the one lbm_forward_record ended with.
 * Synchronising. */
int lbm_backward(lbm_ctx* ctx, const double* d_dL_dF, double* d_grad_disp, double* d_grad_chart,
                 double* d_grad_f0);

/* lbm_step with each kernel of the step bracketed by HIP events on the
 * context's stream: h_ms[k] receives the average duration (ms) of kernel k
 * of the step over the n steps (nslots >= 2: for the two-pass step the
 * moment pass and the collision pass; for the fused step the fused kernel
 * and the end-column passes of a grid with open ends, 0 without them).
 * Synchronising. */
int lbm_step_profiled(lbm_ctx* ctx, int n, double* h_ms, int nslots);

/* Launch shape of the step: zchunk = planes marched per block by the fused
 * step kernel (0 = chosen from the grid size); variant 0 = fused
 * single-kernel step on 64x4 tiles (x by y nodes per block), 1 = two kernels
 * (moment pass, collision pass; what grids with open ends below 2^20 fluid
 * nodes run by default, and otherwise a reference form of the same step).
 * Until this is called the choice is automatic: fused, or two-pass on grids
 * with open ends below 2^20 fluid nodes.  stage = where the fused step keeps
 * a plane's pulled populations between its moment pass and its collision:
 * 0 = nowhere (pulled again, from the caches), 1 = registers (FP32 only;
 * FP64 runs 0), -1 = the default of the precision (1 in FP32, 0 in FP64).
 * Results agree to rounding; only the speed differs.  EINVAL for zchunk < 0,
 * a variant outside 0..1 or a stage outside -1..1. */
int lbm_set_tuning(lbm_ctx* ctx, int zchunk, int variant, int stage);

/* The launch shape the next step will use: *zchunk = planes per block of the
 * fused step (the automatic choice resolved for this device; 0 for the
 * two-kernel variant), *variant as in lbm_set_tuning, *stage = the staging
 * that actually runs (0 in FP64).  EINVAL for a null pointer. */
int lbm_get_tuning(lbm_ctx* ctx, int* zchunk, int* variant, int* stage);

/* Bandwidth calibration, no context: enqueue on hip_stream one kernel that
 * reads 57 planes of n elements from d_in ([57][n]) and writes 29 planes to
 * d_out ([29][n]) with streaming loads and stores, one element per thread:
 * the memory traffic of one fused step over n nodes (populations, history
 * and geometry read; populations and history written) without its
 * arithmetic.  Elements are double for LBM_FP64, float for LBM_FP32_DEV.
 * The caller times it (e.g. with events on the stream).  EINVAL for n < 1,
 * n >= 2^28, null buffers or another precision; EHIP if the launch fails. */
int lbm_stream_probe(int precision, long long n, const void* d_in, void* d_out, void* hip_stream);

/* Wait for the stream and check the instability guard. */
int lbm_sync(lbm_ctx* ctx);

const char* lbm_last_error(const lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */

/*
 * yy.h -- C-ABI of the MI355X (gfx950) library libyy.so: one time step of
 * the second-order artificial-compressibility (AC) direction-splitting
 * scheme for incompressible Navier-Stokes-Boussinesq flow on an overset
 * Yin-Yang spherical shell with MAC finite differences (Takhirov, Frolov &
 * Minev, arXiv 1905.02300).
 *
 * Problem statement (Sec. 1, eq. eq_ns and eq_heat_convec): in the shell
 * R1 <= r <= R2 advance velocity u, pressure p and temperature T under
 *   du/dt + (u.grad)u + grad p - Pr lap u = Pr Ra T e_r,  div u = 0,
 *   dT/dt + u.grad T - lap T = 0,
 * with u = 0 and T = T_wall on both spheres.  The domain is covered by two
 * identical latitude-longitude patches (Sec. 2: Yin, and Yang obtained by
 * (x,y,z) -> (-x,z,y)), each r in [R1,R2], theta in [pi/4-d, 3pi/4+d],
 * phi in [-3pi/4-d, 3pi/4+d], coupled by Schwarz iterations with Lagrange
 * interpolation of boundary data (Sec. 4).  Each step solves the first-order
 * AC system (u1, p1) (eq. ac1) and the bootstrapped second-order system
 * (u2, p2) (eq. ac2); u = u2 and p = p2 are the outputs.
 *
 * General conventions
 *  - Every function returns a yy_status (0 = success).  No exception or
 *    abort crosses the ABI.  A handle is not thread-safe; distinct handles
 *    are independent.
 *  - Memory: the caller allocates one device workspace (size from
 *    yy_workspace_bytes) and owns it and every I/O buffer; the library
 *    allocates no device memory.  The workspace must stay valid until
 *    yy_destroy.  The handle itself is a small host object.
 *  - Streams: all device work is enqueued on the stream passed (NULL = the
 *    default stream) and is asynchronous unless stated.  Only
 *    yy_get_norms synchronises (the stream it is given).
 *  - Field I/O is in double precision whatever the compute precision.
 *    "MAC" layout: the field's unknowns plus its boundary faces, both
 *    patches, [patch][i][j][k], k (phi) fastest: centres (Nr,Nt,Np);
 *    u_r on r-faces (Nr+1,Nt,Np); u_theta on theta-faces (Nr,Nt+1,Np);
 *    u_phi on phi-faces (Nr,Nt,Np+1).  "PADDED" layout: (2,Nr+2,Nt+2,Np+2)
 *    including one ghost layer; logical index -1..N per direction at
 *    storage index 0..N+1, face f at logical index f.
 */
#ifndef YY_H
#define YY_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    YY_OK = 0,
    YY_ERR_ARG = -1,        /* bad argument (null pointer, size, id, value) */
    YY_ERR_GEOMETRY = -2,   /* an overlap-interpolation window would extrapolate */
    YY_ERR_WORKSPACE = -3,  /* workspace too small or misaligned */
    YY_ERR_HIP = -4,        /* a HIP runtime call failed */
    YY_ERR_NONFINITE = -5,  /* a Schwarz or divergence norm was NaN/Inf */
    YY_ERR_STATE = -6       /* call out of order (e.g. step before params) */
} yy_status;

typedef enum { YY_FP64 = 0, YY_FP32_MIXED = 1 } yy_precision;
typedef enum { YY_ADDITIVE = 0, YY_MULTIPLICATIVE = 1 } yy_schwarz_mode;
typedef enum { YY_MAC = 0, YY_PADDED = 1 } yy_layout;
typedef enum { YY_LEVEL_N = 0, YY_LEVEL_NM1 = 1, YY_LEVEL_K = 2 } yy_level;

/* Fields.  T, p1, p2 at cell centres; u*r, u*t, u*p on r-, theta-, phi-faces. */
typedef enum {
    YY_T = 0, YY_U1R, YY_U1T, YY_U1P, YY_P1, YY_U2R, YY_U2T, YY_U2P, YY_P2,
    YY_NFIELDS
} yy_field;

/* Norm slots of yy_get_norms: l2 (midpoint rule, weight r^2 sin(theta)
 * dr dtheta dphi) of each field's iterate increment, and of Div_h u2^k. */
#define YY_NNORMS 10

typedef struct {
    int32_t nr, nt, np;     /* cells per patch along r, theta, phi */
    double r1, r2;          /* shell radii, 0 < r1 < r2 */
    double delta;           /* overlap d; <= 0 selects d = pi/(2(nt-2)),
                               which makes dtheta = d (one-cell overlap) */
} yy_grid;

typedef struct {
    double pr, ra;          /* Prandtl and Rayleigh numbers (Sec. 1) */
    double dt;              /* time step tau > 0 */
    double chi;             /* AC parameter chi > 0 (Sec. 3.3, O(1)) */
    double t_inner, t_outer;/* wall temperatures at r = R1, R2 */
    int32_t mode;           /* yy_schwarz_mode */
} yy_params;

typedef struct yy_shell yy_shell;

/* Bytes of device workspace a shell needs.  prec: yy_precision.
 * Errors: YY_ERR_ARG (null, nr < 2, nt < 6, np < 6, r1 <= 0, r2 <= r1, or
 * one FP64 field -- 2 (nr+2)(nt+2) x (np+2 rounded up to 16) doubles -- of
 * 4 GiB or more, about 2.6e8 cells per patch). */
int yy_workspace_bytes(const yy_grid *g, int32_t prec, uint64_t *bytes);

/* Create a shell on the current device inside the caller's workspace
 * (256-byte aligned, at least yy_workspace_bytes).  Builds, in FP64 on the
 * host, the metric tables (Sec. 2, 3.2) and the overlap-interpolation
 * tables (Sec. 4: donor windows, cubic Lagrange weights, tangential vector
 * rotation per target) and uploads them (synchronously, on the null
 * stream).  Fields start at zero.
 * Errors: YY_ERR_ARG, YY_ERR_GEOMETRY (a target outside its donor span),
 * YY_ERR_WORKSPACE, YY_ERR_HIP.  On error *out is NULL. */
int yy_create(const yy_grid *g, int32_t prec, void *dev_ws, uint64_t ws_bytes, yy_shell **out);

/* Pr, Ra, tau, chi, wall temperatures, Schwarz mode.  Required before
 * yy_step.  Errors: YY_ERR_ARG (dt, chi or pr not > 0, unknown mode). */
int yy_set_params(yy_shell *s, const yy_params *p);

/* Copy one field of one time level from / to a device buffer of doubles in
 * the given layout.  Setting a field marks the shell for a ghost refresh
 * of levels n and n-1 at the next step.  level: yy_level.
 * Errors: YY_ERR_ARG. */
int yy_set_field(yy_shell *s, int32_t field, int32_t level, int32_t layout,
                 const double *dev_src, hipStream_t stream);
int yy_get_field(yy_shell *s, int32_t field, int32_t level, int32_t layout,
                 double *dev_dst, hipStream_t stream);

/* Body forcing of T, u_r, u_theta, u_phi (field = YY_T, YY_U1R, YY_U1T,
 * YY_U1P; it acts on both velocity systems), MAC layout, taken as the value
 * at t^{n+1/2} of the next step; dev_src == NULL removes it.
 * Errors: YY_ERR_ARG. */
int yy_set_forcing(yy_shell *s, int32_t field, const double *dev_src, hipStream_t stream);

/* Dirichlet wall data (the boundary conditions u = u_wall, T = T_wall on
 * r = R1, R2 of eq. eq_ns / eq_heat_convec with given, possibly
 * time-dependent values) of T, u_r, u_theta or u_phi (field = YY_T,
 * YY_U1R, YY_U1T, YY_U1P; both velocity systems take it) for one time
 * level (YY_LEVEL_N: t^n, YY_LEVEL_NM1: t^{n-1}, YY_LEVEL_K: the step's
 * target t^{n+1}) and wall (0: r = R1, 1: r = R2).  dev_src: device doubles
 * [patch][j+1][k+1], j = -1..nt, k = -1..np (2 (nt+2)(np+2) values), at the
 * field's own (theta, phi) positions (theta-faces for u_theta, phi-faces
 * for u_phi, centres otherwise); copied on `stream`.  NULL clears the slot
 * (then T = t_inner / t_outer and u = 0 on that wall).  The fills apply
 * u_r = u_wall on its wall faces and reflection ghosts
 * psi_{-1} = 2 psi_wall - psi_0 for the others.  The slots rotate with the
 * levels at the end of a step; while a field uses wall data, its
 * YY_LEVEL_K slots must be set again before every step (else yy_step
 * returns YY_ERR_STATE).  Errors: YY_ERR_ARG, YY_ERR_HIP. */
int yy_set_wall(yy_shell *s, int32_t field, int32_t level, int32_t wall, const double *dev_src,
                hipStream_t stream);

/* Algorithm step 4 (Sec. 4, optional in the paper): on = 1 corrects, after
 * every velocity fill and for both systems, the interpolated boundary
 * normal velocities of each patch (u_theta on its theta-boundary faces,
 * u_phi on its phi-boundary faces) so that, with the wall data, the
 * patch's boundary carries no net mass flux.  The correction is the
 * minimiser of the paper's functional J (the point its conjugate-gradient
 * iteration converges to): v = u_bd - (F / (eps |dOmega|^2 + a.a)) a, with
 * a the faces' outward flux weights (the face areas of Div_h), F the net
 * flux of u_bd and the wall data, |dOmega| the area of the patch's
 * boundary; by default eps = 0 (the limit: no net flux left) and it is
 * applied whatever F (see yy_set_mass_fix_params).  on = 0 (default) turns
 * it off.  Errors: YY_ERR_ARG. */
int yy_set_mass_fix(yy_shell *s, int32_t on);

/* The parameters of step 4: eps >= 0, the penalty parameter of J (the
 * paper's epsilon; 0: the limit), and tol >= 0, the net flux below which a
 * patch's data are left uncorrected (the paper's test |F| >= tol; 0:
 * always corrected).  Errors: YY_ERR_ARG (negative or NaN). */
int yy_set_mass_fix_params(yy_shell *s, double eps, double tol);

/* Algorithm step 7 (Sec. 4: after the pressure update of a patch,
 * interpolate the pressure near its boundary from the other patch; the
 * remark after the Algorithm states that the exchanged pressure enters the
 * pressure gradient of eqs. r_comp - phi_comp and that skipping it slows
 * the Schwarz iteration).  nring > 0: after every update of p1 and of p2
 * (both systems), the outermost nring cells of each patch in theta and phi
 * (cells with j < nring, j >= nt - nring, k < nring or k >= np - nring, at
 * every radial index) take the other patch's pressure, interpolated at
 * their centres by the cubic Lagrange rule of the ghost fill, instead of
 * the AC update; they leave the pressure increment norms (the divergence
 * norm still covers them).  In the additive mode every target of both
 * patches is gathered before any is written.  (In this MAC layout no
 * momentum stencil reads a pressure ghost, so the exchange acts through
 * the patch's own outermost cells.)  nring = 0 (default) turns it off.
 * Uploads a table synchronously (null stream).
 * Errors: YY_ERR_ARG (nring < 0 or > 8, 2 nring >= nt or np),
 * YY_ERR_GEOMETRY (a ring centre outside the other patch's span of
 * centres: the one-cell overlap leaves room for one ring, two on coarse
 * grids), YY_ERR_HIP. */
int yy_set_pressure_exchange(yy_shell *s, int32_t nring);

/* Wall condition of T on one wall (0: r = R1, 1: r = R2): the Robin form
 * a T + b dT/dn = g (n the outward normal; a, b >= 0, a + b > 0), which
 * the paper states its method can take in place of Dirichlet data
 * (Sec. 1).  g is the wall data of T (yy_set_wall) or else the constant
 * wall temperature of yy_params.  Discretised on the cell pair across the
 * wall (T_wall their mean, dT/dn their outward difference over dr): the
 * ghost is (g - T_in (a/2 - b/dr)) / (a/2 + b/dr), and the r-line
 * corrections of T take c_ghost = -(a/2 - b/dr)/(a/2 + b/dr) c_in.
 * Default (1, 0): Dirichlet.
 * Errors: YY_ERR_ARG. */
int yy_set_t_bc(yy_shell *s, int32_t wall, double a, double b);

/* Wall condition of the tangential velocity (u_theta and u_phi, both
 * systems) on one wall of radius R (0: R1, 1: R2): the Robin form
 * a u + b R dn(u/r) = g (n the outward normal; a, b >= 0, a + b > 0), the
 * Neumann/Robin class the paper states its method can take (Sec. 1).
 * (0, 1) with g = 0 is the stress-free wall: with u_r = 0 on the wall the
 * tangential stress is proportional to R d(u_t/r)/dr.  g is the wall data
 * of u_theta / u_phi (yy_set_wall) or 0.  Discretised on the cell pair
 * across the wall (centres r_g outside, r_i inside): u_wall the mean of
 * the pair, dn(u/r) = (u_g/r_g - u_i/r_i)/dr, so the ghost is
 * u_g = cg g - rho u_i with cg = 1/(a/2 + b R/(r_g dr)) and
 * rho = (a/2 - b R/(r_i dr)) cg; the r-line corrections take
 * c_ghost = -rho c_in.  u_r stays Dirichlet (no penetration).  Default
 * (1, 0): Dirichlet.  Errors: YY_ERR_ARG. */
int yy_set_u_bc(yy_shell *s, int32_t wall, double a, double b);

/* Advance one time step n -> n+1 with n_schwarz Schwarz iterations
 * (Sec. 4 Algorithm with the splitting-error reduction eq. er): per
 * iteration, refresh every field's ghosts from the other patch, solve T,
 * u1 (r, theta, phi), p1, u2 (r, theta, phi), p2, each velocity/T solve as
 * a residual and three direction-split tridiagonal sweeps (Sec. 4).
 * Asynchronous.  Errors: YY_ERR_ARG (n_schwarz < 1 or > 64), YY_ERR_STATE
 * (params not set, or wall data in use without this step's YY_LEVEL_K
 * values), YY_ERR_HIP. */
int yy_step(yy_shell *s, int32_t n_schwarz, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * step of yy_step (same arguments, same result bit for bit), with its
 * scratch arrays -- the residual/correction buffer, the Thomas scratch
 * (each at most 32 MiB: 2 (nr+2)(nt+2) x padded row of compute-precision
 * elements, e.g. grids up to about 2x32x96x288 in FP64), the norm partial
 * sums and the mass-flux partials -- in one static device array of the
 * library (about 67 MiB, one copy per GPU the library runs on, held until
 * the process ends; its address is looked up once per device) instead of
 * the workspace.  It calls no allocating routine.  The array is shared by
 * every call on that GPU and cleared at the start of each call (by a
 * kernel on `stream`): calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.
 * Errors: as yy_step; YY_ERR_WORKSPACE if the grid's scratch does not fit
 * the static array; YY_ERR_HIP if its address cannot be obtained. */
int yy_step_static(yy_shell *s, int32_t n_schwarz, hipStream_t stream);

/* One time step with the paper's tolerance-driven Schwarz loop (Sec. 5.1:
 * iterate until the l2 norm of the difference of two successive iterates
 * of every computed quantity is below a tolerance).  After each iteration
 * the increment norms of T, u1, p1, u2, p2 on both patches come to the
 * host (the stream is synchronised once per iteration); the loop stops at
 * the first iteration whose norms are all below tol, or after kmax.
 * *k_done receives the number of iterations run; yy_get_norms returns
 * their norms.  Not for use under stream capture.
 * Errors: YY_ERR_ARG (null, kmax < 1 or > 64, tol < 0 or not finite),
 * YY_ERR_STATE, YY_ERR_NONFINITE (a norm is NaN/Inf: the step is abandoned
 * and the handle keeps the error), YY_ERR_HIP. */
int yy_step_tol(yy_shell *s, int32_t kmax, double tol, int32_t *k_done, hipStream_t stream);

/* Norms of the last step, synchronising the stream: out[k][patch][slot]
 * for k < n_schwarz, slot order T,u1r,u1t,u1p,p1,u2r,u2t,u2p,p2,div(u2).
 * Returns the number of values available (it writes at most cap), or
 * YY_ERR_NONFINITE if any is NaN/Inf (the values are still written). */
int yy_get_norms(yy_shell *s, double *host_out, int32_t cap, hipStream_t stream);

/* Release the handle (the workspace stays the caller's). */
int yy_destroy(yy_shell *s);

/* Static description of a status code. */
const char *yy_strerror(int status);

/* ---- pieces of the step, for kernel-level tests and benchmarks ---- */

/* Internal padded layout of compute-precision arrays: dims = {2, nr+2,
 * nt+2, pitch} (elements); within each row of `pitch` elements the points
 * k = -1 .. np occupy elements k_first .. k_first+np+1 (k = 0 lands on a
 * 128-byte boundary; the other elements are padding).  elem_bytes = 8 or
 * 4.  elem_bytes and k_first may be NULL. */
int yy_internal_dims(const yy_shell *s, int64_t dims[4], int32_t *elem_bytes, int32_t *k_first);

/* Refresh ghosts and boundary faces of every field at `level` from the
 * other patch, then apply the wall rules. */
int yy_fill(yy_shell *s, int32_t level, hipStream_t stream);

/* psi* = 1.5 psi^n - 0.5 psi^{n-1} for T and both velocities. */
int yy_extrapolate(yy_shell *s, hipStream_t stream);

/* One direction-split solve (I - tau/2 L_{field,dir}) y = x along every
 * line of direction dir (0 = r, 1 = theta, 2 = phi) on both patches, with
 * the coefficients of field's split operator (Sec. 3.2-3.3; advection by
 * the current extrapolated u2).  x, y: device arrays in the internal
 * layout and compute precision; only the field's unknowns are read and
 * written; x == y is allowed.  Errors: YY_ERR_ARG. */
int yy_sweep(yy_shell *s, int32_t field, int32_t dir, const void *dev_x, void *dev_y,
             hipStream_t stream);

/* The same line solve with coefficients from the metric tables only (no
 * advection) for a cell-centred scalar: the factors (I - tau/2 Pr D) with
 * D = D_rr, and for metric = 0 the paper's split operators Dhat_thth,
 * Dhat_phph (Sec. 3.2), for metric = 1 the true D_thth, D_phph.
 * Errors: YY_ERR_ARG, YY_ERR_STATE (params not set). */
int yy_sweep_diffusion(yy_shell *s, int32_t dir, int32_t metric, const void *dev_x, void *dev_y,
                       hipStream_t stream);

/* tau * R^k of a field for the current working iterate (internal layout,
 * compute precision, written at the unknowns only). */
int yy_residual(yy_shell *s, int32_t field, void *dev_out, hipStream_t stream);

/* ---- line-solver autotuning ---- */

/* Time every tile variant of the partitioned line solves of this shell
 * (strided r/theta sweeps: the per-line Thomas kernel, "t", or rows per
 * chunk 4/6/8/12/16 x lane width 64/32/16, "m<rows>w<lanes>", where the
 * lines fit, each also with all loads of a chunk issued together,
 * "m<rows>w<lanes>b"; phi sweeps: one wave per line with 1/2/4 lines per
 * block, "l<lines>", or 2/4/8 waves per line, "v<waves>"), each on the
 * shell's own scratch buffer with its current advecting velocity and in
 * the form the step launches it (the last factor of an unknown fused with
 * its update and norm), and those of the diffusion-only line solves
 * (yy_sweep_diffusion, keys "D.r", "D.t", "D.p"), keep the fastest per
 * (unknown or "D", direction); then the column tile of each residual
 * (keys "res.T", "res.u_r", "res.u_t", "res.u_p": a 256-thread block of
 * k x j columns, "64x4", "128x2", "256x1", "32x8" or "16x16", taken by
 * consecutive blocks k-tile first, "k", or j-tile first, "j"; or 64 x 4,
 * 8 or 16 columns with the theta/phi neighbours staged in LDS, "lds64x4k",
 * "lds64x8k", "lds64x8j", "lds64x16k"); each partitioned line solve
 * is also timed with 1536 and 2048 blocks per patch in place of the
 * default 1024, each block looping over its lines or line tiles, and where
 * one is faster the choice is written as "<unknown>.<dir>.blocks":"<n>"),
 * and
 * write the choices as a JSON object (a NUL-terminated string of at most
 * cap bytes) to json_out if not NULL.
 * Synchronises the stream.  Needs params.  Errors: YY_ERR_ARG,
 * YY_ERR_STATE, YY_ERR_HIP. */
int yy_autotune(yy_shell *s, char *json_out, int32_t cap, hipStream_t stream);

/* The shell's current tile choices in the JSON form of yy_autotune
 * (NUL-terminated).  Errors: YY_ERR_ARG (null, or cap too small). */
int yy_get_tuning(yy_shell *s, char *json_out, int32_t cap);

/* Apply choices written by yy_autotune (a tuning cache).  Unknown keys are
 * ignored.  Optional keys "res.<unknown>.seg":"<n>" (n = 0..64) split each
 * residual column's radial points into n segments run by separate blocks
 * (0, the default: the count that best fills the device's last round of
 * resident blocks, at most 4); every count gives bitwise the same residual.
 * yy_get_tuning writes them only where n > 0.  Likewise optional keys
 * "<unknown>.<dir>.blocks":"<n>" (n = 0 or 8..16384): blocks per patch of
 * that partitioned line solve (0: the default, 1024).  Errors: YY_ERR_ARG
 * (NULL or malformed). */
int yy_set_tuning(yy_shell *s, const char *json);

/* ---- ensembles: many independent shells advanced by one graph ---- */

typedef struct yy_ensemble yy_ensemble;

/* Total workspace of an ensemble of n shells (grids[0..n-1], one
 * precision), each shell's part 256-byte aligned.  Errors: YY_ERR_ARG. */
int yy_ensemble_workspace_bytes(int32_t n, const yy_grid *grids, int32_t prec, uint64_t *bytes);

/* Create n shells inside one caller workspace.  Each shell is then set up
 * and read through the single-shell calls on yy_ensemble_shell(e, s).
 * Errors: as yy_create for any shell; on error *out is NULL. */
int yy_ensemble_create(int32_t n, const yy_grid *grids, int32_t prec, void *dev_ws, uint64_t ws_bytes,
                       yy_ensemble **out);

/* Handle of shell s (0 <= s < n), or NULL. */
yy_shell *yy_ensemble_shell(yy_ensemble *e, int32_t s);

/* Advance every shell one time step with n_schwarz Schwarz iterations.
 * The first call (and the first after any field or parameter change)
 * runs eagerly where a ghost refresh is pending, then captures the step of
 * all shells into hipGraphs (one per phase of the time-level rotation) and
 * replays them on later calls.
 * graph = 1: batched -- each launch of the step covers every shell: the
 * shells' launches at one position of the step are grouped by kernel
 * instance (tile) and block shape, and each group is one launch over a
 * work list in which every shell owns a range of blocks (argument and
 * block tables in the ensemble's workspace); the shells are dealt to up
 * to four branches of similar cell counts, which the graph runs side by
 * side.  Shells whose steps do not line up (different Schwarz modes), with
 * the mass-flux correction or the pressure exchange, n_schwarz > 8, or
 * launch tables that exceed the ensemble's arena fall back to graph = 2.
 * graph = 2: one forked stream per shell inside the graph.
 * graph = 0 enqueues the shells one after another on the stream instead.
 * A single-shell step (yy_step, yy_step_tol, yy_step_static) on a member
 * between graph steps is allowed: the graphs are captured again.  Shells
 * with Dirichlet wall data (yy_set_wall) need new values every step, so
 * graph = 1 and 2 refuse them (YY_ERR_STATE, nothing advanced); graph = 0
 * steps them.  A failed capture leaves every shell's time levels as they
 * were.
 * Errors: YY_ERR_ARG, YY_ERR_STATE (a shell without params, or with wall
 * data under graph = 1 or 2), YY_ERR_HIP. */
int yy_ensemble_step(yy_ensemble *e, int32_t n_schwarz, int32_t graph, hipStream_t stream);

/* Tile autotuning of an ensemble: every shell is tuned (yy_autotune), then
 * one tile is kept per (unknown or diffusion-only, direction, line-length
 * bucket 2^(b-1) < n <= 2^b) -- that of the bucket's largest shell -- and
 * per (unknown, phi-extent bucket) for the residual columns, so that the
 * batched launches group shells of similar lines.  The bucket choices go to
 * json_out (NUL-terminated, at most cap bytes) if not NULL.  Synchronises
 * the stream.  Errors: as yy_autotune. */
int yy_ensemble_autotune(yy_ensemble *e, char *json_out, int32_t cap, hipStream_t stream);

/* Whether the captured graphs hold batched launches (1) or per-shell
 * streams (0, or not captured yet), the number of batched launches per
 * step, and the number of the shells' own launches per step that they
 * replace (both 0 unless batched).  Any output may be NULL.
 * Errors: YY_ERR_ARG. */
int yy_ensemble_info(const yy_ensemble *e, int32_t *batched, int64_t *launches_per_step,
                     int64_t *shell_launches_per_step);

int yy_ensemble_destroy(yy_ensemble *e);

/* ---- measurement ---- */

/* Plain streaming copy of `bytes` bytes from device memory src to dst (both
 * 16-byte aligned, bytes a multiple of 16, non-overlapping) on `stream`:
 * the HBM rate a kernel that reads and writes every word once reaches, the
 * practical ceiling of the step's streaming kernels.  Not part of a step.
 * Errors: YY_ERR_ARG (null, misaligned or bytes not a multiple of 16),
 * YY_ERR_HIP (launch). */
int yy_stream_copy(void *dst, const void *src, uint64_t bytes, hipStream_t stream);

/* ---- live per-kernel timing (HIP events on the caller's stream) ---- */

/* Kernel classes timed by the profiler. */
#define YY_NPROF 17

/* enable != 0: start recording a hipEvent pair around every kernel launch
 * group of later calls (previous records are dropped); 0: stop. */
int yy_profile(yy_shell *s, int32_t enable);

/* Synchronise the stream and return, per kernel class (index < YY_NPROF),
 * the summed elapsed milliseconds and the number of timed launch groups
 * since yy_profile(s, 1).  Returns YY_NPROF. */
int yy_profile_read(yy_shell *s, double *ms, int64_t *count, hipStream_t stream);

/* Name of a kernel class ("sweep_p_last", ...), or NULL if out of range. */
const char *yy_profile_name(int32_t cls);

#ifdef __cplusplus
}
#endif
#endif

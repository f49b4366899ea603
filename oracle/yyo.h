/*
 * yyo.h -- plain FP64 CPU oracle of the Yin-Yang artificial-compressibility
 * direction-splitting time step (Takhirov, Frolov & Minev, "A direction
 * splitting scheme for Navier-Stokes-Boussinesq system in spherical shell
 * geometries", arXiv 1905.02300).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product
 * path (the HIP library declared in include/yy.h) never calls, links or
 * includes anything from this directory, and this directory includes
 * nothing from the product.
 *
 * Conventions (shared with the product only through the written scheme):
 *   - both patches are stored, patch 0 = Yin, patch 1 = Yang;
 *   - every field array of one patch has (nr+2)*(nt+2)*(np+2) doubles,
 *     logical indices -1..N in each direction, phi (k) fastest;
 *     a face index f (0..N) is stored at logical index f;
 *   - "MAC" layout = the field's unknowns plus its boundary faces, no
 *     ghosts: centre (nr,nt,np), r-face (nr+1,nt,np), theta-face
 *     (nr,nt+1,np), phi-face (nr,nt,np+1), per patch, patch slowest.
 */
#ifndef YYO_H
#define YYO_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum { YYO_T = 0, YYO_U1R, YYO_U1T, YYO_U1P, YYO_P1,
       YYO_U2R, YYO_U2T, YYO_U2P, YYO_P2, YYO_NF };
enum { YYO_LEV_N = 0, YYO_LEV_NM1 = 1, YYO_LEV_K = 2 };
enum { YYO_MAC = 0, YYO_PADDED = 1 };
/* explicit one-direction operators for yyo_apply_op */
enum { YYO_OP_DRR = 0, YYO_OP_DTT, YYO_OP_DTT_HAT, YYO_OP_DPP, YYO_OP_DPP_HAT,
       YYO_OP_LR, YYO_OP_LT, YYO_OP_LP };

typedef struct yyo yyo;

/* Create a shell.  delta <= 0 selects the one-cell overlap
 * delta = pi / (2 (nt - 2)).  Returns NULL on bad arguments or when a
 * donor window of the overlap interpolation would extrapolate. */
yyo *yyo_create(int nr, int nt, int np, double r1, double r2, double delta);
void yyo_destroy(yyo *h);
/* pr, ra, tau (time step), chi (AC parameter), wall temperatures */
int yyo_set_params(yyo *h, double pr, double ra, double tau, double chi,
                   double t_inner, double t_outer);
/* 1: print a progress line on stderr after every Schwarz iteration */
int yyo_set_verbose(yyo *h, int on);
/* 0 = additive Schwarz (default), 1 = multiplicative (Yin then Yang) */
int yyo_set_mode(yyo *h, int mode);
/* 1: correct the interpolated boundary normal velocities of every velocity
 * fill so that each patch's boundary carries no net mass flux (Algorithm
 * step 4, optional in the paper); 0 (default): off */
int yyo_set_mass_fix(yyo *h, int on);
/* epsilon of step 4's functional (0: the limit, no net flux left) and the
 * flux below which the correction is skipped (0: always applied) */
int yyo_set_mass_fix_params(yyo *h, double eps, double tol);
/* Algorithm step 7 (pressure exchange): nring > 0 makes the outermost
 * nring cells of each patch (in theta and phi, every radial index) take,
 * after every pressure update of p1 and p2, the other patch's pressure
 * interpolated at their centres, in place of the AC update (they leave
 * the pressure increment norms).  0 (default) turns it off.  Returns -1
 * if nring < 0, 2 nring >= nt or np, or a ring cell lies outside the
 * other patch's centre span. */
int yyo_set_pressure_exchange(yyo *h, int nring);
/* Robin condition a T + b dT/dn = g on a wall (0: R1, 1: R2; n the outward
 * normal), a, b >= 0, a + b > 0; g = the wall data of T or the constant
 * wall temperature.  Default (1, 0): Dirichlet. */
int yyo_set_t_bc(yyo *h, int wall, double a, double b);
/* Robin condition a u + b R dn(u/r) = g of the tangential velocity (both
 * components, both systems) on a wall of radius R (0: R1, 1: R2; n the
 * outward normal), a, b >= 0, a + b > 0; g = the wall data of u_theta /
 * u_phi or 0.  (0, 1): stress-free.  Default (1, 0): Dirichlet.  u_r stays
 * Dirichlet (no penetration). */
int yyo_set_u_bc(yyo *h, int wall, double a, double b);
int64_t yyo_field_count(const yyo *h, int field, int layout);
int yyo_set_field(yyo *h, int field, int level, int layout, const double *src);
int yyo_get_field(const yyo *h, int field, int level, int layout, double *dst);
/* forcing of T, u_r, u_theta, u_phi (fields YYO_T, YYO_U1R, YYO_U1T,
 * YYO_U1P; it applies to both velocity systems), MAC layout; NULL clears */
int yyo_set_forcing(yyo *h, int field, const double *src);
/* Dirichlet wall data of T, u_r, u_theta or u_phi (field YYO_T, YYO_U1R,
 * YYO_U1T, YYO_U1P; both velocity systems take it) for one level (n, n-1,
 * or the iterate k, i.e. time t^{n+1}) and wall (0: r = R1, 1: r = R2):
 * doubles [patch][j+1][k+1], j = -1..nt, k = -1..np, at the field's own
 * (theta, phi) positions.  NULL clears (T = t_inner / t_outer, u = 0).
 * The data rotates with the levels at the end of a step. */
int yyo_set_wall(yyo *h, int field, int level, int wall, const double *src);
/* Advance one time step with K Schwarz iterations. */
int yyo_step(yyo *h, int K);
/* Advance one time step, iterating until every increment norm of an
 * iteration (T, u1, p1, u2, p2, both patches) is below tol, at most kmax
 * (<= 64) iterations.  Returns the iteration count, or -1 on bad input. */
int yyo_step_tol(yyo *h, int kmax, double tol);
/* norms of the last step: out[k][patch][10] = per-field l2 norms of the
 * iterate increment (T,u1r,u1t,u1p,p1,u2r,u2t,u2p,p2) and of Div_h u2^k */
int yyo_get_norms(const yyo *h, double *out, int cap);

/* ---- pieces of the step, exposed for the pin tests ---- */
/* fill ghosts/boundary faces of every field at `level` from the other
 * patch, then apply the wall rules */
int yyo_fill(yyo *h, int level);
/* one direction-split solve (I - tau/2 L_{field,dir}) y = x on every line;
 * x, y padded arrays of both patches (only unknowns are read/written;
 * other points of y are set to zero) */
int yyo_sweep(yyo *h, int field, int dir, const double *x, double *y);
/* apply an explicit operator at the field's unknowns (padded in/out) */
int yyo_apply_op(yyo *h, int field, int op, const double *x, double *y);
/* (I - tau/2 Pr D) y = x along the direction of D = D_rr, D_thth,
 * Dhat_thth, D_phph or Dhat_phph (op YYO_OP_DRR..YYO_OP_DPP_HAT) for the
 * centre unknowns (padded layout); zero at theta/phi ghosts, reflection at
 * the walls.  The line-solve workload with the paper's split operators
 * (hat) or the true metric. */
int yyo_sweep_op(yyo *h, int op, const double *x, double *y);
/* the residual R^k of a field (padded out, zero off the unknowns) for the
 * current working iterate; s = velocity system (1 or 2) */
int yyo_residual(yyo *h, int field, double *out);
/* extrapolated levels psi* = 1.5 psi^n - 0.5 psi^{n-1} for every field */
int yyo_extrapolate(yyo *h);
/* plain Thomas algorithm: lo[0] and up[n-1] are ignored */
int yyo_thomas(int n, const double *lo, const double *di, const double *up,
               const double *rhs, double *x);
/* coordinates of the Yang image of a Yin point (and vice versa) */
void yyo_involution(double th, double ph, double *th2, double *ph2);
/* 2x2 matrix taking (v_th, v_ph) of the other patch at the image point to
 * this patch's components at (th, ph) */
void yyo_rotation(double th, double ph, double m[4]);
int yyo_omp_threads(void);
/* threads of the following calls (n <= 0: one per host core) */
void yyo_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif

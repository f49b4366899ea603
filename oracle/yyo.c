/*
 * yyo.c -- plain FP64 CPU oracle of the Yin-Yang artificial-compressibility
 * direction-splitting time step of Takhirov, Frolov & Minev (arXiv 1905.02300).
 *
 * TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it; the product path never does.  It
 * shares no source with the HIP library.
 *
 * Written for a reader holding the paper.  Every function cites the
 * section / equation it follows.  No blocking, fusion or reordering beyond
 * the scheme itself; lines are solved by the Thomas algorithm; reductions
 * are serial and in a fixed order.  OpenMP only distributes independent
 * points and lines.  Build: -O2 -ffp-contract=off, no fast-math.
 *
 * The discrete scheme (readings of garbled or silent passages are marked
 * "reading"):
 *   grid (Sec. 2): per patch r in [R1,R2], theta in [pi/4-d, 3pi/4+d],
 *     phi in [-3pi/4-d, 3pi/4+d], uniform cells; MAC staggering (Sec. 4):
 *     T, p at centres, u_r / u_theta / u_phi at r / theta / phi faces.
 *   time scheme (Sec. 3, eq. HeatDouglas generalised; reading): for each
 *     unknown psi with split operators L_r + L_t + L_p = Lhat and full
 *     operator F,  (psi^{n+1}-psi^n)/tau = Lhat psi^{n+1/2}
 *     + (F - Lhat) psi^{*} + S, solved by the factored operator
 *     prod_d [I - tau/2 L_d] in the correction form of eq. er (sign read
 *     so that its fixed point is this scheme).
 */
#include "yyo.h"
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NLEV 3
#define MAXK 64
#define NNORM 10

enum { CC = 0, FR = 1, FT = 2, FP = 3 };   /* MAC locations */

struct yyo {
    int nr, nt, np;
    double r1, r2, delta;
    double dr, dth, dph, th0, ph0, th1;
    double pr, ra, tau, chi, t_in, t_out;
    int mode;
    int mass_fix;                /* Algorithm step 4 on every velocity fill */
    double mf_eps, mf_tol;       /* its epsilon (0: the limit) and flux trigger */
    int nring;                   /* Algorithm step 7: rings of pressure cells taken
                                    from the other patch (0: off) */
    double *ptmp;                /* gathered ring pressures (both patches) */
    double t_bc[2][2];           /* T walls: a T + b dT/dn = g, (a, b) per wall */
    double u_bc[2][2];           /* tangential velocity walls: a u + b R dn(u/r) = g */
    int64_t npatch;              /* doubles per patch array */
    double *lev[YYO_NF][NLEV];   /* levels n, n-1, working iterate k */
    double *star[YYO_NF];        /* 1.5 psi^n - 0.5 psi^{n-1} */
    double *force[4];            /* T, u_r, u_theta, u_phi (padded) */
    /* wall data of T, u_r, u_theta, u_phi per level and wall (0: r = R1,
     * 1: r = R2): [patch][j+1][k+1] at the field's own (theta, phi)
     * positions, or NULL (T = t_in / t_out, u = 0) */
    double *wall[4][NLEV][2];
    double *res, *wa, *wb;
    double norms[MAXK][2][NNORM];
    int nk, filled;
    int verbose;                 /* progress line per Schwarz iteration */
};

/* ------------------------------------------------------------------ */
/* grid helpers                                                        */
/* ------------------------------------------------------------------ */
static int loc_of(int f)
{
    switch (f) {
    case YYO_U1R: case YYO_U2R: return FR;
    case YYO_U1T: case YYO_U2T: return FT;
    case YYO_U1P: case YYO_U2P: return FP;
    default: return CC;
    }
}
/* is location `loc` face-centred in direction d (0=r, 1=theta, 2=phi)? */
static int is_face(int loc, int d) { return loc == d + 1; }
static int ncell(const yyo *h, int d) { return d == 0 ? h->nr : (d == 1 ? h->nt : h->np); }
/* first and last unknown index along d: faces 1..N-1, centres 0..N-1 */
static int ulo(int loc, int d) { return is_face(loc, d) ? 1 : 0; }
static int uhi(const yyo *h, int loc, int d) { return ncell(h, d) - 1; }
/* MAC layout range: faces 0..N, centres 0..N-1 */
static int mhi(const yyo *h, int loc, int d) { return is_face(loc, d) ? ncell(h, d) : ncell(h, d) - 1; }

static inline int64_t ix(const yyo *h, int p, int i, int j, int k)
{
    return (int64_t)p * h->npatch +
           ((int64_t)(i + 1) * (h->nt + 2) + (j + 1)) * (h->np + 2) + (k + 1);
}

static double rc(const yyo *h, int i) { return h->r1 + (i + 0.5) * h->dr; }
static double rf(const yyo *h, int f) { return h->r1 + f * h->dr; }
static double tc(const yyo *h, int j) { return h->th0 + (j + 0.5) * h->dth; }
static double tf(const yyo *h, int f) { return h->th0 + f * h->dth; }
static double pc(const yyo *h, int k) { return h->ph0 + (k + 0.5) * h->dph; }
static double pf(const yyo *h, int f) { return h->ph0 + f * h->dph; }
static double r_at(const yyo *h, int loc, int i) { return is_face(loc, 0) ? rf(h, i) : rc(h, i); }
static double t_at(const yyo *h, int loc, int j) { return is_face(loc, 1) ? tf(h, j) : tc(h, j); }
static double p_at(const yyo *h, int loc, int k) { return is_face(loc, 2) ? pf(h, k) : pc(h, k); }

/* ------------------------------------------------------------------ */
/* Yin-Yang geometry (Sec. 2)                                          */
/* ------------------------------------------------------------------ */
/* The Yang map (x,y,z) -> (-x,z,y) is its own inverse, so one formula
 * takes a point of either patch to the other patch's coordinates. */
void yyo_involution(double th, double ph, double *th2, double *ph2)
{
    double x = sin(th) * cos(ph), y = sin(th) * sin(ph), z = cos(th);
    double xb = -x, yb = z, zb = y;          /* other patch's frame */
    if (zb > 1.0) zb = 1.0;
    if (zb < -1.0) zb = -1.0;
    *th2 = acos(zb);
    *ph2 = atan2(yb, xb);
}

/* Local spherical unit vectors of the other patch, expressed in this
 * patch's Cartesian frame, dotted with this patch's unit vectors. */
void yyo_rotation(double th, double ph, double m[4])
{
    double th2, ph2;
    yyo_involution(th, ph, &th2, &ph2);
    double et[3] = { cos(th) * cos(ph), cos(th) * sin(ph), -sin(th) };
    double ep[3] = { -sin(ph), cos(ph), 0.0 };
    /* other frame's basis in its own frame */
    double et2o[3] = { cos(th2) * cos(ph2), cos(th2) * sin(ph2), -sin(th2) };
    double ep2o[3] = { -sin(ph2), cos(ph2), 0.0 };
    /* map back with (x,y,z) -> (-x,z,y) */
    double et2[3] = { -et2o[0], et2o[2], et2o[1] };
    double ep2[3] = { -ep2o[0], ep2o[2], ep2o[1] };
    m[0] = et[0] * et2[0] + et[1] * et2[1] + et[2] * et2[2];
    m[1] = et[0] * ep2[0] + et[1] * ep2[1] + et[2] * ep2[2];
    m[2] = ep[0] * et2[0] + ep[1] * et2[1] + ep[2] * et2[2];
    m[3] = ep[0] * ep2[0] + ep[1] * ep2[1] + ep[2] * ep2[2];
}

/* Donor grid of a location along theta (d=1) or phi (d=2): the other
 * patch's own unknowns only (reading: donors exclude ghosts and boundary
 * faces, which are themselves interpolated). */
static void donor_axis(const yyo *h, int loc, int d, double *x0, double *dx, int *n, int *off)
{
    int N = ncell(h, d);
    double start = d == 1 ? h->th0 : h->ph0;
    double step = d == 1 ? h->dth : h->dph;
    *dx = step;
    if (is_face(loc, d)) { *x0 = start + step; *n = N - 1; *off = 1; }
    else { *x0 = start + 0.5 * step; *n = N; *off = 0; }
}

/* Cubic Lagrange weights on nodes 0..3 at fractional position s. */
static void lagrange4(double s, double w[4])
{
    for (int m = 0; m < 4; m++) {
        double num = 1.0, den = 1.0;
        for (int l = 0; l < 4; l++) {
            if (l == m) continue;
            num *= (s - l);
            den *= (double)(m - l);
        }
        w[m] = num / den;
    }
}

/* Window start and weights along one axis; returns 0 if the point lies
 * outside the donor nodes' span (the interpolation would extrapolate). */
static int window(double x, double x0, double dx, int n, int *m0, double w[4])
{
    double s = (x - x0) / dx;
    if (!(s >= 0.0 && s <= n - 1)) return 0;
    int b = (int)floor(s) - 1;
    if (b < 0) b = 0;
    if (b > n - 4) b = n - 4;
    *m0 = b;
    lagrange4(s - b, w);
    return 1;
}

/* Tensor-product cubic Lagrange interpolation (Sec. 4) of the other
 * patch's field `src` (location loc) at its own coordinates (th2, ph2),
 * at radial index i. */
static double interp(const yyo *h, const double *src, int loc, int pb, int i,
                     double th2, double ph2)
{
    double t0, dt, p0, dp, wt[4], wp[4];
    int nt, np, ot, op, jt, kp;
    donor_axis(h, loc, 1, &t0, &dt, &nt, &ot);
    donor_axis(h, loc, 2, &p0, &dp, &np, &op);
    window(th2, t0, dt, nt, &jt, wt);
    window(ph2, p0, dp, np, &kp, wp);
    double v = 0.0;
    for (int a = 0; a < 4; a++) {
        double row = 0.0;
        for (int b = 0; b < 4; b++)
            row += wp[b] * src[ix(h, pb, i, jt + a + ot, kp + b + op)];
        v += wt[a] * row;
    }
    return v;
}

/* Is every interpolation target of location loc inside the donor span? */
static int target_ok(const yyo *h, int loc, double th, double ph)
{
    double th2, ph2, t0, dt, p0, dp, w[4];
    int nt, np, ot, op, m;
    yyo_involution(th, ph, &th2, &ph2);
    donor_axis(h, loc, 1, &t0, &dt, &nt, &ot);
    donor_axis(h, loc, 2, &p0, &dp, &np, &op);
    if (nt < 4 || np < 4) return 0;
    return window(th2, t0, dt, nt, &m, w) && window(ph2, p0, dp, np, &m, w);
}

/* The (theta, phi) targets of a location, radial index excluded:
 * centre-type in theta and phi: ghost rows j=-1,Nt (k interior) and ghost
 * columns k=-1,Np (j interior); theta-faces: boundary faces j=0,Nt and
 * phi ghosts for interior faces; phi-faces: boundary faces k=0,Np and
 * theta ghosts for interior faces.  Calls fn for each. */
typedef void (*target_fn)(const yyo *h, int loc, int j, int k, void *ctx);
static void for_targets(const yyo *h, int loc, target_fn fn, void *ctx)
{
    int nt = h->nt, np = h->np;
    int jlo = ulo(loc, 1), jhi = uhi(h, loc, 1);
    int klo = ulo(loc, 2), khi = uhi(h, loc, 2);
    int jb0 = is_face(loc, 1) ? 0 : -1, jb1 = nt;   /* theta boundary rows */
    int kb0 = is_face(loc, 2) ? 0 : -1, kb1 = np;
    for (int k = klo; k <= khi; k++) { fn(h, loc, jb0, k, ctx); fn(h, loc, jb1, k, ctx); }
    for (int j = jlo; j <= jhi; j++) { fn(h, loc, j, kb0, ctx); fn(h, loc, j, kb1, ctx); }
}

/* A tangential-velocity target interpolates both of the other patch's
 * components (theta-face and phi-face grids), so both spans are checked. */
static void check_target(const yyo *h, int loc, int j, int k, void *ctx)
{
    int *ok = (int *)ctx;
    double th = t_at(h, loc, j), ph = p_at(h, loc, k);
    if (loc == FT || loc == FP) {
        if (!target_ok(h, FT, th, ph) || !target_ok(h, FP, th, ph)) *ok = 0;
    } else if (!target_ok(h, loc, th, ph)) {
        *ok = 0;
    }
}

/* ------------------------------------------------------------------ */
/* creation and I/O                                                    */
/* ------------------------------------------------------------------ */
yyo *yyo_create(int nr, int nt, int np, double r1, double r2, double delta)
{
    if (nr < 2 || nt < 6 || np < 6 || !(r1 > 0.0) || !(r2 > r1)) return NULL;
    if (nr > 2040 || nt > 2040 || np > 2040) return NULL;   /* line buffers */
    yyo *h = (yyo *)calloc(1, sizeof(yyo));
    if (!h) return NULL;
    h->nr = nr; h->nt = nt; h->np = np;
    h->r1 = r1; h->r2 = r2;
    /* one-cell overlap: delta = pi / (2 (nt - 2)) makes dtheta = delta */
    h->delta = delta > 0.0 ? delta : M_PI / (2.0 * (nt - 2));
    h->dr = (r2 - r1) / nr;
    h->th0 = M_PI / 4.0 - h->delta;
    h->ph0 = -3.0 * M_PI / 4.0 - h->delta;
    h->dth = (M_PI / 2.0 + 2.0 * h->delta) / nt;
    h->dph = (1.5 * M_PI + 2.0 * h->delta) / np;
    h->th1 = M_PI / 4.0 - h->delta;   /* theta_1 of the hat operator */
    h->pr = 1.0; h->ra = 0.0; h->tau = 1e-3; h->chi = 1.0;
    h->npatch = (int64_t)(nr + 2) * (nt + 2) * (np + 2);
    int ok = 1;
    for (int loc = 0; loc < 4; loc++) for_targets(h, loc, check_target, &ok);
    if (!ok) { free(h); return NULL; }
    size_t bytes = sizeof(double) * 2 * (size_t)h->npatch;
    for (int f = 0; f < YYO_NF; f++) {
        for (int l = 0; l < NLEV; l++) h->lev[f][l] = (double *)calloc(1, bytes);
        h->star[f] = (double *)calloc(1, bytes);
    }
    for (int c = 0; c < 4; c++) h->force[c] = NULL;
    for (int w = 0; w < 2; w++) { h->t_bc[w][0] = 1.0; h->t_bc[w][1] = 0.0; }
    for (int w = 0; w < 2; w++) { h->u_bc[w][0] = 1.0; h->u_bc[w][1] = 0.0; }
    for (int c = 0; c < 4; c++)
        for (int l = 0; l < NLEV; l++) h->wall[c][l][0] = h->wall[c][l][1] = NULL;
    h->res = (double *)calloc(1, bytes);
    h->wa = (double *)calloc(1, bytes);
    h->wb = (double *)calloc(1, bytes);
    return h;
}

void yyo_destroy(yyo *h)
{
    if (!h) return;
    for (int f = 0; f < YYO_NF; f++) {
        for (int l = 0; l < NLEV; l++) free(h->lev[f][l]);
        free(h->star[f]);
    }
    for (int c = 0; c < 4; c++) free(h->force[c]);
    for (int c = 0; c < 4; c++)
        for (int l = 0; l < NLEV; l++) { free(h->wall[c][l][0]); free(h->wall[c][l][1]); }
    free(h->res); free(h->wa); free(h->wb); free(h->ptmp);
    free(h);
}

int yyo_set_params(yyo *h, double pr, double ra, double tau, double chi,
                   double t_inner, double t_outer)
{
    if (!h || !(tau > 0.0) || !(chi > 0.0) || !(pr > 0.0)) return -1;
    h->pr = pr; h->ra = ra; h->tau = tau; h->chi = chi;
    h->t_in = t_inner; h->t_out = t_outer;
    return 0;
}

/* 1: print a line on stderr after every Schwarz iteration (long runs) */
int yyo_set_verbose(yyo *h, int on)
{
    if (!h) return -1;
    h->verbose = on != 0;
    return 0;
}

int yyo_set_mode(yyo *h, int mode)
{
    if (!h || (mode != 0 && mode != 1)) return -1;
    h->mode = mode;
    return 0;
}

int yyo_set_t_bc(yyo *h, int wall, double a, double b)
{
    if (!h || wall < 0 || wall > 1 || !(a >= 0.0) || !(b >= 0.0) || !(a + b > 0.0)) return -1;
    h->t_bc[wall][0] = a;
    h->t_bc[wall][1] = b;
    h->filled = 0;
    return 0;
}

/* Robin condition a T + b dT/dn = g on a wall (n the outward normal) with
 * T_wall = (T_ghost + T_in)/2 and dT/dn = (T_ghost - T_in)/dr on the cell
 * pair across it: T_ghost = cg g - rho T_in, cg = 1/(a/2 + b/dr),
 * rho = (a/2 - b/dr)/(a/2 + b/dr).  Dirichlet (1, 0): 2 g - T_in. */
static double t_rho(const yyo *h, int wall)
{
    const double a = h->t_bc[wall][0], b = h->t_bc[wall][1];
    return (0.5 * a - b / h->dr) / (0.5 * a + b / h->dr);
}
static double t_cg(const yyo *h, int wall)
{
    return 1.0 / (0.5 * h->t_bc[wall][0] + h->t_bc[wall][1] / h->dr);
}

int yyo_set_u_bc(yyo *h, int wall, double a, double b)
{
    if (!h || wall < 0 || wall > 1 || !(a >= 0.0) || !(b >= 0.0) || !(a + b > 0.0)) return -1;
    h->u_bc[wall][0] = a;
    h->u_bc[wall][1] = b;
    h->filled = 0;
    return 0;
}

/* Robin condition of the tangential velocity on a wall of radius R,
 * a u + b R dn(u / r) = g (n the outward normal; (0, 1) with g = 0 is the
 * stress-free wall: with u_r = 0 the tangential stress is proportional to
 * R d(u_t / r)/dr), on the cell pair across the wall: u_wall = (u_ghost +
 * u_in)/2 and dn(u/r) = (u_ghost / r_ghost - u_in / r_in)/dr, so
 * u_ghost = cg g - rho u_in with cg = 1/(a/2 + b R/(r_ghost dr)) and
 * rho = (a/2 - b R/(r_in dr)) cg.  Dirichlet (1, 0): 2 g - u_in. */
static void u_wall_rule(const yyo *h, int wall, double *cg, double *rho)
{
    const double a = h->u_bc[wall][0], b = h->u_bc[wall][1];
    const double R = wall == 0 ? h->r1 : h->r2;
    const double rg = wall == 0 ? h->r1 - 0.5 * h->dr : h->r2 + 0.5 * h->dr;
    const double ri = wall == 0 ? h->r1 + 0.5 * h->dr : h->r2 - 0.5 * h->dr;
    *cg = 1.0 / (0.5 * a + b * R / (rg * h->dr));
    *rho = (0.5 * a - b * R / (ri * h->dr)) * *cg;
}
static double u_rho(const yyo *h, int wall)
{
    double cg, rho;
    u_wall_rule(h, wall, &cg, &rho);
    return rho;
}
static double u_cg(const yyo *h, int wall)
{
    double cg, rho;
    u_wall_rule(h, wall, &cg, &rho);
    return cg;
}

/* correction rule c_ghost = -rho c_in of a field's r-lines at a wall */
static double wall_rho(const yyo *h, int field, int wall)
{
    const int loc = loc_of(field);
    if (field == YYO_T) return t_rho(h, wall);
    if (loc == FT || loc == FP) return u_rho(h, wall);
    return 1.0;
}

int yyo_set_mass_fix(yyo *h, int on)
{
    if (!h || (on != 0 && on != 1)) return -1;
    h->mass_fix = on;
    h->filled = 0;
    return 0;
}

int yyo_set_mass_fix_params(yyo *h, double eps, double tol)
{
    if (!h || !(eps >= 0.0) || !(tol >= 0.0)) return -1;
    h->mf_eps = eps;
    h->mf_tol = tol;
    h->filled = 0;
    return 0;
}

/* Algorithm step 7 (Sec. 4): after each pressure update the pressure of
 * the outermost nring cells of a patch (cells with j < nring,
 * j >= nt - nring, k < nring or k >= np - nring, every radial index) is
 * interpolated from the other patch instead of being updated by the AC
 * equation.  Reading: in this MAC layout no momentum stencil reads a
 * pressure ghost, so the exchanged values that reach the pressure gradient
 * of eqs. r_comp - phi_comp are those of the patch's own outermost cells;
 * those cells then act as boundary data of the pressure (they leave the AC
 * update and its increment norm, like ghosts).  Every ring cell must lie
 * inside the other patch's centre span.  0 turns the exchange off. */
int yyo_set_pressure_exchange(yyo *h, int nring)
{
    if (!h || nring < 0 || 2 * nring >= h->nt || 2 * nring >= h->np) return -1;
    for (int j = 0; j < h->nt; j++)
        for (int k = 0; k < h->np; k++) {
            int ring = j < nring || j >= h->nt - nring || k < nring || k >= h->np - nring;
            if (ring && !target_ok(h, CC, tc(h, j), pc(h, k))) return -1;
        }
    if (nring > 0 && !h->ptmp) {
        h->ptmp = (double *)calloc(2 * (size_t)h->npatch, sizeof(double));
        if (!h->ptmp) return -1;
    }
    h->nring = nring;
    return 0;
}

/* is centre (j, k) one of the exchanged pressure cells? */
static int in_ring(const yyo *h, int j, int k)
{
    int n = h->nring;
    return n > 0 && (j < n || j >= h->nt - n || k < n || k >= h->np - n);
}

int64_t yyo_field_count(const yyo *h, int field, int layout)
{
    if (!h || field < 0 || field >= YYO_NF) return -1;
    if (layout == YYO_PADDED) return 2 * h->npatch;
    int loc = loc_of(field);
    return 2LL * (mhi(h, loc, 0) + 1) * (mhi(h, loc, 1) + 1) * (mhi(h, loc, 2) + 1);
}

static int copy_field(const yyo *h, double *pad, int field, int layout, double *mac, int to_pad)
{
    if (layout == YYO_PADDED) {
        if (to_pad) memcpy(pad, mac, sizeof(double) * 2 * h->npatch);
        else memcpy(mac, pad, sizeof(double) * 2 * h->npatch);
        return 0;
    }
    int loc = loc_of(field);
    int64_t n = 0;
    for (int p = 0; p < 2; p++)
        for (int i = 0; i <= mhi(h, loc, 0); i++)
            for (int j = 0; j <= mhi(h, loc, 1); j++)
                for (int k = 0; k <= mhi(h, loc, 2); k++, n++) {
                    if (to_pad) pad[ix(h, p, i, j, k)] = mac[n];
                    else mac[n] = pad[ix(h, p, i, j, k)];
                }
    return 0;
}

int yyo_set_field(yyo *h, int field, int level, int layout, const double *src)
{
    if (!h || field < 0 || field >= YYO_NF || level < 0 || level >= NLEV || !src) return -1;
    copy_field(h, h->lev[field][level], field, layout, (double *)src, 1);
    h->filled = 0;
    return 0;
}

int yyo_get_field(const yyo *h, int field, int level, int layout, double *dst)
{
    if (!h || field < 0 || field >= YYO_NF || level < 0 || level >= NLEV || !dst) return -1;
    copy_field(h, h->lev[field][level], field, layout, dst, 0);
    return 0;
}

int yyo_set_forcing(yyo *h, int field, const double *src)
{
    int c;
    switch (field) {
    case YYO_T: c = 0; break;
    case YYO_U1R: c = 1; break;
    case YYO_U1T: c = 2; break;
    case YYO_U1P: c = 3; break;
    default: return -1;
    }
    if (!src) { free(h->force[c]); h->force[c] = NULL; return 0; }
    if (!h->force[c]) h->force[c] = (double *)calloc(2 * (size_t)h->npatch, sizeof(double));
    copy_field(h, h->force[c], field, YYO_MAC, (double *)src, 1);
    return 0;
}

/* Dirichlet data on the walls (the boundary conditions of eq. eq_ns and
 * eq_heat_convec with given values) for one field and level; NULL clears. */
int yyo_set_wall(yyo *h, int field, int level, int wall, const double *src)
{
    int c;
    switch (field) {
    case YYO_T: c = 0; break;
    case YYO_U1R: c = 1; break;
    case YYO_U1T: c = 2; break;
    case YYO_U1P: c = 3; break;
    default: return -1;
    }
    if (!h || level < 0 || level >= NLEV || wall < 0 || wall > 1) return -1;
    double **w = &h->wall[c][level][wall];
    if (!src) { free(*w); *w = NULL; return 0; }
    size_t n = 2 * (size_t)(h->nt + 2) * (size_t)(h->np + 2);
    if (!*w) *w = (double *)malloc(n * sizeof(double));
    memcpy(*w, src, n * sizeof(double));
    return 0;
}

/* wall value of wall-data slot c at (patch, j, k), or the default */
static double wall_value(const yyo *h, int c, int level, int wall, int p, int j, int k, double dflt)
{
    const double *w = h->wall[c][level][wall];
    if (!w) return dflt;
    return w[((size_t)p * (h->nt + 2) + (size_t)(j + 1)) * (size_t)(h->np + 2) + (size_t)(k + 1)];
}

/* ------------------------------------------------------------------ */
/* overlap interpolation and wall rules (Sec. 4, Algorithm steps 1,3,7) */
/* ------------------------------------------------------------------ */
struct fill_ctx { const yyo *h; int level, pa; };

static void fill_scalar_target(const yyo *h, int loc, int j, int k, void *vctx)
{
    struct fill_ctx *c = (struct fill_ctx *)vctx;
    double th2, ph2;
    yyo_involution(t_at(h, loc, j), p_at(h, loc, k), &th2, &ph2);
    int pb = 1 - c->pa;
    int ilo = ulo(loc, 0), ihi = uhi(h, loc, 0);
    static const int sc_fields[3] = { YYO_T, YYO_P1, YYO_P2 };
    static const int ur_fields[2] = { YYO_U1R, YYO_U2R };
    const int *fl = loc == CC ? sc_fields : ur_fields;
    int nf = loc == CC ? 3 : 2;
    for (int q = 0; q < nf; q++) {
        double *a = h->lev[fl[q]][c->level];
        for (int i = ilo; i <= ihi; i++)
            a[ix(h, c->pa, i, j, k)] = interp(h, a, loc, pb, i, th2, ph2);
    }
}

/* Tangential components: interpolate both of the other patch's
 * components to the target, then rotate into this patch's basis. */
static void fill_vector_target(const yyo *h, int loc, int j, int k, void *vctx)
{
    struct fill_ctx *c = (struct fill_ctx *)vctx;
    double th = t_at(h, loc, j), ph = p_at(h, loc, k), th2, ph2, m[4];
    yyo_involution(th, ph, &th2, &ph2);
    yyo_rotation(th, ph, m);
    int pb = 1 - c->pa;
    for (int s = 0; s < 2; s++) {
        double *ut = h->lev[s == 0 ? YYO_U1T : YYO_U2T][c->level];
        double *up = h->lev[s == 0 ? YYO_U1P : YYO_U2P][c->level];
        double *dst = loc == FT ? ut : up;
        for (int i = 0; i < h->nr; i++) {
            double vt = interp(h, ut, FT, pb, i, th2, ph2);
            double vp = interp(h, up, FP, pb, i, th2, ph2);
            dst[ix(h, c->pa, i, j, k)] = loc == FT ? m[0] * vt + m[1] * vp
                                                   : m[2] * vt + m[3] * vp;
        }
    }
}

/* Wall rules (eq. eq_ns, eq_heat_convec boundary conditions): u = u_wall
 * and T = T_wall on r = R1, R2 (u_wall = 0 and the constant wall
 * temperatures unless wall data is given).  u_r lives on the wall faces;
 * centre-type fields get a reflection ghost psi_{-1} = 2 psi_wall - psi_0.
 * Pressure needs no wall values.  Both velocity systems take the same
 * wall data. */
static void wall_rules(const yyo *h, int level, int p)
{
    int nr = h->nr;
    for (int j = -1; j <= h->nt; j++)
        for (int k = -1; k <= h->np; k++) {
            double *T = h->lev[YYO_T][level];
            T[ix(h, p, -1, j, k)] = t_cg(h, 0) * wall_value(h, 0, level, 0, p, j, k, h->t_in) - t_rho(h, 0) * T[ix(h, p, 0, j, k)];
            T[ix(h, p, nr, j, k)] = t_cg(h, 1) * wall_value(h, 0, level, 1, p, j, k, h->t_out) - t_rho(h, 1) * T[ix(h, p, nr - 1, j, k)];
            static const int tang[4] = { YYO_U1T, YYO_U1P, YYO_U2T, YYO_U2P };
            for (int q = 0; q < 4; q++) {
                const int c = (q % 2 == 0) ? 2 : 3;
                double *a = h->lev[tang[q]][level];
                a[ix(h, p, -1, j, k)] = u_cg(h, 0) * wall_value(h, c, level, 0, p, j, k, 0.0) - u_rho(h, 0) * a[ix(h, p, 0, j, k)];
                a[ix(h, p, nr, j, k)] = u_cg(h, 1) * wall_value(h, c, level, 1, p, j, k, 0.0) - u_rho(h, 1) * a[ix(h, p, nr - 1, j, k)];
            }
            const double w0 = wall_value(h, 1, level, 0, p, j, k, 0.0), w1 = wall_value(h, 1, level, 1, p, j, k, 0.0);
            h->lev[YYO_U1R][level][ix(h, p, 0, j, k)] = w0;
            h->lev[YYO_U1R][level][ix(h, p, nr, j, k)] = w1;
            h->lev[YYO_U2R][level][ix(h, p, 0, j, k)] = w0;
            h->lev[YYO_U2R][level][ix(h, p, nr, j, k)] = w1;
        }
}

/* Algorithm step 4 (mass-flux correction of the interpolated boundary
 * data).  With F(v) the net outward flux of the patch's interpolated
 * boundary normal velocities v (u_theta on the theta-boundary faces, u_phi
 * on the phi-boundary faces) and F_r that of the wall data, the functional
 *   J(v) = |v - u_bd|^2 / 2 + (F(v) + F_r)^2 / (2 eps |dOmega|^2)
 * is quadratic with the Hessian I + c a a^T (a = the faces' flux weights
 * with their outward signs).  Its minimiser, the limit of the conjugate
 * gradient iteration, is v = u_bd - kappa a with
 *   kappa = (F(u_bd) + F_r) / (eps |dOmega|^2 + a.a),
 * |dOmega| the area of the patch's boundary (all its faces).  eps = 0 (the
 * default) is the limit in which the corrected data carry no net flux.  The
 * correction is made when |F(u_bd) + F_r| >= tol (default 0: always).  The
 * flux weights
 * are the face areas of the discrete divergence: r-face r_f^2 sin(theta_j)
 * dtheta dphi, theta-face r_i sin(theta_f) dr dphi, phi-face r_i dr dtheta,
 * so that the volume-weighted sum of Div_h over the patch telescopes to
 * exactly this boundary flux. */
static void mass_fix(yyo *h, int level, int p)
{
    const int nr = h->nr, nt = h->nt, np = h->np;
    for (int s = 0; s < 2; s++) {
        double *ur = h->lev[s == 0 ? YYO_U1R : YYO_U2R][level];
        double *ut = h->lev[s == 0 ? YYO_U1T : YYO_U2T][level];
        double *up = h->lev[s == 0 ? YYO_U1P : YYO_U2P][level];
        double F = 0.0, S = 0.0, A = 0.0;
        for (int j = 0; j < nt; j++)
            for (int k = 0; k < np; k++) {
                const double a0 = rf(h, 0) * rf(h, 0) * sin(tc(h, j)) * h->dth * h->dph;
                const double a1 = rf(h, nr) * rf(h, nr) * sin(tc(h, j)) * h->dth * h->dph;
                F += a1 * ur[ix(h, p, nr, j, k)] - a0 * ur[ix(h, p, 0, j, k)];
                A += a0 + a1;
            }
        for (int i = 0; i < nr; i++) {
            for (int k = 0; k < np; k++) {
                const double a0 = rc(h, i) * sin(tf(h, 0)) * h->dr * h->dph;
                const double a1 = rc(h, i) * sin(tf(h, nt)) * h->dr * h->dph;
                F += a1 * ut[ix(h, p, i, nt, k)] - a0 * ut[ix(h, p, i, 0, k)];
                S += a0 * a0 + a1 * a1;
                A += a0 + a1;
            }
            for (int j = 0; j < nt; j++) {
                const double a = rc(h, i) * h->dr * h->dth;
                F += a * (up[ix(h, p, i, j, np)] - up[ix(h, p, i, j, 0)]);
                S += 2.0 * a * a;
                A += 2.0 * a;
            }
        }
        if (fabs(F) < h->mf_tol) continue;
        const double kappa = F / (h->mf_eps * A * A + S);
        for (int i = 0; i < nr; i++) {
            for (int k = 0; k < np; k++) {
                ut[ix(h, p, i, 0, k)] += kappa * rc(h, i) * sin(tf(h, 0)) * h->dr * h->dph;
                ut[ix(h, p, i, nt, k)] -= kappa * rc(h, i) * sin(tf(h, nt)) * h->dr * h->dph;
            }
            for (int j = 0; j < nt; j++) {
                up[ix(h, p, i, j, 0)] += kappa * rc(h, i) * h->dr * h->dth;
                up[ix(h, p, i, j, np)] -= kappa * rc(h, i) * h->dr * h->dth;
            }
        }
    }
}

static void fill_patch(yyo *h, int level, int pa)
{
    struct fill_ctx c = { h, level, pa };
    for_targets(h, CC, fill_scalar_target, &c);
    for_targets(h, FR, fill_scalar_target, &c);
    for_targets(h, FT, fill_vector_target, &c);
    for_targets(h, FP, fill_vector_target, &c);
    wall_rules(h, level, pa);
    if (h->mass_fix) mass_fix(h, level, pa);
}

/* Additive: both patches read the other's values of the same iterate.
 * Donors are unknowns only and targets are never donors, so the two
 * patches' fills are independent. */
int yyo_fill(yyo *h, int level)
{
    if (!h || level < 0 || level >= NLEV) return -1;
    fill_patch(h, level, 0);
    fill_patch(h, level, 1);
    return 0;
}

/* ------------------------------------------------------------------ */
/* advecting velocity and MAC averaging (Sec. 3.3, 4)                  */
/* ------------------------------------------------------------------ */
/* Value of velocity component c (0=r,1=theta,2=phi; stored on its own
 * faces) at location loc of point (i,j,k): arithmetic mean over the
 * nearest stored points -- faces f, f+1 where loc is a centre, centres
 * f-1, f where loc is a face, the point itself where they agree. */
static double vel_at(const yyo *h, const double *u, int c, int loc, int p, int i, int j, int k)
{
    int cl = c + 1;   /* FR, FT, FP */
    int o0[3], o1[3];
    int idx[3] = { i, j, k };
    for (int d = 0; d < 3; d++) {
        if (is_face(cl, d) && !is_face(loc, d)) { o0[d] = 0; o1[d] = 1; }
        else if (!is_face(cl, d) && is_face(loc, d)) { o0[d] = -1; o1[d] = 0; }
        else { o0[d] = 0; o1[d] = 0; }
    }
    double s = 0.0;
    int cnt = 0;
    for (int a = o0[0]; a <= o1[0]; a++)
        for (int b = o0[1]; b <= o1[1]; b++)
            for (int e = o0[2]; e <= o1[2]; e++) {
                s += u[ix(h, p, idx[0] + a, idx[1] + b, idx[2] + e)];
                cnt++;
            }
    return s / cnt;
}

/* the advecting velocity a = u_2^{*,n+1/2} at a point (Sec. 3.3) */
static void adv_at(const yyo *h, int loc, int p, int i, int j, int k, double a[3])
{
    a[0] = vel_at(h, h->star[YYO_U2R], 0, loc, p, i, j, k);
    a[1] = vel_at(h, h->star[YYO_U2T], 1, loc, p, i, j, k);
    a[2] = vel_at(h, h->star[YYO_U2P], 2, loc, p, i, j, k);
}

/* ------------------------------------------------------------------ */
/* split one-direction operators (Sec. 3.2 hat operators, 3.3.1-3.3.3) */
/* ------------------------------------------------------------------ */
typedef struct { double lo, di, up; } tri;

/* D_rr = r^-2 d_r(r^2 d_r), flux form at the point's r-location */
static tri op_drr(const yyo *h, int loc, int i)
{
    double r0, rm, rp;
    if (is_face(loc, 0)) { r0 = rf(h, i); rm = rc(h, i - 1); rp = rc(h, i); }
    else { r0 = rc(h, i); rm = rf(h, i); rp = rf(h, i + 1); }
    double s = 1.0 / (r0 * r0 * h->dr * h->dr);
    tri t = { rm * rm * s, -(rm * rm + rp * rp) * s, rp * rp * s };
    return t;
}

/* D_thth = (rho^2 sin th)^-1 d_th(sin th d_th), rho = r (true operator)
 * or R1 (hat operator of Sec. 3.2) */
static tri op_dtt(const yyo *h, int loc, int j, double rho)
{
    double s0, sm, sp;
    if (is_face(loc, 1)) { s0 = sin(tf(h, j)); sm = sin(tc(h, j - 1)); sp = sin(tc(h, j)); }
    else { s0 = sin(tc(h, j)); sm = sin(tf(h, j)); sp = sin(tf(h, j + 1)); }
    double s = 1.0 / (rho * rho * s0 * h->dth * h->dth);
    tri t = { sm * s, -(sm + sp) * s, sp * s };
    return t;
}

/* D_phph = d_phph / (r^2 sin^2 th); hat: r -> R1, th -> theta_1 */
static tri op_dpp(const yyo *h, double r, double th)
{
    double s = 1.0 / (r * r * sin(th) * sin(th) * h->dph * h->dph);
    tri t = { s, -2.0 * s, s };
    return t;
}

static tri op_dpp_hat(const yyo *h)
{
    return op_dpp(h, h->r1, h->th1);
}

static tri tri_add(tri a, tri b, double sb)
{
    tri t = { a.lo + sb * b.lo, a.di + sb * b.di, a.up + sb * b.up };
    return t;
}

/* centred first derivative along a direction with grid step g:
 * -a d/dx -> (lo, up) += (+a/(2g), -a/(2g)) */
static tri tri_advect(tri t, double a, double g)
{
    t.lo += a / (2.0 * g);
    t.up -= a / (2.0 * g);
    return t;
}

/* Coefficients of the split operator L_{field,d} at a point
 * (eq. Convect_Douglas for T; eq. r_comp, theta_comp, phi_comp for the
 * velocity components, with readings: viscosity Pr; every grad-div block
 * carries 1/(2 chi); the nonlinear metric terms are linearised with the
 * advecting velocity; advection enters with a minus sign). */
static tri coef(const yyo *h, int field, int d, int p, int i, int j, int k)
{
    int loc = loc_of(field);
    double r = r_at(h, loc, i), th = t_at(h, loc, j);
    double nu = field == YYO_T ? 1.0 : h->pr;
    double ic = 1.0 / (2.0 * h->chi);
    double a[3];
    adv_at(h, loc, p, i, j, k, a);
    tri z = { 0.0, 0.0, 0.0 }, t = z;
    if (d == 0) {
        t = tri_add(z, op_drr(h, loc, i), nu);
        if (loc == FR) {
            /* -2u/r^2 + (2/r^3) d_r(r^2 u), centred at the face */
            double rm = rf(h, i - 1), rp = rf(h, i + 1);
            t.di += nu * (-2.0 / (r * r));
            t.lo += nu * (2.0 / (r * r * r)) * (-rm * rm / (2.0 * h->dr));
            t.up += nu * (2.0 / (r * r * r)) * (rp * rp / (2.0 * h->dr));
            /* D11 = G_r Div_r */
            double cm = rc(h, i - 1), cp = rc(h, i), dr2 = h->dr * h->dr;
            t.lo += ic * rm * rm / (cm * cm * dr2);
            t.up += ic * rp * rp / (cp * cp * dr2);
            t.di += ic * (-r * r * (1.0 / (cp * cp) + 1.0 / (cm * cm)) / dr2);
        }
        t = tri_advect(t, a[0], h->dr);
    } else if (d == 1) {
        t = tri_add(z, op_dtt(h, loc, j, h->r1), nu);
        if (loc == FT) {
            double s0 = sin(th), c0 = cos(th);
            double sm = sin(tf(h, j - 1)), sp = sin(tf(h, j + 1));
            /* -u/(r^2 sin^2) + (2 cos/(r^2 sin^2)) d_th(sin u), centred */
            t.di += nu * (-1.0 / (r * r * s0 * s0));
            t.lo += nu * (2.0 * c0 / (r * r * s0 * s0)) * (-sm / (2.0 * h->dth));
            t.up += nu * (2.0 * c0 / (r * r * s0 * s0)) * (sp / (2.0 * h->dth));
            /* -a_r u / r */
            t.di += -a[0] / r;
            /* D22 = G_th Div_th */
            double scm = sin(tc(h, j - 1)), scp = sin(tc(h, j));
            double q = 1.0 / (r * r * h->dth * h->dth);
            t.lo += ic * sm * q / scm;
            t.up += ic * sp * q / scp;
            t.di += ic * (-s0 * q * (1.0 / scp + 1.0 / scm));
        }
        t = tri_advect(t, a[1] / r, h->dth);
    } else {
        t = tri_add(z, op_dpp_hat(h), nu);
        if (loc == FP) {
            double s0 = sin(th), c0 = cos(th);
            /* -u/(r^2 sin^2) */
            t.di += nu * (-1.0 / (r * r * s0 * s0));
            /* -(a_r + a_th cot th) u / r */
            t.di += -(a[0] + a[1] * c0 / s0) / r;
            /* D33 = G_ph Div_ph */
            tri d33 = op_dpp(h, r, th);
            t = tri_add(t, d33, ic);
        }
        t = tri_advect(t, a[2] / (r * sin(th)), h->dph);
    }
    return t;
}

/* ------------------------------------------------------------------ */
/* divergence and gradient on the MAC grid                              */
/* ------------------------------------------------------------------ */
static double div_rr(const yyo *h, const double *ur, int p, int i, int j, int k)
{
    double a = rf(h, i + 1), b = rf(h, i), r = rc(h, i);
    return (a * a * ur[ix(h, p, i + 1, j, k)] - b * b * ur[ix(h, p, i, j, k)]) / (r * r * h->dr);
}
static double div_th(const yyo *h, const double *ut, int p, int i, int j, int k)
{
    return (sin(tf(h, j + 1)) * ut[ix(h, p, i, j + 1, k)] - sin(tf(h, j)) * ut[ix(h, p, i, j, k)]) /
           (rc(h, i) * sin(tc(h, j)) * h->dth);
}
static double div_ph(const yyo *h, const double *up, int p, int i, int j, int k)
{
    return (up[ix(h, p, i, j, k + 1)] - up[ix(h, p, i, j, k)]) / (rc(h, i) * sin(tc(h, j)) * h->dph);
}

/* Div_h of the average (a + b)/2 of two velocity levels at a centre */
static double div_avg(const yyo *h, double *const a[3], double *const b[3], int p, int i, int j, int k)
{
    double da = div_rr(h, a[0], p, i, j, k) + div_th(h, a[1], p, i, j, k) + div_ph(h, a[2], p, i, j, k);
    double db = div_rr(h, b[0], p, i, j, k) + div_th(h, b[1], p, i, j, k) + div_ph(h, b[2], p, i, j, k);
    return 0.5 * (da + db);
}

/* ------------------------------------------------------------------ */
/* residual R^k (Sec. 3, eq. er in correction form)                    */
/* ------------------------------------------------------------------ */
static double fget(const yyo *h, int c, int p, int i, int j, int k)
{
    return h->force[c] ? h->force[c][ix(h, p, i, j, k)] : 0.0;
}

/* velocity arrays of a system: level l, components r, theta, phi */
static void vel_arrays(const yyo *h, int s, int l, double *u[3])
{
    u[0] = h->lev[s == 1 ? YYO_U1R : YYO_U2R][l];
    u[1] = h->lev[s == 1 ? YYO_U1T : YYO_U2T][l];
    u[2] = h->lev[s == 1 ? YYO_U1P : YYO_U2P][l];
}
static void vel_star(const yyo *h, int s, double *u[3])
{
    u[0] = h->star[s == 1 ? YYO_U1R : YYO_U2R];
    u[1] = h->star[s == 1 ? YYO_U1T : YYO_U2T];
    u[2] = h->star[s == 1 ? YYO_U1P : YYO_U2P];
}

/* p~ of system s at a centre: p1^n for s = 1; p2^n + (p1^k - p1^n)/2 for
 * s = 2 (reading of the bootstrapped system eq. ac2) */
static double p_tilde(const yyo *h, int s, int p, int i, int j, int k)
{
    int64_t q = ix(h, p, i, j, k);
    if (s == 1) return h->lev[YYO_P1][YYO_LEV_N][q];
    return h->lev[YYO_P2][YYO_LEV_N][q] +
           0.5 * (h->lev[YYO_P1][YYO_LEV_K][q] - h->lev[YYO_P1][YYO_LEV_N][q]);
}

static double ubar(const yyo *h, double *const un[3], double *const uk[3], int c, int loc,
                   int p, int i, int j, int k)
{
    return 0.5 * (vel_at(h, un[c], c, loc, p, i, j, k) + vel_at(h, uk[c], c, loc, p, i, j, k));
}

/* explicit part S of a field's equation (Sec. 3.3.1-3.3.3, readings) */
static double source(const yyo *h, int field, int p, int i, int j, int k)
{
    int loc = loc_of(field);
    if (field == YYO_T) return fget(h, 0, p, i, j, k);
    int s = (field >= YYO_U2R) ? 2 : 1;
    double r = r_at(h, loc, i), th = t_at(h, loc, j);
    double ic = 1.0 / (2.0 * h->chi), pr = h->pr;
    double *un[3], *uk[3], *us[3], a[3];
    vel_arrays(h, s, YYO_LEV_N, un);
    vel_arrays(h, s, YYO_LEV_K, uk);
    vel_star(h, s, us);
    adv_at(h, loc, p, i, j, k, a);
    double S = 0.0;
    if (loc == FR) {
        /* (D12 u_th* + D13 u_ph*)/(2 chi): G_r of Div_th, Div_ph */
        double d12 = (div_th(h, us[1], p, i, j, k) - div_th(h, us[1], p, i - 1, j, k)) / h->dr;
        double d13 = (div_ph(h, us[2], p, i, j, k) - div_ph(h, us[2], p, i - 1, j, k)) / h->dr;
        S += ic * (d12 + d13);
        /* (a_th u_th* + a_ph u_ph*) / r */
        S += (a[1] * vel_at(h, us[1], 1, FR, p, i, j, k) + a[2] * vel_at(h, us[2], 2, FR, p, i, j, k)) / r;
        /* -d_r p~ */
        S -= (p_tilde(h, s, p, i, j, k) - p_tilde(h, s, p, i - 1, j, k)) / h->dr;
        /* buoyancy Pr Ra T^{n+1/2} e_r at the face */
        const double *Tn = h->lev[YYO_T][YYO_LEV_N], *Tk = h->lev[YYO_T][YYO_LEV_K];
        double tb = 0.5 * (0.5 * (Tn[ix(h, p, i - 1, j, k)] + Tk[ix(h, p, i - 1, j, k)]) +
                           0.5 * (Tn[ix(h, p, i, j, k)] + Tk[ix(h, p, i, j, k)]));
        S += pr * h->ra * tb;
        S += fget(h, 1, p, i, j, k);
    } else if (loc == FT) {
        double rr = rc(h, i);
        /* (D21 u_r^{n+1/2} + D23 u_ph*)/(2 chi) */
        double d21 = (0.5 * (div_rr(h, un[0], p, i, j, k) + div_rr(h, uk[0], p, i, j, k)) -
                      0.5 * (div_rr(h, un[0], p, i, j - 1, k) + div_rr(h, uk[0], p, i, j - 1, k))) /
                     (rr * h->dth);
        double d23 = (div_ph(h, us[2], p, i, j, k) - div_ph(h, us[2], p, i, j - 1, k)) / (rr * h->dth);
        S += ic * (d21 + d23);
        /* Pr[(2/r^2) d_th u_r + (2 cos/(r^3 sin)) d_r(r^2 u_r)], u_r at n+1/2 */
        double dth_ur = 0.0, dr_r2ur = 0.0;
        for (int lv = 0; lv < 2; lv++) {
            const double *ur = lv == 0 ? un[0] : uk[0];
            double g = 0.5 * ((ur[ix(h, p, i, j, k)] - ur[ix(h, p, i, j - 1, k)]) +
                              (ur[ix(h, p, i + 1, j, k)] - ur[ix(h, p, i + 1, j - 1, k)])) / h->dth;
            double a2 = rf(h, i + 1) * rf(h, i + 1), b2 = rf(h, i) * rf(h, i);
            double q = 0.5 * ((a2 * ur[ix(h, p, i + 1, j - 1, k)] - b2 * ur[ix(h, p, i, j - 1, k)]) +
                              (a2 * ur[ix(h, p, i + 1, j, k)] - b2 * ur[ix(h, p, i, j, k)])) / h->dr;
            dth_ur += 0.5 * g;
            dr_r2ur += 0.5 * q;
        }
        S += pr * (2.0 / (r * r) * dth_ur + 2.0 * cos(th) / (r * r * r * sin(th)) * dr_r2ur);
        /* + a_ph u_ph* cot th / r */
        S += a[2] * vel_at(h, us[2], 2, FT, p, i, j, k) * cos(th) / (sin(th) * r);
        /* -(1/r) d_th p~ */
        S -= (p_tilde(h, s, p, i, j, k) - p_tilde(h, s, p, i, j - 1, k)) / (rr * h->dth);
        S += fget(h, 2, p, i, j, k);
    } else {
        double rr = rc(h, i), sn = sin(tc(h, j));
        /* (D31 u_r^{n+1/2} + D32 u_th^{n+1/2})/(2 chi) */
        double g = rr * sn * h->dph;
        double d31 = (0.5 * (div_rr(h, un[0], p, i, j, k) + div_rr(h, uk[0], p, i, j, k)) -
                      0.5 * (div_rr(h, un[0], p, i, j, k - 1) + div_rr(h, uk[0], p, i, j, k - 1))) / g;
        double d32 = (0.5 * (div_th(h, un[1], p, i, j, k) + div_th(h, uk[1], p, i, j, k)) -
                      0.5 * (div_th(h, un[1], p, i, j, k - 1) + div_th(h, uk[1], p, i, j, k - 1))) / g;
        S += ic * (d31 + d32);
        /* Pr[(2/(r^2 sin)) d_ph u_r + (2 cos/(r^2 sin^2)) d_ph u_th] at n+1/2 */
        double dph_ur = 0.0, dph_ut = 0.0;
        for (int lv = 0; lv < 2; lv++) {
            const double *ur = lv == 0 ? un[0] : uk[0];
            const double *ut = lv == 0 ? un[1] : uk[1];
            dph_ur += 0.5 * 0.5 * ((ur[ix(h, p, i, j, k)] - ur[ix(h, p, i, j, k - 1)]) +
                                   (ur[ix(h, p, i + 1, j, k)] - ur[ix(h, p, i + 1, j, k - 1)])) / h->dph;
            dph_ut += 0.5 * 0.5 * ((ut[ix(h, p, i, j, k)] - ut[ix(h, p, i, j, k - 1)]) +
                                   (ut[ix(h, p, i, j + 1, k)] - ut[ix(h, p, i, j + 1, k - 1)])) / h->dph;
        }
        S += pr * (2.0 / (r * r * sin(th)) * dph_ur + 2.0 * cos(th) / (r * r * sin(th) * sin(th)) * dph_ut);
        /* -(1/(r sin)) d_ph p~ */
        S -= (p_tilde(h, s, p, i, j, k) - p_tilde(h, s, p, i, j, k - 1)) / g;
        S += fget(h, 3, p, i, j, k);
    }
    return S;
}

/* R^k = Lhat psibar + (F - Lhat) psi* + S - (psi^{k-1} - psi^n)/tau,
 * psibar = (psi^n + psi^{k-1})/2, and F - Lhat = nu[(D_thth - Dhat_thth)
 * + (D_phph - Dhat_phph)] (the terms the hat operators change). */
static double residual_at(const yyo *h, int field, int p, int i, int j, int k)
{
    int loc = loc_of(field);
    const double *pn = h->lev[field][YYO_LEV_N], *pk = h->lev[field][YYO_LEV_K];
    const double *ps = h->star[field];
    double nu = field == YYO_T ? 1.0 : h->pr;
    double r = r_at(h, loc, i), th = t_at(h, loc, j);
#define BAR(ii, jj, kk) (0.5 * (pn[ix(h, p, ii, jj, kk)] + pk[ix(h, p, ii, jj, kk)]))
#define STR(ii, jj, kk) (ps[ix(h, p, ii, jj, kk)])
    double R = 0.0;
    tri c;
    c = coef(h, field, 0, p, i, j, k);
    R += c.lo * BAR(i - 1, j, k) + c.di * BAR(i, j, k) + c.up * BAR(i + 1, j, k);
    c = coef(h, field, 1, p, i, j, k);
    R += c.lo * BAR(i, j - 1, k) + c.di * BAR(i, j, k) + c.up * BAR(i, j + 1, k);
    c = coef(h, field, 2, p, i, j, k);
    R += c.lo * BAR(i, j, k - 1) + c.di * BAR(i, j, k) + c.up * BAR(i, j, k + 1);
    tri t1 = op_dtt(h, loc, j, r), t0 = op_dtt(h, loc, j, h->r1);
    tri q1 = op_dpp(h, r, th), q0 = op_dpp_hat(h);
    double dtt = t1.lo * STR(i, j - 1, k) + t1.di * STR(i, j, k) + t1.up * STR(i, j + 1, k);
    double dtt_hat = t0.lo * STR(i, j - 1, k) + t0.di * STR(i, j, k) + t0.up * STR(i, j + 1, k);
    double dpp = q1.lo * STR(i, j, k - 1) + q1.di * STR(i, j, k) + q1.up * STR(i, j, k + 1);
    double dpp_hat = q0.lo * STR(i, j, k - 1) + q0.di * STR(i, j, k) + q0.up * STR(i, j, k + 1);
    R += nu * ((dtt - dtt_hat) + (dpp - dpp_hat));
    R += source(h, field, p, i, j, k);
    R -= (pk[ix(h, p, i, j, k)] - pn[ix(h, p, i, j, k)]) / h->tau;
#undef BAR
#undef STR
    return R;
}

/* ------------------------------------------------------------------ */
/* line solves (Sec. 4: Thomas algorithm per direction)                */
/* ------------------------------------------------------------------ */
int yyo_thomas(int n, const double *lo, const double *di, const double *up,
               const double *rhs, double *x)
{
    if (n <= 0) return 0;
    double *cp = (double *)malloc(sizeof(double) * n);
    double *dp = (double *)malloc(sizeof(double) * n);
    cp[0] = up[0] / di[0];
    dp[0] = rhs[0] / di[0];
    for (int m = 1; m < n; m++) {
        double den = di[m] - lo[m] * cp[m - 1];
        cp[m] = m < n - 1 ? up[m] / den : 0.0;
        dp[m] = (rhs[m] - lo[m] * dp[m - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int m = n - 2; m >= 0; m--) x[m] = dp[m] - cp[m] * x[m + 1];
    free(cp);
    free(dp);
    return 0;
}

/* (I - tau/2 L_{field,d}) y = x along every line of direction d, both
 * patches.  Homogeneous ends: zero at theta/phi ghosts and boundary
 * faces and at the wall faces of u_r; reflection (c_{-1} = -c_0) at the
 * walls for r-centred unknowns. */
static void sweep_range(yyo *h, int field, int d, const double *x, double *y, int p0, int p1)
{
    int loc = loc_of(field);
    int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;   /* the other two directions */
    int n = uhi(h, loc, d) - ulo(loc, d) + 1;
    int a0 = ulo(loc, d1), a1 = uhi(h, loc, d1), b0 = ulo(loc, d2), b1 = uhi(h, loc, d2);
    int reflect = (d == 0 && !is_face(loc, 0));
    /* homogeneous wall rule of the correction: c_ghost = -rho c_in (rho = 1
     * for Dirichlet data, the Robin rules of T and the tangential
     * velocity otherwise) */
    const double rho0 = wall_rho(h, field, 0), rho1 = wall_rho(h, field, 1);
    double ht = 0.5 * h->tau;
    for (int p = p0; p < p1; p++) {
#pragma omp parallel for collapse(2) schedule(static)
        for (int a = a0; a <= a1; a++)
            for (int b = b0; b <= b1; b++) {
                double lo[2048], di[2048], up[2048], rhs[2048], sol[2048];
                for (int m = 0; m < n; m++) {
                    int idx[3];
                    idx[d] = ulo(loc, d) + m; idx[d1] = a; idx[d2] = b;
                    tri c = coef(h, field, d, p, idx[0], idx[1], idx[2]);
                    lo[m] = -ht * c.lo;
                    di[m] = 1.0 - ht * c.di;
                    up[m] = -ht * c.up;
                    if (reflect && m == 0) di[m] = 1.0 - ht * (c.di - rho0 * c.lo);
                    if (reflect && m == n - 1) di[m] = 1.0 - ht * (c.di - rho1 * c.up);
                    rhs[m] = x[ix(h, p, idx[0], idx[1], idx[2])];
                }
                yyo_thomas(n, lo, di, up, rhs, sol);
                for (int m = 0; m < n; m++) {
                    int idx[3];
                    idx[d] = ulo(loc, d) + m; idx[d1] = a; idx[d2] = b;
                    y[ix(h, p, idx[0], idx[1], idx[2])] = sol[m];
                }
            }
    }
}

int yyo_sweep(yyo *h, int field, int dir, const double *x, double *y)
{
    if (!h || field < 0 || field >= YYO_NF || dir < 0 || dir > 2 || !x || !y) return -1;
    if (field == YYO_P1 || field == YYO_P2) return -1;
    memset(y, 0, sizeof(double) * 2 * h->npatch);
    sweep_range(h, field, dir, x, y, 0, 2);
    return 0;
}

/* (I - tau/2 Pr D) y = x along the direction of a plain metric operator D
 * (D_rr, D_thth, Dhat_thth, D_phph, Dhat_phph) for the centre unknowns,
 * every line of both patches; zero at theta/phi ghosts, reflection
 * (c_{-1} = -c_0) at the walls. */
int yyo_sweep_op(yyo *h, int op, const double *x, double *y)
{
    if (!h || !x || !y || op < YYO_OP_DRR || op > YYO_OP_DPP_HAT) return -1;
    const int d = op == YYO_OP_DRR ? 0 : (op == YYO_OP_DTT || op == YYO_OP_DTT_HAT) ? 1 : 2;
    const int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
    const int n = ncell(h, d);
    const double ht = 0.5 * h->tau;
    memset(y, 0, sizeof(double) * 2 * h->npatch);
    for (int p = 0; p < 2; p++) {
#pragma omp parallel for collapse(2) schedule(static)
        for (int a = 0; a < ncell(h, d1); a++)
            for (int b = 0; b < ncell(h, d2); b++) {
                double lo[2048], di[2048], up[2048], rhs[2048], sol[2048];
                for (int m = 0; m < n; m++) {
                    int idx[3];
                    idx[d] = m; idx[d1] = a; idx[d2] = b;
                    const double r = rc(h, idx[0]), th = tc(h, idx[1]);
                    tri c;
                    switch (op) {
                    case YYO_OP_DRR: c = op_drr(h, CC, idx[0]); break;
                    case YYO_OP_DTT: c = op_dtt(h, CC, idx[1], r); break;
                    case YYO_OP_DTT_HAT: c = op_dtt(h, CC, idx[1], h->r1); break;
                    case YYO_OP_DPP: c = op_dpp(h, r, th); break;
                    default: c = op_dpp_hat(h); break;
                    }
                    lo[m] = -ht * h->pr * c.lo;
                    di[m] = 1.0 - ht * h->pr * c.di;
                    up[m] = -ht * h->pr * c.up;
                    if (d == 0 && m == 0) di[m] = 1.0 - ht * h->pr * (c.di - c.lo);
                    if (d == 0 && m == n - 1) di[m] = 1.0 - ht * h->pr * (c.di - c.up);
                    rhs[m] = x[ix(h, p, idx[0], idx[1], idx[2])];
                }
                yyo_thomas(n, lo, di, up, rhs, sol);
                for (int m = 0; m < n; m++) {
                    int idx[3];
                    idx[d] = m; idx[d1] = a; idx[d2] = b;
                    y[ix(h, p, idx[0], idx[1], idx[2])] = sol[m];
                }
            }
    }
    return 0;
}

/* explicit operator at the unknowns with homogeneous neighbours outside
 * the unknown set (the operator whose inverse factor a sweep applies) */
int yyo_apply_op(yyo *h, int field, int op, const double *x, double *y)
{
    if (!h || field < 0 || field >= YYO_NF || !x || !y) return -1;
    int loc = loc_of(field);
    memset(y, 0, sizeof(double) * 2 * h->npatch);
    int d = (op == YYO_OP_DRR || op == YYO_OP_LR) ? 0
          : (op == YYO_OP_DTT || op == YYO_OP_DTT_HAT || op == YYO_OP_LT) ? 1 : 2;
    for (int p = 0; p < 2; p++)
        for (int i = ulo(loc, 0); i <= uhi(h, loc, 0); i++)
            for (int j = ulo(loc, 1); j <= uhi(h, loc, 1); j++)
                for (int k = ulo(loc, 2); k <= uhi(h, loc, 2); k++) {
                    tri c;
                    double r = r_at(h, loc, i), th = t_at(h, loc, j);
                    switch (op) {
                    case YYO_OP_DRR: c = op_drr(h, loc, i); break;
                    case YYO_OP_DTT: c = op_dtt(h, loc, j, r); break;
                    case YYO_OP_DTT_HAT: c = op_dtt(h, loc, j, h->r1); break;
                    case YYO_OP_DPP: c = op_dpp(h, r, th); break;
                    case YYO_OP_DPP_HAT: c = op_dpp_hat(h); break;
                    default: c = coef(h, field, d, p, i, j, k); break;
                    }
                    int idx[3] = { i, j, k };
                    int lo_i = ulo(loc, d), hi_i = uhi(h, loc, d), m = idx[d];
                    int reflect = (d == 0 && !is_face(loc, 0));
                    const double rho0 = wall_rho(h, field, 0), rho1 = wall_rho(h, field, 1);
                    double xm, xp, x0 = x[ix(h, p, i, j, k)];
                    int im[3] = { i, j, k }, ip[3] = { i, j, k };
                    im[d]--; ip[d]++;
                    xm = (m > lo_i) ? x[ix(h, p, im[0], im[1], im[2])] : (reflect ? -rho0 * x0 : 0.0);
                    xp = (m < hi_i) ? x[ix(h, p, ip[0], ip[1], ip[2])] : (reflect ? -rho1 * x0 : 0.0);
                    y[ix(h, p, i, j, k)] = c.lo * xm + c.di * x0 + c.up * xp;
                }
    return 0;
}

/* ------------------------------------------------------------------ */
/* one field's solve, pressure update, norms                            */
/* ------------------------------------------------------------------ */
/* sweep orders = factor orders of eq. Convect_Douglas, r_comp,
 * theta_comp, phi_comp */
static void sweep_order(int field, int ord[3])
{
    int loc = loc_of(field);
    if (loc == FR) { ord[0] = 1; ord[1] = 2; ord[2] = 0; }
    else if (loc == FT) { ord[0] = 2; ord[1] = 0; ord[2] = 1; }
    else { ord[0] = 0; ord[1] = 1; ord[2] = 2; }
}

static double vol(const yyo *h, int loc, int i, int j)
{
    double r = r_at(h, loc, i), th = t_at(h, loc, j);
    return r * r * sin(th) * h->dr * h->dth * h->dph;
}

/* l2 (midpoint rule) norm over a patch's unknowns of a padded array */
static double l2_unknowns(const yyo *h, int loc, const double *x, int p)
{
    double s = 0.0;
    for (int i = ulo(loc, 0); i <= uhi(h, loc, 0); i++)
        for (int j = ulo(loc, 1); j <= uhi(h, loc, 1); j++)
            for (int k = ulo(loc, 2); k <= uhi(h, loc, 2); k++) {
                double v = x[ix(h, p, i, j, k)];
                s += vol(h, loc, i, j) * v * v;
            }
    return sqrt(s);
}

static int norm_slot(int field)
{
    return field;   /* T,u1r,u1t,u1p,p1,u2r,u2t,u2p,p2 in enum order */
}

/* Solve one field on patches [p0,p1): residual, three sweeps in the
 * field's factor order, psi^k = psi^{k-1} + c (Sec. 4 steps xi->eta->zeta,
 * with eq. er). */
static void solve_field(yyo *h, int field, int p0, int p1, int kk)
{
    int loc = loc_of(field);
    double *pk = h->lev[field][YYO_LEV_K];
    for (int p = p0; p < p1; p++) {
        memset(h->res + p * h->npatch, 0, sizeof(double) * h->npatch);
#pragma omp parallel for collapse(2) schedule(static)
        for (int i = ulo(loc, 0); i <= uhi(h, loc, 0); i++)
            for (int j = ulo(loc, 1); j <= uhi(h, loc, 1); j++)
                for (int k = ulo(loc, 2); k <= uhi(h, loc, 2); k++)
                    h->res[ix(h, p, i, j, k)] = h->tau * residual_at(h, field, p, i, j, k);
    }
    int ord[3];
    sweep_order(field, ord);
    sweep_range(h, field, ord[0], h->res, h->wa, p0, p1);
    sweep_range(h, field, ord[1], h->wa, h->wb, p0, p1);
    sweep_range(h, field, ord[2], h->wb, h->wa, p0, p1);
    for (int p = p0; p < p1; p++) {
        for (int i = ulo(loc, 0); i <= uhi(h, loc, 0); i++)
            for (int j = ulo(loc, 1); j <= uhi(h, loc, 1); j++)
                for (int k = ulo(loc, 2); k <= uhi(h, loc, 2); k++)
                    pk[ix(h, p, i, j, k)] += h->wa[ix(h, p, i, j, k)];
        if (kk < MAXK) h->norms[kk][p][norm_slot(field)] = l2_unknowns(h, loc, h->wa, p);
    }
}

/* eq. nst_Mass1 and its bootstrapped form (eq. ac2, reading):
 * p1^k = p1^n - Div_h u1^{n+1/2} / chi;
 * p2^k = p2^n + (p1^k - p1^n) - Div_h u2^{n+1/2} / chi. */
static void pressure(yyo *h, int s, int p0, int p1, int kk)
{
    double *un[3], *uk[3];
    vel_arrays(h, s, YYO_LEV_N, un);
    vel_arrays(h, s, YYO_LEV_K, uk);
    int pf_ = s == 1 ? YYO_P1 : YYO_P2;
    double *pn = h->lev[pf_][YYO_LEV_N], *pk = h->lev[pf_][YYO_LEV_K];
    const double *p1n = h->lev[YYO_P1][YYO_LEV_N], *p1k = h->lev[YYO_P1][YYO_LEV_K];
    for (int p = p0; p < p1; p++) {
        double sinc = 0.0, sdiv = 0.0;
        for (int i = 0; i < h->nr; i++)
            for (int j = 0; j < h->nt; j++)
                for (int k = 0; k < h->np; k++) {
                    int64_t q = ix(h, p, i, j, k);
                    double w = vol(h, CC, i, j);
                    if (!in_ring(h, j, k)) {
                        double nv = pn[q] - div_avg(h, un, uk, p, i, j, k) / h->chi;
                        if (s == 2) nv += p1k[q] - p1n[q];
                        double inc = nv - pk[q];
                        pk[q] = nv;
                        sinc += w * inc * inc;
                    }
                    if (s == 2) {
                        double dv = div_rr(h, uk[0], p, i, j, k) + div_th(h, uk[1], p, i, j, k) +
                                    div_ph(h, uk[2], p, i, j, k);
                        sdiv += w * dv * dv;
                    }
                }
        if (kk < MAXK) {
            h->norms[kk][p][norm_slot(pf_)] = sqrt(sinc);
            if (s == 2) h->norms[kk][p][9] = sqrt(sdiv);
        }
    }
}

/* Algorithm step 7: the ring cells of pressure `field` on patches
 * [p0,p1) take the other patch's pressure, interpolated like every other
 * boundary value (cubic Lagrange at the same radial index).  All targets
 * are gathered before any is replaced, so in the additive mode each patch
 * reads the other's values as its pressure update left them. */
static void exchange_pressure(yyo *h, int field, int p0, int p1)
{
    double *a = h->lev[field][YYO_LEV_K];
    for (int pass = 0; pass < 2; pass++)
        for (int p = p0; p < p1; p++)
            for (int i = 0; i < h->nr; i++)
                for (int j = 0; j < h->nt; j++)
                    for (int k = 0; k < h->np; k++) {
                        if (!in_ring(h, j, k)) continue;
                        int64_t q = ix(h, p, i, j, k);
                        if (pass == 0) {
                            double th2, ph2;
                            yyo_involution(tc(h, j), pc(h, k), &th2, &ph2);
                            h->ptmp[q] = interp(h, a, CC, 1 - p, i, th2, ph2);
                        } else {
                            a[q] = h->ptmp[q];
                        }
                    }
}

int yyo_extrapolate(yyo *h)
{
    if (!h) return -1;
    int64_t n = 2 * h->npatch;
    for (int f = 0; f < YYO_NF; f++) {
        const double *a = h->lev[f][YYO_LEV_N], *b = h->lev[f][YYO_LEV_NM1];
        double *s = h->star[f];
        for (int64_t q = 0; q < n; q++) s[q] = 1.5 * a[q] - 0.5 * b[q];
    }
    return 0;
}

int yyo_residual(yyo *h, int field, double *out)
{
    if (!h || !out || field < 0 || field >= YYO_NF || field == YYO_P1 || field == YYO_P2) return -1;
    int loc = loc_of(field);
    memset(out, 0, sizeof(double) * 2 * h->npatch);
    for (int p = 0; p < 2; p++)
        for (int i = ulo(loc, 0); i <= uhi(h, loc, 0); i++)
            for (int j = ulo(loc, 1); j <= uhi(h, loc, 1); j++)
                for (int k = ulo(loc, 2); k <= uhi(h, loc, 2); k++)
                    out[ix(h, p, i, j, k)] = residual_at(h, field, p, i, j, k);
    return 0;
}

/* Solve every quantity on patches [p0,p1) in the order of the Algorithm
 * of Sec. 4: T, then u1 (r, theta, phi; Gauss-Seidel), p1 (and its
 * exchange, step 7, when on), then u2, p2. */
static void solve_all(yyo *h, int p0, int p1, int kk)
{
    solve_field(h, YYO_T, p0, p1, kk);
    solve_field(h, YYO_U1R, p0, p1, kk);
    solve_field(h, YYO_U1T, p0, p1, kk);
    solve_field(h, YYO_U1P, p0, p1, kk);
    pressure(h, 1, p0, p1, kk);
    if (h->nring > 0) exchange_pressure(h, YYO_P1, p0, p1);
    solve_field(h, YYO_U2R, p0, p1, kk);
    solve_field(h, YYO_U2T, p0, p1, kk);
    solve_field(h, YYO_U2P, p0, p1, kk);
    pressure(h, 2, p0, p1, kk);
    if (h->nring > 0) exchange_pressure(h, YYO_P2, p0, p1);
}

/* One time step n -> n+1 with K Schwarz iterations. */
/* largest increment norm of iteration kk over the computed quantities
 * (T, u1, p1, u2, p2) and both patches; the divergence slot is not one */
static double max_increment(const yyo *h, int kk)
{
    double m = 0.0;
    for (int p = 0; p < 2; p++)
        for (int q = 0; q < 9; q++)
            if (h->norms[kk][p][q] > m || h->norms[kk][p][q] != h->norms[kk][p][q]) m = h->norms[kk][p][q];
    return m;
}

/* One time step.  tol < 0: exactly K Schwarz iterations.  tol >= 0: stop
 * after the first iteration whose increments are all below tol (the stop
 * test of the numerical-tests section), at most K.  Returns the count. */
static int step_run(yyo *h, int K, double tol)
{
    size_t bytes = sizeof(double) * 2 * (size_t)h->npatch;
    if (!h->filled) {
        yyo_fill(h, YYO_LEV_N);
        yyo_fill(h, YYO_LEV_NM1);
        h->filled = 1;
    }
    yyo_extrapolate(h);
    for (int f = 0; f < YYO_NF; f++) memcpy(h->lev[f][YYO_LEV_K], h->lev[f][YYO_LEV_N], bytes);
    memset(h->norms, 0, sizeof(h->norms));
    int done = 0;
    for (int kk = 0; kk < K; kk++) {
        if (h->mode == 0) {
            yyo_fill(h, YYO_LEV_K);
            solve_all(h, 0, 2, kk);
        } else {
            for (int p = 0; p < 2; p++) {
                fill_patch(h, YYO_LEV_K, p);
                solve_all(h, p, p + 1, kk);
            }
        }
        done = kk + 1;
        if (h->verbose) {
            fprintf(stderr, "oracle: Schwarz iteration %d done\n", kk + 1);
            fflush(stderr);
        }
        if (tol >= 0.0 && kk < MAXK && max_increment(h, kk) < tol) break;
    }
    h->nk = done < MAXK ? done : MAXK;
    yyo_fill(h, YYO_LEV_K);
    for (int f = 0; f < YYO_NF; f++) {
        memcpy(h->lev[f][YYO_LEV_NM1], h->lev[f][YYO_LEV_N], bytes);
        memcpy(h->lev[f][YYO_LEV_N], h->lev[f][YYO_LEV_K], bytes);
    }
    /* wall data moves with its level: n-1 <- n <- k; the k slot keeps the
     * old n-1 data until the caller sets the next step's values */
    for (int c = 0; c < 4; c++)
        for (int w = 0; w < 2; w++) {
            double *t = h->wall[c][YYO_LEV_NM1][w];
            h->wall[c][YYO_LEV_NM1][w] = h->wall[c][YYO_LEV_N][w];
            h->wall[c][YYO_LEV_N][w] = h->wall[c][YYO_LEV_K][w];
            h->wall[c][YYO_LEV_K][w] = t;
        }
    return done;
}

int yyo_step(yyo *h, int K)
{
    if (!h || K < 1) return -1;
    step_run(h, K, -1.0);
    return 0;
}

int yyo_step_tol(yyo *h, int kmax, double tol)
{
    if (!h || kmax < 1 || kmax > MAXK || !(tol >= 0.0)) return -1;
    return step_run(h, kmax, tol);
}

int yyo_get_norms(const yyo *h, double *out, int cap)
{
    if (!h || !out) return -1;
    int n = 0;
    for (int kk = 0; kk < h->nk; kk++)
        for (int p = 0; p < 2; p++)
            for (int q = 0; q < NNORM; q++) {
                if (n < cap) out[n] = h->norms[kk][p][q];
                n++;
            }
    return n;
}

void yyo_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}

int yyo_omp_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

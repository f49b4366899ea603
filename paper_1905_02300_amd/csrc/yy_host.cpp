// yy_host.cpp -- host side of libyy.so: C-ABI entry points (include/yy.h),
// metric and overlap-interpolation tables, workspace layout, and the
// schedule of one time step (Sec. 4 Algorithm, additive Schwarz).
#include <algorithm>
#include <cctype>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/yy.h"
#include "yy_internal.h"

using namespace yy;

namespace {

constexpr int MAXK = 64;
constexpr int64_t ALIGN = 256;
// independent chains of batched launches in an ensemble graph (one per
// hardware queue a process gets by default)
constexpr size_t BATCH_BRANCHES = 4;

int64_t align_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct Layout {
    Dims d;
    int64_t field_elems;     // elements of one field array (both patches)
    int prec;
    int64_t ncc, nvt, nvp;   // interpolation targets per class
    // byte offsets
    int64_t off_fields, off_p, off_tab_r, off_tab_d, off_ptab_r, off_ptab_d, off_fill, off_partial,
        off_norms, off_wall, off_mf, off_ring, off_tref, total;
    int64_t nring_max;       // ring targets of the pressure exchange at NRING_MAX rings
    int64_t wall_elems;      // doubles of one wall-data slot: 2 (nt+2)(np+2)
    int64_t elem;            // bytes per compute element
    int nR;                  // compute-precision arrays
};

int64_t ntab_r(const Dims &d) { return (d.nr + 2) + (d.nr + 3) + (int64_t)NTAB_R * (d.nr + 3); }
int64_t ntab_t(const Dims &d) { return 2 * (d.nt + 2) + 2 * (d.nt + 3) + (int64_t)NTAB_T * (d.nt + 3); }

// compute-precision arrays: T (3 levels) + T*, u (2x3x3) + u* (2x3),
// forcing (4), residual, Thomas scratch
constexpr int N_R_ARRAYS = 4 + 18 + 6 + 4 + 2;

bool valid_grid(const yy_grid *g, int prec)
{
    if (!(g && g->nr >= 2 && g->nt >= 6 && g->np >= 6 && g->nr <= 4096 && g->nt <= 4096 &&
          g->np <= 8192 && g->r1 > 0.0 && g->r2 > g->r1 && std::isfinite(g->r1) &&
          std::isfinite(g->r2)))
        return false;
    // kernels address a field by a 32-bit byte offset: one FP64 array (both
    // patches, ghosts and row padding; the pressures are FP64 in both
    // precisions) must stay below 4 GiB
    const int64_t field =
        2 * (int64_t)(g->nr + 2) * (g->nt + 2) * row_pitch(g->np, prec == YY_FP64 ? 8 : 4) * 8;
    return field < ((int64_t)1 << 32);
}

Layout make_layout(const yy_grid *g, int prec)
{
    Layout L{};
    L.prec = prec;
    L.d.nr = g->nr;
    L.d.nt = g->nt;
    L.d.np = g->np;
    L.d.ko = row_origin(prec == YY_FP64 ? 8 : 4);
    L.d.sJ = row_pitch(g->np, prec == YY_FP64 ? 8 : 4);
    L.d.sI = (int64_t)(g->nt + 2) * L.d.sJ;
    L.d.sP = (int64_t)(g->nr + 2) * L.d.sI;
    L.d.p0 = 0;
    L.d.npatch = 2;
    L.field_elems = 2 * L.d.sP;
    L.elem = prec == YY_FP64 ? 8 : 4;
    L.ncc = 2LL * g->np + 2LL * g->nt;
    L.nvt = 2LL * g->np + 2LL * (g->nt - 1);
    L.nvp = 2LL * g->nt + 2LL * (g->np - 1);
    int64_t o = 0;
    L.off_fields = o;
    o += align_up(N_R_ARRAYS * L.field_elems * L.elem, ALIGN);
    L.off_p = o;
    o += align_up(4 * L.field_elems * 8, ALIGN);
    L.off_tab_r = o;
    o += align_up((ntab_r(L.d) + ntab_t(L.d)) * L.elem, ALIGN);
    L.off_tab_d = o;
    o += align_up((ntab_r(L.d) + ntab_t(L.d)) * 8, ALIGN);
    L.off_ptab_r = o;
    o += align_up(3 * ((int64_t)g->nr + 3 + g->nt + 3) * L.elem, ALIGN);
    L.off_ptab_d = o;
    o += align_up(3 * ((int64_t)g->nr + 3 + g->nt + 3) * 8, ALIGN);
    L.off_fill = o;
    o += align_up(L.ncc * (int64_t)sizeof(FillScalar) + (L.nvt + L.nvp) * (int64_t)sizeof(FillVector), ALIGN);
    L.off_partial = o;
    o += align_up((int64_t)NSLOT * 2 * NBMAX * 8, ALIGN);
    L.off_norms = o;
    o += align_up((int64_t)MAXK * 2 * NSLOT * 8, ALIGN);
    // wall data: T, u_r, u_theta, u_phi x 3 levels x 2 walls
    L.wall_elems = 2 * (int64_t)(g->nt + 2) * (g->np + 2);
    L.off_wall = o;
    o += 24 * align_up(L.wall_elems * 8, ALIGN);
    L.off_mf = o;
    o += align_up((int64_t)4 * MF_BLOCKS * 8, ALIGN);
    // targets of the pressure exchange (Algorithm step 7), up to NRING_MAX rings
    {
        const int64_t it = std::max<int64_t>(0, g->nt - 2 * NRING_MAX), ip = std::max<int64_t>(0, g->np - 2 * NRING_MAX);
        L.nring_max = (int64_t)g->nt * g->np - it * ip;
    }
    L.off_ring = o;
    o += align_up(L.nring_max * (int64_t)sizeof(FillScalar), ALIGN);
    // T's reference profile (FP64) and its radial difference (compute
    // precision), i = -1..nr
    L.off_tref = o;
    o += 2 * align_up(((int64_t)g->nr + 2) * 8, ALIGN);
    L.total = o;
    return L;
}

// ---------------- geometry (Sec. 2) ----------------
struct Frame {
    double th0, ph0, dth, dph, dr, r1, r2, delta;
};

// The Yin <-> Yang map (x,y,z) -> (-x,z,y) is an involution: the same
// formula gives the other patch's (theta, phi) of a point of either patch.
void other_coords(double th, double ph, double &th2, double &ph2)
{
    const double st = std::sin(th);
    double c = st * std::sin(ph);       // y = cos(theta')
    c = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
    th2 = std::acos(c);
    ph2 = std::atan2(std::cos(th), -st * std::cos(ph));
}

// Rows of the 2x2 matrix taking the other patch's (v_theta', v_phi') at the
// image point to this patch's (v_theta, v_phi): dot products of the local
// unit vectors, the other patch's expressed in this patch's frame.
void rotation(double th, double ph, double m[2][2])
{
    double th2, ph2;
    other_coords(th, ph, th2, ph2);
    const double et[3] = {std::cos(th) * std::cos(ph), std::cos(th) * std::sin(ph), -std::sin(th)};
    const double ep[3] = {-std::sin(ph), std::cos(ph), 0.0};
    const double eto[3] = {-std::cos(th2) * std::cos(ph2), -std::sin(th2), std::cos(th2) * std::sin(ph2)};
    const double epo[3] = {std::sin(ph2), 0.0, std::cos(ph2)};
    auto dot = [](const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
    m[0][0] = dot(et, eto);
    m[0][1] = dot(et, epo);
    m[1][0] = dot(ep, eto);
    m[1][1] = dot(ep, epo);
}

// Cubic Lagrange window on n uniform donor nodes x0 + m h: first node
// (clamped so the four nodes exist) and weights.  false = outside the span.
bool window(double x, double x0, double h, int n, int &m0, double w[4])
{
    const double s = (x - x0) / h;
    if (!(s >= 0.0 && s <= (double)(n - 1)) || n < 4) return false;
    int b = (int)std::floor(s) - 1;
    if (b < 0) b = 0;
    if (b > n - 4) b = n - 4;
    m0 = b;
    const double u = s - b;
    w[0] = -(u - 1.0) * (u - 2.0) * (u - 3.0) / 6.0;
    w[1] = u * (u - 2.0) * (u - 3.0) / 2.0;
    w[2] = -u * (u - 1.0) * (u - 3.0) / 2.0;
    w[3] = u * (u - 1.0) * (u - 2.0) / 6.0;
    return true;
}

// donor grid of the other patch along theta or phi: its unknowns only
struct Axis {
    double x0, h;
    int n, off;
};
Axis centres(double start, double h, int N) { return {start + 0.5 * h, h, N, 0}; }
Axis faces(double start, double h, int N) { return {start + h, h, N - 1, 1}; }

bool build_fill(const Frame &F, const Dims &d, std::vector<FillScalar> &cc,
                std::vector<FillVector> &vt, std::vector<FillVector> &vp)
{
    const Axis tc = centres(F.th0, F.dth, d.nt), tfc = faces(F.th0, F.dth, d.nt);
    const Axis pc = centres(F.ph0, F.dph, d.np), pfc = faces(F.ph0, F.dph, d.np);
    auto thc = [&](int j) { return F.th0 + (j + 0.5) * F.dth; };
    auto thf = [&](int j) { return F.th0 + j * F.dth; };
    auto phc = [&](int k) { return F.ph0 + (k + 0.5) * F.dph; };
    auto phf = [&](int k) { return F.ph0 + k * F.dph; };
    bool ok = true;
    auto add_scalar = [&](int j, int k) {
        double a, b;
        other_coords(thc(j), phc(k), a, b);
        FillScalar e{};
        int mt = 0, mp = 0;
        ok = ok && window(a, tc.x0, tc.h, tc.n, mt, e.wt) && window(b, pc.x0, pc.h, pc.n, mp, e.wp);
        e.tj = j; e.tk = k; e.dj = mt + tc.off; e.dk = mp + pc.off;
        cc.push_back(e);
    };
    auto add_vector = [&](std::vector<FillVector> &v, double th, double ph, int j, int k, int row) {
        double a, b, m[2][2];
        other_coords(th, ph, a, b);
        rotation(th, ph, m);
        FillVector e{};
        int m1 = 0, m2 = 0, m3 = 0, m4 = 0;
        ok = ok && window(a, tfc.x0, tfc.h, tfc.n, m1, e.wtA) && window(b, pc.x0, pc.h, pc.n, m2, e.wpA);
        ok = ok && window(a, tc.x0, tc.h, tc.n, m3, e.wtB) && window(b, pfc.x0, pfc.h, pfc.n, m4, e.wpB);
        e.tj = j; e.tk = k;
        e.tjA = m1 + tfc.off; e.tkA = m2 + pc.off;
        e.tjB = m3 + tc.off; e.tkB = m4 + pfc.off;
        e.ma = m[row][0];
        e.mb = m[row][1];
        v.push_back(e);
    };
    // centre-type in theta and phi: ghost rows, then ghost columns
    for (int k = 0; k < d.np; k++) { add_scalar(-1, k); add_scalar(d.nt, k); }
    for (int j = 0; j < d.nt; j++) { add_scalar(j, -1); add_scalar(j, d.np); }
    // u_theta: boundary faces j = 0, Nt; phi ghosts of interior faces
    for (int k = 0; k < d.np; k++) {
        add_vector(vt, thf(0), phc(k), 0, k, 0);
        add_vector(vt, thf(d.nt), phc(k), d.nt, k, 0);
    }
    for (int j = 1; j < d.nt; j++) {
        add_vector(vt, thf(j), phc(-1), j, -1, 0);
        add_vector(vt, thf(j), phc(d.np), j, d.np, 0);
    }
    // u_phi: boundary faces k = 0, Np; theta ghosts of interior faces
    for (int j = 0; j < d.nt; j++) {
        add_vector(vp, thc(j), phf(0), j, 0, 1);
        add_vector(vp, thc(j), phf(d.np), j, d.np, 1);
    }
    for (int k = 1; k < d.np; k++) {
        add_vector(vp, thc(-1), phf(k), -1, k, 1);
        add_vector(vp, thc(d.nt), phf(k), d.nt, k, 1);
    }
    return ok;
}

// Targets of the pressure exchange (Algorithm step 7): the centres of the
// outermost nring cells in theta and phi, each interpolated from the other
// patch's centres.  false if one lies outside the donor span.
bool build_ring(const Frame &F, const Dims &d, int nring, std::vector<FillScalar> &ring)
{
    const Axis tc = centres(F.th0, F.dth, d.nt), pc = centres(F.ph0, F.dph, d.np);
    ring.clear();
    for (int j = 0; j < d.nt; j++)
        for (int k = 0; k < d.np; k++) {
            if (!(j < nring || j >= d.nt - nring || k < nring || k >= d.np - nring)) continue;
            double a, b;
            other_coords(F.th0 + (j + 0.5) * F.dth, F.ph0 + (k + 0.5) * F.dph, a, b);
            FillScalar e{};
            int mt = 0, mp = 0;
            if (!window(a, tc.x0, tc.h, tc.n, mt, e.wt) || !window(b, pc.x0, pc.h, pc.n, mp, e.wp)) return false;
            e.tj = j; e.tk = k; e.dj = mt + tc.off; e.dk = mp + pc.off;
            ring.push_back(e);
        }
    return true;
}

double safe_inv(double x) { return x != 0.0 ? 1.0 / x : 0.0; }

// Position tables, then the coefficient tables of the split operators
// (unit viscosity) in the order of the Geo members, all in FP64.
template <typename R> void host_tables(const Frame &F, const Dims &d, std::vector<R> &v)
{
    v.clear();
    auto rc = [&](int i) { return F.r1 + (i + 0.5) * F.dr; };
    auto rf = [&](int f) { return F.r1 + f * F.dr; };
    auto sc = [&](int j) { return std::sin(F.th0 + (j + 0.5) * F.dth); };
    auto cc = [&](int j) { return std::cos(F.th0 + (j + 0.5) * F.dth); };
    auto sf = [&](int f) { return std::sin(F.th0 + f * F.dth); };
    auto cf = [&](int f) { return std::cos(F.th0 + f * F.dth); };
    for (int i = -1; i <= d.nr; i++) v.push_back((R)rc(i));
    for (int f = -1; f <= d.nr + 1; f++) v.push_back((R)rf(f));
    for (int j = -1; j <= d.nt; j++) v.push_back((R)sc(j));
    for (int j = -1; j <= d.nt; j++) v.push_back((R)cc(j));
    for (int f = -1; f <= d.nt + 1; f++) v.push_back((R)sf(f));
    for (int f = -1; f <= d.nt + 1; f++) v.push_back((R)cf(f));
    const double dr2 = F.dr * F.dr, dt2 = F.dth * F.dth, R12 = F.r1 * F.r1;
    std::vector<std::vector<double>> tr(NTAB_R), tt(NTAB_T);
    for (int e = -1; e <= d.nr + 1; e++) {
        const double c0 = rc(e), f0 = rf(e), cm = rc(e - 1), fm = rf(e - 1), fp = rf(e + 1), c1 = rc(e + 1);
        (void)c1;
        tr[0].push_back(safe_inv(c0));
        tr[1].push_back(safe_inv(f0));
        tr[2].push_back(safe_inv(c0 * c0));
        tr[3].push_back(safe_inv(f0 * f0));
        // D_rr at centre i = e: faces e, e+1
        tr[4].push_back(f0 * f0 * safe_inv(c0 * c0 * dr2));
        tr[5].push_back(fp * fp * safe_inv(c0 * c0 * dr2));
        // u_r at face f = e: D_rr(face) - 2/r^2 + (2/r^3) d_r(r^2 .)
        const double lo0 = cm * cm * safe_inv(f0 * f0 * dr2), up0 = c0 * c0 * safe_inv(f0 * f0 * dr2);
        const double k3 = 2.0 * safe_inv(f0 * f0 * f0) / (2.0 * F.dr);
        tr[6].push_back(lo0 - k3 * fm * fm);
        tr[7].push_back(up0 + k3 * fp * fp);
        tr[8].push_back(-(lo0 + up0) - 2.0 * safe_inv(f0 * f0));
        // D11 = G_r Div_r at face f = e
        tr[9].push_back(fm * fm * safe_inv(cm * cm * dr2));
        tr[10].push_back(fp * fp * safe_inv(c0 * c0 * dr2));
        tr[11].push_back(-f0 * f0 * (safe_inv(c0 * c0) + safe_inv(cm * cm)) / dr2);
        // Div_r at centre i = e
        tr[12].push_back(fp * fp * safe_inv(c0 * c0 * F.dr));
        tr[13].push_back(f0 * f0 * safe_inv(c0 * c0 * F.dr));
    }
    for (int e = -1; e <= d.nt + 1; e++) {
        const double s0 = sc(e), sF = sf(e), sFm = sf(e - 1), sFp = sf(e + 1), sCm = sc(e - 1);
        // Dhat_thth at theta-centre j = e and theta-face f = e
        tt[0].push_back(sF * safe_inv(R12 * s0 * dt2));
        tt[1].push_back(sFp * safe_inv(R12 * s0 * dt2));
        tt[2].push_back(sCm * safe_inv(R12 * sF * dt2));
        tt[3].push_back(s0 * safe_inv(R12 * sF * dt2));
        // u_theta: -u/sin^2 + (2 cos/sin^2) d_th(sin u), times 1/r^2
        const double w = 2.0 * cf(e) * safe_inv(sF * sF) / (2.0 * F.dth);
        tt[4].push_back(-w * sFm);
        tt[5].push_back(w * sFp);
        tt[6].push_back(-safe_inv(sF * sF));
        // D22 = G_th Div_th at theta-face f = e, times 1/r^2
        tt[7].push_back(sFm * safe_inv(sCm * dt2));
        tt[8].push_back(sFp * safe_inv(s0 * dt2));
        tt[9].push_back(-sF * (safe_inv(s0) + safe_inv(sCm)) / dt2);
        tt[10].push_back(safe_inv(2.0 * s0 * F.dph));
        tt[11].push_back(safe_inv(2.0 * sF * F.dph));
        tt[12].push_back(safe_inv(s0 * s0));
        tt[13].push_back(safe_inv(sF * sF));
        tt[14].push_back(cc(e) * safe_inv(s0));
        // Div_th at centre j = e (times 1/r), Div_ph factor, cot at faces, 1/sin
        tt[15].push_back(sFp * safe_inv(s0 * F.dth));
        tt[16].push_back(sF * safe_inv(s0 * F.dth));
        tt[17].push_back(safe_inv(s0 * F.dph));
        tt[18].push_back(cf(e) * safe_inv(sF));
        tt[19].push_back(safe_inv(s0));
    }
    for (auto &t : tr)
        for (double x : t) v.push_back((R)x);
    for (auto &t : tt)
        for (double x : t) v.push_back((R)x);
}

template <typename R> void bind_geo(Geo<R> &g, const R *base, const Dims &d, const Frame &F)
{
    g.rc = base;
    g.rf = base + (d.nr + 2);
    g.sc = (const R *)g.rf + (d.nr + 3);
    g.cc = (const R *)g.sc + (d.nt + 2);
    g.sf = (const R *)g.cc + (d.nt + 2);
    g.cf = (const R *)g.sf + (d.nt + 3);
    const R *tr = (const R *)g.cf + (d.nt + 3);
    const int64_t lr = d.nr + 3, lt = d.nt + 3;
    CPtr<R> *rt[NTAB_R] = {&g.ir_c, &g.ir_f, &g.ir2_c, &g.ir2_f, &g.rc_lo, &g.rc_up,
                            &g.rf_lo, &g.rf_up, &g.rf_di, &g.gf_lo, &g.gf_up, &g.gf_di,
                            &g.dr_p, &g.dr_m};
    for (int q = 0; q < NTAB_R; q++) *rt[q] = tr + q * lr;
    const R *tt = tr + NTAB_R * lr;
    CPtr<R> *tp[NTAB_T] = {&g.tc_lo, &g.tc_up, &g.tf_lo, &g.tf_up, &g.ef_lo, &g.ef_up, &g.ef_di,
                            &g.gt_lo, &g.gt_up, &g.gt_di, &g.h2p_c, &g.h2p_f, &g.is2_c, &g.is2_f,
                            &g.cot_c, &g.dt_p, &g.dt_m, &g.dp_c, &g.cot_f, &g.is_c};
    for (int q = 0; q < NTAB_T; q++) *tp[q] = tt + q * lt;
    g.h2r = (R)(1.0 / (2.0 * F.dr));
    g.h2t = (R)(1.0 / (2.0 * F.dth));
    g.idph2 = (R)(1.0 / (F.dph * F.dph));
    g.idr = (R)(1.0 / F.dr);
    g.idth = (R)(1.0 / F.dth);
    g.idph = (R)(1.0 / F.dph);
    g.r12 = (R)(F.r1 * F.r1);
    g.dr = (R)F.dr;
    g.dth = (R)F.dth;
    g.dph = (R)F.dph;
    g.r1 = (R)F.r1;
    const double th1 = M_PI / 4.0 - F.delta;
    g.cphat = (R)(1.0 / (F.r1 * F.r1 * std::sin(th1) * std::sin(th1) * F.dph * F.dph));
    g.rho_t[0] = g.rho_t[1] = R(1);   // Dirichlet until yy_set_t_bc
    g.rho_u[0] = g.rho_u[1] = R(1);   // Dirichlet until yy_set_u_bc
}

// parameter-dependent tables: Pr * (u_r radial) + (1/(2 chi)) * D11 per
// r-face, and Pr * (u_theta extra) + (1/(2 chi)) * D22 per theta-face
template <typename R>
int upload_param_tables(Geo<R> &g, const Frame &F, const Dims &d, const yy_params &p, char *dev)
{
    std::vector<double> td;
    host_tables<double>(F, d, td);
    const int64_t lr = d.nr + 3, lt = d.nt + 3;
    const double *tr = td.data() + (d.nr + 2) + (d.nr + 3) + 2 * (d.nt + 2) + 2 * (d.nt + 3);
    const double *tt = tr + NTAB_R * lr;
    const double pr = p.pr, ic = 1.0 / (2.0 * p.chi);
    std::vector<R> v;
    for (int q = 0; q < 3; q++)
        for (int64_t e = 0; e < lr; e++) v.push_back((R)(pr * tr[(6 + q) * lr + e] + ic * tr[(9 + q) * lr + e]));
    for (int q = 0; q < 3; q++)
        for (int64_t e = 0; e < lt; e++) v.push_back((R)(pr * tt[(4 + q) * lt + e] + ic * tt[(7 + q) * lt + e]));
    if (hipMemcpy(dev, v.data(), v.size() * sizeof(R), hipMemcpyHostToDevice) != hipSuccess) return YY_ERR_HIP;
    const R *b = (const R *)dev;
    g.fr_lo = b; g.fr_up = b + lr; g.fr_di = b + 2 * lr;
    g.ft_lo = b + 3 * lr; g.ft_up = b + 3 * lr + lt; g.ft_di = b + 3 * lr + 2 * lt;
    return YY_OK;
}

template <typename R> void set_coefs(Geo<R> &g, const yy_params &p)
{
    g.ht = (R)(0.5 * p.dt);
    g.tau = (R)p.dt;
    g.inv_tau = (R)(1.0 / p.dt);
    g.pr = (R)p.pr;
    g.ic = (R)(1.0 / (2.0 * p.chi));
    g.prra = (R)(p.pr * p.ra);
    g.inv_chi = 1.0 / p.chi;
    g.prra_d = p.pr * p.ra;
}

}  // namespace

enum ProfClass {
    PC_START = 0, PC_EXTRAP, PC_FILL, PC_RES_T, PC_RES_UR, PC_RES_UT, PC_RES_UP,
    PC_SW_R, PC_SW_T, PC_SW_P, PC_SW_R_LAST, PC_SW_T_LAST, PC_SW_P_LAST,
    PC_PRESS1, PC_PRESS2, PC_REDUCE, PC_SW_P_LAST_T
};
// step_start: extrapolation and working level of a step (extrap: the
// extrapolation alone, yy_extrapolate); sweep_p_last: the last (phi) factor
// of u_phi; sweep_p_last_T: that of T
static const char *prof_names[YY_NPROF] = {
    "step_start", "extrap", "fill", "residual_T", "residual_ur", "residual_ut", "residual_up",
    "sweep_r", "sweep_t", "sweep_p", "sweep_r_last", "sweep_t_last", "sweep_p_last",
    "pressure_1", "pressure_2", "norm_reduce", "sweep_p_last_T"};

struct yy_shell {
    uint64_t version = 0;    // bumped by every state or parameter change
    // live timing: event pairs around launch groups
    bool prof = false;
    std::vector<hipEvent_t> ev;
    std::vector<int> ev_cls;
    size_t ev_used = 0;
    Layout L;
    Frame F;
    yy_params prm;
    bool have_params = false, need_fill = true;
    int sticky = YY_OK;
    int last_k = 0;
    char *ws = nullptr;
    Geo<double> gd, g64;
    Geo<float> g32;
    State<double> s64;
    State<float> s32;
    double *pres[2][2];
    FillScalar *fcc = nullptr;
    FillVector *fvt = nullptr, *fvp = nullptr;
    double *partial = nullptr, *norms = nullptr;
    int nblocks[NSLOT];
    bool has_force[4] = {false, false, false, false};
    void *force_ptr[4];
    // Dirichlet wall data per (T, u_r, u_theta, u_phi) x level x wall: device
    // slot, whether it holds data, and whether the iterate's (level k) data
    // was set since the last step; slots rotate with the levels
    double *wall[4][3][2];
    bool wall_on[4][3][2] = {};
    bool wall_fresh[4][2] = {};
    // T's wall conditions a T + b dT/dn = g, (a, b) per wall, and the
    // derived ghost coefficients
    double t_ab[2][2] = {{1.0, 0.0}, {1.0, 0.0}};
    TRobin tb = {{2.0, 2.0}, {1.0, 1.0}, {0.0, 0.0}};
    // the tangential velocity's walls a u + b R dn(u/r) = g
    URobin ub = {{2.0, 2.0}, {1.0, 1.0}};
    // FP32-mixed: T is stored as T - Tref, Tref the discrete conductive
    // profile of the wall temperatures (host copy, i = -1..nr)
    std::vector<double> tref;
    // Algorithm step 7: rings of pressure cells taken from the other patch
    int nring = 0;
    int nptab = 0;
    FillScalar *ptab = nullptr;
    // Algorithm step 4 on every velocity fill
    bool mass_fix = false;
    double mf_S = 0.0;           // sum of the squared boundary flux weights
    double mf_A = 0.0;           // area of a patch's boundary
    double mf_eps = 0.0, mf_tol = 0.0;   // step 4's epsilon (0: the limit) and flux trigger
    double *mfp = nullptr;       // partial net fluxes
};

namespace {

template <typename R> State<R> &state_of(yy_shell *s);
template <> State<double> &state_of<double>(yy_shell *s) { return s->s64; }
template <> State<float> &state_of<float>(yy_shell *s) { return s->s32; }
template <typename R> Geo<R> &geo_of(yy_shell *s);
template <> Geo<double> &geo_of<double>(yy_shell *s) { return s->g64; }
template <> Geo<float> &geo_of<float>(yy_shell *s) { return s->g32; }

template <typename R> void bind_state(yy_shell *s)
{
    State<R> &st = state_of<R>(s);
    R *base = (R *)(s->ws + s->L.off_fields);
    const int64_t n = s->L.field_elems;
    int a = 0;
    auto next = [&]() { return base + (a++) * n; };
    for (int l = 0; l < 3; l++) st.T[l] = next();
    st.Ts = next();
    for (int y = 0; y < 2; y++)
        for (int c = 0; c < 3; c++)
            for (int l = 0; l < 3; l++) st.u[y][c][l] = next();
    for (int y = 0; y < 2; y++)
        for (int c = 0; c < 3; c++) st.us[y][c] = next();
    for (int c = 0; c < 4; c++) {
        s->force_ptr[c] = next();
        st.force[c] = nullptr;
    }
    st.res = next();
    st.cb = next();
    double *pb = (double *)(s->ws + s->L.off_p);
    for (int y = 0; y < 2; y++)
        for (int l = 0; l < 2; l++) st.p[y][l] = pb + (y * 2 + l) * n;
}

int loc_of(int f)
{
    switch (f) {
    case YY_U1R: case YY_U2R: return FR;
    case YY_U1T: case YY_U2T: return FT;
    case YY_U1P: case YY_U2P: return FP;
    default: return CC;
    }
}

int hip_status(hipError_t e) { return e == hipSuccess ? YY_OK : YY_ERR_HIP; }

template <typename R> R *field_ptr(yy_shell *s, int f, int lev)
{
    State<R> &st = state_of<R>(s);
    if (f == YY_T) return st.T[lev];
    const int y = f >= YY_U2R ? 1 : 0;
    const int c = f - (y ? YY_U2R : YY_U1R);
    return st.u[y][c][lev];
}

// RAII pair of timing events around a launch group (no-op unless enabled)
struct Timed {
    yy_shell *s;
    hipStream_t st;
    size_t slot;
    Timed(yy_shell *s_, int cls, hipStream_t st_) : s(s_), st(st_), slot((size_t)-1)
    {
        if (!s->prof || s->ev_used + 2 > s->ev.size()) return;
        slot = s->ev_used;
        s->ev_used += 2;
        s->ev_cls[slot / 2] = cls;
        (void)hipEventRecord(s->ev[slot], st);
    }
    ~Timed()
    {
        if (slot != (size_t)-1) (void)hipEventRecord(s->ev[slot + 1], st);
    }
};

WallLev walls_of(const yy_shell *s, int lev)
{
    WallLev w;
    for (int c = 0; c < 4; c++)
        for (int side = 0; side < 2; side++)
            w.v[c][side] = s->wall_on[c][lev][side] ? s->wall[c][lev][side] : nullptr;
    return w;
}

template <typename R> void do_fill(yy_shell *s, int lev, int pmask, hipStream_t st)
{
    Timed tm(s, PC_FILL, st);
    Ops<R>::fill(s->L.d, state_of<R>(s), lev, s->fcc, (int)s->L.ncc, s->fvt, (int)s->L.nvt, s->fvp,
                 (int)s->L.nvp, s->prm.t_inner, s->prm.t_outer, s->tb, s->ub, walls_of(s, lev), pmask, st);
    if (s->mass_fix)
        Ops<R>::mass_fix(s->L.d, s->gd, state_of<R>(s), lev, s->mf_S + s->mf_eps * s->mf_A * s->mf_A, s->mf_tol,
                         s->mfp, pmask, st);
}

template <typename R> void solve_field(yy_shell *s, const Dims &d, int f, hipStream_t st)
{
    State<R> &S = state_of<R>(s);
    const int loc = loc_of(f);
    static const int order[4][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 1, 2}};
    {
        Timed tm(s, PC_RES_T + loc, st);
        Ops<R>::residual(d, geo_of<R>(s), S, f, S.res, st);
    }
    for (int q = 0; q < 2; q++) {
        Timed tm(s, PC_SW_R + order[loc][q], st);
        Ops<R>::sweep(d, geo_of<R>(s), s->gd, S, f, order[loc][q], S.res, S.res, 0, nullptr, nullptr, 0, st);
    }
    Timed tm(s, loc == CC ? PC_SW_P_LAST_T : PC_SW_R_LAST + order[loc][2], st);
    Ops<R>::sweep(d, geo_of<R>(s), s->gd, S, f, order[loc][2], S.res, S.res, 1,
                  s->partial + (int64_t)f * 2 * NBMAX, &s->nblocks[f], 0, st);
}

template <typename R> void rotate_levels(yy_shell *s);

// one time step: extrapolation, Schwarz iterations, post-step fill, level
// rotation.  tol < 0: exactly K iterations.  tol >= 0: after each iteration
// the increment norms come to the host (a stream synchronisation) and the
// loop stops at the first iteration whose increments of every computed
// quantity (T, u1, p1, u2, p2; both patches) are below tol, at most K.
template <typename R> int step_impl(yy_shell *s, int K, double tol, int *k_done, hipStream_t st)
{
    State<R> &S = state_of<R>(s);
    if (s->need_fill) {
        do_fill<R>(s, 0, 3, st);
        do_fill<R>(s, 1, 3, st);
        s->need_fill = false;
    }
    {
        Timed tm(s, PC_START, st);
        Ops<R>::extrap_copy(s->L.d, S, st);
    }
    int done = 0;
    for (int k = 0; k < K; k++) {
        // additive: both patches at once from the other's iterate k-1;
        // multiplicative (Algorithm of Sec. 4): Yin, then Yang from Yin's k
        const int passes = s->prm.mode == YY_MULTIPLICATIVE ? 2 : 1;
        for (int pass = 0; pass < passes; pass++) {
            Dims d = s->L.d;
            int pmask = 3;
            if (passes == 2) {
                d.p0 = pass;
                d.npatch = 1;
                pmask = 1 << pass;
            }
            do_fill<R>(s, 2, pmask, st);
            solve_field<R>(s, d, YY_T, st);
            solve_field<R>(s, d, YY_U1R, st);
            solve_field<R>(s, d, YY_U1T, st);
            solve_field<R>(s, d, YY_U1P, st);
            {
                Timed tm(s, PC_PRESS1, st);
                Ops<R>::pressure(d, geo_of<R>(s), s->gd, S, 1, s->partial + (int64_t)YY_P1 * 2 * NBMAX,
                                 nullptr, &s->nblocks[YY_P1], s->nring, st);
                if (s->nring > 0) pressure_exchange(d, S.p[0][1], s->ptab, s->nptab, (double *)S.cb, st);
            }
            solve_field<R>(s, d, YY_U2R, st);
            solve_field<R>(s, d, YY_U2T, st);
            solve_field<R>(s, d, YY_U2P, st);
            {
                Timed tm(s, PC_PRESS2, st);
                Ops<R>::pressure(d, geo_of<R>(s), s->gd, S, 2, s->partial + (int64_t)YY_P2 * 2 * NBMAX,
                                 s->partial + (int64_t)9 * 2 * NBMAX, &s->nblocks[YY_P2], s->nring, st);
                if (s->nring > 0) pressure_exchange(d, S.p[1][1], s->ptab, s->nptab, (double *)S.cb, st);
            }
        }
        s->nblocks[9] = s->nblocks[YY_P2];
        {
            Timed tm(s, PC_REDUCE, st);
            reduce_norms(s->partial, s->nblocks, s->norms + (int64_t)k * 2 * NSLOT, st);
        }
        done = k + 1;
        if (tol >= 0.0) {
            double h[2 * NSLOT];
            hipError_t e = hipMemcpyAsync(h, s->norms + (int64_t)k * 2 * NSLOT, sizeof h,
                                          hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) return YY_ERR_HIP;
            double m = 0.0;
            for (int p = 0; p < 2; p++)
                for (int q = 0; q < NSLOT - 1; q++) {
                    const double v = h[p * NSLOT + q];
                    if (!std::isfinite(v)) {
                        s->sticky = YY_ERR_NONFINITE;
                        return YY_ERR_NONFINITE;
                    }
                    m = std::max(m, v);
                }
            if (m < tol) break;
        }
    }
    do_fill<R>(s, 2, 3, st);
    rotate_levels<R>(s);
    s->last_k = done;
    if (k_done) *k_done = done;
    return hip_status(hipGetLastError());
}

// rotate time levels: n-1 <- n <- k; the old n-1 becomes the next working
// level (host pointers only; the period is 6 = lcm of 3 and 2 levels)
template <typename R> void rotate_levels(yy_shell *s)
{
    State<R> &S = state_of<R>(s);
    R *t = S.T[1];
    S.T[1] = S.T[0]; S.T[0] = S.T[2]; S.T[2] = t;
    for (int y = 0; y < 2; y++)
        for (int c = 0; c < 3; c++) {
            R *u = S.u[y][c][1];
            S.u[y][c][1] = S.u[y][c][0];
            S.u[y][c][0] = S.u[y][c][2];
            S.u[y][c][2] = u;
        }
    for (int y = 0; y < 2; y++) {
        double *p = S.p[y][0];
        S.p[y][0] = S.p[y][1];
        S.p[y][1] = p;
    }
    // wall data moves with its level (n-1 <- n <- k); the k slot keeps the
    // old n-1 data, which the caller must replace before the next step
    for (int c = 0; c < 4; c++)
        for (int w = 0; w < 2; w++) {
            double *t = s->wall[c][1][w];
            const bool o = s->wall_on[c][1][w];
            s->wall[c][1][w] = s->wall[c][0][w];
            s->wall_on[c][1][w] = s->wall_on[c][0][w];
            s->wall[c][0][w] = s->wall[c][2][w];
            s->wall_on[c][0][w] = s->wall_on[c][2][w];
            s->wall[c][2][w] = t;
            s->wall_on[c][2][w] = o;
            s->wall_fresh[c][w] = false;
        }
}

// shift of T's wall ghost under deviation storage (zero in FP64)
void update_tshift(yy_shell *s)
{
    const int nr = s->L.d.nr;
    const bool dev = s->L.prec == YY_FP32_MIXED;
    s->tb.shift[0] = dev ? s->tb.rho[0] * s->tref[1] + s->tref[0] : 0.0;
    s->tb.shift[1] = dev ? s->tb.rho[1] * s->tref[nr] + s->tref[nr + 1] : 0.0;
}

// FP32-mixed: the discrete conductive profile of the wall temperatures
// (D_rr Tref = 0 at every centre with the reflection ghosts of Dirichlet
// walls: the flux r_f^2 dT is the same through every face), uploaded with
// its centred radial difference; stored T levels are shifted from the old
// reference to the new one.  Synchronous.
int set_reference_profile(yy_shell *s, double t_in, double t_out)
{
    if (s->L.prec != YY_FP32_MIXED) return YY_OK;
    const int nr = s->L.d.nr;
    const double dr = s->F.dr, r1 = s->F.r1;
    auto rf = [&](int f) { return r1 + f * dr; };
    double sum = 0.5 / (rf(0) * rf(0)) + 0.5 / (rf(nr) * rf(nr));
    for (int f = 1; f < nr; f++) sum += 1.0 / (rf(f) * rf(f));
    const double F = (t_out - t_in) / sum;
    std::vector<double> t(nr + 2);
    t[1] = t_in + 0.5 * F / (rf(0) * rf(0));
    for (int i = 1; i < nr; i++) t[i + 1] = t[i] + F / (rf(i) * rf(i));
    t[0] = 2.0 * t_in - t[1];
    t[nr + 1] = 2.0 * t_out - t[nr];
    std::vector<float> dtf(nr + 2, 0.0f);
    for (int i = 0; i < nr; i++) dtf[i + 1] = (float)((t[i + 2] - t[i]) / (2.0 * dr));
    std::vector<double> diff(nr + 2);
    bool moved = false;
    for (int i = 0; i < nr + 2; i++) {
        diff[i] = s->tref[i] - t[i];
        moved = moved || diff[i] != 0.0;
    }
    double *dev_t = (double *)(s->ws + s->L.off_tref);
    char *dev_d = s->ws + s->L.off_tref + align_up(((int64_t)nr + 2) * 8, ALIGN);
    hipError_t e = hipSuccess;
    if (moved) {
        // shift the stored deviations: T - old = (T - new) + (new - old)
        e = hipMemcpy(dev_t, diff.data(), diff.size() * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            State<float> &S = s->s32;
            for (int l = 0; l < 3; l++) Ops<float>::add_profile(s->L.d, S.T[l], dev_t, nullptr);
            Ops<float>::add_profile(s->L.d, S.Ts, dev_t, nullptr);
            e = hipDeviceSynchronize();
        }
    }
    if (e == hipSuccess) e = hipMemcpy(dev_t, t.data(), t.size() * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dev_d, dtf.data(), dtf.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) return YY_ERR_HIP;
    s->tref = t;
    update_tshift(s);
    return YY_OK;
}

// wall data in use for a field but not set for the step's iterate
bool walls_stale(const yy_shell *s)
{
    for (int c = 0; c < 4; c++)
        for (int w = 0; w < 2; w++)
            if ((s->wall_on[c][0][w] || s->wall_on[c][2][w]) && !s->wall_fresh[c][w]) return true;
    return false;
}

}  // namespace

extern "C" {

const char *yy_strerror(int st)
{
    switch (st) {
    case YY_OK: return "ok";
    case YY_ERR_ARG: return "invalid argument";
    case YY_ERR_GEOMETRY: return "overlap interpolation would extrapolate (overlap too small)";
    case YY_ERR_WORKSPACE: return "workspace too small or misaligned";
    case YY_ERR_HIP: return "HIP runtime error";
    case YY_ERR_NONFINITE: return "non-finite norm (the step diverged)";
    case YY_ERR_STATE: return "call out of order";
    default: return "unknown status";
    }
}

int yy_workspace_bytes(const yy_grid *g, int32_t prec, uint64_t *bytes)
{
    if (!valid_grid(g, prec) || !bytes || (prec != YY_FP64 && prec != YY_FP32_MIXED)) return YY_ERR_ARG;
    *bytes = (uint64_t)make_layout(g, prec).total;
    return YY_OK;
}

int yy_create(const yy_grid *g, int32_t prec, void *dev_ws, uint64_t ws_bytes, yy_shell **out)
{
    if (!out) return YY_ERR_ARG;
    *out = nullptr;
    if (!valid_grid(g, prec) || !dev_ws || (prec != YY_FP64 && prec != YY_FP32_MIXED)) return YY_ERR_ARG;
    Layout L = make_layout(g, prec);
    if ((uintptr_t)dev_ws % ALIGN) return YY_ERR_WORKSPACE;
    if (ws_bytes < (uint64_t)L.total) return YY_ERR_WORKSPACE;
    Frame F;
    F.r1 = g->r1;
    F.r2 = g->r2;
    F.delta = g->delta > 0.0 ? g->delta : M_PI / (2.0 * (g->nt - 2));
    F.dr = (g->r2 - g->r1) / g->nr;
    F.th0 = M_PI / 4.0 - F.delta;
    F.ph0 = -3.0 * M_PI / 4.0 - F.delta;
    F.dth = (M_PI / 2.0 + 2.0 * F.delta) / g->nt;
    F.dph = (1.5 * M_PI + 2.0 * F.delta) / g->np;
    std::vector<FillScalar> cc;
    std::vector<FillVector> vt, vp;
    if (!build_fill(F, L.d, cc, vt, vp)) return YY_ERR_GEOMETRY;
    yy_shell *s = new (std::nothrow) yy_shell();
    if (!s) return YY_ERR_ARG;
    s->L = L;
    s->F = F;
    s->ws = (char *)dev_ws;
    // occupancy queries of the launchers, here rather than under a capture
    if (prec == YY_FP64) Ops<double>::prepare();
    else Ops<float>::prepare();
    // zero the whole workspace (fields start at zero)
    zero_doubles((double *)s->ws, L.total / 8, nullptr);
    // tables
    std::vector<double> td;
    host_tables<double>(F, L.d, td);
    hipError_t e = hipMemcpy(s->ws + L.off_tab_d, td.data(), td.size() * 8, hipMemcpyHostToDevice);
    bind_geo<double>(s->gd, (const double *)(s->ws + L.off_tab_d), L.d, F);
    if (prec == YY_FP64) {
        bind_geo<double>(s->g64, (const double *)(s->ws + L.off_tab_d), L.d, F);
        bind_state<double>(s);
    } else {
        std::vector<float> tf;
        host_tables<float>(F, L.d, tf);
        if (e == hipSuccess)
            e = hipMemcpy(s->ws + L.off_tab_r, tf.data(), tf.size() * 4, hipMemcpyHostToDevice);
        bind_geo<float>(s->g32, (const float *)(s->ws + L.off_tab_r), L.d, F);
        bind_state<float>(s);
    }
    char *fb = s->ws + L.off_fill;
    s->fcc = (FillScalar *)fb;
    s->fvt = (FillVector *)(fb + cc.size() * sizeof(FillScalar));
    s->fvp = s->fvt + vt.size();
    if (e == hipSuccess) e = hipMemcpy(s->fcc, cc.data(), cc.size() * sizeof(FillScalar), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->fvt, vt.data(), vt.size() * sizeof(FillVector), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(s->fvp, vp.data(), vp.size() * sizeof(FillVector), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        delete s;
        return YY_ERR_HIP;
    }
    s->partial = (double *)(s->ws + L.off_partial);
    s->norms = (double *)(s->ws + L.off_norms);
    for (int c = 0; c < 4; c++)
        for (int l = 0; l < 3; l++)
            for (int w = 0; w < 2; w++)
                s->wall[c][l][w] = (double *)(s->ws + L.off_wall + ((c * 3 + l) * 2 + w) * align_up(L.wall_elems * 8, ALIGN));
    s->mfp = (double *)(s->ws + L.off_mf);
    s->ptab = (FillScalar *)(s->ws + L.off_ring);
    {
        const double *tr = (const double *)(s->ws + L.off_tref);
        char *dt = s->ws + L.off_tref + align_up(((int64_t)L.d.nr + 2) * 8, ALIGN);
        s->tref.assign(L.d.nr + 2, 0.0);
        s->gd.tref = tr; s->gd.dtref = (const double *)dt; s->gd.tdev = 0;
        s->g64.tref = tr; s->g64.dtref = (const double *)dt; s->g64.tdev = 0;
        s->g32.tref = tr; s->g32.dtref = (const float *)dt; s->g32.tdev = prec == YY_FP32_MIXED ? 1 : 0;
    }
    {
        // squared flux weights of the interpolated boundary faces (theta- and
        // phi-boundary), the same for both patches
        double S = 0.0, A = 0.0;
        const double s0 = std::sin(F.th0), s1 = std::sin(F.th0 + L.d.nt * F.dth);
        for (int i = 0; i < L.d.nr; i++) {
            const double rc = F.r1 + (i + 0.5) * F.dr;
            const double a0 = rc * s0 * F.dr * F.dph, a1 = rc * s1 * F.dr * F.dph, a2 = rc * F.dr * F.dth;
            S += L.d.np * (a0 * a0 + a1 * a1) + 2.0 * L.d.nt * a2 * a2;
            A += L.d.np * (a0 + a1) + 2.0 * L.d.nt * a2;
        }
        // the r walls (their data enter the flux, they are not corrected)
        const double r2 = F.r1 + L.d.nr * F.dr;
        for (int j = 0; j < L.d.nt; j++)
            A += (F.r1 * F.r1 + r2 * r2) * L.d.np * std::sin(F.th0 + (j + 0.5) * F.dth) * F.dth * F.dph;
        s->mf_S = S;
        s->mf_A = A;
    }
    for (int q = 0; q < NSLOT; q++) s->nblocks[q] = 0;
    *out = s;
    return YY_OK;
}

int yy_set_params(yy_shell *s, const yy_params *p)
{
    if (!s || !p) return YY_ERR_ARG;
    if (!(p->dt > 0.0) || !(p->chi > 0.0) || !(p->pr > 0.0) || !std::isfinite(p->ra) ||
        !std::isfinite(p->dt) || !std::isfinite(p->t_inner) || !std::isfinite(p->t_outer))
        return YY_ERR_ARG;
    if (p->mode != YY_ADDITIVE && p->mode != YY_MULTIPLICATIVE) return YY_ERR_ARG;
    s->prm = *p;
    set_coefs<double>(s->gd, *p);
    set_coefs<double>(s->g64, *p);
    set_coefs<float>(s->g32, *p);
    int st = upload_param_tables<double>(s->gd, s->F, s->L.d, *p, s->ws + s->L.off_ptab_d);
    if (st != YY_OK) return st;
    if (s->L.prec == YY_FP64) {
        s->g64.fr_lo = s->gd.fr_lo; s->g64.fr_up = s->gd.fr_up; s->g64.fr_di = s->gd.fr_di;
        s->g64.ft_lo = s->gd.ft_lo; s->g64.ft_up = s->gd.ft_up; s->g64.ft_di = s->gd.ft_di;
    } else {
        st = upload_param_tables<float>(s->g32, s->F, s->L.d, *p, s->ws + s->L.off_ptab_r);
        if (st != YY_OK) return st;
    }
    st = set_reference_profile(s, p->t_inner, p->t_outer);
    if (st != YY_OK) return st;
    s->have_params = true;
    s->need_fill = true;   // wall values may have changed
    s->version++;
    return YY_OK;
}

static bool field_ok(int f) { return f >= 0 && f < YY_NFIELDS; }

int yy_set_field(yy_shell *s, int32_t field, int32_t level, int32_t layout, const double *src,
                 hipStream_t st)
{
    if (!s || !field_ok(field) || !src || (layout != YY_MAC && layout != YY_PADDED) || level < 0 || level > 2)
        return YY_ERR_ARG;
    const int loc = loc_of(field);
    if (field == YY_P1 || field == YY_P2) {
        if (level == YY_LEVEL_NM1) return YY_ERR_ARG;
        const int y = field == YY_P2;
        double *dst = s->L.prec == YY_FP64 ? s->s64.p[y][level == 0 ? 0 : 1] : s->s32.p[y][level == 0 ? 0 : 1];
        io_double(s->L.d, dst, src, nullptr, loc, layout, st);
    } else if (s->L.prec == YY_FP64) {
        Ops<double>::io(s->L.d, field_ptr<double>(s, field, level), src, nullptr, loc, layout, nullptr, st);
    } else {
        Ops<float>::io(s->L.d, field_ptr<float>(s, field, level), src, nullptr, loc, layout,
                       field == YY_T ? (const double *)s->g32.tref : nullptr, st);
    }
    s->need_fill = true;
    s->version++;
    return hip_status(hipGetLastError());
}

int yy_get_field(yy_shell *s, int32_t field, int32_t level, int32_t layout, double *dst,
                 hipStream_t st)
{
    if (!s || !field_ok(field) || !dst || (layout != YY_MAC && layout != YY_PADDED) || level < 0 || level > 2)
        return YY_ERR_ARG;
    const int loc = loc_of(field);
    if (field == YY_P1 || field == YY_P2) {
        if (level == YY_LEVEL_NM1) return YY_ERR_ARG;
        const int y = field == YY_P2;
        double *src = s->L.prec == YY_FP64 ? s->s64.p[y][level == 0 ? 0 : 1] : s->s32.p[y][level == 0 ? 0 : 1];
        io_double(s->L.d, src, nullptr, dst, loc, layout, st);
    } else if (s->L.prec == YY_FP64) {
        Ops<double>::io(s->L.d, field_ptr<double>(s, field, level), nullptr, dst, loc, layout, nullptr, st);
    } else {
        Ops<float>::io(s->L.d, field_ptr<float>(s, field, level), nullptr, dst, loc, layout,
                       field == YY_T ? (const double *)s->g32.tref : nullptr, st);
    }
    return hip_status(hipGetLastError());
}

int yy_set_forcing(yy_shell *s, int32_t field, const double *src, hipStream_t st)
{
    if (!s) return YY_ERR_ARG;
    int c;
    switch (field) {
    case YY_T: c = 0; break;
    case YY_U1R: c = 1; break;
    case YY_U1T: c = 2; break;
    case YY_U1P: c = 3; break;
    default: return YY_ERR_ARG;
    }
    const int loc = loc_of(field);
    s->version++;
    if (s->L.prec == YY_FP64) {
        s->s64.force[c] = src ? (double *)s->force_ptr[c] : nullptr;
        if (src) Ops<double>::io(s->L.d, (double *)s->force_ptr[c], src, nullptr, loc, YY_MAC, nullptr, st);
    } else {
        s->s32.force[c] = src ? (float *)s->force_ptr[c] : nullptr;
        if (src) Ops<float>::io(s->L.d, (float *)s->force_ptr[c], src, nullptr, loc, YY_MAC, nullptr, st);
    }
    return hip_status(hipGetLastError());
}

int yy_set_t_bc(yy_shell *s, int32_t wall, double a, double b)
{
    if (!s || wall < 0 || wall > 1 || !(a >= 0.0) || !(b >= 0.0) || !(a + b > 0.0) || !std::isfinite(a) ||
        !std::isfinite(b))
        return YY_ERR_ARG;
    const double dr = s->F.dr;
    s->t_ab[wall][0] = a;
    s->t_ab[wall][1] = b;
    s->tb.cg[wall] = 1.0 / (0.5 * a + b / dr);
    s->tb.rho[wall] = (0.5 * a - b / dr) / (0.5 * a + b / dr);
    s->gd.rho_t[wall] = s->tb.rho[wall];
    s->g64.rho_t[wall] = s->tb.rho[wall];
    s->g32.rho_t[wall] = (float)s->tb.rho[wall];
    update_tshift(s);
    s->need_fill = true;
    s->version++;
    return YY_OK;
}

int yy_set_u_bc(yy_shell *s, int32_t wall, double a, double b)
{
    if (!s || wall < 0 || wall > 1 || !(a >= 0.0) || !(b >= 0.0) || !(a + b > 0.0) || !std::isfinite(a) ||
        !std::isfinite(b))
        return YY_ERR_ARG;
    const double dr = s->F.dr, R = wall == 0 ? s->F.r1 : s->F.r2;
    const double rg = wall == 0 ? R - 0.5 * dr : R + 0.5 * dr, ri = wall == 0 ? R + 0.5 * dr : R - 0.5 * dr;
    s->ub.cg[wall] = 1.0 / (0.5 * a + b * R / (rg * dr));
    s->ub.rho[wall] = (0.5 * a - b * R / (ri * dr)) * s->ub.cg[wall];
    s->gd.rho_u[wall] = s->ub.rho[wall];
    s->g64.rho_u[wall] = s->ub.rho[wall];
    s->g32.rho_u[wall] = (float)s->ub.rho[wall];
    s->need_fill = true;
    s->version++;
    return YY_OK;
}

int yy_set_mass_fix(yy_shell *s, int32_t on)
{
    if (!s || (on != 0 && on != 1)) return YY_ERR_ARG;
    if ((on != 0) != s->mass_fix) s->version++;
    s->mass_fix = on != 0;
    s->need_fill = true;
    return YY_OK;
}

int yy_set_mass_fix_params(yy_shell *s, double eps, double tol)
{
    if (!s || !(eps >= 0.0) || !(tol >= 0.0)) return YY_ERR_ARG;
    if (eps != s->mf_eps || tol != s->mf_tol) s->version++;
    s->mf_eps = eps;
    s->mf_tol = tol;
    s->need_fill = true;
    return YY_OK;
}

int yy_set_pressure_exchange(yy_shell *s, int32_t nring)
{
    if (!s || nring < 0 || nring > NRING_MAX || 2 * nring >= s->L.d.nt || 2 * nring >= s->L.d.np)
        return YY_ERR_ARG;
    std::vector<FillScalar> ring;
    if (nring > 0) {
        if (!build_ring(s->F, s->L.d, nring, ring)) return YY_ERR_GEOMETRY;
        // gathered values (2 patches x nr x targets doubles) go to the Thomas
        // scratch array, which no kernel uses between the pressure update and
        // the next sweep
        if ((int64_t)ring.size() > s->L.nring_max ||
            2 * (int64_t)ring.size() * s->L.d.nr * 8 > s->L.field_elems * s->L.elem)
            return YY_ERR_ARG;
        if (hipMemcpy(s->ptab, ring.data(), ring.size() * sizeof(FillScalar), hipMemcpyHostToDevice) != hipSuccess)
            return YY_ERR_HIP;
    }
    if (nring != s->nring) s->version++;
    s->nring = nring;
    s->nptab = (int)ring.size();
    return YY_OK;
}

int yy_set_wall(yy_shell *s, int32_t field, int32_t level, int32_t wall, const double *src, hipStream_t st)
{
    int c;
    switch (field) {
    case YY_T: c = 0; break;
    case YY_U1R: c = 1; break;
    case YY_U1T: c = 2; break;
    case YY_U1P: c = 3; break;
    default: return YY_ERR_ARG;
    }
    if (!s || level < 0 || level > 2 || wall < 0 || wall > 1) return YY_ERR_ARG;
    const bool on = src != nullptr;
    if (on && hipMemcpyAsync(s->wall[c][level][wall], src, s->L.wall_elems * 8, hipMemcpyDeviceToDevice,
                             st) != hipSuccess)
        return YY_ERR_HIP;
    if (on != s->wall_on[c][level][wall]) s->version++;   // kernel arguments change
    s->wall_on[c][level][wall] = on;
    if (level == YY_LEVEL_K) s->wall_fresh[c][wall] = true;
    else s->need_fill = true;
    return YY_OK;
}

int yy_step(yy_shell *s, int32_t K, hipStream_t st)
{
    if (!s || K < 1 || K > MAXK) return YY_ERR_ARG;
    if (!s->have_params || walls_stale(s)) return YY_ERR_STATE;
    if (s->sticky != YY_OK) return s->sticky;
    // the level pointers rotate here, outside any captured ensemble graph
    s->version++;
    return s->L.prec == YY_FP64 ? step_impl<double>(s, K, -1.0, nullptr, st)
                                : step_impl<float>(s, K, -1.0, nullptr, st);
}

}  // extern "C"

namespace yy {
// yy_step whose scratch arrays (residual/correction buffer, Thomas scratch,
// norm partial sums, mass-flux partials) live at `scratch`.  The region in
// use is cleared first (a kernel, so a captured graph replays it), so each
// call starts from the same zeroed scratch as a fresh workspace.
template <typename R> int step_scratch_impl(yy_shell *s, int K, char *scratch, hipStream_t st)
{
    State<R> &S = state_of<R>(s);
    const int64_t fb = align_up(s->L.field_elems * s->L.elem, ALIGN);
    R *res = S.res, *cb = S.cb;
    double *partial = s->partial, *mfp = s->mfp;
    S.res = (R *)scratch;
    S.cb = (R *)(scratch + fb);
    s->partial = (double *)(scratch + 2 * fb);
    s->mfp = (double *)(scratch + 2 * fb + STATIC_PARTIAL_BYTES);
    zero_doubles((double *)scratch, (2 * fb + STATIC_PARTIAL_BYTES + STATIC_MF_BYTES) / 8, st);
    const int rc = step_impl<R>(s, K, -1.0, nullptr, st);
    S.res = res;
    S.cb = cb;
    s->partial = partial;
    s->mfp = mfp;
    return rc;
}

int step_with_scratch(yy_shell *s, int K, char *scratch, int64_t cap, hipStream_t st)
{
    if (!s || !scratch || K < 1 || K > MAXK) return YY_ERR_ARG;
    const int64_t fb = align_up(s->L.field_elems * s->L.elem, ALIGN);
    if (fb > STATIC_FIELD_BYTES || 2 * fb + STATIC_PARTIAL_BYTES + STATIC_MF_BYTES > cap)
        return YY_ERR_WORKSPACE;
    if (!s->have_params || walls_stale(s)) return YY_ERR_STATE;
    if (s->sticky != YY_OK) return s->sticky;
    s->version++;
    return s->L.prec == YY_FP64 ? step_scratch_impl<double>(s, K, scratch, st)
                                : step_scratch_impl<float>(s, K, scratch, st);
}
}  // namespace yy

extern "C" {

int yy_step_tol(yy_shell *s, int32_t kmax, double tol, int32_t *k_done, hipStream_t st)
{
    if (!s || !k_done || kmax < 1 || kmax > MAXK || !(tol >= 0.0) || !std::isfinite(tol)) return YY_ERR_ARG;
    *k_done = 0;
    if (!s->have_params || walls_stale(s)) return YY_ERR_STATE;
    if (s->sticky != YY_OK) return s->sticky;
    s->version++;
    int k = 0;
    const int r = s->L.prec == YY_FP64 ? step_impl<double>(s, kmax, tol, &k, st)
                                       : step_impl<float>(s, kmax, tol, &k, st);
    *k_done = k;
    return r;
}

int yy_get_norms(yy_shell *s, double *out, int32_t cap, hipStream_t st)
{
    if (!s || !out || cap < 0) return YY_ERR_ARG;
    const int n = s->last_k * 2 * NSLOT;
    std::vector<double> h(n > 0 ? n : 1);
    hipError_t e = hipSuccess;
    if (n > 0) e = hipMemcpyAsync(h.data(), s->norms, n * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return YY_ERR_HIP;
    bool finite = true;
    for (int q = 0; q < n; q++) {
        if (q < cap) out[q] = h[q];
        if (!std::isfinite(h[q])) finite = false;
    }
    if (!finite) {
        s->sticky = YY_ERR_NONFINITE;
        return YY_ERR_NONFINITE;
    }
    return n;
}

int yy_destroy(yy_shell *s)
{
    if (!s) return YY_ERR_ARG;
    for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
    delete s;
    return YY_OK;
}

int yy_profile(yy_shell *s, int32_t enable)
{
    if (!s) return YY_ERR_ARG;
    if (enable && s->ev.empty()) {
        const size_t n = 2 * 8192;
        s->ev.resize(n);
        s->ev_cls.resize(n / 2);
        for (size_t q = 0; q < n; q++)
            if (hipEventCreate(&s->ev[q]) != hipSuccess) return YY_ERR_HIP;
    }
    s->prof = enable != 0;
    if (enable) s->ev_used = 0;
    return YY_OK;
}

int yy_profile_read(yy_shell *s, double *ms, int64_t *count, hipStream_t st)
{
    if (!s || !ms || !count) return YY_ERR_ARG;
    if (hipStreamSynchronize(st) != hipSuccess) return YY_ERR_HIP;
    for (int c = 0; c < YY_NPROF; c++) {
        ms[c] = 0.0;
        count[c] = 0;
    }
    for (size_t q = 0; q + 1 < s->ev_used; q += 2) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, s->ev[q], s->ev[q + 1]) != hipSuccess) return YY_ERR_HIP;
        const int c = s->ev_cls[q / 2];
        ms[c] += t;
        count[c] += 1;
    }
    return YY_NPROF;
}

const char *yy_profile_name(int32_t c)
{
    return (c >= 0 && c < YY_NPROF) ? prof_names[c] : nullptr;
}

int yy_internal_dims(const yy_shell *s, int64_t dims[4], int32_t *elem_bytes, int32_t *k_first)
{
    if (!s || !dims) return YY_ERR_ARG;
    dims[0] = 2;
    dims[1] = s->L.d.nr + 2;
    dims[2] = s->L.d.nt + 2;
    dims[3] = s->L.d.sJ;
    if (elem_bytes) *elem_bytes = (int32_t)s->L.elem;
    if (k_first) *k_first = s->L.d.ko - 1;
    return YY_OK;
}

int yy_fill(yy_shell *s, int32_t level, hipStream_t st)
{
    if (!s || level < 0 || level > 2) return YY_ERR_ARG;
    if (s->L.prec == YY_FP64) do_fill<double>(s, level, 3, st);
    else do_fill<float>(s, level, 3, st);
    return hip_status(hipGetLastError());
}

int yy_extrapolate(yy_shell *s, hipStream_t st)
{
    if (!s) return YY_ERR_ARG;
    {
        Timed tm(s, PC_EXTRAP, st);
        if (s->L.prec == YY_FP64) Ops<double>::extrap(s->L.d, s->s64, st);
        else Ops<float>::extrap(s->L.d, s->s32, st);
    }
    return hip_status(hipGetLastError());
}

int yy_sweep(yy_shell *s, int32_t field, int32_t dir, const void *x, void *y, hipStream_t st)
{
    if (!s || !x || !y || dir < 0 || dir > 2 || !field_ok(field) || field == YY_P1 || field == YY_P2)
        return YY_ERR_ARG;
    if (!s->have_params) return YY_ERR_STATE;
    if (s->L.prec == YY_FP64)
        Ops<double>::sweep(s->L.d, s->g64, s->gd, s->s64, field, dir, (const double *)x, (double *)y, 0,
                           nullptr, nullptr, 0, st);
    else
        Ops<float>::sweep(s->L.d, s->g32, s->gd, s->s32, field, dir, (const float *)x, (float *)y, 0,
                          nullptr, nullptr, 0, st);
    return hip_status(hipGetLastError());
}

int yy_sweep_diffusion(yy_shell *s, int32_t dir, int32_t metric, const void *x, void *y, hipStream_t st)
{
    if (!s || !x || !y || dir < 0 || dir > 2 || (metric != 0 && metric != 1)) return YY_ERR_ARG;
    if (!s->have_params) return YY_ERR_STATE;
    if (s->L.prec == YY_FP64)
        Ops<double>::sweep(s->L.d, s->g64, s->gd, s->s64, YY_T, dir, (const double *)x, (double *)y, 0,
                           nullptr, nullptr, 1 + metric, st);
    else
        Ops<float>::sweep(s->L.d, s->g32, s->gd, s->s32, YY_T, dir, (const float *)x, (float *)y, 0,
                          nullptr, nullptr, 1 + metric, st);
    return hip_status(hipGetLastError());
}

int yy_residual(yy_shell *s, int32_t field, void *out, hipStream_t st)
{
    if (!s || !out || !field_ok(field) || field == YY_P1 || field == YY_P2) return YY_ERR_ARG;
    if (!s->have_params) return YY_ERR_STATE;
    if (s->L.prec == YY_FP64) Ops<double>::residual(s->L.d, s->g64, s->s64, field, (double *)out, st);
    else Ops<float>::residual(s->L.d, s->g32, s->s32, field, (float *)out, st);
    return hip_status(hipGetLastError());
}

// ---------------------------------------------------------------------------
// autotuning of the line-solver tiles
// ---------------------------------------------------------------------------
// tile slots: the four unknowns' sweeps and ("D") the diffusion-only line
// solves of the line-solve workload
static const char *tune_field_name[5] = {"T", "u_r", "u_t", "u_p", "D"};
static const int tune_field_id[5] = {YY_T, YY_U2R, YY_U2T, YY_U2P, -1};
static const char dir_name[3] = {'r', 't', 'p'};

static Tune &tune_of(yy_shell *s) { return s->L.prec == YY_FP64 ? s->s64.tune : s->s32.tune; }

// One sweep as the step launches it.  The direction that comes last in the
// field's factor order always runs fused with psi^k += c and the increment
// norm, so it is timed in that form, with psi^k redirected to the Thomas
// scratch array so that the field itself is left untouched.
static const int last_dir[4] = {2, 0, 1, 2};   // T: r,t,p; u_r: t,p,r; u_t: p,r,t; u_p: r,t,p

extern "C++" template <typename R> static int sweep_in_step(yy_shell *s, int field, int dir, hipStream_t st)
{
    State<R> S = state_of<R>(s);
    if (field < 0) {   // the diffusion-only solve (split operators)
        Ops<R>::sweep(s->L.d, geo_of<R>(s), s->gd, S, YY_T, dir, S.res, S.res, 0, nullptr, nullptr, 1, st);
        return hip_status(hipGetLastError());
    }
    const int loc = loc_of(field);
    if (dir != last_dir[loc]) {
        Ops<R>::sweep(s->L.d, geo_of<R>(s), s->gd, S, field, dir, S.res, S.res, 0, nullptr, nullptr, 0, st);
    } else {
        if (field == YY_T) S.T[2] = S.cb;
        else S.u[field >= YY_U2R ? 1 : 0][(field - 1) % 4][2] = S.cb;
        int nb = 0;
        Ops<R>::sweep(s->L.d, geo_of<R>(s), s->gd, S, field, dir, S.res, S.res, 1, s->partial, &nb, 0, st);
    }
    return hip_status(hipGetLastError());
}

static int sweep_as_in_step(yy_shell *s, int field, int dir, hipStream_t st)
{
    return s->L.prec == YY_FP64 ? sweep_in_step<double>(s, field, dir, st)
                                : sweep_in_step<float>(s, field, dir, st);
}

// time one sweep configuration: mean of 3 runs after one warm-up (ms)
// mean time of the residual of `field` (into the scratch buffer), as the step launches it
extern "C++" template <typename R> static double time_residual_t(yy_shell *s, int field, hipStream_t st, hipEvent_t a, hipEvent_t b)
{
    State<R> &S = state_of<R>(s);
    Ops<R>::residual(s->L.d, geo_of<R>(s), S, field, S.res, st);
    (void)hipEventRecord(a, st);
    for (int q = 0; q < 3; q++) Ops<R>::residual(s->L.d, geo_of<R>(s), S, field, S.res, st);
    (void)hipEventRecord(b, st);
    if (hipEventSynchronize(b) != hipSuccess) return 1e30;
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, a, b);
    return ms / 3.0;
}
static double time_residual(yy_shell *s, int field, hipStream_t st, hipEvent_t a, hipEvent_t b)
{
    return s->L.prec == YY_FP64 ? time_residual_t<double>(s, field, st, a, b)
                                : time_residual_t<float>(s, field, st, a, b);
}

static double time_sweep(yy_shell *s, int field, int dir, hipStream_t st, hipEvent_t a, hipEvent_t b)
{
    if (sweep_as_in_step(s, field, dir, st) != YY_OK) return 1e30;
    (void)hipEventRecord(a, st);
    for (int q = 0; q < 3; q++)
        if (sweep_as_in_step(s, field, dir, st) != YY_OK) return 1e30;
    (void)hipEventRecord(b, st);
    if (hipEventSynchronize(b) != hipSuccess) return 1e30;
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, a, b);
    return ms / 3.0;
}

extern "C" int yy_autotune(yy_shell *s, char *json_out, int32_t cap, hipStream_t st)
{
    if (!s) return YY_ERR_ARG;
    if (!s->have_params) return YY_ERR_STATE;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return YY_ERR_HIP;
    if (hipEventCreate(&b) != hipSuccess) return YY_ERR_HIP;
    const bool prof = s->prof;
    s->prof = false;
    Tune &T = tune_of(s);
    std::string js = "{";
    for (int L = 0; L < 5; L++) {
        for (int dir = 0; dir < 3; dir++) {
            char key[16];
            std::snprintf(key, sizeof key, "%s.%c", tune_field_name[L], dir_name[dir]);
            char val[32];
            T.sb[L][dir] = 0;
            if (dir < 2) {
                // the per-line Thomas kernel, then every partitioned tile
                // that fits the lines
                const int n = (dir == 0 ? s->L.d.nr : s->L.d.nt) - (L == dir + 1 ? 1 : 0);
                T.m[L][dir] = 1;
                T.w[L][dir] = 0;
                T.bl[L][dir] = 0;
                int bm = 1, bw = 0, bb = 0;
                double best = time_sweep(s, tune_field_id[L], dir, st, a, b);
                const int ms[5] = {4, 6, 8, 12, 16}, ws[3] = {64, 32, 16};
                for (int im = 0; im < 5; im++)
                    for (int iw = 0; iw < 3; iw++)
                        for (int ib = 0; ib < 2; ib++) {
                            int W = 0, P = 0;
                            if (!strided_tile(n, ms[im], ws[iw], W, P)) continue;
                            T.m[L][dir] = (int8_t)ms[im];
                            T.w[L][dir] = (int8_t)ws[iw];
                            T.bl[L][dir] = (int8_t)ib;
                            const double t = time_sweep(s, tune_field_id[L], dir, st, a, b);
                            if (t < best) { best = t; bm = ms[im]; bw = ws[iw]; bb = ib; }
                        }
                T.m[L][dir] = (int8_t)bm;
                T.w[L][dir] = (int8_t)bw;
                T.bl[L][dir] = (int8_t)bb;
                if (bm == 1) std::snprintf(val, sizeof val, "t");
                else std::snprintf(val, sizeof val, "m%dw%d%s", bm, bw, bb ? "b" : "");
            } else {
                // one wave per line with 1, 2 or 4 lines per block, or 2, 4 or
                // 8 waves per line
                int bl = 0, bv = 0;
                double best = 1e30;
                const int ls[6] = {1, 2, 4, 1, 1, 1}, vs[6] = {0, 0, 0, 2, 4, 8};
                for (int il = 0; il < 6; il++) {
                    T.lpb[L] = (int8_t)ls[il];
                    T.wpl[L] = (int8_t)vs[il];
                    const double t = time_sweep(s, tune_field_id[L], dir, st, a, b);
                    if (t < best) { best = t; bl = ls[il]; bv = vs[il]; }
                }
                T.lpb[L] = (int8_t)bl;
                T.wpl[L] = (int8_t)bv;
                if (bv) std::snprintf(val, sizeof val, "v%d", bv);
                else std::snprintf(val, sizeof val, "l%d", bl);
            }
            if (js.size() > 1) js += ",";
            js += "\"";
            js += key;
            js += "\":\"";
            js += val;
            js += "\"";
            // blocks per patch of the chosen partitioned solve: the default,
            // 1.5 or 2 times it, whichever runs fastest (all timed afresh)
            T.sb[L][dir] = 0;
            if (dir == 2 || T.m[L][dir] != 1) {
                double tb = time_sweep(s, tune_field_id[L], dir, st, a, b);
                int best_sb = 0;
                for (const int nb : {SWEEP_BLOCKS * 3 / 2, SWEEP_BLOCKS * 2}) {
                    T.sb[L][dir] = (int16_t)nb;
                    const double t1 = time_sweep(s, tune_field_id[L], dir, st, a, b);
                    if (t1 < tb) { tb = t1; best_sb = nb; }
                }
                T.sb[L][dir] = (int16_t)best_sb;
                if (best_sb > 0) {
                    char bv[64];
                    std::snprintf(bv, sizeof bv, ",\"%s.blocks\":\"%d\"", key, best_sb);
                    js += bv;
                }
            }
        }
    }
    // column tiles of the residuals (one per unknown location)
    for (int L = 0; L < 4; L++) {
        int best_t = 0;
        double best = 1e30;
        for (int t = 0; t < N_RES_TILES; t++) {
            T.rt[L] = (int8_t)t;
            const double tm = time_residual(s, tune_field_id[L], st, a, b);
            if (tm < best) { best = tm; best_t = t; }
        }
        T.rt[L] = (int8_t)best_t;
        js += ",\"res.";
        js += tune_field_name[L];
        js += "\":\"";
        js += RES_TILES[best_t].name;
        js += "\"";
    }
    js += "}";
    s->prof = prof;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    s->version++;
    if (json_out && cap > 0) {
        std::strncpy(json_out, js.c_str(), (size_t)cap - 1);
        json_out[cap - 1] = 0;
    }
    return hip_status(hipGetLastError());
}

// the current tile choices of a shell, in the JSON form of yy_autotune
static std::string tuning_json(yy_shell *s)
{
    const Tune &T = tune_of(s);
    std::string js = "{";
    for (int L = 0; L < 5; L++)
        for (int dir = 0; dir < 3; dir++) {
            char val[48];
            if (dir < 2) {
                const int m = T.m[L][dir] ? T.m[L][dir] : ((L == 2 && dir == 1) ? 12 : 16);
                if (m == 1) std::snprintf(val, sizeof val, "t");
                else std::snprintf(val, sizeof val, "m%dw%d%s", m, T.w[L][dir] ? T.w[L][dir] : 64, T.bl[L][dir] ? "b" : "");
            } else {
                if (T.wpl[L]) std::snprintf(val, sizeof val, "v%d", T.wpl[L]);
                else std::snprintf(val, sizeof val, "l%d", T.lpb[L] ? T.lpb[L] : 1);
            }
            char key[16];
            std::snprintf(key, sizeof key, "%s.%c", tune_field_name[L], dir_name[dir]);
            if (js.size() > 1) js += ",";
            js += "\"";
            js += key;
            js += "\":\"";
            js += val;
            js += "\"";
            if (T.sb[L][dir] > 0) {
                char bv[64];
                std::snprintf(bv, sizeof bv, ",\"%s.blocks\":\"%d\"", key, (int)T.sb[L][dir]);
                js += bv;
            }
        }
    for (int L = 0; L < 4; L++) {
        js += ",\"res.";
        js += tune_field_name[L];
        js += "\":\"";
        js += RES_TILES[T.rt[L] >= 0 && T.rt[L] < N_RES_TILES ? T.rt[L] : 0].name;
        js += "\"";
        if (T.rseg[L] > 0) {
            char val[48];
            std::snprintf(val, sizeof val, ",\"res.%s.seg\":\"%d\"", tune_field_name[L], (int)T.rseg[L]);
            js += val;
        }
    }
    return js + "}";
}

extern "C" int yy_get_tuning(yy_shell *s, char *json_out, int32_t cap)
{
    if (!s || !json_out || cap < 1) return YY_ERR_ARG;
    const std::string js = tuning_json(s);
    if ((int64_t)js.size() >= cap) return YY_ERR_ARG;
    std::memcpy(json_out, js.c_str(), js.size() + 1);
    return YY_OK;
}

extern "C" int yy_set_tuning(yy_shell *s, const char *json)
{
    if (!s || !json) return YY_ERR_ARG;
    Tune &T = tune_of(s);
    // keys and values hold no blanks: drop every blank, so that JSON written
    // with separators ", " and ": " matches like the compact form
    std::string js;
    for (const char *c = json; *c; c++)
        if (!std::isspace((unsigned char)*c)) js += *c;
    for (int L = 0; L < 5; L++)
        for (int dir = 0; dir < 3; dir++) {
            char key[24];
            std::snprintf(key, sizeof key, "\"%s.%c\":\"", tune_field_name[L], dir_name[dir]);
            const size_t at = js.find(key);
            if (at == std::string::npos) continue;
            const char *v = js.c_str() + at + std::strlen(key);
            int m = 0, w = 0, l = 0;
            if (dir < 2) {
                if (v[0] == 't' && v[1] == '"') {
                    T.m[L][dir] = 1;
                    T.w[L][dir] = 0;
                    T.bl[L][dir] = 0;
                    continue;
                }
                int used = 0;
                if (std::sscanf(v, "m%dw%d%n", &m, &w, &used) != 2) return YY_ERR_ARG;
                if ((m != 4 && m != 6 && m != 8 && m != 12 && m != 16) || (w != 16 && w != 32 && w != 64))
                    return YY_ERR_ARG;
                const bool bl = v[used] == 'b';
                if (v[used + (bl ? 1 : 0)] != '"') return YY_ERR_ARG;
                T.m[L][dir] = (int8_t)m;
                T.w[L][dir] = (int8_t)w;
                T.bl[L][dir] = (int8_t)bl;
            } else {
                if (std::sscanf(v, "l%d", &l) == 1 && (l == 1 || l == 2 || l == 4)) {
                    T.lpb[L] = (int8_t)l;
                    T.wpl[L] = 0;
                } else if (std::sscanf(v, "v%d", &l) == 1 && (l == 2 || l == 4 || l == 8)) {
                    T.lpb[L] = 1;
                    T.wpl[L] = (int8_t)l;
                } else {
                    return YY_ERR_ARG;
                }
            }
        }
    for (int L = 0; L < 4; L++) {
        const std::string key = std::string("\"res.") + tune_field_name[L] + "\":\"";
        const size_t at = js.find(key);
        if (at == std::string::npos) continue;
        const std::string v = js.substr(at + key.size(), js.find('"', at + key.size()) - at - key.size());
        int found = -1;
        for (int t = 0; t < N_RES_TILES; t++)
            if (v == RES_TILES[t].name) found = t;
        if (found < 0) return YY_ERR_ARG;
        T.rt[L] = (int8_t)found;
    }
    // radial segments of the residual columns: "0" = from the occupancy
    for (int L = 0; L < 4; L++) {
        const std::string key = std::string("\"res.") + tune_field_name[L] + ".seg\":\"";
        const size_t at = js.find(key);
        if (at == std::string::npos) continue;
        int n = -1, used = 0;
        if (std::sscanf(js.c_str() + at + key.size(), "%d%n", &n, &used) != 1 || n < 0 || n > 64 ||
            js[at + key.size() + used] != '"')
            return YY_ERR_ARG;
        T.rseg[L] = (int8_t)n;
    }
    // blocks per patch of a partitioned line solve: "0" = the default
    for (int L = 0; L < 5; L++)
        for (int dir = 0; dir < 3; dir++) {
            char key[32];
            std::snprintf(key, sizeof key, "\"%s.%c.blocks\":\"", tune_field_name[L], dir_name[dir]);
            const size_t at = js.find(key);
            if (at == std::string::npos) continue;
            const size_t v0 = at + std::strlen(key);
            int n = -1, used = 0;
            if (std::sscanf(js.c_str() + v0, "%d%n", &n, &used) != 1 || n < 0 || n > NBMAX ||
                (n > 0 && n < 8) || js[v0 + used] != '"')
                return YY_ERR_ARG;
            T.sb[L][dir] = (int16_t)n;
        }
    s->version++;
    return YY_OK;
}

// ---------------------------------------------------------------------------
// ensembles
// ---------------------------------------------------------------------------
}  // extern "C"

struct yy_ensemble {
    std::vector<yy_shell *> sh;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> join;
    hipStream_t cap = nullptr;
    hipEvent_t fork = nullptr;
    hipGraph_t graph[6] = {};
    hipGraphExec_t exec[6] = {};
    bool captured = false;
    bool batched = false;    // the graphs hold batched launches (else one stream per shell)
    int phase = 0, K = 0, how = 0;
    std::vector<uint64_t> versions;
    // device arena of the batched launches' argument and block tables
    char *arena = nullptr;
    uint64_t arena_bytes = 0;
    int64_t batched_launches = 0;   // launches per captured step (all phases: / 6)
    int64_t shell_launches = 0;     // the shells' own launches they replace (all phases)
};

namespace {

int shell_step(yy_shell *s, int K, hipStream_t st)
{
    if (!s->have_params || walls_stale(s)) return YY_ERR_STATE;
    if (s->sticky != YY_OK) return s->sticky;
    return s->L.prec == YY_FP64 ? step_impl<double>(s, K, -1.0, nullptr, st) : step_impl<float>(s, K, -1.0, nullptr, st);
}

void shell_rotate(yy_shell *s)
{
    if (s->L.prec == YY_FP64) rotate_levels<double>(s);
    else rotate_levels<float>(s);
}

void drop_graphs(yy_ensemble *e)
{
    for (int f = 0; f < 6; f++) {
        if (e->exec[f]) (void)hipGraphExecDestroy(e->exec[f]);
        if (e->graph[f]) (void)hipGraphDestroy(e->graph[f]);
        e->exec[f] = nullptr;
        e->graph[f] = nullptr;
    }
    e->captured = false;
}

// host-side time-level state of a shell that a step rotates
struct LevelState {
    State<double> s64;
    State<float> s32;
    double *wall[4][3][2];
    bool wall_on[4][3][2];
    bool wall_fresh[4][2];
};
LevelState save_levels(const yy_shell *s)
{
    LevelState v;
    v.s64 = s->s64;
    v.s32 = s->s32;
    std::memcpy(v.wall, s->wall, sizeof v.wall);
    std::memcpy(v.wall_on, s->wall_on, sizeof v.wall_on);
    std::memcpy(v.wall_fresh, s->wall_fresh, sizeof v.wall_fresh);
    return v;
}
void restore_levels(yy_shell *s, const LevelState &v)
{
    s->s64 = v.s64;
    s->s32 = v.s32;
    std::memcpy(s->wall, v.wall, sizeof v.wall);
    std::memcpy(s->wall_on, v.wall_on, sizeof v.wall_on);
    std::memcpy(s->wall_fresh, v.wall_fresh, sizeof v.wall_fresh);
}

// does any level of the shell use Dirichlet wall data?  (Wall data must be
// set for every step, which a replayed graph cannot do.)
bool uses_walls(const yy_shell *s)
{
    for (int c = 0; c < 4; c++)
        for (int l = 0; l < 3; l++)
            for (int w = 0; w < 2; w++)
                if (s->wall_on[c][l][w]) return true;
    return false;
}

// capture the six rotation phases of one ensemble step; every shell's
// kernels go on its own stream, forked from and joined to the capture
// stream.  Capturing runs the host side of six steps: the level pointers
// come back to where they were (the rotation has period 6), and on any
// failure they are restored from a snapshot, so no shell's levels move
// without device work.
int capture(yy_ensemble *e, int K)
{
    drop_graphs(e);
    for (yy_shell *s : e->sh)
        if (uses_walls(s) || walls_stale(s)) return YY_ERR_STATE;
    std::vector<LevelState> snap;
    for (yy_shell *s : e->sh) snap.push_back(save_levels(s));
    std::vector<bool> prof(e->sh.size());
    for (size_t q = 0; q < e->sh.size(); q++) {
        prof[q] = e->sh[q]->prof;
        e->sh[q]->prof = false;
    }
    int st = YY_OK;
    for (int f = 0; f < 6 && st == YY_OK; f++) {
        hipError_t h = hipStreamBeginCapture(e->cap, hipStreamCaptureModeThreadLocal);
        if (h == hipSuccess) h = hipEventRecord(e->fork, e->cap);
        for (size_t q = 0; q < e->sh.size() && h == hipSuccess; q++) {
            h = hipStreamWaitEvent(e->streams[q], e->fork, 0);
            if (h == hipSuccess) {
                const int r = shell_step(e->sh[q], K, e->streams[q]);
                if (r != YY_OK) { st = r; h = hipErrorUnknown; }
            }
            if (h == hipSuccess) h = hipEventRecord(e->join[q], e->streams[q]);
            if (h == hipSuccess) h = hipStreamWaitEvent(e->cap, e->join[q], 0);
        }
        hipGraph_t g = nullptr;
        const hipError_t h2 = hipStreamEndCapture(e->cap, &g);
        if (h == hipSuccess) h = h2;
        if (h == hipSuccess) h = hipGraphInstantiate(&e->exec[f], g, nullptr, nullptr, 0);
        e->graph[f] = g;
        if (h != hipSuccess && st == YY_OK) st = YY_ERR_HIP;
    }
    for (size_t q = 0; q < e->sh.size(); q++) e->sh[q]->prof = prof[q];
    for (size_t q = 0; q < e->sh.size(); q++) restore_levels(e->sh[q], snap[q]);
    if (st != YY_OK) {
        drop_graphs(e);
        return st;
    }
    e->captured = true;
    e->phase = 0;
    e->K = K;
    for (size_t q = 0; q < e->sh.size(); q++) e->versions[q] = e->sh[q]->version;
    return YY_OK;
}

// Batched capture (the ensemble's "one launch per phase"): the host side of
// one step of every shell is run with the launch recorder installed, for
// each of the six rotation phases.  At each position of the step's launch
// sequence the shells' records are grouped by kernel instance (tile), block
// shape and argument size; each group becomes one launch of the kernel's
// batched twin over a 1-D grid in which each shell owns its own block range
// (work list: off, nx, ny per shell).  The shells are dealt to up to four
// branches of similar cell counts, each a chain of such launches, and the
// branches run side by side (so one launch's tail overlaps another's
// work).  The argument structs and block tables are uploaded once into the
// arena; the six graphs hold only the launches.
// Returns YY_ERR_STATE if the shells' step sequences do not line up (then
// the per-shell stream capture is used).
int capture_batched(yy_ensemble *e, int K)
{
    drop_graphs(e);
    for (yy_shell *s : e->sh)
        if (uses_walls(s) || walls_stale(s)) return YY_ERR_STATE;
    const size_t n = e->sh.size();
    std::vector<LevelState> snap;
    for (yy_shell *s : e->sh) snap.push_back(save_levels(s));
    std::vector<bool> prof(n);
    for (size_t q = 0; q < n; q++) {
        prof[q] = e->sh[q]->prof;
        e->sh[q]->prof = false;
    }
    std::vector<std::vector<LaunchRecorder>> rec(6, std::vector<LaunchRecorder>(n));
    int st = YY_OK;
    for (int f = 0; f < 6 && st == YY_OK; f++)
        for (size_t q = 0; q < n && st == YY_OK; q++) {
            set_launch_recorder(&rec[f][q]);
            st = shell_step(e->sh[q], K, e->cap);
            set_launch_recorder(nullptr);
        }
    for (size_t q = 0; q < n; q++) {
        restore_levels(e->sh[q], snap[q]);
        e->sh[q]->prof = prof[q];
    }
    if (st != YY_OK) return st;
    // every launch of the step needs a batched twin (the mass fix and the
    // pressure exchange have none: such shells take the stream graph)
    for (int f = 0; f < 6; f++)
        for (size_t q = 0; q < n; q++)
            if (rec[f][q].foreign) return YY_ERR_STATE;
    // the step sequences must line up position by position
    for (int f = 0; f < 6; f++)
        for (size_t q = 1; q < n; q++)
            if (rec[f][q].recs.size() != rec[f][0].recs.size()) return YY_ERR_STATE;
    struct Group {
        const void *multi;
        dim3 block;
        size_t lds;
        uint64_t total;          // blocks
        int nq;
        std::vector<unsigned char> args;
        std::vector<BatchEnt> ents;
        uint64_t arg_off, ent_off;
    };
    // branches: the shells are dealt to up to BATCH_BRANCHES independent
    // chains of batched launches (largest shells first, each to the chain
    // with the fewest cells so far), which the graph runs side by side
    const int nbr = (int)std::min<size_t>(BATCH_BRANCHES, n);
    std::vector<std::vector<size_t>> branch(nbr);
    {
        std::vector<size_t> order(n);
        for (size_t q = 0; q < n; q++) order[q] = q;
        auto cells = [&](size_t q) { return (int64_t)e->sh[q]->L.d.nr * e->sh[q]->L.d.nt * e->sh[q]->L.d.np; };
        std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return cells(a) > cells(b); });
        std::vector<int64_t> load(nbr, 0);
        for (size_t q : order) {
            const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            branch[b].push_back(q);
            load[b] += cells(q);
        }
        for (auto &br : branch) std::sort(br.begin(), br.end());
    }
    // groups[f][b]: the launches of branch b in phase f, in order
    std::vector<std::vector<std::vector<Group>>> groups(6, std::vector<std::vector<Group>>(nbr));
    uint64_t need = 0;
    for (int f = 0; f < 6; f++) {
        const size_t npos = rec[f][0].recs.size();
        for (int br = 0; br < nbr; br++)
        for (size_t i = 0; i < npos; i++) {
            // members of each group: the shells whose launch at this
            // position is the same kernel instance, block shape and
            // argument size
            std::vector<Group> gs;
            std::vector<std::vector<size_t>> mem;
            for (size_t q : branch[br]) {
                const LaunchRec &r = rec[f][q].recs[i];
                if (r.grid.z != 1) return YY_ERR_STATE;
                size_t gi = gs.size();
                for (size_t c = 0; c < gs.size(); c++)
                    if (gs[c].multi == r.multi && gs[c].block.x == r.block.x && gs[c].block.y == r.block.y &&
                        gs[c].block.z == r.block.z && rec[f][mem[c][0]].recs[i].arg_size == r.arg_size)
                        gi = c;
                if (gi == gs.size()) {
                    gs.push_back(Group{r.multi, r.block, 0, 0, 0, {}, {}, 0, 0});
                    mem.emplace_back();
                }
                mem[gi].push_back(q);
            }
            // the heaviest blocks (most cells per block) are dispatched
            // first; each shell's range starts on a multiple of 8 blocks and
            // is padded to one, so that its blocks spread evenly over the
            // 8 XCDs (the batched kernel remaps within the shell's range)
            for (size_t c = 0; c < gs.size(); c++) {
                Group &g = gs[c];
                auto weight = [&](size_t q) {
                    const LaunchRec &r = rec[f][q].recs[i];
                    const Dims &d = e->sh[q]->L.d;
                    return (double)d.nr * d.nt * d.np / ((double)r.grid.x * r.grid.y);
                };
                std::stable_sort(mem[c].begin(), mem[c].end(),
                                 [&](size_t a, size_t b) { return weight(a) > weight(b); });
                for (size_t q : mem[c]) {
                    const LaunchRec &r = rec[f][q].recs[i];
                    const uint64_t nb = (uint64_t)r.grid.x * r.grid.y;
                    const uint64_t padded = (nb + 7) & ~7ull;
                    if (g.total + padded >= (1ull << 31)) return YY_ERR_STATE;
                    g.ents.push_back(BatchEnt{(int32_t)g.total, (int32_t)r.grid.x, (int32_t)r.grid.y,
                                              (int32_t)padded});
                    g.total += padded;
                    g.lds = std::max(g.lds, r.lds);
                    g.nq++;
                    const unsigned char *a = rec[f][q].args.data() + r.arg_off;
                    g.args.insert(g.args.end(), a, a + r.arg_size);
                }
            }
            for (Group &g : gs) {
                g.arg_off = need;
                need += (uint64_t)align_up((int64_t)g.args.size(), ALIGN);
                g.ent_off = need;
                need += (uint64_t)align_up((int64_t)(g.ents.size() * sizeof(BatchEnt)), ALIGN);
                groups[f][br].push_back(std::move(g));
            }
        }
    }
    if (need > e->arena_bytes) return YY_ERR_STATE;
    std::vector<unsigned char> host(need, 0);
    int64_t launches = 0;
    for (int f = 0; f < 6; f++)
        for (auto &gb : groups[f])
            for (Group &g : gb) {
                std::memcpy(host.data() + g.arg_off, g.args.data(), g.args.size());
                std::memcpy(host.data() + g.ent_off, g.ents.data(), g.ents.size() * sizeof(BatchEnt));
                launches++;
            }
    if (hipMemcpy(e->arena, host.data(), need, hipMemcpyHostToDevice) != hipSuccess) return YY_ERR_HIP;
    for (int f = 0; f < 6 && st == YY_OK; f++) {
        hipError_t h = hipStreamBeginCapture(e->cap, hipStreamCaptureModeThreadLocal);
        if (h == hipSuccess) h = hipEventRecord(e->fork, e->cap);
        for (int br = 0; br < nbr && h == hipSuccess; br++) {
            hipStream_t bs = e->streams[br];
            h = hipStreamWaitEvent(bs, e->fork, 0);
            for (Group &g : groups[f][br]) {
                if (h != hipSuccess) break;
                const void *list = e->arena + g.arg_off;
                const BatchEnt *ents = (const BatchEnt *)(e->arena + g.ent_off);
                int nq = g.nq;
                void *args[3] = {(void *)&list, (void *)&ents, (void *)&nq};
                h = hipLaunchKernel(g.multi, dim3((unsigned)g.total), g.block, args, g.lds, bs);
            }
            if (h == hipSuccess) h = hipEventRecord(e->join[br], bs);
            if (h == hipSuccess) h = hipStreamWaitEvent(e->cap, e->join[br], 0);
        }
        hipGraph_t gr = nullptr;
        const hipError_t h2 = hipStreamEndCapture(e->cap, &gr);
        if (h == hipSuccess) h = h2;
        if (h == hipSuccess) h = hipGraphInstantiate(&e->exec[f], gr, nullptr, nullptr, 0);
        e->graph[f] = gr;
        if (h != hipSuccess) st = YY_ERR_HIP;
    }
    if (st != YY_OK) {
        drop_graphs(e);
        return st;
    }
    e->captured = true;
    e->batched = true;
    e->phase = 0;
    e->K = K;
    e->batched_launches = launches;
    e->shell_launches = 0;
    for (int f = 0; f < 6; f++)
        for (size_t q = 0; q < n; q++) e->shell_launches += (int64_t)rec[f][q].recs.size();
    for (size_t q = 0; q < n; q++) e->versions[q] = e->sh[q]->version;
    return YY_OK;
}

// arena of the batched launches: every recorded launch of one step for K
// <= 8 iterations, 6 phases, with the largest argument struct, per shell
uint64_t arena_bytes_for(int32_t n)
{
    const uint64_t launches = 41ull * 8 + 16;     // fill 10, 7 solves x 4, 2 pressures, 1 reduce per iteration
    return 6ull * launches * (uint64_t)n * (4096 + 64) + (1u << 20);
}

}  // namespace

extern "C" {

int yy_ensemble_workspace_bytes(int32_t n, const yy_grid *grids, int32_t prec, uint64_t *bytes)
{
    if (n < 1 || !grids || !bytes) return YY_ERR_ARG;
    uint64_t tot = 0;
    for (int q = 0; q < n; q++) {
        uint64_t b = 0;
        const int st = yy_workspace_bytes(&grids[q], prec, &b);
        if (st != YY_OK) return st;
        tot += (uint64_t)align_up((int64_t)b, ALIGN);
    }
    *bytes = tot + (uint64_t)align_up((int64_t)arena_bytes_for(n), ALIGN);
    return YY_OK;
}

int yy_ensemble_create(int32_t n, const yy_grid *grids, int32_t prec, void *dev_ws, uint64_t ws_bytes,
                       yy_ensemble **out)
{
    if (!out) return YY_ERR_ARG;
    *out = nullptr;
    uint64_t need = 0;
    int st = yy_ensemble_workspace_bytes(n, grids, prec, &need);
    if (st != YY_OK) return st;
    if (!dev_ws || (uintptr_t)dev_ws % ALIGN) return YY_ERR_WORKSPACE;
    if (ws_bytes < need) return YY_ERR_WORKSPACE;
    // validate every geometry before touching the device
    for (int q = 0; q < n; q++) {
        Layout L = make_layout(&grids[q], prec);
        Frame F;
        F.r1 = grids[q].r1;
        F.r2 = grids[q].r2;
        F.delta = grids[q].delta > 0.0 ? grids[q].delta : M_PI / (2.0 * (grids[q].nt - 2));
        F.dr = (F.r2 - F.r1) / grids[q].nr;
        F.th0 = M_PI / 4.0 - F.delta;
        F.ph0 = -3.0 * M_PI / 4.0 - F.delta;
        F.dth = (M_PI / 2.0 + 2.0 * F.delta) / grids[q].nt;
        F.dph = (1.5 * M_PI + 2.0 * F.delta) / grids[q].np;
        std::vector<FillScalar> cc;
        std::vector<FillVector> vt, vp;
        if (!build_fill(F, L.d, cc, vt, vp)) return YY_ERR_GEOMETRY;
    }
    yy_ensemble *e = new (std::nothrow) yy_ensemble();
    if (!e) return YY_ERR_ARG;
    char *base = (char *)dev_ws;
    for (int q = 0; q < n && st == YY_OK; q++) {
        uint64_t b = 0;
        yy_workspace_bytes(&grids[q], prec, &b);
        yy_shell *sh = nullptr;
        st = yy_create(&grids[q], prec, base, b, &sh);
        if (st == YY_OK) e->sh.push_back(sh);
        base += align_up((int64_t)b, ALIGN);
    }
    e->arena = base;
    e->arena_bytes = arena_bytes_for(n);
    hipError_t h = hipSuccess;
    if (st == YY_OK) {
        e->streams.resize(n, nullptr);
        e->join.resize(n, nullptr);
        e->versions.resize(n, 0);
        for (int q = 0; q < n && h == hipSuccess; q++) {
            h = hipStreamCreateWithFlags(&e->streams[q], hipStreamNonBlocking);
            if (h == hipSuccess) h = hipEventCreateWithFlags(&e->join[q], hipEventDisableTiming);
        }
        if (h == hipSuccess) h = hipStreamCreateWithFlags(&e->cap, hipStreamNonBlocking);
        if (h == hipSuccess) h = hipEventCreateWithFlags(&e->fork, hipEventDisableTiming);
        if (h != hipSuccess) st = YY_ERR_HIP;
    }
    if (st != YY_OK) {
        yy_ensemble_destroy(e);
        return st;
    }
    *out = e;
    return YY_OK;
}

yy_shell *yy_ensemble_shell(yy_ensemble *e, int32_t s)
{
    if (!e || s < 0 || s >= (int32_t)e->sh.size()) return nullptr;
    return e->sh[s];
}

int yy_ensemble_step(yy_ensemble *e, int32_t K, int32_t graph, hipStream_t stream)
{
    if (!e || K < 1 || K > MAXK) return YY_ERR_ARG;
    for (yy_shell *s : e->sh) {
        if (!s->have_params) return YY_ERR_STATE;
        if (s->sticky != YY_OK) return s->sticky;
    }
    if (!graph) {
        for (yy_shell *s : e->sh) {
            const int st = shell_step(s, K, stream);
            if (st != YY_OK) return st;
        }
        return YY_OK;
    }
    // wall data must be set before every step, which a replay cannot do
    for (yy_shell *s : e->sh)
        if (uses_walls(s)) return YY_ERR_STATE;
    bool stale = !e->captured || e->K != K || e->how != graph;
    for (size_t q = 0; q < e->sh.size() && !stale; q++)
        if (e->sh[q]->version != e->versions[q]) stale = true;
    bool pending = false;
    for (yy_shell *s : e->sh) pending = pending || s->need_fill;
    // graph 1: batched launches (one per phase and tile bin), else, or if
    // the shells' steps do not line up, one forked stream per shell; 2:
    // forked streams
    auto capture_any = [&]() -> int {
        e->how = graph;
        if (graph == 1 && K <= 8 && capture_batched(e, K) == YY_OK) return YY_OK;
        e->batched = false;
        return capture(e, K);
    };
    if (stale && pending) {
        // this step runs eagerly (it performs the pending ghost refresh);
        // the graphs are captured for the following steps
        for (yy_shell *s : e->sh) {
            const int st = shell_step(s, K, stream);
            if (st != YY_OK) return st;
        }
        return capture_any();
    }
    if (stale) {
        const int st = capture_any();
        if (st != YY_OK) return st;
    }
    for (yy_shell *s : e->sh)
        if (walls_stale(s)) return YY_ERR_STATE;
    if (hipGraphLaunch(e->exec[e->phase], stream) != hipSuccess) return YY_ERR_HIP;
    for (yy_shell *s : e->sh) shell_rotate(s);
    e->phase = (e->phase + 1) % 6;
    return YY_OK;
}

int yy_ensemble_autotune(yy_ensemble *e, char *json_out, int32_t cap, hipStream_t stream)
{
    if (!e) return YY_ERR_ARG;
    const size_t n = e->sh.size();
    for (yy_shell *s : e->sh) {
        const int st = yy_autotune(s, nullptr, 0, stream);
        if (st != YY_OK) return st;
    }
    auto cells = [](const yy_shell *s) { return (int64_t)s->L.d.nr * s->L.d.nt * s->L.d.np; };
    auto bucket = [](int len) {
        int b = 0;
        while ((1 << b) < len) b++;
        return b;
    };
    std::string js = "{";
    // line-solve tiles per (unknown or diffusion-only, direction, line-length bucket)
    for (int L = 0; L < 5; L++)
        for (int dir = 0; dir < 3; dir++) {
            std::vector<int> rep(64, -1);
            std::vector<int> bk(n);
            for (size_t q = 0; q < n; q++) {
                const Dims &d = e->sh[q]->L.d;
                const int len = (dir == 0 ? d.nr : dir == 1 ? d.nt : d.np) - (L == dir + 1 ? 1 : 0);
                bk[q] = bucket(len);
                if (rep[bk[q]] < 0 || cells(e->sh[q]) > cells(e->sh[rep[bk[q]]])) rep[bk[q]] = (int)q;
            }
            for (size_t q = 0; q < n; q++) {
                const Tune &src = tune_of(e->sh[rep[bk[q]]]);
                Tune &dst = tune_of(e->sh[q]);
                dst.sb[L][dir] = 0;      // ensembles keep the default block counts
                if (dir < 2) {
                    dst.m[L][dir] = src.m[L][dir];
                    dst.w[L][dir] = src.w[L][dir];
                    dst.bl[L][dir] = src.bl[L][dir];
                } else {
                    dst.lpb[L] = src.lpb[L];
                    dst.wpl[L] = src.wpl[L];
                }
            }
            for (int b = 0; b < 64; b++) {
                if (rep[b] < 0) continue;
                const Tune &t = tune_of(e->sh[rep[b]]);
                char val[64];
                if (dir < 2) {
                    if (t.m[L][dir] == 1) std::snprintf(val, sizeof val, "t");
                    else std::snprintf(val, sizeof val, "m%dw%d%s", t.m[L][dir], t.w[L][dir], t.bl[L][dir] ? "b" : "");
                } else {
                    if (t.wpl[L]) std::snprintf(val, sizeof val, "v%d", t.wpl[L]);
                    else std::snprintf(val, sizeof val, "l%d", t.lpb[L]);
                }
                char key[48];
                std::snprintf(key, sizeof key, "%s.%c.n<=%d", tune_field_name[L], dir_name[dir], 1 << b);
                js += js.size() > 1 ? ",\"" : "\"";
                js += key;
                js += "\":\"";
                js += val;
                js += "\"";
            }
        }
    // residual column tiles per (unknown, phi-extent bucket)
    for (int L = 0; L < 4; L++) {
        std::vector<int> rep(64, -1);
        std::vector<int> bk(n);
        for (size_t q = 0; q < n; q++) {
            bk[q] = bucket(e->sh[q]->L.d.np);
            if (rep[bk[q]] < 0 || cells(e->sh[q]) > cells(e->sh[rep[bk[q]]])) rep[bk[q]] = (int)q;
        }
        for (size_t q = 0; q < n; q++) tune_of(e->sh[q]).rt[L] = tune_of(e->sh[rep[bk[q]]]).rt[L];
        for (int b = 0; b < 64; b++) {
            if (rep[b] < 0) continue;
            char key[48];
            std::snprintf(key, sizeof key, "res.%s.np<=%d", tune_field_name[L], 1 << b);
            js += ",\"";
            js += key;
            js += "\":\"";
            js += RES_TILES[tune_of(e->sh[rep[b]]).rt[L]].name;
            js += "\"";
        }
    }
    js += "}";
    for (yy_shell *s : e->sh) s->version++;
    if (json_out && cap > 0) {
        std::strncpy(json_out, js.c_str(), (size_t)cap - 1);
        json_out[cap - 1] = 0;
    }
    return YY_OK;
}

int yy_stream_copy(void *dst, const void *src, uint64_t bytes, hipStream_t stream)
{
    if (!dst || !src || bytes % 16 || ((uintptr_t)dst | (uintptr_t)src) % 16) return YY_ERR_ARG;
    if (bytes / 16 > (uint64_t)0xffffffffu * 1024) return YY_ERR_ARG;     // grid limit
    if (bytes == 0) return YY_OK;
    stream_copy(dst, src, (int64_t)(bytes / 16), stream);
    return hip_status(hipGetLastError());
}

int yy_ensemble_info(const yy_ensemble *e, int32_t *batched, int64_t *launches_per_step,
                     int64_t *shell_launches_per_step)
{
    if (!e) return YY_ERR_ARG;
    const bool b = e->captured && e->batched;
    if (batched) *batched = b ? 1 : 0;
    if (launches_per_step) *launches_per_step = b ? e->batched_launches / 6 : 0;
    if (shell_launches_per_step) *shell_launches_per_step = b ? e->shell_launches / 6 : 0;
    return YY_OK;
}

int yy_ensemble_destroy(yy_ensemble *e)
{
    if (!e) return YY_ERR_ARG;
    drop_graphs(e);
    for (hipStream_t s : e->streams)
        if (s) (void)hipStreamDestroy(s);
    for (hipEvent_t v : e->join)
        if (v) (void)hipEventDestroy(v);
    if (e->cap) (void)hipStreamDestroy(e->cap);
    if (e->fork) (void)hipEventDestroy(e->fork);
    for (yy_shell *s : e->sh) yy_destroy(s);
    delete e;
    return YY_OK;
}

}  // extern "C"

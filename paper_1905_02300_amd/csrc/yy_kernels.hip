// yy_kernels.hip -- gfx950 kernels of one Yin-Yang AC direction-splitting
// time step (Takhirov, Frolov & Minev, arXiv 1905.02300).
//
// Every kernel is templated on the compute precision R (double, or float in
// the FP32-mixed mode, where pressure accumulation, the divergence and all
// norms stay in double).  Memory-bound throughout: no dense contraction, so
// no MFMA; coalescing is along phi (k), the fastest index.
#include "yy_internal.h"

namespace yy {

template <typename R> struct Tri { R lo, di, up; };

// ---------------------------------------------------------------------------
// MAC averaging: component C (0 = r, 1 = theta, 2 = phi; stored on its own
// faces) at location L of the point with storage index q.  Faces f, f+1 are
// averaged where L is centred, centres f-1, f where L is a face.
// ---------------------------------------------------------------------------
template <int C, int L, typename R>
__device__ __forceinline__ R vel(const R *__restrict__ a, int64_t q, const Dims &d)
{
    const int64_t sI = d.sI, sJ = d.sJ;
    if (C == 0) {
        if (L == FR) return a[q];
        if (L == CC) return R(0.5) * (a[q] + a[q + sI]);
        if (L == FT) return R(0.25) * ((a[q - sJ] + a[q - sJ + sI]) + (a[q] + a[q + sI]));
        return R(0.25) * ((a[q - 1] + a[q - 1 + sI]) + (a[q] + a[q + sI]));
    } else if (C == 1) {
        if (L == FT) return a[q];
        if (L == CC) return R(0.5) * (a[q] + a[q + sJ]);
        if (L == FR) return R(0.25) * ((a[q - sI] + a[q - sI + sJ]) + (a[q] + a[q + sJ]));
        return R(0.25) * ((a[q - 1] + a[q - 1 + sJ]) + (a[q] + a[q + sJ]));
    } else {
        if (L == FP) return a[q];
        if (L == CC) return R(0.5) * (a[q] + a[q + 1]);
        if (L == FR) return R(0.25) * ((a[q - sI] + a[q - sI + 1]) + (a[q] + a[q + 1]));
        return R(0.25) * ((a[q - sJ] + a[q - sJ + 1]) + (a[q] + a[q + 1]));
    }
}

template <int L, typename R> __device__ __forceinline__ R r_of(const Geo<R> &g, int i)
{
    return L == FR ? g.rf[i + 1] : g.rc[i + 1];
}
template <int L, typename R> __device__ __forceinline__ R s_of(const Geo<R> &g, int j)
{
    return L == FT ? g.sf[j + 1] : g.sc[j + 1];
}
template <int L, typename R> __device__ __forceinline__ R c_of(const Geo<R> &g, int j)
{
    return L == FT ? g.cf[j + 1] : g.cc[j + 1];
}

// ---------------------------------------------------------------------------
// Coefficients (lower, diagonal, upper) of the split operator L_{L,D} at a
// point: T (eq. Convect_Douglas) and u_r, u_theta, u_phi (eq. r_comp,
// theta_comp, phi_comp), hat metrics (Sec. 3.2) in the theta/phi diffusion,
// grad-div blocks D_cc/(2 chi) in the own direction, advection by the
// extrapolated u2 (ar, at, ap at the point) with a minus sign.
// ---------------------------------------------------------------------------
template <int L, int D, typename R>
__device__ __forceinline__ Tri<R> coef(const Geo<R> &g, int i, int j, R ar, R at, R ap, R nu)
{
    Tri<R> c;
    const R r0 = r_of<L>(g, i);
    if (D == 0) {
        const R q = R(1) / (r0 * r0 * g.dr * g.dr);
        if (L == FR) {
            const R rm = g.rc[i], rp = g.rc[i + 1];           // centres i-1, i
            const R fm = g.rf[i], fp = g.rf[i + 2];           // faces i-1, i+1
            c.lo = nu * rm * rm * q;
            c.up = nu * rp * rp * q;
            c.di = -nu * (rm * rm + rp * rp) * q - nu * R(2) / (r0 * r0);
            const R k3 = nu * R(2) / (r0 * r0 * r0) / (R(2) * g.dr);
            c.lo -= k3 * fm * fm;
            c.up += k3 * fp * fp;
            const R dr2 = g.dr * g.dr;
            c.lo += g.ic * fm * fm / (rm * rm * dr2);
            c.up += g.ic * fp * fp / (rp * rp * dr2);
            c.di -= g.ic * r0 * r0 * (R(1) / (rp * rp) + R(1) / (rm * rm)) / dr2;
        } else {
            const R fm = g.rf[i + 1], fp = g.rf[i + 2];       // faces i, i+1
            c.lo = nu * fm * fm * q;
            c.up = nu * fp * fp * q;
            c.di = -nu * (fm * fm + fp * fp) * q;
        }
        const R a = ar / (R(2) * g.dr);
        c.lo += a;
        c.up -= a;
    } else if (D == 1) {
        const R s0 = s_of<L>(g, j);
        const R q = R(1) / (g.r1 * g.r1 * s0 * g.dth * g.dth);
        if (L == FT) {
            const R sm = g.sc[j], sp = g.sc[j + 1];           // centres j-1, j
            const R fm = g.sf[j], fp = g.sf[j + 2];           // faces j-1, j+1
            const R c0 = g.cf[j + 1];
            c.lo = nu * sm * q;
            c.up = nu * sp * q;
            c.di = -nu * (sm + sp) * q;
            const R e = nu / (r0 * r0 * s0 * s0);
            c.di -= e;
            const R k2 = R(2) * c0 * e / (R(2) * g.dth);
            c.lo -= k2 * fm;
            c.up += k2 * fp;
            c.di -= ar / r0;
            const R q2 = R(1) / (r0 * r0 * g.dth * g.dth);
            c.lo += g.ic * fm * q2 / sm;
            c.up += g.ic * fp * q2 / sp;
            c.di -= g.ic * s0 * q2 * (R(1) / sp + R(1) / sm);
        } else {
            const R fm = g.sf[j + 1], fp = g.sf[j + 2];       // faces j, j+1
            c.lo = nu * fm * q;
            c.up = nu * fp * q;
            c.di = -nu * (fm + fp) * q;
        }
        const R a = at / (R(2) * r0 * g.dth);
        c.lo += a;
        c.up -= a;
    } else {
        const R s0 = s_of<L>(g, j);
        c.lo = nu * g.cphat;
        c.up = nu * g.cphat;
        c.di = R(-2) * nu * g.cphat;
        if (L == FP) {
            const R c0 = c_of<L>(g, j);
            const R e = R(1) / (r0 * r0 * s0 * s0);
            c.di -= nu * e;
            c.di -= (ar + at * c0 / s0) / r0;
            const R q3 = g.ic * e / (g.dph * g.dph);
            c.lo += q3;
            c.up += q3;
            c.di -= R(2) * q3;
        }
        const R a = ap / (R(2) * r0 * s0 * g.dph);
        c.lo += a;
        c.up -= a;
    }
    return c;
}

template <int L, typename R>
__device__ __forceinline__ void adv(const State<R> &s, const Dims &d, int64_t q, R &ar, R &at, R &ap)
{
    ar = vel<0, L>(s.us[1][0], q, d);
    at = vel<1, L>(s.us[1][1], q, d);
    ap = vel<2, L>(s.us[1][2], q, d);
}

template <int L> __host__ __device__ constexpr int ulo(int dir) { return L == dir + 1 ? 1 : 0; }
__host__ __device__ inline int ncell(const Dims &d, int dir) { return dir == 0 ? d.nr : dir == 1 ? d.nt : d.np; }

// ---------------------------------------------------------------------------
// block reduction of a double (blockDim.x multiple of 64, <= 1024)
// ---------------------------------------------------------------------------
__device__ double block_sum(double v)
{
    __shared__ double red[16];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        for (int q = 0; q < nw; q++) t += red[q];
    }
    __syncthreads();
    return t;
}

// ---------------------------------------------------------------------------
// a1: extrapolation psi* = 1.5 psi^n - 0.5 psi^{n-1} (all padded points)
// ---------------------------------------------------------------------------
template <typename R> struct Ptr7 { R *s[7]; const R *n[7]; const R *m[7]; };

template <typename R>
__global__ void k_extrap(Ptr7<R> a, int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int f = 0; f < 7; f++) a.s[f][q] = R(1.5) * a.n[f][q] - R(0.5) * a.m[f][q];
    }
}

template <typename R>
__global__ void k_copy(Ptr7<R> a, int nf, const double *p0, double *p0d, const double *p1,
                       double *p1d, int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        for (int f = 0; f < nf; f++) a.s[f][q] = a.n[f][q];
        p0d[q] = p0[q];
        p1d[q] = p1[q];
    }
}

static int grid_for(int64_t n, int bs = 256)
{
    int64_t b = (n + bs - 1) / bs;
    return (int)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

template <typename R> void Ops<R>::extrap(const Dims &d, const State<R> &s, hipStream_t st)
{
    Ptr7<R> a;
    a.s[0] = s.Ts; a.n[0] = s.T[0]; a.m[0] = s.T[1];
    int f = 1;
    for (int y = 0; y < 2; y++)
        for (int c = 0; c < 3; c++, f++) {
            a.s[f] = s.us[y][c];
            a.n[f] = s.u[y][c][0];
            a.m[f] = s.u[y][c][1];
        }
    const int64_t n = 2 * d.sP;
    hipLaunchKernelGGL(k_extrap<R>, dim3(grid_for(n)), dim3(256), 0, st, a, n);
}

template <typename R>
void Ops<R>::copy_levels(const Dims &d, const State<R> &s, int from, int to, hipStream_t st)
{
    Ptr7<R> a;
    a.s[0] = s.T[to]; a.n[0] = s.T[from];
    int f = 1;
    for (int y = 0; y < 2; y++)
        for (int c = 0; c < 3; c++, f++) {
            a.s[f] = s.u[y][c][to];
            a.n[f] = s.u[y][c][from];
        }
    const int pf = from == 0 ? 0 : 1, pt = to == 0 ? 0 : 1;
    const int64_t n = 2 * d.sP;
    hipLaunchKernelGGL(k_copy<R>, dim3(grid_for(n)), dim3(256), 0, st, a, 7,
                       (const double *)s.p[0][pf], s.p[0][pt], (const double *)s.p[1][pf],
                       s.p[1][pt], n);
}


// ---------------------------------------------------------------------------
// a2: overlap interpolation (Sec. 4: Lagrange interpolation of boundary data
// from the other patch, at the same radial index) and wall rules
// ---------------------------------------------------------------------------
template <typename TT>
__device__ __forceinline__ double gather16(const TT *__restrict__ a, int64_t base, int64_t sJ,
                                           const double *wt, const double *wp)
{
    double v = 0.0;
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const TT *row = a + base + u * sJ;
        const double rsum = wp[0] * (double)row[0] + wp[1] * (double)row[1] +
                            wp[2] * (double)row[2] + wp[3] * (double)row[3];
        v += wt[u] * rsum;
    }
    return v;
}

// Targets of one scalar field (targets of patch blockIdx.y read the other
// patch); thread = (target, radial index).
template <typename TT>
__global__ void k_fill_scalar(Dims d, const FillScalar *__restrict__ tab, int ntab, TT *a,
                              int ilo, int ni, int pmask)
{
    const int p = blockIdx.y;
    if (!((pmask >> p) & 1)) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntab * ni) return;
    const int e = t % ntab;
    const int i = ilo + t / ntab;
    const FillScalar &f = tab[e];
    const double v = gather16(a, ix(d, 1 - p, i, f.dj, f.dk), d.sJ, f.wt, f.wp);
    a[ix(d, p, i, f.tj, f.tk)] = (TT)v;
}

// Tangential velocity targets: interpolate the other patch's u_theta (on
// its theta-face grid) and u_phi (on its phi-face grid) to the target and
// rotate into this patch's basis.
template <typename R>
__global__ void k_fill_vector(Dims d, const FillVector *__restrict__ tab, int ntab, const R *ut,
                              const R *up, R *dst, int ni, int pmask)
{
    const int p = blockIdx.y;
    if (!((pmask >> p) & 1)) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntab * ni) return;
    const int e = t % ntab;
    const int i = t / ntab;
    const FillVector &f = tab[e];
    const double vt = gather16(ut, ix(d, 1 - p, i, f.tjA, f.tkA), d.sJ, f.wtA, f.wpA);
    const double vp = gather16(up, ix(d, 1 - p, i, f.tjB, f.tkB), d.sJ, f.wtB, f.wpB);
    dst[ix(d, p, i, f.tj, f.tk)] = (R)(f.ma * vt + f.mb * vp);
}

// Walls r = R1, R2 (eq. eq_ns, eq_heat_convec): u_r = 0 on the wall faces;
// reflection ghosts psi_{-1} = 2 psi_wall - psi_0 for T and the tangential
// velocities.  Thread = padded (j, k) point of patch blockIdx.y.
template <typename R>
__global__ void k_walls(Dims d, State<R> s, int lev, R t_in, R t_out, int pmask)
{
    const int p = blockIdx.y;
    if (!((pmask >> p) & 1)) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int nk = d.np + 2, nj = d.nt + 2;
    if (t >= nk * nj) return;
    const int j = t / nk - 1, k = t % nk - 1;
    const int64_t q0 = ix(d, p, 0, j, k), qm = q0 - d.sI;
    const int64_t q1 = ix(d, p, d.nr - 1, j, k), qp = q1 + d.sI;
    R *T = s.T[lev];
    T[qm] = R(2) * t_in - T[q0];
    T[qp] = R(2) * t_out - T[q1];
    for (int y = 0; y < 2; y++) {
        R *a = s.u[y][1][lev], *b = s.u[y][2][lev], *c = s.u[y][0][lev];
        a[qm] = -a[q0];
        a[qp] = -a[q1];
        b[qm] = -b[q0];
        b[qp] = -b[q1];
        c[q0] = R(0);
        c[ix(d, p, d.nr, j, k)] = R(0);
    }
}

template <typename R>
void Ops<R>::fill(const Dims &d, const State<R> &s, int lev, const FillScalar *cc, int ncc,
                  const FillVector *vt, int nvt, const FillVector *vp, int nvp, double t_in,
                  double t_out, int pmask, hipStream_t st)
{
    const int pl = lev == 0 ? 0 : 1;     // pressure keeps levels n and k
    // centre-type scalars: T, p1, p2 (radial 0..nr-1); u_r (faces 1..nr-1)
    int n = ncc * d.nr;
    dim3 g((n + 255) / 256, 2);
    hipLaunchKernelGGL(k_fill_scalar<R>, g, dim3(256), 0, st, d, cc, ncc, s.T[lev], 0, d.nr, pmask);
    hipLaunchKernelGGL(k_fill_scalar<double>, g, dim3(256), 0, st, d, cc, ncc, s.p[0][pl], 0, d.nr, pmask);
    hipLaunchKernelGGL(k_fill_scalar<double>, g, dim3(256), 0, st, d, cc, ncc, s.p[1][pl], 0, d.nr, pmask);
    n = ncc * (d.nr - 1);
    dim3 g1((n + 255) / 256, 2);
    for (int y = 0; y < 2; y++)
        hipLaunchKernelGGL(k_fill_scalar<R>, g1, dim3(256), 0, st, d, cc, ncc, s.u[y][0][lev], 1,
                           d.nr - 1, pmask);
    for (int y = 0; y < 2; y++) {
        R *ut = s.u[y][1][lev], *up = s.u[y][2][lev];
        n = nvt * d.nr;
        hipLaunchKernelGGL(k_fill_vector<R>, dim3((n + 255) / 256, 2), dim3(256), 0, st, d, vt, nvt,
                           (const R *)ut, (const R *)up, ut, d.nr, pmask);
        n = nvp * d.nr;
        hipLaunchKernelGGL(k_fill_vector<R>, dim3((n + 255) / 256, 2), dim3(256), 0, st, d, vp, nvp,
                           (const R *)ut, (const R *)up, up, d.nr, pmask);
    }
    n = (d.np + 2) * (d.nt + 2);
    hipLaunchKernelGGL(k_walls<R>, dim3((n + 255) / 256, 2), dim3(256), 0, st, d, s, lev, (R)t_in,
                       (R)t_out, pmask);
}

// ---------------------------------------------------------------------------
// a3/a4: residual tau R^k = tau [Lhat psibar + (F - Lhat) psi* + S
//                                 - (psi^{k-1} - psi^n)/tau]
// ---------------------------------------------------------------------------
template <typename R> struct RhsIn {
    const R *pn, *pk, *ps, *f;
    const R *un[3], *uk[3], *us[3];   // velocity of the solved system
    const R *Tn, *Tk;
    const double *psn, *p1n, *p1k;
    int sys;                          // 0 (T), 1, 2
};

// Div_r, Div_theta, Div_phi of one stored velocity component at the centre
// with storage index q (centre (i, j, k))
template <typename R, typename A>
__device__ __forceinline__ A div_r(const Geo<R> &g, const R *a, int64_t q, int64_t sI, int i)
{
    const A fp = g.rf[i + 2], fm = g.rf[i + 1], rc = g.rc[i + 1];
    return (fp * fp * (A)a[q + sI] - fm * fm * (A)a[q]) / (rc * rc * (A)g.dr);
}
template <typename R, typename A>
__device__ __forceinline__ A div_t(const Geo<R> &g, const R *a, int64_t q, int64_t sJ, int i, int j)
{
    return ((A)g.sf[j + 2] * (A)a[q + sJ] - (A)g.sf[j + 1] * (A)a[q]) /
           ((A)g.rc[i + 1] * (A)g.sc[j + 1] * (A)g.dth);
}
template <typename R, typename A>
__device__ __forceinline__ A div_p(const Geo<R> &g, const R *a, int64_t q, int i, int j)
{
    return ((A)a[q + 1] - (A)a[q]) / ((A)g.rc[i + 1] * (A)g.sc[j + 1] * (A)g.dph);
}

template <typename R>
__device__ __forceinline__ double ptilde(const RhsIn<R> &in, int64_t q)
{
    if (in.sys == 1) return in.psn[q];
    return in.psn[q] + 0.5 * (in.p1k[q] - in.p1n[q]);
}

template <typename R, int L>
__device__ R source(const Dims &d, const Geo<R> &g, const RhsIn<R> &in, int64_t q, int i, int j,
                    R ar, R at, R ap)
{
    const int64_t sI = d.sI, sJ = d.sJ;
    R S = in.f ? in.f[q] : R(0);
    if (L == CC) return S;
    if (L == FR) {
        // grad-div with the extrapolated upper blocks: (D12 u_t* + D13 u_p*)/(2 chi)
        const R d12 = (div_t<R, R>(g, in.us[1], q, sJ, i, j) - div_t<R, R>(g, in.us[1], q - sI, sJ, i - 1, j)) / g.dr;
        const R d13 = (div_p<R, R>(g, in.us[2], q, i, j) - div_p<R, R>(g, in.us[2], q - sI, i - 1, j)) / g.dr;
        S += g.ic * (d12 + d13);
        const R r0 = g.rf[i + 1];
        S += (at * vel<1, FR>(in.us[1], q, d) + ap * vel<2, FR>(in.us[2], q, d)) / r0;
        S -= (R)((ptilde(in, q) - ptilde(in, q - sI)) / (double)g.dr);
        S += g.prra * R(0.25) * ((in.Tn[q - sI] + in.Tk[q - sI]) + (in.Tn[q] + in.Tk[q]));
    } else if (L == FT) {
        const R r0 = g.rc[i + 1], s0 = g.sf[j + 1], c0 = g.cf[j + 1];
        // (D21 u_r^{n+1/2} + D23 u_p*)/(2 chi)
        const R dj0 = R(0.5) * (div_r<R, R>(g, in.un[0], q, sI, i) + div_r<R, R>(g, in.uk[0], q, sI, i));
        const R dj1 = R(0.5) * (div_r<R, R>(g, in.un[0], q - sJ, sI, i) + div_r<R, R>(g, in.uk[0], q - sJ, sI, i));
        const R d21 = (dj0 - dj1) / (r0 * g.dth);
        const R d23 = (div_p<R, R>(g, in.us[2], q, i, j) - div_p<R, R>(g, in.us[2], q - sJ, i, j - 1)) / (r0 * g.dth);
        S += g.ic * (d21 + d23);
        // Pr[(2/r^2) d_th u_r + (2 cos/(r^3 sin)) d_r(r^2 u_r)] at n+1/2
        auto ub = [&](int64_t qq) { return R(0.5) * (in.un[0][qq] + in.uk[0][qq]); };
        const R dth_ur = R(0.5) * ((ub(q) - ub(q - sJ)) + (ub(q + sI) - ub(q + sI - sJ))) / g.dth;
        const R fp2 = g.rf[i + 2] * g.rf[i + 2], fm2 = g.rf[i + 1] * g.rf[i + 1];
        const R dr_r2ur = R(0.5) * ((fp2 * ub(q - sJ + sI) - fm2 * ub(q - sJ)) +
                                    (fp2 * ub(q + sI) - fm2 * ub(q))) / g.dr;
        S += g.pr * (R(2) / (r0 * r0) * dth_ur + R(2) * c0 / (r0 * r0 * r0 * s0) * dr_r2ur);
        S += ap * vel<2, FT>(in.us[2], q, d) * c0 / (s0 * r0);
        S -= (R)((ptilde(in, q) - ptilde(in, q - sJ)) / ((double)r0 * (double)g.dth));
    } else {
        const R r0 = g.rc[i + 1], s0 = g.sc[j + 1], c0 = g.cc[j + 1];
        const R gg = r0 * s0 * g.dph;
        // (D31 u_r^{n+1/2} + D32 u_t^{n+1/2})/(2 chi)
        const R a0 = R(0.5) * (div_r<R, R>(g, in.un[0], q, sI, i) + div_r<R, R>(g, in.uk[0], q, sI, i));
        const R a1 = R(0.5) * (div_r<R, R>(g, in.un[0], q - 1, sI, i) + div_r<R, R>(g, in.uk[0], q - 1, sI, i));
        const R b0 = R(0.5) * (div_t<R, R>(g, in.un[1], q, sJ, i, j) + div_t<R, R>(g, in.uk[1], q, sJ, i, j));
        const R b1 = R(0.5) * (div_t<R, R>(g, in.un[1], q - 1, sJ, i, j) + div_t<R, R>(g, in.uk[1], q - 1, sJ, i, j));
        S += g.ic * ((a0 - a1) / gg + (b0 - b1) / gg);
        auto ubr = [&](int64_t qq) { return R(0.5) * (in.un[0][qq] + in.uk[0][qq]); };
        auto ubt = [&](int64_t qq) { return R(0.5) * (in.un[1][qq] + in.uk[1][qq]); };
        const R dph_ur = R(0.5) * ((ubr(q) - ubr(q - 1)) + (ubr(q + sI) - ubr(q + sI - 1))) / g.dph;
        const R dph_ut = R(0.5) * ((ubt(q) - ubt(q - 1)) + (ubt(q + sJ) - ubt(q + sJ - 1))) / g.dph;
        S += g.pr * (R(2) / (r0 * r0 * s0) * dph_ur + R(2) * c0 / (r0 * r0 * s0 * s0) * dph_ut);
        S -= (R)((ptilde(in, q) - ptilde(in, q - 1)) / ((double)r0 * (double)s0 * (double)g.dph));
    }
    return S;
}

template <typename R, int L>
__global__ void k_residual(Dims d, Geo<R> g, State<R> s, RhsIn<R> in, R *out)
{
    const int p = blockIdx.y;
    const int i0 = ulo<L>(0), j0 = ulo<L>(1), k0 = ulo<L>(2);
    const int ni = d.nr - i0, nj = d.nt - j0, nk = d.np - k0;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)ni * nj * nk) return;
    const int k = k0 + (int)(t % nk);
    const int j = j0 + (int)((t / nk) % nj);
    const int i = i0 + (int)(t / ((int64_t)nk * nj));
    const int64_t q = ix(d, p, i, j, k);
    const int64_t sI = d.sI, sJ = d.sJ;
    const R nu = L == CC ? R(1) : g.pr;
    R ar, at, ap;
    adv<L>(s, d, q, ar, at, ap);
    auto bar = [&](int64_t qq) { return R(0.5) * (in.pn[qq] + in.pk[qq]); };
    const Tri<R> c0 = coef<L, 0>(g, i, j, ar, at, ap, nu);
    const Tri<R> c1 = coef<L, 1>(g, i, j, ar, at, ap, nu);
    const Tri<R> c2 = coef<L, 2>(g, i, j, ar, at, ap, nu);
    const R b0 = bar(q);
    R Rv = c0.lo * bar(q - sI) + c0.di * b0 + c0.up * bar(q + sI);
    Rv += c1.lo * bar(q - sJ) + c1.di * b0 + c1.up * bar(q + sJ);
    Rv += c2.lo * bar(q - 1) + c2.di * b0 + c2.up * bar(q + 1);
    // (F - Lhat) psi* = nu [(D_thth - Dhat_thth) + (D_phph - Dhat_phph)] psi*
    const R r0 = r_of<L>(g, i), s0 = s_of<L>(g, j);
    const R sm = L == FT ? g.sc[j] : g.sf[j + 1];
    const R sp = L == FT ? g.sc[j + 1] : g.sf[j + 2];
    const R x0 = in.ps[q];
    const R lt = (sp * (in.ps[q + sJ] - x0) - sm * (x0 - in.ps[q - sJ])) / (s0 * g.dth * g.dth);
    const R lp = in.ps[q + 1] - R(2) * x0 + in.ps[q - 1];
    Rv += nu * ((R(1) / (r0 * r0) - R(1) / (g.r1 * g.r1)) * lt +
                (R(1) / (r0 * r0 * s0 * s0 * g.dph * g.dph) - g.cphat) * lp);
    Rv += source<R, L>(d, g, in, q, i, j, ar, at, ap);
    Rv -= (in.pk[q] - in.pn[q]) * g.inv_tau;
    out[q] = g.tau * Rv;
}

// ---------------------------------------------------------------------------
// a5: line sweeps (I - tau/2 L_{L,D}) y = x, Thomas algorithm per line.
// Homogeneous ends: correction 0 at theta/phi ghosts, boundary faces and
// u_r wall faces; reflection c_{-1} = -c_0 for r-centred unknowns.
// MODE 0: y = solution; MODE 1 (last factor): psi^k += solution and the
// l2 norm of the increment into per-block partial sums.
// Thread = line; lines along r and theta are coalesced over k.
// ---------------------------------------------------------------------------
template <typename R, int L, int D, int MODE, bool DIFF>
__global__ void __launch_bounds__(256) k_sweep(Dims d, Geo<R> g, Geo<double> gd, State<R> s,
                                               const R *x, R *y, R *cb, R *psi, double *partial)
{
    const int p = blockIdx.y;
    const int i0 = ulo<L>(0), j0 = ulo<L>(1), k0 = ulo<L>(2);
    // the two indices that label a line, and the along-line range
    const int nA = D == 0 ? d.nt - j0 : d.nr - i0;          // slow label
    const int nB = D == 2 ? d.nt - j0 : d.np - k0;          // fast label
    const int m0 = D == 0 ? i0 : (D == 1 ? j0 : k0);
    const int n = ncell(d, D) - m0;
    const int64_t stride = D == 0 ? d.sI : (D == 1 ? d.sJ : 1);
    const bool reflect = (D == 0) && (L != FR);
    const R nu = (L == CC && !DIFF) ? R(1) : g.pr;
    const R ht = g.ht;
    double acc = 0.0;
    const int64_t nlines = (int64_t)nA * nB;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nlines;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int a = (int)(t / nB), b = (int)(t % nB);
        int i, j, k;
        if (D == 0) { j = j0 + a; k = k0 + b; i = m0; }
        else if (D == 1) { i = i0 + a; k = k0 + b; j = m0; }
        else { i = i0 + a; j = j0 + b; k = m0; }
        int64_t q = ix(d, p, i, j, k);
        R cprev = R(0), dprev = R(0);
        for (int m = 0; m < n; m++, q += stride) {
            const int ii = D == 0 ? m0 + m : i, jj = D == 1 ? m0 + m : j;
            R ar = R(0), at = R(0), ap = R(0);
            if (!DIFF) adv<L>(s, d, q, ar, at, ap);
            const Tri<R> c = coef<L, D>(g, ii, jj, ar, at, ap, nu);
            const R lo = -ht * c.lo, up = -ht * c.up;
            R di = R(1) - ht * c.di;
            if (reflect && m == 0) di = R(1) - ht * (c.di - c.lo);
            if (reflect && m == n - 1) di = R(1) - ht * (c.di - c.up);
            const R den = di - lo * cprev;
            const R cp = (m < n - 1) ? up / den : R(0);
            const R dp = (x[q] - lo * dprev) / den;
            cb[q] = cp;
            y[q] = dp;
            cprev = cp;
            dprev = dp;
        }
        q -= stride;
        R xn = R(0);
        for (int m = n - 1; m >= 0; m--, q -= stride) {
            const R xm = y[q] - cb[q] * xn;
            xn = xm;
            if (MODE == 0) {
                y[q] = xm;
            } else {
                psi[q] += xm;
                const int ii = D == 0 ? m0 + m : i, jj = D == 1 ? m0 + m : j;
                const double r0 = L == FR ? gd.rf[ii + 1] : gd.rc[ii + 1];
                const double s0 = L == FT ? gd.sf[jj + 1] : gd.sc[jj + 1];
                acc += r0 * r0 * s0 * gd.dr * gd.dth * gd.dph * (double)xm * (double)xm;
            }
        }
    }
    if (MODE == 1) {
        const double tot = block_sum(acc);
        if (threadIdx.x == 0) partial[p * NBMAX + blockIdx.x] = tot;
    }
}

template <typename R, int L, int D, int MODE, bool DIFF>
static void launch_sweep(const Dims &d, const Geo<R> &g, const Geo<double> &gd, const State<R> &s,
                         const R *x, R *y, R *psi, double *partial, int *nblocks, hipStream_t st)
{
    const int i0 = ulo<L>(0), j0 = ulo<L>(1), k0 = ulo<L>(2);
    const int nA = D == 0 ? d.nt - j0 : d.nr - i0;
    const int nB = D == 2 ? d.nt - j0 : d.np - k0;
    int64_t b = ((int64_t)nA * nB + 255) / 256;
    if (MODE == 1 && b > NBMAX) b = NBMAX;
    if (nblocks) *nblocks = (int)b;
    hipLaunchKernelGGL((k_sweep<R, L, D, MODE, DIFF>), dim3((unsigned)b, 2), dim3(256), 0, st, d, g,
                       gd, s, x, y, s.cb, psi, partial);
}

template <typename R, int L, int MODE>
static void sweep_dir(int dir, const Dims &d, const Geo<R> &g, const Geo<double> &gd,
                      const State<R> &s, const R *x, R *y, R *psi, double *partial, int *nb,
                      hipStream_t st)
{
    if (dir == 0) launch_sweep<R, L, 0, MODE, false>(d, g, gd, s, x, y, psi, partial, nb, st);
    else if (dir == 1) launch_sweep<R, L, 1, MODE, false>(d, g, gd, s, x, y, psi, partial, nb, st);
    else launch_sweep<R, L, 2, MODE, false>(d, g, gd, s, x, y, psi, partial, nb, st);
}

static int loc_of_field(int f)
{
    switch (f) {
    case 1: case 5: return FR;
    case 2: case 6: return FT;
    case 3: case 7: return FP;
    default: return CC;
    }
}

template <typename R> static R *field_level(const State<R> &s, int f, int lev)
{
    if (f == 0) return s.T[lev];
    const int y = f >= 5 ? 1 : 0, c = (f - (y ? 5 : 1));
    return s.u[y][c][lev];
}

template <typename R>
void Ops<R>::sweep(const Dims &d, const Geo<R> &g, const Geo<double> &gd, const State<R> &s,
                   int field, int dir, const R *x, R *y, int mode, double *partial, int *nb,
                   int diffusion_only, hipStream_t st)
{
    if (diffusion_only) {
        if (dir == 0) launch_sweep<R, CC, 0, 0, true>(d, g, gd, s, x, y, nullptr, nullptr, nullptr, st);
        else if (dir == 1) launch_sweep<R, CC, 1, 0, true>(d, g, gd, s, x, y, nullptr, nullptr, nullptr, st);
        else launch_sweep<R, CC, 2, 0, true>(d, g, gd, s, x, y, nullptr, nullptr, nullptr, st);
        return;
    }
    const int L = loc_of_field(field);
    R *psi = mode ? field_level(s, field, 2) : nullptr;
#define YY_SW(LL)                                                                              \
    if (mode) sweep_dir<R, LL, 1>(dir, d, g, gd, s, x, y, psi, partial, nb, st);                  \
    else sweep_dir<R, LL, 0>(dir, d, g, gd, s, x, y, psi, partial, nb, st);
    if (L == CC) { YY_SW(CC) }
    else if (L == FR) { YY_SW(FR) }
    else if (L == FT) { YY_SW(FT) }
    else { YY_SW(FP) }
#undef YY_SW
}

template <typename R>
void Ops<R>::residual(const Dims &d, const Geo<R> &g, const State<R> &s, int field, R *out,
                      hipStream_t st)
{
    RhsIn<R> in;
    const int L = loc_of_field(field);
    const int sys = field == 0 ? 0 : (field >= 5 ? 2 : 1);
    in.pn = field_level(s, field, 0);
    in.pk = field_level(s, field, 2);
    in.ps = field == 0 ? s.Ts : s.us[sys - 1][L - 1];
    in.f = s.force[L];
    const int y = sys == 2 ? 1 : 0;
    for (int c = 0; c < 3; c++) {
        in.un[c] = s.u[y][c][0];
        in.uk[c] = s.u[y][c][2];
        in.us[c] = s.us[y][c];
    }
    in.Tn = s.T[0];
    in.Tk = s.T[2];
    in.psn = s.p[y][0];
    in.p1n = s.p[0][0];
    in.p1k = s.p[0][1];
    in.sys = sys;
    const int i0 = L == FR, j0 = L == FT, k0 = L == FP;
    const int64_t n = (int64_t)(d.nr - i0) * (d.nt - j0) * (d.np - k0);
    dim3 gr((unsigned)((n + 255) / 256), 2);
    if (L == CC) hipLaunchKernelGGL((k_residual<R, CC>), gr, dim3(256), 0, st, d, g, s, in, out);
    else if (L == FR) hipLaunchKernelGGL((k_residual<R, FR>), gr, dim3(256), 0, st, d, g, s, in, out);
    else if (L == FT) hipLaunchKernelGGL((k_residual<R, FT>), gr, dim3(256), 0, st, d, g, s, in, out);
    else hipLaunchKernelGGL((k_residual<R, FP>), gr, dim3(256), 0, st, d, g, s, in, out);
}

// ---------------------------------------------------------------------------
// a6: pressure (eq. nst_Mass1; bootstrapped form of eq. ac2), FP64:
//   p1^k = p1^n - Div_h u1^{n+1/2}/chi,
//   p2^k = p2^n + (p1^k - p1^n) - Div_h u2^{n+1/2}/chi,
// with the l2 norms of the increment and (system 2) of Div_h u2^k.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ double div_h(const Geo<double> &gd, const R *ur, const R *ut, const R *up,
                                        int64_t q, const Dims &d, int i, int j)
{
    const double fp = gd.rf[i + 2], fm = gd.rf[i + 1], rc = gd.rc[i + 1];
    const double sc = gd.sc[j + 1];
    const double a = (fp * fp * (double)ur[q + d.sI] - fm * fm * (double)ur[q]) / (rc * rc * gd.dr);
    const double b = (gd.sf[j + 2] * (double)ut[q + d.sJ] - gd.sf[j + 1] * (double)ut[q]) / (rc * sc * gd.dth);
    const double c = ((double)up[q + 1] - (double)up[q]) / (rc * sc * gd.dph);
    return a + b + c;
}

template <typename R>
__global__ void __launch_bounds__(256) k_pressure(Dims d, Geo<double> gd, State<R> s, int sys,
                                                  double *pinc, double *pdiv)
{
    const int p = blockIdx.y;
    const int y = sys - 1;
    const int64_t n = (int64_t)d.nr * d.nt * d.np;
    double ai = 0.0, ad = 0.0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(t % d.np);
        const int j = (int)((t / d.np) % d.nt);
        const int i = (int)(t / ((int64_t)d.np * d.nt));
        const int64_t q = ix(d, p, i, j, k);
        const double dn = div_h(gd, s.u[y][0][0], s.u[y][1][0], s.u[y][2][0], q, d, i, j);
        const double dk = div_h(gd, s.u[y][0][2], s.u[y][1][2], s.u[y][2][2], q, d, i, j);
        double nv = s.p[y][0][q] - 0.5 * (dn + dk) * gd.inv_chi;
        if (sys == 2) nv += s.p[0][1][q] - s.p[0][0][q];
        const double inc = nv - s.p[y][1][q];
        s.p[y][1][q] = nv;
        const double rc = gd.rc[i + 1];
        const double w = rc * rc * gd.sc[j + 1] * gd.dr * gd.dth * gd.dph;
        ai += w * inc * inc;
        if (sys == 2) ad += w * dk * dk;
    }
    const double ti = block_sum(ai);
    const double td = block_sum(ad);
    if (threadIdx.x == 0) {
        pinc[p * NBMAX + blockIdx.x] = ti;
        if (sys == 2) pdiv[p * NBMAX + blockIdx.x] = td;
    }
}

template <typename R>
void Ops<R>::pressure(const Dims &d, const Geo<R> &g, const Geo<double> &gd, const State<R> &s,
                      int sys, double *pinc, double *pdiv, int *nb, hipStream_t st)
{
    (void)g;
    const int64_t n = (int64_t)d.nr * d.nt * d.np;
    int64_t b = (n + 255) / 256;
    if (b > NBMAX) b = NBMAX;
    *nb = (int)b;
    hipLaunchKernelGGL(k_pressure<R>, dim3((unsigned)b, 2), dim3(256), 0, st, d, gd, s, sys, pinc, pdiv);
}

// ---------------------------------------------------------------------------
// norms: fixed-order reduction of the per-block partial sums
// ---------------------------------------------------------------------------
struct NB { int n[NSLOT]; };

__global__ void k_reduce(const double *partial, NB nb, double *out)
{
    const int slot = blockIdx.x >> 1, p = blockIdx.x & 1;
    const double *src = partial + (int64_t)(slot * 2 + p) * NBMAX;
    double v = 0.0;
    for (int b = threadIdx.x; b < nb.n[slot]; b += blockDim.x) v += src[b];
    const double t = block_sum(v);
    if (threadIdx.x == 0) out[p * NSLOT + slot] = sqrt(t);
}

void reduce_norms(const double *partial, const int *nblocks, double *out, hipStream_t st)
{
    NB nb;
    for (int q = 0; q < NSLOT; q++) nb.n[q] = nblocks[q];
    hipLaunchKernelGGL(k_reduce, dim3(2 * NSLOT), dim3(256), 0, st, partial, nb, out);
}

__global__ void k_zero(double *p, int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        p[q] = 0.0;
}

void zero_doubles(double *p, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero, dim3(grid_for(n)), dim3(256), 0, st, p, n);
}

// ---------------------------------------------------------------------------
// field I/O: MAC or padded double arrays <-> internal layout
// ---------------------------------------------------------------------------
template <typename TT>
__global__ void k_io(Dims d, TT *in, const double *src, double *dst, int loc, int layout)
{
    const int fr = loc == FR, ft = loc == FT, fp = loc == FP;
    int n0, n1, n2, o;
    if (layout == 0) { n0 = d.nr + fr; n1 = d.nt + ft; n2 = d.np + fp; o = 0; }
    else { n0 = d.nr + 2; n1 = d.nt + 2; n2 = d.np + 2; o = -1; }
    const int64_t per = (int64_t)n0 * n1 * n2;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < 2 * per;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(t / per);
        const int64_t u = t % per;
        const int k = (int)(u % n2) + o, j = (int)((u / n2) % n1) + o, i = (int)(u / ((int64_t)n2 * n1)) + o;
        const int64_t q = ix(d, p, i, j, k);
        if (src) in[q] = (TT)src[t];
        else dst[t] = (double)in[q];
    }
}

template <typename R>
void Ops<R>::io(const Dims &d, R *internal, const double *src, double *dst, int loc, int layout,
                hipStream_t st)
{
    const int64_t n = 2LL * (d.nr + 2) * (d.nt + 2) * (d.np + 2);
    hipLaunchKernelGGL(k_io<R>, dim3(grid_for(n)), dim3(256), 0, st, d, internal, src, dst, loc, layout);
}

void io_double(const Dims &d, double *internal, const double *src, double *dst, int loc, int layout,
               hipStream_t st)
{
    const int64_t n = 2LL * (d.nr + 2) * (d.nt + 2) * (d.np + 2);
    hipLaunchKernelGGL(k_io<double>, dim3(grid_for(n)), dim3(256), 0, st, d, internal, src, dst, loc, layout);
}

template struct Ops<double>;
template struct Ops<float>;

}  // namespace yy

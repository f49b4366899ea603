// yy_kernels.hip -- gfx950 kernels of one Yin-Yang AC direction-splitting
// time step (Takhirov, Frolov & Minev, arXiv 1905.02300).
//
// Every kernel is templated on the compute precision R (double, or float in
// the FP32-mixed mode, where pressure accumulation, the divergence and all
// norms stay in double).  Memory-bound throughout: no dense contraction, so
// no MFMA; coalescing is along phi (k), the fastest index.
#include <type_traits>

#include "yy_internal.h"

namespace yy {

// This file is compiled twice, once per compute precision (YY_ONLY_DOUBLE,
// YY_ONLY_FLOAT), so that the two halves build in parallel; the functions
// that are not templates live in the FP64 object.
#if !defined(YY_ONLY_FLOAT)
// the launch recorder of the calling thread (null: launch normally)
static thread_local LaunchRecorder *t_recorder = nullptr;
void set_launch_recorder(LaunchRecorder *r) { t_recorder = r; }
LaunchRecorder *launch_recorder() { return t_recorder; }
#endif

template <typename R> struct Tri { R lo, di, up; };

// ---------------------------------------------------------------------------
// Field access by 32-bit element index: the byte offset is formed in 32 bits,
// so a load is one wave-uniform 64-bit base (SGPRs) plus a 32-bit lane
// offset, with no per-lane 64-bit address arithmetic.
// ---------------------------------------------------------------------------
template <typename T> struct FV {
    const T *p;
    __device__ __forceinline__ explicit FV(const T *q) : p(q) {}
    __device__ __forceinline__ T operator[](uint32_t e) const
    {
        return *(const T *)((const char *)p + e * (uint32_t)sizeof(T));
    }
};
template <typename T> __device__ __forceinline__ void st(T *b, uint32_t e, T v)
{
    *(T *)((char *)b + e * (uint32_t)sizeof(T)) = v;
}

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
// Per-row coefficient tables of L_{L,D} along an r-line (D = 0, index i+1)
// or a theta-line (D = 1, index j+1), in a fixed order: D = 0: u_r (FR)
// fr_lo, fr_up, fr_di, else rc_lo, rc_up; D = 1: u_theta (FT) tf_lo, tf_up,
// ft_lo, ft_up, ft_di, else tc_lo, tc_up.  The strided line solves stage
// them in LDS (Tab = an LDS row); everyone else reads the tables (GTab).
template <int L, int D> __host__ __device__ constexpr int ntabs()
{
    return D == 0 ? (L == FR ? 3 : 2) : (D == 1 ? (L == FT ? 5 : 2) : 0);
}
template <int L, int D, typename R> __device__ __forceinline__ const R *row_table(const Geo<R> &g, int t)
{
    if (D == 0) {
        if (L == FR) return t == 0 ? (const R *)g.fr_lo : (t == 1 ? (const R *)g.fr_up : (const R *)g.fr_di);
        return t == 0 ? (const R *)g.rc_lo : (const R *)g.rc_up;
    }
    if (L == FT)
        return t == 0 ? (const R *)g.tf_lo : t == 1 ? (const R *)g.tf_up : t == 2 ? (const R *)g.ft_lo
                                                                          : t == 3 ? (const R *)g.ft_up
                                                                                   : (const R *)g.ft_di;
    return t == 0 ? (const R *)g.tc_lo : (const R *)g.tc_up;
}
// table t of the row through the Geo tables
template <int L, int D, typename R> struct GTab {
    const Geo<R> &g;
    int idx;
    __device__ __forceinline__ R operator()(int t) const
    {
        if (D == 0) {
            if (L == FR) return t == 0 ? g.fr_lo[idx] : (t == 1 ? g.fr_up[idx] : g.fr_di[idx]);
            return t == 0 ? g.rc_lo[idx] : g.rc_up[idx];
        }
        if (L == FT)
            return t == 0 ? g.tf_lo[idx] : t == 1 ? g.tf_up[idx] : t == 2 ? g.ft_lo[idx] : t == 3 ? g.ft_up[idx] : g.ft_di[idx];
        return t == 0 ? g.tc_lo[idx] : g.tc_up[idx];
    }
};
// table t of the row from LDS (row-major: table t at base[t * ld])
template <typename R> struct LTab {
    const R *base;
    int ld;
    __device__ __forceinline__ R operator()(int t) const { return base[t * ld]; }
};

template <int L, int D, typename R, typename TB>
__device__ __forceinline__ Tri<R> coef_t(const Geo<R> &g, int i, int j, R ar, R at, R ap, R nu, const TB &tb)
{
    Tri<R> c;
    if (D == 0) {
        if (L == FR) {
            // u_r is always a velocity unknown: nu = Pr, combined on the host
            c.lo = tb(0);
            c.up = tb(1);
            c.di = tb(2);
        } else {
            const R lo = tb(0), up = tb(1);
            c.lo = nu * lo;
            c.up = nu * up;
            c.di = -nu * (lo + up);
        }
        const R a = ar * g.h2r;
        c.lo += a;
        c.up -= a;
    } else if (D == 1) {
        const R ir = L == FR ? g.ir_f[i + 1] : g.ir_c[i + 1];
        if (L == FT) {
            const R lo = tb(0), up = tb(1);
            const R ir2 = g.ir2_c[i + 1];
            c.lo = nu * lo + ir2 * tb(2);
            c.up = nu * up + ir2 * tb(3);
            c.di = -nu * (lo + up) + ir2 * tb(4) - ar * ir;
        } else {
            const R lo = tb(0), up = tb(1);
            c.lo = nu * lo;
            c.up = nu * up;
            c.di = -nu * (lo + up);
        }
        const R a = at * ir * g.h2t;
        c.lo += a;
        c.up -= a;
    } else {
        const R ir = L == FR ? g.ir_f[i + 1] : g.ir_c[i + 1];
        c.lo = nu * g.cphat;
        c.up = nu * g.cphat;
        c.di = R(-2) * nu * g.cphat;
        if (L == FP) {
            const R ir2 = g.ir2_c[i + 1], e = g.is2_c[j + 1];
            const R q3 = g.ic * e * g.idph2 * ir2;
            c.di += -nu * e * ir2 - (ar + at * g.cot_c[j + 1]) * ir - R(2) * q3;
            c.lo += q3;
            c.up += q3;
        }
        const R a = ap * ir * (L == FT ? g.h2p_f[j + 1] : g.h2p_c[j + 1]);
        c.lo += a;
        c.up -= a;
    }
    return c;
}

template <int L, int D, typename R>
__device__ __forceinline__ Tri<R> coef(const Geo<R> &g, int i, int j, R ar, R at, R ap, R nu)
{
    return coef_t<L, D>(g, i, j, ar, at, ap, nu, GTab<L, D, R>{g, D == 0 ? i + 1 : j + 1});
}

// Coefficients of the diffusion-only line solves (DIFF = 1: the paper's
// split operators Dhat_thth, Dhat_phph; DIFF = 2: the true D_thth =
// (R1/r)^2 Dhat_thth and D_phph = 1/(r^2 sin^2(theta) dphi^2)) for the
// centre unknowns; D_rr is common.
template <int D, int DIFF, typename R>
__device__ __forceinline__ Tri<R> true_metric(const Geo<R> &g, int i, int j, Tri<R> c, R nu)
{
    if (DIFF == 2 && D == 1) {
        const R f = g.r12 * g.ir2_c[i + 1];
        c.lo *= f;
        c.up *= f;
        c.di *= f;
    } else if (DIFF == 2 && D == 2) {
        const R q = nu * g.ir2_c[i + 1] * g.is2_c[j + 1] * g.idph2;
        c.lo = q;
        c.up = q;
        c.di = R(-2) * q;
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

// The same averages split into a fetch of the raw face values and their
// combination (same operands, same order: bitwise equal to vel<C, L>), so
// that a line solve can issue the loads of every row of a chunk before any
// arithmetic waits on them.  nvel: raw values of component C at location L.
template <int C, int L> __host__ __device__ constexpr int nvel()
{
    return (C == 0 && L == FR) || (C == 1 && L == FT) || (C == 2 && L == FP) ? 1 : (L == CC ? 2 : 4);
}
template <int C, int L, typename R>
__device__ __forceinline__ void vel_fetch(const R *__restrict__ a, int64_t q, const Dims &d, R *v)
{
    const int64_t sI = d.sI, sJ = d.sJ;
    constexpr int N = nvel<C, L>();
    const int64_t sa = C == 0 ? sI : (C == 1 ? sJ : 1);          // the component's own face step
    // the other step of a 4-point average (face-centred L in another direction)
    const int64_t sb = L == FR ? sI : (L == FT ? sJ : 1);
    if (N == 1) {
        v[0] = a[q];
    } else if (N == 2) {
        v[0] = a[q];
        v[1] = a[q + sa];
    } else {
        v[0] = a[q - sb];
        v[1] = a[q - sb + sa];
        v[2] = a[q];
        v[3] = a[q + sa];
    }
}
template <int C, int L, typename R> __device__ __forceinline__ R vel_combine(const R *v)
{
    constexpr int N = nvel<C, L>();
    if (N == 1) return v[0];
    if (N == 2) return R(0.5) * (v[0] + v[1]);
    return R(0.25) * ((v[0] + v[1]) + (v[2] + v[3]));
}

// Advecting-velocity components the split operator L_{L,D} uses: the one
// along the line, and u_r (u_theta on theta-faces, D = 1; u_phi on
// phi-faces, D = 2) and u_theta (u_phi, D = 2) for the metric terms.
template <int L, int D> struct AdvNeed {
    static constexpr bool r = D == 0 || (D == 1 && L == FT) || (D == 2 && L == FP);
    static constexpr bool t = D == 1 || (D == 2 && L == FP);
    static constexpr bool p = D == 2;
    static constexpr int N = (r ? nvel<0, L>() : 0) + (t ? nvel<1, L>() : 0) + (p ? nvel<2, L>() : 0);
};
template <int L, int D, typename R>
__device__ __forceinline__ void adv_fetch(const State<R> &s, const Dims &d, int64_t q, R *v)
{
    using A = AdvNeed<L, D>;
    int o = 0;
    if (A::r) { vel_fetch<0, L>(s.us[1][0], q, d, v + o); o += nvel<0, L>(); }
    if (A::t) { vel_fetch<1, L>(s.us[1][1], q, d, v + o); o += nvel<1, L>(); }
    if (A::p) { vel_fetch<2, L>(s.us[1][2], q, d, v + o); }
}
template <int L, int D, typename R>
__device__ __forceinline__ void adv_combine(const R *v, R &ar, R &at, R &ap)
{
    using A = AdvNeed<L, D>;
    int o = 0;
    ar = at = ap = R(0);
    if (A::r) { ar = vel_combine<0, L>(v + o); o += nvel<0, L>(); }
    if (A::t) { at = vel_combine<1, L>(v + o); o += nvel<1, L>(); }
    if (A::p) { ap = vel_combine<2, L>(v + o); }
}

template <int L> __host__ __device__ constexpr int ulo(int dir) { return L == dir + 1 ? 1 : 0; }
__host__ __device__ inline int ncell(const Dims &d, int dir) { return dir == 0 ? d.nr : dir == 1 ? d.nt : d.np; }

// ---------------------------------------------------------------------------
// XCD-aware block order.  Workgroups are handed to the 8 XCDs round-robin
// in linear dispatch order, and each XCD has its own L2.  This bijection
// gives XCD x the contiguous logical range [x*n/8, (x+1)*n/8) of the grid,
// so that blocks which share stencil halos (neighbouring theta rows) run on
// the same XCD and meet their neighbours' rows in its L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void xcd_block(unsigned &bx, unsigned &by)
{
    const unsigned gx = gridDim.x, n = gx * gridDim.y;
    const unsigned b = blockIdx.x + blockIdx.y * gx;
    const unsigned x = b & 7u, pos = b >> 3, q = n >> 3, r = n & 7u;
    const unsigned l = (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + pos;
    bx = l % gx;
    by = l / gx;
}

// ---------------------------------------------------------------------------
// Launches.  Every kernel of the step is a body taking its argument struct
// and a virtual block (x, y of a grid nx x ny).  k_single runs one shell: its
// hardware grid is the virtual grid (XCD-remapped where the body asks for
// it).  k_multi runs many shells in one launch: shell q owns the blocks
// [off_q, off_q + padded_q) of a 1-D grid (multiples of 8; XCD-remapped
// within the range where the body asks for it, the padding blocks exit) and
// reads its arguments from a device table.
// ---------------------------------------------------------------------------
struct Blk { unsigned x, y, nx, ny; };

__device__ __forceinline__ unsigned xcd_linear(unsigned b, unsigned n)
{
    const unsigned x = b & 7u, pos = b >> 3, q = n >> 3, r = n & 7u;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + pos;
}

// waves per SIMD a kernel asks to keep (its register budget), 1 if it names none
template <class K, class = void> struct WpeOf { static constexpr int v = 1; };
template <class K> struct WpeOf<K, std::void_t<decltype(K::wpe)>> { static constexpr int v = K::wpe; };

template <class K>
__global__ void __launch_bounds__(K::bounds) __attribute__((amdgpu_waves_per_eu(WpeOf<K>::v)))
k_single(typename K::Args a)
{
    Blk b = {blockIdx.x, blockIdx.y, gridDim.x, gridDim.y};
    if (K::xcd) {
        const unsigned l = xcd_linear(b.x + b.y * b.nx, b.nx * b.ny);
        b.x = l % b.nx;
        b.y = l / b.nx;
    }
    K::body(a, b);
}

template <class K>
__global__ void __launch_bounds__(K::bounds) __attribute__((amdgpu_waves_per_eu(WpeOf<K>::v)))
k_multi(const typename K::Args *__restrict__ list, const BatchEnt *__restrict__ ents, int nq)
{
    const unsigned hb = blockIdx.x;
    int lo = 0, hi = nq - 1;                 // last entry with off <= hb
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((unsigned)ents[mid].off <= hb) lo = mid;
        else hi = mid - 1;
    }
    const BatchEnt e = ents[lo];
    // the shell's range starts on a multiple of 8, so hb - off keeps the
    // XCD residue: the remap spreads the shell evenly over the XCDs
    unsigned loc = hb - (unsigned)e.off;
    if (K::xcd) loc = xcd_linear(loc, (unsigned)e.padded);
    if (loc >= (unsigned)e.nx * (unsigned)e.ny) return;
    const Blk b = {loc % (unsigned)e.nx, loc / (unsigned)e.nx, (unsigned)e.nx, (unsigned)e.ny};
    K::body(list[lo], b);
}

// launch one shell's kernel, or hand it to the launch recorder
template <class K> void launch(dim3 grid, dim3 block, size_t lds, hipStream_t st, const typename K::Args &a)
{
    if (LaunchRecorder *r = launch_recorder()) {
        r->push((const void *)k_multi<K>, grid, block, lds, &a, sizeof a);
        return;
    }
    hipLaunchKernelGGL(k_single<K>, grid, block, lds, st, a);
}

// Column kernels: a block of (COL_K, COL_J) threads owns a COL_K x COL_J tile
// of (k, j) columns, so the theta neighbours j-1, j+1 of most columns are read
// by waves of the same block.  (Holding the waves at one radial level with a
// barrier per level cuts the re-fetched halo rows by a quarter but costs more
// time than it saves, so the waves run free.)
constexpr int COL_K = 64, COL_J = 4;

// tile of block (bx) over the columns j0 <= j < j0 + nj, k0 <= k < np; the
// k-tiles are aligned to the row storage (k = tk COL_K + x); false if the
// thread's column is outside
__device__ __forceinline__ bool col_of(unsigned bx, int nj, int np, int j0, int k0, int &j, int &k)
{
    const int ntk = (np + COL_K - 1) / COL_K;
    const int tk = (int)(bx % (unsigned)ntk), tj = (int)(bx / (unsigned)ntk);
    k = tk * COL_K + (int)threadIdx.x;
    j = j0 + tj * COL_J + (int)threadIdx.y;
    return k >= k0 && k < np && (j - j0) < nj;
}
__host__ __device__ inline int64_t col_blocks(int nj, int np)
{
    return (int64_t)((np + COL_K - 1) / COL_K) * ((nj + COL_J - 1) / COL_J);
}

// the same for a block of (blockDim.x, blockDim.y) columns, tiles taken
// k-fastest or (jfast) j-fastest by consecutive logical blocks
__device__ __forceinline__ bool col_of_t(unsigned bx, int nj, int np, int j0, int k0, int jfast, int &j, int &k)
{
    const int ck = (int)blockDim.x, cj = (int)blockDim.y;
    const unsigned ntk = (unsigned)((np + ck - 1) / ck), ntj = (unsigned)((nj + cj - 1) / cj);
    const int tk = (int)(jfast ? bx / ntj : bx % ntk), tj = (int)(jfast ? bx % ntj : bx / ntk);
    k = tk * ck + (int)threadIdx.x;
    j = j0 + tj * cj + (int)threadIdx.y;
    return k >= k0 && k < np && (j - j0) < nj;
}
inline int64_t col_blocks_t(int nj, int np, const ResTile &t)
{
    return (int64_t)((np + t.ck - 1) / t.ck) * ((nj + t.cj - 1) / t.cj);
}

// ---------------------------------------------------------------------------
// block reduction of a double (blockDim.x * blockDim.y a multiple of 64,
// <= 1024, blockDim.x a multiple of 64 or blockDim.y == 1); the sum is
// returned on the block's first thread
// ---------------------------------------------------------------------------
__device__ double block_sum(double v)
{
    __shared__ double red[16];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int f = threadIdx.x + blockDim.x * threadIdx.y;
    const int w = f >> 6, l = f & 63;
    if (l == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    if (f == 0) {
        const int nw = (blockDim.x * blockDim.y) >> 6;
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

// start of a step: the extrapolated levels and the working iterate k = n in
// one pass over level n (T, u1, u2; p1 and p2 copied)
template <typename R> struct PtrStep {
    R *s[7], *k[7];
    const R *n[7], *m[7];
    const double *p0, *p1;
    double *p0k, *p1k;
};

template <typename R>
struct ExtrapCopyArgs { PtrStep<R> p; int64_t n; };
template <typename R> struct KExtrapCopy {
    using Args = ExtrapCopyArgs<R>;
    static constexpr int bounds = 256;
    static constexpr bool xcd = false;
    static __device__ __forceinline__ void body(const Args &a, const Blk &blk)
    {
        const PtrStep<R> &pa = a.p;
        const int64_t n = a.n;

    // one 16-byte word of every compute-precision array per thread (VN
    // elements; the FP64 pressures as VN doubles), all loads issued before
    // the stores; n is a multiple of VN (rows are 128-byte aligned)
    constexpr int VN = 16 / (int)sizeof(R);
    const int64_t q = (blk.x * (int64_t)blockDim.x + threadIdx.x) * VN;
    if (q >= n) return;
    R vn[7][VN], vm[7][VN];
    double pp[2][VN];
#pragma unroll
    for (int f = 0; f < 7; f++) {
        *(uint4 *)vn[f] = *(const uint4 *)(pa.n[f] + q);
        *(uint4 *)vm[f] = *(const uint4 *)(pa.m[f] + q);
    }
#pragma unroll
    for (int h = 0; h < VN; h += 2) {
        *(double2 *)&pp[0][h] = *(const double2 *)(pa.p0 + q + h);
        *(double2 *)&pp[1][h] = *(const double2 *)(pa.p1 + q + h);
    }
    asm volatile("" ::: "memory");
#pragma unroll
    for (int f = 0; f < 7; f++) {
        R vs[VN];
#pragma unroll
        for (int e = 0; e < VN; e++) vs[e] = R(1.5) * vn[f][e] - R(0.5) * vm[f][e];
        *(uint4 *)(pa.s[f] + q) = *(const uint4 *)vs;
        *(uint4 *)(pa.k[f] + q) = *(const uint4 *)vn[f];
    }
#pragma unroll
    for (int h = 0; h < VN; h += 2) {
        *(double2 *)(pa.p0k + q + h) = *(const double2 *)&pp[0][h];
        *(double2 *)(pa.p1k + q + h) = *(const double2 *)&pp[1][h];
    }
    }
};

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
    if (LaunchRecorder *r = launch_recorder()) {
        r->foreign = true;
        return;
    }
    hipLaunchKernelGGL(k_extrap<R>, dim3(grid_for(n)), dim3(256), 0, st, a, n);
}

template <typename R> void Ops<R>::extrap_copy(const Dims &d, const State<R> &s, hipStream_t st)
{
    PtrStep<R> a;
    a.s[0] = s.Ts; a.k[0] = s.T[2]; a.n[0] = s.T[0]; a.m[0] = s.T[1];
    int f = 1;
    for (int y = 0; y < 2; y++)
        for (int c = 0; c < 3; c++, f++) {
            a.s[f] = s.us[y][c];
            a.k[f] = s.u[y][c][2];
            a.n[f] = s.u[y][c][0];
            a.m[f] = s.u[y][c][1];
        }
    a.p0 = s.p[0][0]; a.p0k = s.p[0][1];
    a.p1 = s.p[1][0]; a.p1k = s.p[1][1];
    const int64_t n = 2 * d.sP;
    const int64_t words = n / (16 / (int64_t)sizeof(R));
    launch<KExtrapCopy<R>>(dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st, ExtrapCopyArgs<R>{a, n});
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
struct FillScalarArgs { Dims d; const FillScalar *tab; int ntab; TT *a; int ilo, ni, pmask; };
template <typename TT> struct KFillScalar {
    using Args = FillScalarArgs<TT>;
    static constexpr int bounds = 256;
    static constexpr bool xcd = false;
    static __device__ __forceinline__ void body(const Args &a, const Blk &blk)
    {
        const Dims &d = a.d;
        const FillScalar *__restrict__ tab = a.tab;
        const int ntab = a.ntab, ilo = a.ilo, ni = a.ni, pmask = a.pmask;
        TT *fa = a.a;

    const int p = blk.y;
    if (!((pmask >> p) & 1)) return;
    const int t = blk.x * blockDim.x + threadIdx.x;
    if (t >= ntab * ni) return;
    const int e = t % ntab;
    const int i = ilo + t / ntab;
    const FillScalar &f = tab[e];
    const double v = gather16(fa, ix(d, 1 - p, i, f.dj, f.dk), d.sJ, f.wt, f.wp);
    fa[ix(d, p, i, f.tj, f.tk)] = (TT)v;
    }
};

// Tangential velocity targets: interpolate the other patch's u_theta (on
// its theta-face grid) and u_phi (on its phi-face grid) to the target and
// rotate into this patch's basis.
template <typename R>
struct FillVectorArgs { Dims d; const FillVector *tab; int ntab; const R *ut, *up; R *dst; int ni, pmask; };
template <typename R> struct KFillVector {
    using Args = FillVectorArgs<R>;
    static constexpr int bounds = 256;
    static constexpr bool xcd = false;
    static __device__ __forceinline__ void body(const Args &a, const Blk &blk)
    {
        const Dims &d = a.d;
        const FillVector *__restrict__ tab = a.tab;
        const int ntab = a.ntab, ni = a.ni, pmask = a.pmask;
        const R *ut = a.ut, *up = a.up;
        R *dst = a.dst;

    const int p = blk.y;
    if (!((pmask >> p) & 1)) return;
    const int t = blk.x * blockDim.x + threadIdx.x;
    if (t >= ntab * ni) return;
    const int e = t % ntab;
    const int i = t / ntab;
    const FillVector &f = tab[e];
    const double vt = gather16(ut, ix(d, 1 - p, i, f.tjA, f.tkA), d.sJ, f.wtA, f.wpA);
    const double vp = gather16(up, ix(d, 1 - p, i, f.tjB, f.tkB), d.sJ, f.wtB, f.wpB);
    dst[ix(d, p, i, f.tj, f.tk)] = (R)(f.ma * vt + f.mb * vp);
    }
};

// Walls r = R1, R2 (eq. eq_ns, eq_heat_convec): u_r = 0 on the wall faces;
// reflection ghosts psi_{-1} = 2 psi_wall - psi_0 for T and the tangential
// velocities, psi_wall from the level's wall data where given (else the
// constant wall temperature, zero velocity); u_r takes the wall value on
// its wall faces.  Both velocity systems take the same data.  Thread =
// padded (j, k) point of patch blockIdx.y.
template <typename R>
struct WallsArgs { Dims d; State<R> s; int lev; double t_in, t_out; TRobin tb; URobin ub; WallLev w; int pmask; };
template <typename R> struct KWalls {
    using Args = WallsArgs<R>;
    static constexpr int bounds = 256;
    static constexpr bool xcd = false;
    static __device__ __forceinline__ void body(const Args &a, const Blk &blk)
    {
        const Dims &d = a.d;
        const State<R> &s = a.s;
        const int lev = a.lev, pmask = a.pmask;
        const double t_in = a.t_in, t_out = a.t_out;
        const TRobin &tb = a.tb;
        const URobin &ub = a.ub;
        const WallLev &w = a.w;

    const int p = blk.y;
    if (!((pmask >> p) & 1)) return;
    const int t = blk.x * blockDim.x + threadIdx.x;
    const int nk = d.np + 2, nj = d.nt + 2;
    if (t >= nk * nj) return;
    const int j = t / nk - 1, k = t % nk - 1;
    const int64_t q0 = ix(d, p, 0, j, k), qm = q0 - d.sI;
    const int64_t q1 = ix(d, p, d.nr - 1, j, k), qp = q1 + d.sI;
    const int64_t wq = ((int64_t)p * nj + (j + 1)) * nk + (k + 1);
    auto wv = [&](int c, int side, R dflt) { return w.v[c][side] ? (R)w.v[c][side][wq] : dflt; };
    R *T = s.T[lev];
    // the wall value and the reference profile's part in FP64, rounded once
    const double g0 = w.v[0][0] ? w.v[0][0][wq] : t_in, g1 = w.v[0][1] ? w.v[0][1][wq] : t_out;
    T[qm] = (R)(tb.cg[0] * g0 - tb.shift[0]) - (R)tb.rho[0] * T[q0];
    T[qp] = (R)(tb.cg[1] * g1 - tb.shift[1]) - (R)tb.rho[1] * T[q1];
    // tangential velocity: cg g - rho u_in (Robin; Dirichlet cg = 2, rho = 1)
    auto wd = [&](int c, int side) { return w.v[c][side] ? w.v[c][side][wq] : 0.0; };
    const R a0 = (R)(ub.cg[0] * wd(2, 0)), a1 = (R)(ub.cg[1] * wd(2, 1));
    const R b0 = (R)(ub.cg[0] * wd(3, 0)), b1 = (R)(ub.cg[1] * wd(3, 1));
    const R r0 = (R)ub.rho[0], r1 = (R)ub.rho[1];
    const R c0 = wv(1, 0, R(0)), c1 = wv(1, 1, R(0));
    for (int y = 0; y < 2; y++) {
        R *a = s.u[y][1][lev], *b = s.u[y][2][lev], *c = s.u[y][0][lev];
        a[qm] = a0 - r0 * a[q0];
        a[qp] = a1 - r1 * a[q1];
        b[qm] = b0 - r0 * b[q0];
        b[qp] = b1 - r1 * b[q1];
        c[q0] = c0;
        c[ix(d, p, d.nr, j, k)] = c1;
    }
    }
};

template <typename R>
void Ops<R>::fill(const Dims &d, const State<R> &s, int lev, const FillScalar *cc, int ncc,
                  const FillVector *vt, int nvt, const FillVector *vp, int nvp, double t_in,
                  double t_out, const TRobin &tb, const URobin &ub, const WallLev &walls, int pmask,
                  hipStream_t st)
{
    const int pl = lev == 0 ? 0 : 1;     // pressure keeps levels n and k
    // centre-type scalars: T, p1, p2 (radial 0..nr-1); u_r (faces 1..nr-1)
    int n = ncc * d.nr;
    dim3 g((n + 255) / 256, 2);
    launch<KFillScalar<R>>(g, dim3(256), 0, st, FillScalarArgs<R>{d, cc, ncc, s.T[lev], 0, d.nr, pmask});
    launch<KFillScalar<double>>(g, dim3(256), 0, st, FillScalarArgs<double>{d, cc, ncc, s.p[0][pl], 0, d.nr, pmask});
    launch<KFillScalar<double>>(g, dim3(256), 0, st, FillScalarArgs<double>{d, cc, ncc, s.p[1][pl], 0, d.nr, pmask});
    n = ncc * (d.nr - 1);
    dim3 g1((n + 255) / 256, 2);
    for (int y = 0; y < 2; y++)
        launch<KFillScalar<R>>(g1, dim3(256), 0, st, FillScalarArgs<R>{d, cc, ncc, s.u[y][0][lev], 1, d.nr - 1, pmask});
    for (int y = 0; y < 2; y++) {
        R *ut = s.u[y][1][lev], *up = s.u[y][2][lev];
        n = nvt * d.nr;
        launch<KFillVector<R>>(dim3((n + 255) / 256, 2), dim3(256), 0, st,
                               FillVectorArgs<R>{d, vt, nvt, ut, up, ut, d.nr, pmask});
        n = nvp * d.nr;
        launch<KFillVector<R>>(dim3((n + 255) / 256, 2), dim3(256), 0, st,
                               FillVectorArgs<R>{d, vp, nvp, ut, up, up, d.nr, pmask});
    }
    n = (d.np + 2) * (d.nt + 2);
    launch<KWalls<R>>(dim3((n + 255) / 256, 2), dim3(256), 0, st,
                      WallsArgs<R>{d, s, lev, t_in, t_out, tb, ub, walls, pmask});
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
// with storage index q (centre (i, j, k)), from the metric tables
template <typename R>
__device__ __forceinline__ R div_r(const Geo<R> &g, const R *a, int64_t q, int64_t sI, int i)
{
    return g.dr_p[i + 1] * a[q + sI] - g.dr_m[i + 1] * a[q];
}
template <typename R>
__device__ __forceinline__ R div_t(const Geo<R> &g, const R *a, int64_t q, int64_t sJ, int i, int j)
{
    return g.ir_c[i + 1] * (g.dt_p[j + 1] * a[q + sJ] - g.dt_m[j + 1] * a[q]);
}
template <typename R>
__device__ __forceinline__ R div_p(const Geo<R> &g, const R *a, int64_t q, int i, int j)
{
    return g.ir_c[i + 1] * g.dp_c[j + 1] * (a[q + 1] - a[q]);
}

template <typename R>
__device__ __forceinline__ double ptilde(const RhsIn<R> &in, int64_t q)
{
    if (in.sys == 1) return in.psn[q];
    return in.psn[q] + 0.5 * (in.p1k[q] - in.p1n[q]);
}

// Residual, column-marching form: a thread owns one (patch, j, k) column
// and walks i upwards, keeping every value it needs at i-1 / i / i+1 of the
// same (j, k) offset in registers (sliding windows), so each r-neighbour is
// fetched once.  The arithmetic is the point form above, term by term; it
// is written once (res_point) and fed by two kernels that differ only in
// where the theta and phi neighbours come from: memory (KResidual) or
// planes staged in LDS (KResidualLds).
template <typename R> struct Col {
    // psibar = (psi^n + psi^{k-1})/2 at i-1, i, i+1
    R bm, b0, bp;
    // averaged-velocity windows: value at offset (dj,dk) and radial i+e
    R a0, a1, c0, c1, e0, e1, f0, f1, g0, g1, h0, h1;
    double p0, pm;   // p~ at i and i-1 (FR)
    double tg;       // T^n + T^k at i-1 (FR), in FP64
};

// The values one point update at (i, j, k) reads besides its windows.
// Common: psibar at i+1 (own) and at the theta/phi neighbours at i; psi* at
// the point and its four neighbours; forcing; psi^k - psi^n at the point.
// Location-specific (names as in res_point):
//   CC  wr1 = w_r at face i+1; t0, t1 = w_t at j, j+1; p0, p1 = w_p at k, k+1
//   FR  wr0 = w_r; t0, t1, p0, p1 as CC; e0, e1 = u*_t at j, j+1;
//       f0, f1 = u*_p at k, k+1; Tn, Tk; pt = p~
//   FT  r0, r1 = w_r at (i+1, j-1), (i+1, j); t0 = w_t; p0..p3 = w_p at
//       (j-1,k), (j-1,k+1), (j,k), (j,k+1); u0, u1 = 2 ubar_r at (i+1, j-1),
//       (i+1, j); s0..s3 = u*_p at (j,k+1), (j,k), (j-1,k+1), (j-1,k);
//       pt, pm = p~ at j, j-1
//   FP  r0, r1 = w_r at (i+1, k-1), (i+1, k); p0 = w_p; t0..t3 = w_t at
//       (j,k-1), (j+1,k-1), (j,k), (j+1,k); u0, u1 = 2 ubar_r at (i+1, k-1),
//       (i+1, k); h0..h3 = u^n_t + u^k_t at (j,k), (j+1,k), (j,k-1),
//       (j+1,k-1); pt, pm = p~ at k, k-1
template <typename R> struct ResNb {
    R bp, bjm, bjp, bkm, bkp;
    R x0, xjm, xjp, xkm, xkp;
    R f, dk;
    R wr0, wr1, r0, r1, u0, u1;
    R t0, t1, t2, t3, p0, p1, p2, p3;
    R e0, e1, f0, f1, s0, s1, s2, s3, h0, h1, h2, h3;
    R Tn, Tk;
    double pt, pm;
};

// one point update; returns tau R^k and advances the radial windows
template <typename R, int L>
__device__ __forceinline__ R res_point(const Geo<R> &g, int i, int j, const ResNb<R> &n, Col<R> &w)
{
    const R nu = L == CC ? R(1) : g.pr;
    w.bp = n.bp;
    R ar, at, ap, S = n.f;
    if (L == CC) {
        const R wr1 = n.wr1;
        ar = R(0.5) * (w.a0 + wr1);
        at = R(0.5) * (n.t0 + n.t1);
        ap = R(0.5) * (n.p0 + n.p1);
        w.a0 = wr1;
    } else if (L == FR) {
        const R t0 = n.t0, t1 = n.t1, p0 = n.p0, p1 = n.p1;
        ar = n.wr0;
        at = R(0.25) * ((w.a0 + w.a1) + (t0 + t1));
        ap = R(0.25) * ((w.c0 + w.c1) + (p0 + p1));
        const R e0 = n.e0, e1 = n.e1, f0 = n.f0, f1 = n.f1;
        // (D12 u_t* + D13 u_p*)/(2 chi)
        const R dtc = g.ir_c[i + 1] * (g.dt_p[j + 1] * e1 - g.dt_m[j + 1] * e0);
        const R dtm = g.ir_c[i] * (g.dt_p[j + 1] * w.e1 - g.dt_m[j + 1] * w.e0);
        const R dpc = g.ir_c[i + 1] * g.dp_c[j + 1] * (f1 - f0);
        const R dpm = g.ir_c[i] * g.dp_c[j + 1] * (w.f1 - w.f0);
        S += g.ic * g.idr * ((dtc - dtm) + (dpc - dpm));
        const R vt = R(0.25) * ((w.e0 + w.e1) + (e0 + e1));
        const R vp = R(0.25) * ((w.f0 + w.f1) + (f0 + f1));
        S += (at * vt + ap * vp) * g.ir_f[i + 1];
        // -d_r p~ + Pr Ra T^{n+1/2}: the hydrostatic balance cancels
        // two large terms, so they are combined in FP64 before rounding
        const double pt = n.pt;
        const double tg = (double)n.Tn + (double)n.Tk + 2.0 * g.tref[i + 1];
        S += (R)(g.prra_d * 0.25 * (w.tg + tg) - (pt - w.pm) * (double)g.idr);
        w.a0 = t0; w.a1 = t1; w.c0 = p0; w.c1 = p1;
        w.e0 = e0; w.e1 = e1; w.f0 = f0; w.f1 = f1;
        w.tg = tg; w.pm = pt;
    } else if (L == FT) {
        const R r0 = n.r0, r1 = n.r1;
        ar = R(0.25) * ((w.a0 + r0) + (w.a1 + r1));
        at = n.t0;
        ap = R(0.25) * ((n.p0 + n.p1) + (n.p2 + n.p3));
        const R ir = g.ir_c[i + 1], ir2 = g.ir2_c[i + 1], cot = g.cot_f[j + 1];
        const R u0 = n.u0;                        // 2 ubar_r at (i+1, j-1)
        const R u1 = n.u1;                        // 2 ubar_r at (i+1, j)
        // Div_r of ubar at centres (i, j) and (i, j-1), times 2
        const R dj0 = g.dr_p[i + 1] * u1 - g.dr_m[i + 1] * w.c1;
        const R dj1 = g.dr_p[i + 1] * u0 - g.dr_m[i + 1] * w.c0;
        const R d23 = g.ir_c[i + 1] * (g.dp_c[j + 1] * (n.s0 - n.s1) -
                                       g.dp_c[j] * (n.s2 - n.s3));
        S += g.ic * ir * g.idth * (R(0.5) * (dj0 - dj1) + d23);
        const R dth_ur = R(0.5) * ((R(0.5) * w.c1 - R(0.5) * w.c0) + (R(0.5) * u1 - R(0.5) * u0)) * g.idth;
        const R fp2 = g.rf[i + 2] * g.rf[i + 2], fm2 = g.rf[i + 1] * g.rf[i + 1];
        const R dr_r2ur = R(0.5) * ((fp2 * R(0.5) * u0 - fm2 * R(0.5) * w.c0) +
                                    (fp2 * R(0.5) * u1 - fm2 * R(0.5) * w.c1)) * g.idr;
        S += g.pr * R(2) * ir2 * (dth_ur + cot * ir * dr_r2ur);
        const R vp = R(0.25) * ((n.s3 + n.s2) + (n.s1 + n.s0));
        S += ap * vp * cot * ir;
        S -= (R)((n.pt - n.pm) * (double)ir * (double)g.idth);
        w.a0 = r0; w.a1 = r1; w.c0 = u0; w.c1 = u1;
    } else {
        const R r0 = n.r0, r1 = n.r1;
        ar = R(0.25) * ((w.a0 + r0) + (w.a1 + r1));
        at = R(0.25) * ((n.t0 + n.t1) + (n.t2 + n.t3));
        ap = n.p0;
        const R ir = g.ir_c[i + 1], ir2 = g.ir2_c[i + 1], isn = g.is_c[j + 1], cot = g.cot_c[j + 1];
        const R igg = ir * g.dp_c[j + 1];
        const R u0 = n.u0;                        // 2 ubar_r at (i+1, k-1)
        const R u1 = n.u1;                        // 2 ubar_r at (i+1, k)
        const R a0 = g.dr_p[i + 1] * u1 - g.dr_m[i + 1] * w.c1;
        const R a1 = g.dr_p[i + 1] * u0 - g.dr_m[i + 1] * w.c0;
        const R th00 = n.h0, th01 = n.h1, thm0 = n.h2, thm1 = n.h3;
        const R b0 = ir * (g.dt_p[j + 1] * th01 - g.dt_m[j + 1] * th00);
        const R b1 = ir * (g.dt_p[j + 1] * thm1 - g.dt_m[j + 1] * thm0);
        S += g.ic * igg * R(0.5) * ((a0 - a1) + (b0 - b1));
        const R dph_ur = R(0.5) * ((R(0.5) * w.c1 - R(0.5) * w.c0) + (R(0.5) * u1 - R(0.5) * u0)) * g.idph;
        const R dph_ut = R(0.5) * ((R(0.5) * th00 - R(0.5) * thm0) + (R(0.5) * th01 - R(0.5) * thm1)) * g.idph;
        S += g.pr * R(2) * ir2 * isn * (dph_ur + cot * dph_ut);
        S -= (R)((n.pt - n.pm) * (double)igg);
        w.a0 = r0; w.a1 = r1; w.c0 = u0; w.c1 = u1;
    }
    const Tri<R> c0 = coef<L, 0>(g, i, j, ar, at, ap, nu);
    const Tri<R> c1 = coef<L, 1>(g, i, j, ar, at, ap, nu);
    const Tri<R> c2 = coef<L, 2>(g, i, j, ar, at, ap, nu);
    R Rv = c0.lo * w.bm + c0.di * w.b0 + c0.up * w.bp;
    Rv += c1.lo * n.bjm + c1.di * w.b0 + c1.up * n.bjp;
    Rv += c2.lo * n.bkm + c2.di * w.b0 + c2.up * n.bkp;
    const R ir2 = L == FR ? g.ir2_f[i + 1] : g.ir2_c[i + 1];
    const R hlo = L == FT ? g.tf_lo[j + 1] : g.tc_lo[j + 1];
    const R hup = L == FT ? g.tf_up[j + 1] : g.tc_up[j + 1];
    const R is2 = L == FT ? g.is2_f[j + 1] : g.is2_c[j + 1];
    const R x0 = n.x0;
    const R lt = hup * (n.xjp - x0) - hlo * (x0 - n.xjm);
    const R lp = n.xkp - R(2) * x0 + n.xkm;
    Rv += nu * ((g.r12 * ir2 - R(1)) * lt + (ir2 * is2 * g.idph2 - g.cphat) * lp);
    Rv += S;
    // T's deviation storage: the advection of the reference profile
    // (its diffusion vanishes: Tref is the discrete conductive state)
    if (L == CC && g.tdev) Rv -= ar * g.dtref[i + 1];
    Rv -= n.dk * g.inv_tau;
    w.bm = w.b0;
    w.b0 = w.bp;
    return g.tau * Rv;
}

// nseg: each column's radial points are split into nseg segments of
// ceil((nr - i0) / nseg) points, one block per (segment, column tile), so
// that the block count fills the last round of resident blocks; ntile:
// column tiles per patch.  Virtual block x = segment * ntile + tile.
template <typename R>
struct ResArgs { Dims d; Geo<R> g; State<R> s; RhsIn<R> in; R *out; int jfast, nseg, ntile; };

// radial range [is, ie) of segment seg of a column starting at i0
__device__ __forceinline__ void res_segment(int i0, int nr, int nseg, int seg, int &is, int &ie)
{
    const int len = (nr - i0 + nseg - 1) / nseg;
    is = i0 + seg * len;
    ie = min(nr, is + len);
}

// the arrays a residual reads, as 32-bit-indexed views
template <typename R> struct ResSrc {
    FV<R> pn, pk, ps, fin, wr, wt, wp, un0, uk0, un1, uk1, us1, us2, Tn, Tk;
    FV<double> psn, p1n, p1k;
    int sys;
    __device__ __forceinline__ explicit ResSrc(const ResArgs<R> &a)
        : pn(a.in.pn), pk(a.in.pk), ps(a.in.ps), fin(a.in.f), wr(a.s.us[1][0]), wt(a.s.us[1][1]),
          wp(a.s.us[1][2]), un0(a.in.un[0]), uk0(a.in.uk[0]), un1(a.in.un[1]), uk1(a.in.uk[1]),
          us1(a.in.us[1]), us2(a.in.us[2]), Tn(a.in.Tn), Tk(a.in.Tk), psn(a.in.psn), p1n(a.in.p1n),
          p1k(a.in.p1k), sys(a.in.sys)
    {
    }
    __device__ __forceinline__ R bar(uint32_t q) const { return R(0.5) * (pn[q] + pk[q]); }
    __device__ __forceinline__ double ptl(uint32_t q) const
    {
        return sys == 1 ? psn[q] : psn[q] + 0.5 * (p1k[q] - p1n[q]);
    }
    // the radial windows at the column's first point (q = point i0)
    template <int L> __device__ __forceinline__ void prime(const Geo<R> &g, int i0, uint32_t q, uint32_t sI,
                                                           uint32_t sJ, Col<R> &w) const
    {
        w.bm = bar(q - sI);
        w.b0 = bar(q);
        // windows whose lower radial point is i-1 (FR) are primed with i-1
        if (L == FR) {
            w.a0 = wt[q - sI]; w.a1 = wt[q - sI + sJ];       // w_t at (i-1, j), (i-1, j+1)
            w.c0 = wp[q - sI]; w.c1 = wp[q - sI + 1];        // w_p at (i-1, k), (i-1, k+1)
            w.e0 = us1[q - sI]; w.e1 = us1[q - sI + sJ];
            w.f0 = us2[q - sI]; w.f1 = us2[q - sI + 1];
            w.tg = (double)Tn[q - sI] + (double)Tk[q - sI] + 2.0 * g.tref[i0];
            w.pm = ptl(q - sI);
        } else if (L == CC) {
            w.a0 = wr[q];                                    // w_r at face i
        } else if (L == FT) {
            w.a0 = wr[q - sJ]; w.a1 = wr[q];                 // w_r at face i, (j-1) and j
            w.c0 = un0[q - sJ] + uk0[q - sJ];      // 2 ubar_r at face i, j-1
            w.c1 = un0[q] + uk0[q];                // 2 ubar_r at face i, j
        } else {
            w.a0 = wr[q - 1]; w.a1 = wr[q];                  // w_r at face i, (k-1) and k
            w.c0 = un0[q - 1] + uk0[q - 1];
            w.c1 = un0[q] + uk0[q];
        }
    }
    // the values of the point only this column reads
    template <int L> __device__ __forceinline__ void own(uint32_t q, uint32_t sI, ResNb<R> &n) const
    {
        n.bp = bar(q + sI);
        n.f = fin.p ? fin[q] : R(0);
        n.dk = pk[q] - pn[q];
        if (L == CC) n.wr1 = wr[q + sI];
        if (L == FR) {
            n.wr0 = wr[q];
            n.Tn = Tn[q];
            n.Tk = Tk[q];
            n.pt = ptl(q);
        }
        if (L == FT) n.t0 = wt[q];
        if (L == FP) n.p0 = wp[q];
    }
    // the neighbour values, from memory
    template <int L> __device__ __forceinline__ void nbrs(uint32_t q, uint32_t sI, uint32_t sJ, ResNb<R> &n) const
    {
        n.bjm = bar(q - sJ); n.bjp = bar(q + sJ); n.bkm = bar(q - 1); n.bkp = bar(q + 1);
        n.x0 = ps[q]; n.xjm = ps[q - sJ]; n.xjp = ps[q + sJ]; n.xkm = ps[q - 1]; n.xkp = ps[q + 1];
        if (L == CC) {
            n.t0 = wt[q]; n.t1 = wt[q + sJ];
            n.p0 = wp[q]; n.p1 = wp[q + 1];
        } else if (L == FR) {
            n.t0 = wt[q]; n.t1 = wt[q + sJ]; n.p0 = wp[q]; n.p1 = wp[q + 1];
            n.e0 = us1[q]; n.e1 = us1[q + sJ]; n.f0 = us2[q]; n.f1 = us2[q + 1];
        } else if (L == FT) {
            n.r0 = wr[q - sJ + sI]; n.r1 = wr[q + sI];
            n.p0 = wp[q - sJ]; n.p1 = wp[q - sJ + 1]; n.p2 = wp[q]; n.p3 = wp[q + 1];
            n.u0 = un0[q - sJ + sI] + uk0[q - sJ + sI];
            n.u1 = un0[q + sI] + uk0[q + sI];
            n.s0 = us2[q + 1]; n.s1 = us2[q]; n.s2 = us2[q - sJ + 1]; n.s3 = us2[q - sJ];
            n.pt = ptl(q); n.pm = ptl(q - sJ);
        } else {
            n.r0 = wr[q - 1 + sI]; n.r1 = wr[q + sI];
            n.t0 = wt[q - 1]; n.t1 = wt[q - 1 + sJ]; n.t2 = wt[q]; n.t3 = wt[q + sJ];
            n.u0 = un0[q - 1 + sI] + uk0[q - 1 + sI];
            n.u1 = un0[q + sI] + uk0[q + sI];
            n.h0 = un1[q] + uk1[q]; n.h1 = un1[q + sJ] + uk1[q + sJ];
            n.h2 = un1[q - 1] + uk1[q - 1]; n.h3 = un1[q - 1 + sJ] + uk1[q - 1 + sJ];
            n.pt = ptl(q); n.pm = ptl(q - 1);
        }
    }
};

template <typename R, int L> struct KResidual {
    using Args = ResArgs<R>;
    static constexpr int bounds = 256;
    static constexpr bool xcd = true;
    static __device__ __forceinline__ void body(const Args &a, const Blk &blk)
    {
        const Dims &d = a.d;
        const Geo<R> &g = a.g;
        const int p = d.p0 + (int)blk.y;
        const int j0 = ulo<L>(1), k0 = ulo<L>(2), i0 = ulo<L>(0);
        const int nj = d.nt - j0;
        int j, k, is, ie;
        const unsigned seg = blk.x / (unsigned)a.ntile;
        res_segment(i0, d.nr, a.nseg, (int)seg, is, ie);
        if (is >= ie) return;
        if (!col_of_t(blk.x - seg * (unsigned)a.ntile, nj, d.np, j0, k0, a.jfast, j, k)) return;
        // 32-bit element indices (each field is below 4 GiB: checked on the host)
        const uint32_t sI = (uint32_t)d.sI, sJ = (uint32_t)d.sJ;
        const ResSrc<R> src(a);
        uint32_t q = (uint32_t)ix(d, p, is, j, k);
        Col<R> w;
        src.template prime<L>(g, is, q, sI, sJ, w);
        for (int i = is; i < ie; i++, q += sI) {
            ResNb<R> n;
            src.template own<L>(q, sI, n);
            src.template nbrs<L>(q, sI, sJ, n);
            st(a.out, q, res_point<R, L>(g, i, j, n, w));
        }
    }
};

// Residual with the theta and phi neighbours staged in LDS.  A block of
// 64 x CJ threads owns a 64 (k) x CJ (j) tile of columns and walks i with
// them.  At each radial point every quantity read at a neighbour (psibar,
// psi* and the location's velocity and pressure terms) is written into an
// LDS plane covering the tile and the halo cells read from outside it; each
// thread writes its own cell, and the halo cells are dealt one per thread.
// The plane values of the next point are loaded while the current point is
// computed.  So a value is fetched from memory once per tile rather than
// once per column that reads it.  Two barriers per point: before the planes
// are overwritten and before they are read.
enum : int { QBAR, QPS, QWR, QWT, QWP, QUS1, QUS2, QUBR, QTH };
// quantity, radial offset (0: at the point, 1: at i+1), halo sides held
// (jm/jp: the rows j0-1 / j0+CJ over k0-1 .. k0+64; km/kp: the columns
// k0-1 / k0+64 over the tile's rows)
struct PlaneSpec { int q, off, jm, jp, km, kp; };
template <int L> __host__ __device__ constexpr int res_nplanes() { return L == CC ? 4 : 6; }
template <int L> __host__ __device__ constexpr PlaneSpec res_plane(int p)
{
    if (p == 0) return PlaneSpec{QBAR, 0, 1, 1, 1, 1};
    if (p == 1) return PlaneSpec{QPS, 0, 1, 1, 1, 1};
    if (L == CC) return p == 2 ? PlaneSpec{QWT, 0, 0, 1, 0, 0} : PlaneSpec{QWP, 0, 0, 0, 0, 1};
    if (L == FR)
        return p == 2 ? PlaneSpec{QWT, 0, 0, 1, 0, 0} : p == 3 ? PlaneSpec{QWP, 0, 0, 0, 0, 1}
             : p == 4 ? PlaneSpec{QUS1, 0, 0, 1, 0, 0} : PlaneSpec{QUS2, 0, 0, 0, 0, 1};
    if (L == FT)
        return p == 2 ? PlaneSpec{QWR, 1, 1, 0, 0, 0} : p == 3 ? PlaneSpec{QWP, 0, 1, 0, 0, 1}
             : p == 4 ? PlaneSpec{QUBR, 1, 1, 0, 0, 0} : PlaneSpec{QUS2, 0, 1, 0, 0, 1};
    return p == 2 ? PlaneSpec{QWR, 1, 0, 0, 1, 0} : p == 3 ? PlaneSpec{QWT, 0, 0, 1, 1, 0}
         : p == 4 ? PlaneSpec{QUBR, 1, 0, 0, 1, 0} : PlaneSpec{QTH, 0, 0, 1, 1, 0};
}
// the FP64 p~ plane (FT: its row j0-1; FP: its column k0-1)
template <int L> __host__ __device__ constexpr PlaneSpec res_pplane()
{
    return L == FT ? PlaneSpec{0, 0, 1, 0, 0, 0} : PlaneSpec{0, 0, 0, 0, 1, 0};
}

template <typename R>
__device__ __forceinline__ R plane_val(const ResSrc<R> &s, int qid, uint32_t q)
{
    switch (qid) {
    case QBAR: return s.bar(q);
    case QPS: return s.ps[q];
    case QWR: return s.wr[q];
    case QWT: return s.wt[q];
    case QWP: return s.wp[q];
    case QUS1: return s.us1[q];
    case QUS2: return s.us2[q];
    case QUBR: return s.un0[q] + s.uk0[q];
    default: return s.un1[q] + s.uk1[q];
    }
}

// halo cell h of a plane (rows first, then columns); false if h is past
// the plane's halo
template <int CJ>
__device__ __forceinline__ bool halo_cell(const PlaneSpec &s, int h, int &jj, int &kk)
{
    if (s.jm) { if (h < 66) { jj = -1; kk = h - 1; return true; } h -= 66; }
    if (s.jp) { if (h < 66) { jj = CJ; kk = h - 1; return true; } h -= 66; }
    if (s.km) { if (h < CJ) { jj = h; kk = -1; return true; } h -= CJ; }
    if (s.kp) { if (h < CJ) { jj = h; kk = 64; return true; } }
    return false;
}

template <typename R, int L, int CJ> struct KResidualLds {
    using Args = ResArgs<R>;
    static constexpr int bounds = 64 * CJ;
    // register budget: 4 waves per SIMD (128 VGPRs) where that holds the
    // prefetched planes without spilling, else 3 (the FP64 velocities)
    static constexpr int wpe = (L == CC || sizeof(R) == 4) ? 4 : 3;
    static constexpr bool xcd = true;
    static constexpr int W = 66, PL = (CJ + 2) * W, NT = 64 * CJ;
    // every halo cell of a group has its own thread (at most two rows of
    // 66 and two columns of CJ)
    static_assert(2 * W + 2 * CJ <= NT, "LDS residual tiles need at least 4 rows");
    static constexpr int NPL = res_nplanes<L>();
    static constexpr bool HASP = L == FT || L == FP;
    // halo groups: psibar and psi* (all four sides); CC/FR: j+1 and k+1
    // planes; FT/FP: the one-sided planes with p~, and the two-sided ones
    // (plane NPL: p~)
    static constexpr int NG = 3;
    static __host__ __device__ constexpr int grp(int c) { return c < 2 ? 0 : (c == NPL || c % 2 == 0) ? 1 : 2; }
    static __host__ __device__ constexpr int group_head(int c) { return c == 0 ? 0 : c == 1 ? 2 : 3; }
    static __host__ __device__ constexpr int halo_count(const PlaneSpec &s)
    {
        return s.jm * W + s.jp * W + s.km * CJ + s.kp * CJ;
    }
    static __device__ __forceinline__ void body(const Args &a, const Blk &blk)
    {
        __shared__ R pl[NPL][PL];
        __shared__ double pd[HASP ? PL : 1];
        const Dims &d = a.d;
        const Geo<R> &g = a.g;
        const int p = d.p0 + (int)blk.y;
        const int j0 = ulo<L>(1), k0 = ulo<L>(2), i0 = ulo<L>(0);
        const int nj = d.nt - j0;
        const unsigned ntk = (unsigned)((d.np + 63) / 64), ntj = (unsigned)((nj + CJ - 1) / CJ);
        // segment (block-uniform, so the early exit keeps every barrier whole)
        const unsigned seg = blk.x / (ntk * ntj), bt = blk.x - seg * (ntk * ntj);
        int is, ie;
        res_segment(i0, d.nr, a.nseg, (int)seg, is, ie);
        if (is >= ie) return;
        const int tk = (int)(a.jfast ? bt / ntj : bt % ntk);
        const int tj = (int)(a.jfast ? bt % ntj : bt / ntk);
        const int kt0 = tk * 64, jt0 = j0 + tj * CJ;
        const int x = (int)threadIdx.x, y = (int)threadIdx.y, t = x + 64 * y;
        const int j = jt0 + y, k = kt0 + x;
        const bool active = j < d.nt && k >= k0 && k < d.np;
        const uint32_t sI = (uint32_t)d.sI, sJ = (uint32_t)d.sJ;
        const ResSrc<R> src(a);
        // own cell (loads clamped to the ghost row / column past the tile)
        const uint32_t ql = (uint32_t)ix(d, p, i0, j < d.nt ? j : d.nt, k < d.np ? k : d.np);
        // this thread's halo cell of each group of planes with the same
        // halo sides (if any); the groups' cells are dealt from staggered
        // threads, so the halo loads spread over the waves
        uint32_t qh[NG];
        int hl[NG];
        int base = 0;
#pragma unroll
        for (int c = 0; c < NG; c++) {
            hl[c] = -1;
            qh[c] = ql;
            const PlaneSpec s = res_plane<L>(group_head(c));
            const int h = (t + NT - base % NT) % NT;
            base += halo_count(s);
            int jj, kk;
            if (halo_cell<CJ>(s, h, jj, kk)) {
                const int jg = min(jt0 + jj, d.nt), kg = min(kt0 + kk, d.np);
                hl[c] = (jj + 1) * W + (kk + 1);
                qh[c] = (uint32_t)ix(d, p, i0, jg, kg);
            }
        }
        // values of the next point: the planes (own cell and halo cell), the
        // own psi^k - psi^n and forcing, and the location's own-cell terms
        R ov[NPL], hv[NPL];
        double pov = 0.0, phv = 0.0;
        R dkn = R(0), fn = R(0), wrn = R(0), owa = R(0), Tnn = R(0), Tkn = R(0);
        double ptn = 0.0;
        // full: everything of point lev; else only psibar and psi^k - psi^n
        // of the own cell (the last point's psibar at i+1)
        auto fetch = [&](uint32_t lev, bool full) {
            const R pkv = src.pk[ql + lev], pnv = src.pn[ql + lev];
            ov[0] = R(0.5) * (pnv + pkv);
            dkn = pkv - pnv;
            if (!full) return;
            hv[0] = hl[0] >= 0 ? src.bar(qh[0] + lev) : R(0);
#pragma unroll
            for (int c = 1; c < NPL; c++) {
                const PlaneSpec s = res_plane<L>(c);
                const uint32_t o = lev + (uint32_t)s.off * sI;
                ov[c] = plane_val<R>(src, s.q, ql + o);
                hv[c] = hl[grp(c)] >= 0 ? plane_val<R>(src, s.q, qh[grp(c)] + o) : R(0);
            }
            if (HASP) {
                pov = src.ptl(ql + lev);
                phv = hl[grp(NPL)] >= 0 ? src.ptl(qh[grp(NPL)] + lev) : 0.0;
            }
            fn = src.fin.p ? src.fin[ql + lev] : R(0);
            if (L == CC) wrn = src.wr[ql + lev + sI];
            if (L == FR) {
                wrn = src.wr[ql + lev];
                Tnn = src.Tn[ql + lev];
                Tkn = src.Tk[ql + lev];
                ptn = src.ptl(ql + lev);
            }
            if (L == FT) owa = src.wt[ql + lev];
            if (L == FP) owa = src.wp[ql + lev];
        };
        Col<R> w;
        uint32_t lev = (uint32_t)(is - i0) * sI;   // (i - i0) sI
        uint32_t q = ql + lev;
        if (active) src.template prime<L>(g, is, q, sI, sJ, w);
        fetch(lev, true);
        const int me = (y + 1) * W + (x + 1);
        for (int i = is; i < ie; i++, q += sI) {
            if (i > is) __syncthreads();
#pragma unroll
            for (int c = 0; c < NPL; c++) {
                pl[c][me] = ov[c];
                if (hl[grp(c)] >= 0) pl[c][hl[grp(c)]] = hv[c];
            }
            if (HASP) {
                pd[me] = pov;
                if (hl[grp(NPL)] >= 0) pd[hl[grp(NPL)]] = phv;
            }
            ResNb<R> n;
            n.dk = dkn;
            n.f = fn;
            if (L == CC) n.wr1 = wrn;
            if (L == FR) {
                n.wr0 = wrn;
                n.Tn = Tnn;
                n.Tk = Tkn;
                n.pt = ptn;
            }
            if (L == FT) n.t0 = owa;
            if (L == FP) n.p0 = owa;
            lev += sI;
            fetch(lev, i + 1 < ie);
            n.bp = ov[0];
            __syncthreads();
            if (active) {
                auto P = [&](int c, int dj, int dk) { return pl[c][me + dj * W + dk]; };
                n.bjm = P(0, -1, 0); n.bjp = P(0, 1, 0); n.bkm = P(0, 0, -1); n.bkp = P(0, 0, 1);
                n.x0 = P(1, 0, 0); n.xjm = P(1, -1, 0); n.xjp = P(1, 1, 0);
                n.xkm = P(1, 0, -1); n.xkp = P(1, 0, 1);
                if (L == CC) {
                    n.t0 = P(2, 0, 0); n.t1 = P(2, 1, 0);
                    n.p0 = P(3, 0, 0); n.p1 = P(3, 0, 1);
                } else if (L == FR) {
                    n.t0 = P(2, 0, 0); n.t1 = P(2, 1, 0); n.p0 = P(3, 0, 0); n.p1 = P(3, 0, 1);
                    n.e0 = P(4, 0, 0); n.e1 = P(4, 1, 0); n.f0 = P(5, 0, 0); n.f1 = P(5, 0, 1);
                } else if (L == FT) {
                    n.r0 = P(2, -1, 0); n.r1 = P(2, 0, 0);
                    n.p0 = P(3, -1, 0); n.p1 = P(3, -1, 1); n.p2 = P(3, 0, 0); n.p3 = P(3, 0, 1);
                    n.u0 = P(4, -1, 0); n.u1 = P(4, 0, 0);
                    n.s0 = P(5, 0, 1); n.s1 = P(5, 0, 0); n.s2 = P(5, -1, 1); n.s3 = P(5, -1, 0);
                    n.pt = pd[me]; n.pm = pd[me - W];
                } else {
                    n.r0 = P(2, 0, -1); n.r1 = P(2, 0, 0);
                    n.t0 = P(3, 0, -1); n.t1 = P(3, 1, -1); n.t2 = P(3, 0, 0); n.t3 = P(3, 1, 0);
                    n.u0 = P(4, 0, -1); n.u1 = P(4, 0, 0);
                    n.h0 = P(5, 0, 0); n.h1 = P(5, 1, 0); n.h2 = P(5, 0, -1); n.h3 = P(5, 1, -1);
                    n.pt = pd[me]; n.pm = pd[me - 1];
                }
                st(a.out, q, res_point<R, L>(g, i, j, n, w));
            }
        }
    }
};

// ---------------------------------------------------------------------------
// a5: line sweeps (I - tau/2 L_{L,D}) y = x, Thomas algorithm per line.
// Homogeneous ends: correction 0 at theta/phi ghosts, boundary faces and
// u_r wall faces; reflection c_{-1} = -c_0 for r-centred unknowns.
// MODE 0: y = solution; MODE 1 (last factor): psi^k += solution and the
// l2 norm of the increment into per-block partial sums.
// Thread = line; lines along r and theta are coalesced over k.
// ---------------------------------------------------------------------------
template <typename R>
struct SweepArgs { Dims d; Geo<R> g; Geo<double> gd; State<R> s; const R *x; R *y; R *cb; R *psi; double *partial; int P, mc, ld; };
template <typename R, int L, int D, int MODE, int DIFF> struct KThomas {
    using Args = SweepArgs<R>;
    static constexpr int bounds = 256;
    static constexpr bool xcd = false;
    static __device__ __forceinline__ void body(const Args &a, const Blk &blk)
    {
        const Dims &d = a.d;
        const Geo<R> &g = a.g;
        const Geo<double> &gd = a.gd;
        const State<R> &s = a.s;
        const R *x = a.x;
        R *y = a.y;
        R *cb = a.cb;
        R *psi = a.psi;
        double *partial = a.partial;
        (void)cb; (void)gd; (void)partial;

    const int p = d.p0 + blk.y;
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
    for (int64_t t = blk.x * (int64_t)blockDim.x + threadIdx.x; t < nlines;
         t += (int64_t)blk.nx * blockDim.x) {
        const int a = (int)(t / nB), b = (int)(t % nB);
        int i, j, k;
        if (D == 0) { j = j0 + a; k = k0 + b; i = m0; }
        else if (D == 1) { i = i0 + a; k = k0 + b; j = m0; }
        else { i = i0 + a; j = j0 + b; k = m0; }
        const int64_t q0 = ix(d, p, i, j, k);
        // rows go in batches of TB: the loads of a batch are unconditional
        // (rows past the line's end repeat its last row) and in flight
        // together; the recurrences then run over the batch
        constexpr int TB = 4;
        R cprev = R(0), dprev = R(0);
        for (int mb = 0; mb < n; mb += TB) {
            R lo[TB], di[TB], up[TB], xv[TB];
#pragma unroll
            for (int b = 0; b < TB; b++) {
                const int m = mb + b < n ? mb + b : n - 1;
                const int64_t q = q0 + (int64_t)m * stride;
                const int ii = D == 0 ? m0 + m : i, jj = D == 1 ? m0 + m : j;
                R ar = R(0), at = R(0), ap = R(0);
                if (!DIFF) adv<L>(s, d, q, ar, at, ap);
                const Tri<R> c = true_metric<D, DIFF>(g, ii, jj, coef<L, D>(g, ii, jj, ar, at, ap, nu), nu);
                lo[b] = -ht * c.lo;
                up[b] = -ht * c.up;
                di[b] = R(1) - ht * c.di;
                const R rw0 = DIFF ? R(1) : (L == CC ? g.rho_t[0] : g.rho_u[0]);
                const R rw1 = DIFF ? R(1) : (L == CC ? g.rho_t[1] : g.rho_u[1]);
                if (reflect && m == 0) di[b] = R(1) - ht * (c.di - rw0 * c.lo);
                if (reflect && m == n - 1) di[b] = R(1) - ht * (c.di - rw1 * c.up);
                xv[b] = x[q];
            }
#pragma unroll
            for (int b = 0; b < TB; b++) {
                const int m = mb + b;
                if (m < n) {
                    const int64_t q = q0 + (int64_t)m * stride;
                    const R den = di[b] - lo[b] * cprev;
                    const R cp = (m < n - 1) ? up[b] / den : R(0);
                    const R dp = (xv[b] - lo[b] * dprev) / den;
                    cb[q] = cp;
                    y[q] = dp;
                    cprev = cp;
                    dprev = dp;
                }
            }
        }
        R xn = R(0);
        for (int mb = n - 1; mb >= 0; mb -= TB) {
            R yv[TB], cv[TB], pv[TB];
#pragma unroll
            for (int b = 0; b < TB; b++) {
                const int m = mb - b >= 0 ? mb - b : 0;
                const int64_t q = q0 + (int64_t)m * stride;
                yv[b] = y[q];
                cv[b] = cb[q];
                if (MODE == 1) pv[b] = psi[q];
            }
#pragma unroll
            for (int b = 0; b < TB; b++) {
                const int m = mb - b;
                if (m >= 0) {
                    const int64_t q = q0 + (int64_t)m * stride;
                    const R xm = yv[b] - cv[b] * xn;
                    xn = xm;
                    if (MODE == 0) {
                        y[q] = xm;
                    } else {
                        psi[q] = pv[b] + xm;
                        const int ii = D == 0 ? m0 + m : i, jj = D == 1 ? m0 + m : j;
                        const double r0 = L == FR ? gd.rf[ii + 1] : gd.rc[ii + 1];
                        const double s0 = L == FT ? gd.sf[jj + 1] : gd.sc[jj + 1];
                        acc += r0 * r0 * s0 * gd.dr * gd.dth * gd.dph * (double)xm * (double)xm;
                    }
                }
            }
        }
    }
    if (MODE == 1) {
        const double tot = block_sum(acc);
        if (threadIdx.x == 0) partial[p * NBMAX + blk.x] = tot;
    }
    }
};

// ---------------------------------------------------------------------------
// a5 (register-resident form): partitioned line solve.  A line of n
// unknowns is split into P chunks of 2..M consecutive rows, one chunk per
// thread, held in registers.  Each chunk is reduced by two-way elimination
// (forward, then backward) to rows written through its own first and last
// unknowns; the 2P reduced rows form a tridiagonal system solved by one
// thread per line (Thomas), after which every chunk recovers its interior.
// The line is read once and written once: no c'/d' round trip to memory.
// ---------------------------------------------------------------------------
// Forward elimination of row m of a chunk as it is assembled (row m:
// lo x_{m-1} + di x_m + up x_{m+1} = rhs).  Rows 0 and 1 are normalised;
// rows m >= 2 are rewritten through the chunk's first unknown x_0.
// 1/x for the pivots of the line solvers: the hardware reciprocal refined
// by two Newton steps r <- r (2 - x r) in FP64 (each squares the relative
// error), the 1-ulp hardware reciprocal in FP32.  The pivots of these
// diagonally dominant systems are O(1), far from zero and from overflow, so
// the scaling an IEEE division performs is not needed.
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = r * (2.0 - x * r);
    return r * (2.0 - x * r);
}
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename R, int M>
__device__ __forceinline__ void chunk_forward(R (&a)[M], R (&c)[M], R (&d)[M], int m, R lo, R di,
                                              R up, R rhs)
{
    if (m < 2) {
        const R r = recip(di);
        a[m] = lo * r;
        c[m] = up * r;
        d[m] = rhs * r;
    } else {
        const R r = recip(di - lo * c[m - 1]);
        d[m] = r * (rhs - lo * d[m - 1]);
        c[m] = r * up;
        a[m] = -r * lo * a[m - 1];
    }
}

// Backward elimination: rows 1..mt-2 become a_i x_0 + x_i + c_i x_{mt-1} =
// d_i; row 0 becomes a_0 x_{-1} + x_0 + c_0 x_{mt-1} = d_0 (two-way
// elimination of a partitioned tridiagonal solve).
template <typename R, int M>
__device__ __forceinline__ void chunk_backward(R (&a)[M], R (&c)[M], R (&d)[M], int mt)
{
#pragma unroll
    for (int i = M - 3; i >= 1; i--) {
        if (i <= mt - 3) {
            d[i] = d[i] - c[i] * d[i + 1];
            a[i] = a[i] - c[i] * a[i + 1];
            c[i] = -c[i] * c[i + 1];
        }
    }
    if (mt >= 3) {
        const R r = recip(R(1) - c[0] * a[1]);
        d[0] = r * (d[0] - c[0] * d[1]);
        a[0] = r * a[0];
        c[0] = -r * c[0] * c[1];
    }
}

// Reduced system of a partitioned solve.  Chunk t keeps two rows,
//   S_t: al_t x_{e(t-1)} + x_{s(t)} + be_t x_{e(t)}   = de_t   (its first row)
//   E_t: ga_t x_{s(t)}   + x_{e(t)} + et_t x_{s(t+1)} = ze_t   (its last row)
// Eliminating the first unknowns x_s with S_t and S_{t+1} leaves one row per
// chunk in the last unknowns only:
//   A_t x_{e(t-1)} + B_t x_{e(t)} + C_t x_{e(t+1)} = D_t,
// solved by parallel cyclic reduction (all chunks at once, log2 P levels).
template <typename R> struct Row4 { R a, b, c, d; };

template <typename R>
__device__ __forceinline__ Row4<R> erow(R al, R be, R de, R ga, R et, R ze, R al1, R be1, R de1)
{
    Row4<R> r;
    r.a = -ga * al;
    r.b = R(1) - ga * be - et * al1;
    r.c = -et * be1;
    r.d = ze - ga * de - et * de1;
    return r;
}

// one PCR level: combine row t with rows t-h (m) and t+h (p)
template <typename R>
__device__ __forceinline__ Row4<R> pcr_level(const Row4<R> &t, const Row4<R> &m, const Row4<R> &p)
{
    const R k1 = t.a * recip(m.b), k2 = t.c * recip(p.b);
    Row4<R> o;
    o.a = -k1 * m.a;
    o.c = -k2 * p.c;
    o.b = t.b - k1 * m.c - k2 * p.a;
    o.d = t.d - k1 * m.d - k2 * p.d;
    return o;
}

template <typename R> __device__ __forceinline__ R shfl_r(R v, int src)
{
    return __shfl(v, src, 64);
}

// last row of a chunk (runtime index into a register array)
template <typename R, int M>
__device__ __forceinline__ void chunk_last(const R (&a)[M], const R (&c)[M], const R (&d)[M], int mt,
                                           R &ga, R &gc, R &gd)
{
    ga = a[0]; gc = c[0]; gd = d[0];
#pragma unroll
    for (int i = 1; i < M; i++)
        if (i == mt - 1) { ga = a[i]; gc = c[i]; gd = d[i]; }
}

// Thomas over the 2P reduced rows (lower, upper, rhs; unit diagonal) kept in
// a strided array: row r at base[r * rs]; overwrites rhs with the solution.
template <typename R>
__device__ __forceinline__ void reduced_solve(R *lo, R *up, R *rhs, int nrow, int rs)
{
    R cp = R(0), dp = R(0);
    for (int r = 0; r < nrow; r++) {
        const R l = lo[r * rs];
        const R den = R(1) - l * cp;
        cp = up[r * rs] / den;
        dp = (rhs[r * rs] - l * dp) / den;
        up[r * rs] = cp;
        rhs[r * rs] = dp;
    }
    R xn = R(0);
    for (int r = nrow - 1; r >= 0; r--) {
        xn = rhs[r * rs] - up[r * rs] * xn;
        rhs[r * rs] = xn;
    }
}

// one row of the line system (I - tau/2 L) at global row g of n, from the
// advecting velocity at the point
template <typename R, int L, int D, int DIFF, typename TB>
__device__ __forceinline__ void line_row_t(const Geo<R> &g, int ii, int jj, int gr, int n, R nu, R ar, R at,
                                           R ap, const TB &tb, R &lo, R &di, R &up)
{
    const Tri<R> c = true_metric<D, DIFF>(g, ii, jj, coef_t<L, D>(g, ii, jj, ar, at, ap, nu, tb), nu);
    lo = gr > 0 ? -g.ht * c.lo : R(0);
    up = gr < n - 1 ? -g.ht * c.up : R(0);
    di = R(1) - g.ht * c.di;
    if (D == 0 && L != FR) {
        // wall rule of the correction c_ghost = -rho c_in: rho = 1 for
        // Dirichlet walls, the Robin rules of T and of the tangential
        // velocity otherwise
        const R rw0 = DIFF ? R(1) : (L == CC ? g.rho_t[0] : g.rho_u[0]);
        const R rw1 = DIFF ? R(1) : (L == CC ? g.rho_t[1] : g.rho_u[1]);
        if (gr == 0) di = R(1) - g.ht * (c.di - rw0 * c.lo);
        if (gr == n - 1) di = R(1) - g.ht * (c.di - rw1 * c.up);
    }
}

template <typename R, int L, int D, int DIFF>
__device__ __forceinline__ void line_row(const Dims &d, const Geo<R> &g, const State<R> &s, int64_t q,
                                         int ii, int jj, int gr, int n, R nu, R &lo, R &di, R &up)
{
    R ar = R(0), at = R(0), ap = R(0);
    if (!DIFF) adv<L>(s, d, q, ar, at, ap);
    line_row_t<R, L, D, DIFF>(g, ii, jj, gr, n, nu, ar, at, ap, GTab<L, D, R>{g, D == 0 ? ii + 1 : jj + 1}, lo,
                              di, up);
}

template <int L, int D> __device__ __forceinline__ double vol_at(const Geo<double> &gd, int ii, int jj)
{
    const double r0 = L == FR ? gd.rf[ii + 1] : gd.rc[ii + 1];
    const double s0 = L == FT ? gd.sf[jj + 1] : gd.sc[jj + 1];
    return r0 * r0 * s0 * gd.dr * gd.dth * gd.dph;
}

// number of W-wide k-tiles (tile q: k = q W .. q W + W - 1, aligned to the
// row storage) that cover the unknowns k < np
__host__ __device__ inline int sweep_ktiles(int np, int W) { return (np + W - 1) / W; }

// Strided lines (D = 0: r, D = 1: theta).  Block (W, P): lane x <-> k (W
// consecutive k, coalesced), y <-> chunk.  A task = (k-tile, other index).
// BL: every load of a chunk (and its psi, last factor) is issued before the
// elimination, rows past the chunk's end repeating its last row, so that
// they are in flight together (more registers); otherwise each row is
// loaded as it is eliminated.  The autotuner picks per sweep.
template <typename R, int L, int D, int MODE, int DIFF, int M, bool BL> struct KStrided {
    using Args = SweepArgs<R>;
    static constexpr int bounds = 512;
    static constexpr bool xcd = true;
    static __device__ __forceinline__ void body(const Args &a, const Blk &blk)
    {
        const Dims &d = a.d;
        const Geo<R> &g = a.g;
        const Geo<double> &gd = a.gd;
        const State<R> &s = a.s;
        const R *x = a.x;
        R *y = a.y;
        R *cb = a.cb;
        R *psi = a.psi;
        double *partial = a.partial;
        (void)cb; (void)gd; (void)partial;

    extern __shared__ unsigned char smem_raw[];
    R *sm = reinterpret_cast<R *>(smem_raw);
    const int W = blockDim.x, P = blockDim.y;
    const int lane = threadIdx.x, t = threadIdx.y;
    unsigned bx, by;
    bx = blk.x;
    by = blk.y;
    const int p = d.p0 + (int)by;
    const int i0 = ulo<L>(0), j0 = ulo<L>(1), k0 = ulo<L>(2);
    const int m0 = D == 0 ? i0 : j0;
    const int n = ncell(d, D) - m0;
    const int nother = D == 0 ? d.nt - j0 : d.nr - i0;
    const int ntile = sweep_ktiles(d.np, W);
    const int64_t stride = D == 0 ? d.sI : d.sJ;
    const R nu = (L == CC && !DIFF) ? R(1) : g.pr;
    // chunk rows [r0, r1)
    const int r0 = (int)((int64_t)t * n / P), r1 = (int)((int64_t)(t + 1) * n / P);
    const int mt = r1 - r0;
    // reduced-system exchange in LDS: four [P][W] arrays; then the line's
    // per-row coefficient tables (ntabs x n, row gr at gr), staged once
    R *sA = sm, *sB = sm + P * W, *sC = sm + 2 * P * W, *sD = sm + 3 * P * W;
    constexpr int NT = ntabs<L, D>();
    R *stab = sm + 4 * P * W;
    for (int e = t * W + lane; e < NT * n; e += W * P) {
        const int tt = e / n, gr = e % n;
        stab[e] = row_table<L, D>(g, tt)[m0 + gr + 1];
    }
    __syncthreads();
    double acc = 0.0;
    for (int task = (int)bx; task < ntile * nother; task += blk.nx) {
        const int tile = task % ntile, oth = task / ntile;
        const int k = tile * W + lane;
        const bool live = k >= k0 && k < d.np;
        int i = 0, j = 0;
        if (D == 0) j = j0 + oth; else i = i0 + oth;
        R a[M], c[M], dd[M];
#pragma unroll
        for (int m = 0; m < M; m++) { a[m] = R(0); c[m] = R(0); dd[m] = R(0); }
        const int64_t qf = ix(d, p, D == 0 ? m0 + r0 : i, D == 1 ? m0 + r0 : j, k);
        R pv[M];                           // psi of the chunk (BL, last factor)
        if (live) {
            if (BL) {
                // every raw load of the chunk first (right-hand side, psi,
                // advecting-velocity face values); the empty asm with a
                // memory clobber keeps the scheduler from sinking any of
                // them below the arithmetic, so they are in flight together
                constexpr int NA = DIFF ? 1 : AdvNeed<L, D>::N;
                R xv[M], av[M][NA];
#pragma unroll
                for (int m = 0; m < M; m++) {
                    const int mm = m < mt ? m : mt - 1;
                    const int64_t q = qf + (int64_t)mm * stride;
                    xv[m] = x[q];
                    if (MODE == 1) pv[m] = psi[q];
                    if (!DIFF) adv_fetch<L, D>(s, d, q, av[m]);
                }
                asm volatile("" ::: "memory");
#pragma unroll
                for (int m = 0; m < M; m++) {
                    const int mm = m < mt ? m : mt - 1;
                    const int gr = r0 + mm;
                    const int ii = D == 0 ? m0 + gr : i, jj = D == 1 ? m0 + gr : j;
                    R ar = R(0), at = R(0), ap = R(0);
                    if (!DIFF) adv_combine<L, D>(av[m], ar, at, ap);
                    R lo, di, up;
                    line_row_t<R, L, D, DIFF>(g, ii, jj, gr, n, nu, ar, at, ap, LTab<R>{stab + gr, n}, lo, di, up);
                    chunk_forward<R, M>(a, c, dd, m, lo, di, up, xv[m]);
                    if (m >= mt) { a[m] = R(0); c[m] = R(0); dd[m] = R(0); }
                }
            } else {
#pragma unroll
                for (int m = 0; m < M; m++) {
                    if (m < mt) {
                        const int gr = r0 + m;
                        const int ii = D == 0 ? m0 + gr : i, jj = D == 1 ? m0 + gr : j;
                        const int64_t q = qf + (int64_t)m * stride;
                        R ar = R(0), at = R(0), ap = R(0);
                        if (!DIFF) adv<L>(s, d, q, ar, at, ap);
                        R lo, di, up;
                        line_row_t<R, L, D, DIFF>(g, ii, jj, gr, n, nu, ar, at, ap, LTab<R>{stab + gr, n}, lo, di,
                                                  up);
                        chunk_forward<R, M>(a, c, dd, m, lo, di, up, x[q]);
                    }
                }
            }
            chunk_backward<R, M>(a, c, dd, mt);
        }
        // reduced rows: S_t in registers, S_{t+1} through LDS
        R ga = R(0), gc = R(0), gdv = R(0);
        if (live) chunk_last<R, M>(a, c, dd, mt, ga, gc, gdv);
        sA[t * W + lane] = a[0];
        sB[t * W + lane] = c[0];
        sC[t * W + lane] = dd[0];
        __syncthreads();
        R al1 = R(0), be1 = R(0), de1 = R(0);
        if (t + 1 < P) {
            al1 = sA[(t + 1) * W + lane];
            be1 = sB[(t + 1) * W + lane];
            de1 = sC[(t + 1) * W + lane];
        }
        Row4<R> row = erow<R>(a[0], c[0], dd[0], ga, gc, gdv, al1, be1, de1);
        if (!live) { row.a = R(0); row.b = R(1); row.c = R(0); row.d = R(0); }
        for (int h = 1; h < P; h <<= 1) {
            __syncthreads();
            sA[t * W + lane] = row.a;
            sB[t * W + lane] = row.b;
            sC[t * W + lane] = row.c;
            sD[t * W + lane] = row.d;
            __syncthreads();
            Row4<R> rm = {R(0), R(1), R(0), R(0)}, rp = {R(0), R(1), R(0), R(0)};
            if (t - h >= 0) {
                const int o = (t - h) * W + lane;
                rm.a = sA[o]; rm.b = sB[o]; rm.c = sC[o]; rm.d = sD[o];
            }
            if (t + h < P) {
                const int o = (t + h) * W + lane;
                rp.a = sA[o]; rp.b = sB[o]; rp.c = sC[o]; rp.d = sD[o];
            }
            row = pcr_level<R>(row, rm, rp);
        }
        const R xe = row.d * recip(row.b);
        __syncthreads();
        sA[t * W + lane] = xe;
        __syncthreads();
        const R xem = t > 0 ? sA[(t - 1) * W + lane] : R(0);
        const R xs = dd[0] - a[0] * xem - c[0] * xe;
        if (live) {
#pragma unroll
            for (int m = 0; m < M; m++) {
                if (m < mt) {
                    const R v = (m == 0) ? xs : (m == mt - 1 ? xe : dd[m] - a[m] * xs - c[m] * xe);
                    const int gr = r0 + m;
                    const int ii = D == 0 ? m0 + gr : i, jj = D == 1 ? m0 + gr : j;
                    const int64_t q = qf + (int64_t)m * stride;
                    if (MODE == 0) {
                        y[q] = v;
                    } else {
                        psi[q] = (BL ? pv[m] : psi[q]) + v;
                        acc += vol_at<L, D>(gd, ii, jj) * (double)v * (double)v;
                    }
                }
            }
        }
        __syncthreads();
    }
    if (MODE == 1) {
        // block_sum needs a 1-D thread index: flatten
        double v = acc;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        __shared__ double red[16];
        const int flat = t * W + lane;
        if ((flat & 63) == 0) red[flat >> 6] = v;
        __syncthreads();
        if (flat == 0) {
            double tot = 0.0;
            const int nw = (W * P) >> 6;
            for (int w = 0; w < nw; w++) tot += red[w];
            partial[p * NBMAX + bx] = tot;
        }
    }
    }
};

// Contiguous lines (D = 2, phi).  One wave per line (LPB lines per block).
// Phase A, coalesced: lane e%64 assembles row e (coefficients from the
// tables and the advecting velocity) and stores (lo, di, up, x) in LDS,
// transposed to [row-in-chunk][chunk] (padded) so that phase B reads are
// conflict-free.  Phase B: lane c eliminates chunk c (rows c*m .. c*m+m-1)
// in registers, the reduced system is solved by PCR over wave shuffles, and
// the chunk's solution goes back to LDS.  Phase C, coalesced: write y (or
// psi += y and the increment norm).
template <typename R, int L, int MODE, int DIFF, int M> struct KContig {
    using Args = SweepArgs<R>;
    static constexpr int bounds = 256;
    static constexpr bool xcd = false;
    static __device__ __forceinline__ void body(const Args &a, const Blk &blk)
    {
        const Dims &d = a.d;
        const Geo<R> &g = a.g;
        const Geo<double> &gd = a.gd;
        const State<R> &s = a.s;
        const R *x = a.x;
        R *y = a.y;
        R *cb = a.cb;
        R *psi = a.psi;
        double *partial = a.partial;
        (void)cb; (void)gd; (void)partial;
        const int P = a.P, mc = a.mc;

    extern __shared__ unsigned char smem_raw[];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, lpb = blockDim.x >> 6;
    const int p = d.p0 + blk.y;
    const int i0 = ulo<L>(0), j0 = ulo<L>(1), k0 = ulo<L>(2);
    const int n = d.np - k0;
    const int ni = d.nr - i0, nj = d.nt - j0;
    const int64_t nlines = (int64_t)ni * nj;
    const int ld = a.ld;                       // row pitch of the transposed arrays (host-chosen)
    const int per = 4 * mc * ld;               // elements per line
    R *sl = reinterpret_cast<R *>(smem_raw) + (int64_t)w * per;
    R *tlo = sl, *tdi = sl + mc * ld, *tup = sl + 2 * mc * ld, *tx = sl + 3 * mc * ld;
    const R nu = (L == CC && !DIFF) ? R(1) : g.pr;
    const int mt = lane < P ? (lane < P - 1 ? mc : n - (P - 1) * mc) : 0;
    double acc = 0.0;
    for (int64_t base = (int64_t)blk.x * lpb; base < nlines; base += (int64_t)blk.nx * lpb) {
        const int64_t line = base + w;
        const bool lv = line < nlines;
        const int i = i0 + (int)(lv ? line / nj : 0), j = j0 + (int)(lv ? line % nj : 0);
        const int64_t q0 = ix(d, p, i, j, k0);
        if (lv) {
            // batches of CB rows per lane, all loads of a batch in flight
            // together (rows past the end repeat the last one)
            constexpr int CB = 4;
            for (int e0 = lane; e0 < n; e0 += 64 * CB) {
#pragma unroll
                for (int b = 0; b < CB; b++) {
                    const int e = e0 + 64 * b, ec = e < n ? e : n - 1;
                    R lo, di, up;
                    line_row<R, L, 2, DIFF>(d, g, s, q0 + ec, i, j, ec, n, nu, lo, di, up);
                    const R xv = x[q0 + ec];
                    if (e < n) {
                        const int cc = e / mc, rr = e - cc * mc;
                        const int o = rr * ld + cc;
                        tlo[o] = lo;
                        tdi[o] = di;
                        tup[o] = up;
                        tx[o] = xv;
                    }
                }
            }
        }
        __syncthreads();
        R a[M], c[M], dd[M];
#pragma unroll
        for (int m = 0; m < M; m++) {
            a[m] = R(0); c[m] = R(0); dd[m] = R(0);
            if (lv && m < mt) {
                const int o = m * ld + lane;
                chunk_forward<R, M>(a, c, dd, m, tlo[o], tdi[o], tup[o], tx[o]);
            }
        }
        if (lv && mt > 0) chunk_backward<R, M>(a, c, dd, mt);
        R ga = R(0), gc = R(0), gdv = R(0);
        if (mt > 0) chunk_last<R, M>(a, c, dd, mt, ga, gc, gdv);
        const R al1 = shfl_r(a[0], (lane + 1) & 63), be1 = shfl_r(c[0], (lane + 1) & 63),
                de1 = shfl_r(dd[0], (lane + 1) & 63);
        Row4<R> row;
        if (lane < P) row = erow<R>(a[0], c[0], dd[0], ga, gc, gdv, lane + 1 < P ? al1 : R(0),
                                    lane + 1 < P ? be1 : R(0), lane + 1 < P ? de1 : R(0));
        else { row.a = R(0); row.b = R(1); row.c = R(0); row.d = R(0); }
        for (int h = 1; h < P; h <<= 1) {
            Row4<R> rm, rp;
            rm.a = shfl_r(row.a, (lane - h) & 63); rm.b = shfl_r(row.b, (lane - h) & 63);
            rm.c = shfl_r(row.c, (lane - h) & 63); rm.d = shfl_r(row.d, (lane - h) & 63);
            rp.a = shfl_r(row.a, (lane + h) & 63); rp.b = shfl_r(row.b, (lane + h) & 63);
            rp.c = shfl_r(row.c, (lane + h) & 63); rp.d = shfl_r(row.d, (lane + h) & 63);
            if (lane - h < 0) { rm.a = R(0); rm.b = R(1); rm.c = R(0); rm.d = R(0); }
            if (lane + h >= P) { rp.a = R(0); rp.b = R(1); rp.c = R(0); rp.d = R(0); }
            row = pcr_level<R>(row, rm, rp);
        }
        const R xe = row.d * recip(row.b);
        const R xem0 = shfl_r(xe, (lane - 1) & 63);
        const R xem = lane > 0 ? xem0 : R(0);
        const R xs = dd[0] - a[0] * xem - c[0] * xe;
        __syncthreads();
#pragma unroll
        for (int m = 0; m < M; m++) {
            if (lv && m < mt) {
                const R v = (m == 0) ? xs : (m == mt - 1 ? xe : dd[m] - a[m] * xs - c[m] * xe);
                tx[m * ld + lane] = v;
            }
        }
        __syncthreads();
        if (lv) {
            const double vol = MODE == 1 ? vol_at<L, 2>(gd, i, j) : 0.0;
            if (MODE == 0) {
                for (int e = lane; e < n; e += 64) {
                    const int cc = e / mc, rr = e - cc * mc;
                    y[q0 + e] = tx[rr * ld + cc];
                }
            } else {
                constexpr int CB = 4;
                for (int e0 = lane; e0 < n; e0 += 64 * CB) {
                    R pv[CB];
#pragma unroll
                    for (int b = 0; b < CB; b++) {
                        const int e = e0 + 64 * b;
                        pv[b] = psi[q0 + (e < n ? e : n - 1)];
                    }
#pragma unroll
                    for (int b = 0; b < CB; b++) {
                        const int e = e0 + 64 * b;
                        if (e < n) {
                            const int cc = e / mc, rr = e - cc * mc;
                            const R v = tx[rr * ld + cc];
                            psi[q0 + e] = pv[b] + v;
                            acc += vol * (double)v * (double)v;
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (MODE == 1) {
        const double tot = block_sum(acc);
        if (threadIdx.x == 0) partial[p * NBMAX + blk.x] = tot;
    }
    }
};

// Contiguous lines, V = blockDim.x / 64 waves per line (one line per block
// at a time): P = 64 V chunks of mc rows, so each lane holds a few rows
// (fewer registers, more waves per SIMD).  Phases as in k_sweep_contig; the
// reduced system spans the waves, so its PCR goes through LDS, reusing the
// staging arrays of the coefficients once the chunks have consumed them.
template <typename R, int L, int MODE, int DIFF, int M> struct KContigMw {
    using Args = SweepArgs<R>;
    static constexpr int bounds = 512;
    static constexpr bool xcd = false;
    static __device__ __forceinline__ void body(const Args &a, const Blk &blk)
    {
        const Dims &d = a.d;
        const Geo<R> &g = a.g;
        const Geo<double> &gd = a.gd;
        const State<R> &s = a.s;
        const R *x = a.x;
        R *y = a.y;
        R *cb = a.cb;
        R *psi = a.psi;
        double *partial = a.partial;
        (void)cb; (void)gd; (void)partial;
        const int P = a.P, mc = a.mc;

    extern __shared__ unsigned char smem_raw[];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int p = d.p0 + blk.y;
    const int i0 = ulo<L>(0), j0 = ulo<L>(1), k0 = ulo<L>(2);
    const int n = d.np - k0;
    const int ni = d.nr - i0, nj = d.nt - j0;
    const int64_t nlines = (int64_t)ni * nj;
    const int ld = a.ld;                       // row pitch of the transposed arrays (host-chosen)
    R *tlo = reinterpret_cast<R *>(smem_raw);
    R *tdi = tlo + mc * ld, *tup = tlo + 2 * mc * ld, *tx = tlo + 3 * mc * ld;
    // reduced rows (after the chunks are eliminated): aliases of tlo/tdi/tup
    R *sA = tlo, *sB = tdi, *sC = tup, *sD = tlo + ld;
    const R nu = (L == CC && !DIFF) ? R(1) : g.pr;
    const int mt = tid < P ? (tid < P - 1 ? mc : n - (P - 1) * mc) : 0;
    // a thread stages rows tid + r nthr, r < M (n <= P mc <= nthr M).  PRE:
    // every raw load of the thread's rows is issued first (x, psi of the
    // last factor, the advecting-velocity face values), in flight together;
    // the empty asm keeps the scheduler from sinking them into the
    // arithmetic.  u_phi's own line needs 9 velocity values a row: there
    // the registers would cost more occupancy than the prefetch gains, and
    // each row is loaded as it is staged.
    constexpr bool PRE = DIFF || AdvNeed<L, 2>::N <= 4;
    constexpr int NA = (PRE && !DIFF) ? AdvNeed<L, 2>::N : 1;
    double acc = 0.0;
    for (int64_t line = blk.x; line < nlines; line += blk.nx) {
        const int i = i0 + (int)(line / nj), j = j0 + (int)(line % nj);
        const int64_t q0 = ix(d, p, i, j, k0);
        // the diffusion-only operators have one (lower, diagonal, upper)
        // per phi line (the ends drop their outer coupling): only x is staged
        R clo = R(0), cdi = R(0), cup = R(0);
        if (DIFF) line_row<R, L, 2, DIFF>(d, g, s, q0 + 1, i, j, 1, n, nu, clo, cdi, cup);
        R pv[M];
        if (PRE) {
            R xv[M], av[M][NA];
#pragma unroll
            for (int r = 0; r < M; r++) {
                const int e = tid + r * nthr, ec = e < n ? e : n - 1;
                xv[r] = x[q0 + ec];
                if (MODE == 1) pv[r] = psi[q0 + ec];
                if (!DIFF) adv_fetch<L, 2>(s, d, q0 + ec, av[r]);
            }
            asm volatile("" ::: "memory");
#pragma unroll
            for (int r = 0; r < M; r++) {
                const int e = tid + r * nthr;
                if (e < n) {
                    const int cc = e / mc, rr = e - cc * mc;
                    const int o = rr * ld + cc;
                    if (!DIFF) {
                        R ar, at, ap, lo, di, up;
                        adv_combine<L, 2>(av[r], ar, at, ap);
                        line_row_t<R, L, 2, DIFF>(g, i, j, e, n, nu, ar, at, ap, GTab<L, 2, R>{g, 0}, lo, di, up);
                        tlo[o] = lo;
                        tdi[o] = di;
                        tup[o] = up;
                    }
                    tx[o] = xv[r];
                }
            }
        } else {
            for (int e = tid; e < n; e += nthr) {
                const int cc = e / mc, rr = e - cc * mc;
                const int o = rr * ld + cc;
                R lo, di, up;
                line_row<R, L, 2, DIFF>(d, g, s, q0 + e, i, j, e, n, nu, lo, di, up);
                tlo[o] = lo;
                tdi[o] = di;
                tup[o] = up;
                tx[o] = x[q0 + e];
            }
        }
        __syncthreads();
        R a[M], c[M], dd[M];
#pragma unroll
        for (int m = 0; m < M; m++) {
            a[m] = R(0); c[m] = R(0); dd[m] = R(0);
            if (m < mt) {
                const int o = m * ld + tid;
                if (DIFF) {
                    const int gr = tid * mc + m;
                    chunk_forward<R, M>(a, c, dd, m, gr > 0 ? clo : R(0), cdi, gr < n - 1 ? cup : R(0), tx[o]);
                } else {
                    chunk_forward<R, M>(a, c, dd, m, tlo[o], tdi[o], tup[o], tx[o]);
                }
            }
        }
        if (mt > 0) chunk_backward<R, M>(a, c, dd, mt);
        R ga = R(0), gc = R(0), gdv = R(0);
        if (mt > 0) chunk_last<R, M>(a, c, dd, mt, ga, gc, gdv);
        __syncthreads();                       // staging arrays are free from here
        if (tid < P) {
            sA[tid] = a[0];
            sB[tid] = c[0];
            sC[tid] = dd[0];
        }
        __syncthreads();
        Row4<R> row = {R(0), R(1), R(0), R(0)};
        if (tid < P) {
            const bool nx = tid + 1 < P;
            row = erow<R>(a[0], c[0], dd[0], ga, gc, gdv, nx ? sA[tid + 1] : R(0), nx ? sB[tid + 1] : R(0),
                          nx ? sC[tid + 1] : R(0));
        }
        // The levels alternate between two sets of row arrays, so a level
        // needs one barrier: the odd levels (h = 1, 4, 16, ...) use the second
        // rows of tdi and tup and the first two rows of tx, which the reads
        // above do not touch, the even ones sA..sD; a thread writes a set
        // again only after the next level's barrier, which every thread
        // reaches after its reads of the level before.  (Each call site names
        // its arrays, so they stay LDS addresses.)
        auto level = [&](R *bA, R *bB, R *bC, R *bD, int h) {
            if (tid < P) {
                bA[tid] = row.a;
                bB[tid] = row.b;
                bC[tid] = row.c;
                bD[tid] = row.d;
            }
            __syncthreads();
            if (tid < P) {
                Row4<R> rm = {R(0), R(1), R(0), R(0)}, rp = {R(0), R(1), R(0), R(0)};
                if (tid - h >= 0) { rm.a = bA[tid - h]; rm.b = bB[tid - h]; rm.c = bC[tid - h]; rm.d = bD[tid - h]; }
                if (tid + h < P) { rp.a = bA[tid + h]; rp.b = bB[tid + h]; rp.c = bC[tid + h]; rp.d = bD[tid + h]; }
                row = pcr_level<R>(row, rm, rp);
            }
        };
        for (int h = 1; h < P; h <<= 2) {
            level(tdi + ld, tup + ld, tx, tx + ld, h);
            if (2 * h < P) level(sA, sB, sC, sD, 2 * h);
        }
        const R xe = tid < P ? row.d * recip(row.b) : R(0);
        __syncthreads();
        if (tid < P) sA[tid] = xe;
        __syncthreads();
        const R xem = (tid > 0 && tid < P) ? sA[tid - 1] : R(0);
        const R xs = dd[0] - a[0] * xem - c[0] * xe;
#pragma unroll
        for (int m = 0; m < M; m++) {
            if (m < mt) {
                const R v = (m == 0) ? xs : (m == mt - 1 ? xe : dd[m] - a[m] * xs - c[m] * xe);
                tx[m * ld + tid] = v;
            }
        }
        __syncthreads();
        const double vol = MODE == 1 ? vol_at<L, 2>(gd, i, j) : 0.0;
#pragma unroll
        for (int r = 0; r < M; r++) {
            const int e = tid + r * nthr;
            if (e < n) {
                const int cc = e / mc, rr = e - cc * mc;
                const R v = tx[rr * ld + cc];
                if (MODE == 0) {
                    y[q0 + e] = v;
                } else {
                    psi[q0 + e] = (PRE ? pv[r] : psi[q0 + e]) + v;
                    acc += vol * (double)v * (double)v;
                }
            }
        }
        __syncthreads();
    }
    if (MODE == 1) {
        const double tot = block_sum(acc);
        if (tid == 0) partial[p * NBMAX + blk.x] = tot;
    }
    }
};

// Row pitch (>= P + 1) of the chunk-transposed staging arrays of the phi
// solvers.  Row e of a line goes to (e mod mc) * ld + e / mc, so the lanes
// of a wave, holding consecutive rows, write mc-strided runs: with ld = P + 1
// most pitches put several lanes of a wave on one LDS bank (6-way for 6-row
// chunks of 1152-point lines).  The pitch kept is the one among P+1 .. P+32
// with the fewest lanes per bank over the waves' access groups (32 banks of
// 4 bytes; 8-byte elements in half-waves).
#if !defined(YY_ONLY_FLOAT)
int contig_pitch(int n, int P, int mc, int elem_bytes)
{
    // a few (n, P, mc, size) keys recur every step: remember them
    struct Key { int n, P, mc, eb, ld; };
    thread_local Key memo[16] = {};
    thread_local int nmemo = 0;
    for (int q = 0; q < nmemo; q++)
        if (memo[q].n == n && memo[q].P == P && memo[q].mc == mc && memo[q].eb == elem_bytes) return memo[q].ld;
    const int group = elem_bytes == 8 ? 32 : 64, words = elem_bytes / 4;
    int best_ld = P + 1, best = 1 << 30;
    for (int ld = P + 1; ld <= P + 32; ld++) {
        int worst = 0;
        for (int e0 = 0; e0 < n && e0 < 64 * 8; e0 += group) {
            int cnt[32] = {0};
            for (int e = e0; e < e0 + group && e < n; e++) {
                const int o = (e % mc) * ld + e / mc;
                for (int w = 0; w < words; w++) {
                    const int b = (o * words + w) & 31;
                    if (++cnt[b] > worst) worst = cnt[b];
                }
            }
        }
        if (worst < best) {
            best = worst;
            best_ld = ld;
        }
    }
    memo[nmemo < 16 ? nmemo++ : (n + P + mc) & 15] = Key{n, P, mc, elem_bytes, best_ld};
    return best_ld;
}
#endif

// Block shape of a strided partitioned solve of lines of n unknowns with
// chunks of <= M rows: W lanes (consecutive k) x P chunks, W * P <= 512 and
// a whole number of 64-lane waves, every chunk >= 2 rows.  False if the
// line does not fit (then the per-line Thomas kernel runs).
#if !defined(YY_ONLY_FLOAT)
bool strided_tile(int n, int M, int wmax, int &W, int &P)
{
    P = (n + M - 1) / M;
    if (P < 1) P = 1;
    if (wmax != 16 && wmax != 32 && wmax != 64) wmax = 64;
    W = wmax;
    while (W * P > 512 && W > 8) W >>= 1;
    const int q = 64 / W;
    P = (P + q - 1) / q * q;
    if (W * P > 512 || P > n) return false;
    if (2 * P > n && n > 1) return false;
    return true;
}
#endif

// Launch the partitioned solver when the line fits the register chunks,
// else the per-line Thomas kernel.  Returns false if it fell back.
template <typename R, int L, int D, int MODE, int DIFF>
static bool launch_partitioned(const Dims &d, const Geo<R> &g, const Geo<double> &gd,
                               const State<R> &s, const R *x, R *y, R *psi, double *partial,
                               int *nblocks, hipStream_t st)
{
    const int i0 = ulo<L>(0), j0 = ulo<L>(1), k0 = ulo<L>(2);
    if (D < 2) {
        // rows per chunk: tuned (1 = per-line Thomas), else 12 for the
        // u_theta polar sweep (the most per-row data) and 16 otherwise
        const int TL = DIFF ? 4 : L;   // tile slot
        int M = s.tune.m[TL][D];
        if (M == 1) return false;
        if (M != 4 && M != 6 && M != 8 && M != 12 && M != 16) M = (L == FT && D == 1) ? 12 : 16;
        const int n = ncell(d, D) - (D == 0 ? i0 : j0);
        int W = 0, P = 0;
        if (!strided_tile(n, M, s.tune.w[TL][D], W, P)) return false;
        const int nother = D == 0 ? d.nt - j0 : d.nr - i0;
        int64_t tasks = (int64_t)sweep_ktiles(d.np, W) * nother;
        int64_t b = tasks;
        const int64_t cap = s.tune.sb[TL][D] > 0 ? s.tune.sb[TL][D] : SWEEP_BLOCKS;
        if (b > cap) b = cap;
        if (nblocks) *nblocks = (int)b;
        const size_t lds = ((size_t)4 * P * W + (size_t)ntabs<L, D>() * n) * sizeof(R);
        const bool bl = s.tune.bl[TL][D] != 0;
        const SweepArgs<R> sa{d, g, gd, s, x, y, s.cb, psi, partial, P, 0};
#define YY_ST(MM, BB)                                                                                     \
    launch<KStrided<R, L, D, MODE, DIFF, MM, BB>>(dim3((unsigned)b, d.npatch), dim3(W, P), lds, st, sa)
#define YY_STM(MM) \
    do { if (bl) YY_ST(MM, true); else YY_ST(MM, false); } while (0)
        if (M == 4) YY_STM(4);
        else if (M == 6) YY_STM(6);
        else if (M == 8) YY_STM(8);
        else if (M == 12) YY_STM(12);
        else YY_STM(16);
#undef YY_STM
#undef YY_ST
        return true;
    } else {
        const int n = d.np - k0;
        // uniform chunks of mc rows (last chunk >= 2 rows), P <= 64 lanes
        int mc = (n + 63) / 64;
        if (mc < 2) mc = 2;
        int P = (n + mc - 1) / mc;
        while (P > 1 && n - (P - 1) * mc < 2) {
            mc++;
            P = (n + mc - 1) / mc;
        }
        if (mc > 32 || P > 64) return false;
        const int64_t nlines = (int64_t)(d.nr - i0) * (d.nt - j0);
        const int V = s.tune.wpl[DIFF ? 4 : L];
        if ((V == 2 || V == 4 || V == 8) && n >= 64 * V) {
            // V waves per line: uniform chunks of mcv rows (last >= 2)
            int mcv = (n + 64 * V - 1) / (64 * V);
            if (mcv < 2) mcv = 2;
            int Pv = (n + mcv - 1) / mcv;
            while (Pv > 1 && n - (Pv - 1) * mcv < 2) {
                mcv++;
                Pv = (n + mcv - 1) / mcv;
            }
            if (mcv <= 12 && Pv <= 64 * V) {
                int64_t b = nlines;
                const int64_t cap = s.tune.sb[DIFF ? 4 : L][2] > 0 ? s.tune.sb[DIFF ? 4 : L][2] : SWEEP_BLOCKS;
                if (b > cap) b = cap;
                if (nblocks) *nblocks = (int)b;
                const int ldv = contig_pitch(n, Pv, mcv, (int)sizeof(R));
                const size_t lds = (size_t)4 * mcv * ldv * sizeof(R);
                const dim3 grid((unsigned)b, d.npatch), block(64 * V);
                const SweepArgs<R> sa{d, g, gd, s, x, y, s.cb, psi, partial, Pv, mcv, ldv};
#define YY_MW(MM) launch<KContigMw<R, L, MODE, DIFF, MM>>(grid, block, lds, st, sa)
                if (mcv <= 4) YY_MW(4);
                else if (mcv <= 6) YY_MW(6);
                else if (mcv <= 8) YY_MW(8);
                else YY_MW(12);
#undef YY_MW
                return true;
            }
        }
        const int ld = contig_pitch(n, P, mc, (int)sizeof(R));
        const size_t per_line = (size_t)4 * mc * ld * sizeof(R);
        int lpb = (int)(65536 / per_line);
        if (lpb > 4) lpb = 4;
        if (lpb < 1) return false;
        const int want = s.tune.lpb[DIFF ? 4 : L];
        if ((want == 1 || want == 2 || want == 4) && want < lpb) lpb = want;
        int64_t b = (nlines + lpb - 1) / lpb;
        const int64_t cap = s.tune.sb[DIFF ? 4 : L][2] > 0 ? s.tune.sb[DIFF ? 4 : L][2] : SWEEP_BLOCKS;
        if (b > cap) b = cap;
        if (nblocks) *nblocks = (int)b;
        const size_t lds = per_line * lpb;
        const dim3 grid((unsigned)b, d.npatch), block(64 * lpb);
        const SweepArgs<R> sa{d, g, gd, s, x, y, s.cb, psi, partial, P, mc, ld};
        if (mc <= 8) launch<KContig<R, L, MODE, DIFF, 8>>(grid, block, lds, st, sa);
        else if (mc <= 16) launch<KContig<R, L, MODE, DIFF, 16>>(grid, block, lds, st, sa);
        else if (mc <= 24) launch<KContig<R, L, MODE, DIFF, 24>>(grid, block, lds, st, sa);
        else launch<KContig<R, L, MODE, DIFF, 32>>(grid, block, lds, st, sa);
        return true;
    }
}

bool partitioned_on();
#if !defined(YY_ONLY_FLOAT)
static bool use_partitioned = true;
void set_partitioned(bool on) { use_partitioned = on; }
bool partitioned_on() { return use_partitioned; }
#endif

template <typename R, int L, int D, int MODE, int DIFF>
static void launch_sweep(const Dims &d, const Geo<R> &g, const Geo<double> &gd, const State<R> &s,
                         const R *x, R *y, R *psi, double *partial, int *nblocks, hipStream_t st)
{
    const int i0 = ulo<L>(0), j0 = ulo<L>(1), k0 = ulo<L>(2);
    const int nA = D == 0 ? d.nt - j0 : d.nr - i0;
    const int nB = D == 2 ? d.nt - j0 : d.np - k0;
    if (partitioned_on() && launch_partitioned<R, L, D, MODE, DIFF>(d, g, gd, s, x, y, psi, partial, nblocks, st))
        return;
    int64_t b = ((int64_t)nA * nB + 255) / 256;
    if (MODE == 1 && b > SWEEP_BLOCKS) b = SWEEP_BLOCKS;
    if (nblocks) *nblocks = (int)b;
    launch<KThomas<R, L, D, MODE, DIFF>>(dim3((unsigned)b, d.npatch), dim3(256), 0, st,
                                         SweepArgs<R>{d, g, gd, s, x, y, s.cb, psi, partial, 0, 0});
}

template <typename R, int L, int MODE>
static void sweep_dir(int dir, const Dims &d, const Geo<R> &g, const Geo<double> &gd,
                      const State<R> &s, const R *x, R *y, R *psi, double *partial, int *nb,
                      hipStream_t st)
{
    if (dir == 0) launch_sweep<R, L, 0, MODE, 0>(d, g, gd, s, x, y, psi, partial, nb, st);
    else if (dir == 1) launch_sweep<R, L, 1, MODE, 0>(d, g, gd, s, x, y, psi, partial, nb, st);
    else launch_sweep<R, L, 2, MODE, 0>(d, g, gd, s, x, y, psi, partial, nb, st);
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
    if (diffusion_only == 1) {
        if (dir == 0) launch_sweep<R, CC, 0, 0, 1>(d, g, gd, s, x, y, nullptr, nullptr, nullptr, st);
        else if (dir == 1) launch_sweep<R, CC, 1, 0, 1>(d, g, gd, s, x, y, nullptr, nullptr, nullptr, st);
        else launch_sweep<R, CC, 2, 0, 1>(d, g, gd, s, x, y, nullptr, nullptr, nullptr, st);
        return;
    }
    if (diffusion_only == 2) {
        // D_rr is the same in both metrics
        if (dir == 0) launch_sweep<R, CC, 0, 0, 1>(d, g, gd, s, x, y, nullptr, nullptr, nullptr, st);
        else if (dir == 1) launch_sweep<R, CC, 1, 0, 2>(d, g, gd, s, x, y, nullptr, nullptr, nullptr, st);
        else launch_sweep<R, CC, 2, 0, 2>(d, g, gd, s, x, y, nullptr, nullptr, nullptr, st);
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

// Resident blocks of a residual kernel on the whole device (blocks per CU
// from its registers and LDS, times the CU count), per location and tile
// kind (0..2: LDS tiles of 4, 8, 16 rows; 3: memory-read, 256 threads);
// 0 until prepare() has run, which then leaves every column whole.
template <typename R> struct ResSlots { static int v[4][4]; };
template <typename R> int ResSlots<R>::v[4][4] = {};

template <class K> static int device_slots(int threads, int cus)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_single<K>, threads, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb * cus;
}

template <typename R, int L> static void res_slots_of(int cus)
{
    ResSlots<R>::v[L][0] = device_slots<KResidualLds<R, L, 4>>(256, cus);
    ResSlots<R>::v[L][1] = device_slots<KResidualLds<R, L, 8>>(512, cus);
    ResSlots<R>::v[L][2] = device_slots<KResidualLds<R, L, 16>>(1024, cus);
    ResSlots<R>::v[L][3] = device_slots<KResidual<R, L>>(256, cus);
}

template <typename R> void Ops<R>::prepare()
{
    static const bool once = [] {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        res_slots_of<R, CC>(cus);
        res_slots_of<R, FR>(cus);
        res_slots_of<R, FT>(cus);
        res_slots_of<R, FP>(cus);
        return true;
    }();
    (void)once;
}

// Radial segments per column: blocks run in rounds of `slots`, and a last
// round that is partly empty leaves CUs idle for a whole block time.  Cost
// model: rounds x (points per segment + 2, the priming and pipeline fill of
// a segment); the fewest segments of least cost, at most 4.  forced > 0
// (tuning) overrides.
static int res_segments(int forced, int64_t blocks, int ni, int slots)
{
    if (forced > 0) return forced < ni ? forced : (ni > 0 ? ni : 1);
    if (slots <= 0 || ni < 8) return 1;
    int best = 1;
    double bc = 0.0;
    for (int ns = 1; ns <= 4 && ns <= ni / 4; ns++) {
        const int64_t rounds = (blocks * ns + slots - 1) / slots;
        const double c = (double)rounds * ((ni + ns - 1) / ns + 2);
        if (ns == 1 || c < bc) {
            bc = c;
            best = ns;
        }
    }
    return best;
}

template <typename R, int L>
void launch_res_lds(int cj, dim3 gr, dim3 bl, hipStream_t st, const ResArgs<R> &ra)
{
    if (cj == 4) launch<KResidualLds<R, L, 4>>(gr, bl, 0, st, ra);
    else if (cj == 8) launch<KResidualLds<R, L, 8>>(gr, bl, 0, st, ra);
    else launch<KResidualLds<R, L, 16>>(gr, bl, 0, st, ra);
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
    const int j0 = L == FT, k0 = L == FP;
    int ti = s.tune.rt[L];
    if (ti < 0 || ti >= N_RES_TILES) ti = 0;
    const ResTile &t = RES_TILES[ti];
    const int64_t ntile = col_blocks_t(d.nt - j0, d.np, t);
    const int kind = t.lds ? (t.cj == 4 ? 0 : t.cj == 8 ? 1 : 2) : 3;
    const int nseg = res_segments(s.tune.rseg[L], ntile * d.npatch, d.nr - (L == FR ? 1 : 0),
                                  ResSlots<R>::v[L][kind]);
    const dim3 gr((unsigned)(ntile * nseg), d.npatch), bl(t.ck, t.cj);
    const int jf = t.jfast;
    const ResArgs<R> ra{d, g, s, in, out, jf, nseg, (int)ntile};
    if (t.lds) {
        if (L == CC) launch_res_lds<R, CC>(t.cj, gr, bl, st, ra);
        else if (L == FR) launch_res_lds<R, FR>(t.cj, gr, bl, st, ra);
        else if (L == FT) launch_res_lds<R, FT>(t.cj, gr, bl, st, ra);
        else launch_res_lds<R, FP>(t.cj, gr, bl, st, ra);
        return;
    }
    if (L == CC) launch<KResidual<R, CC>>(gr, bl, 0, st, ra);
    else if (L == FR) launch<KResidual<R, FR>>(gr, bl, 0, st, ra);
    else if (L == FT) launch<KResidual<R, FT>>(gr, bl, 0, st, ra);
    else launch<KResidual<R, FP>>(gr, bl, 0, st, ra);
}

// ---------------------------------------------------------------------------
// a6: pressure (eq. nst_Mass1; bootstrapped form of eq. ac2), FP64:
//   p1^k = p1^n - Div_h u1^{n+1/2}/chi,
//   p2^k = p2^n + (p1^k - p1^n) - Div_h u2^{n+1/2}/chi,
// with the l2 norms of the increment and (system 2) of Div_h u2^k.
// ---------------------------------------------------------------------------
// Column-marching form: a thread owns one (patch, j, k) column and walks i
// upwards; the radial face value at i+1 is reused at the next i.
// With the pressure exchange on (nring > 0), the outermost nring cells in
// theta and phi take the other patch's pressure instead (Algorithm step 7):
// they are not updated and leave the increment norm; the divergence norm
// still covers every cell.
template <typename R>
struct PressArgs { Dims d; Geo<double> gd; State<R> s; int sys; double *pinc, *pdiv; int nring; };
template <typename R> struct KPressure {
    using Args = PressArgs<R>;
    static constexpr int bounds = 256;
    static constexpr bool xcd = true;
    static __device__ __forceinline__ void body(const Args &a, const Blk &blk)
    {
        const Dims &d = a.d;
        const Geo<double> &gd = a.gd;
        const State<R> &s = a.s;
        const int sys = a.sys, nring = a.nring;
        double *pinc = a.pinc, *pdiv = a.pdiv;

    unsigned bx, by;
    bx = blk.x;
    by = blk.y;
    const int p = d.p0 + (int)by;
    const int y = sys - 1;
    double ai = 0.0, ad = 0.0;
    const unsigned ntile = (unsigned)col_blocks(d.nt, d.np);
    for (unsigned tile = bx; tile < ntile; tile += blk.nx) {
        int j, k;
        if (!col_of(tile, d.nt, d.np, 0, 0, j, k)) continue;
        const uint32_t sI = (uint32_t)d.sI, sJ = (uint32_t)d.sJ;
        const FV<R> rn(s.u[y][0][0]), tn(s.u[y][1][0]), pn(s.u[y][2][0]);
        const FV<R> rk(s.u[y][0][2]), tk(s.u[y][1][2]), pk(s.u[y][2][2]);
        const FV<double> pyn(s.p[y][0]), pyk(s.p[y][1]), p1n(s.p[0][0]), p1k(s.p[0][1]);
        const double dtp = gd.dt_p[j + 1], dtm = gd.dt_m[j + 1], dpc = gd.dp_c[j + 1];
        const double wj = gd.sc[j + 1] * gd.dr * gd.dth * gd.dph;
        const bool upd = !(j < nring || j >= d.nt - nring || k < nring || k >= d.np - nring);
        uint32_t q = (uint32_t)ix(d, p, 0, j, k);
        double rn0 = (double)rn[q], rk0 = (double)rk[q];
        for (int i = 0; i < d.nr; i++, q += sI) {
            // Div_h of u^n and u^k at the centre (i, j, k)
            const double rn1 = (double)rn[q + sI], rk1 = (double)rk[q + sI];
            const double drp = gd.dr_p[i + 1], drm = gd.dr_m[i + 1], ir = gd.ir_c[i + 1];
            const double dn = (drp * rn1 - drm * rn0) +
                              ir * ((dtp * (double)tn[q + sJ] - dtm * (double)tn[q]) +
                                    dpc * ((double)pn[q + 1] - (double)pn[q]));
            const double dk = (drp * rk1 - drm * rk0) +
                              ir * ((dtp * (double)tk[q + sJ] - dtm * (double)tk[q]) +
                                    dpc * ((double)pk[q + 1] - (double)pk[q]));
            rn0 = rn1;
            rk0 = rk1;
            const double rc = gd.rc[i + 1];
            const double w = rc * rc * wj;
            if (upd) {
                double nv = pyn[q] - 0.5 * (dn + dk) * gd.inv_chi;
                if (sys == 2) nv += p1k[q] - p1n[q];
                const double inc = nv - pyk[q];
                st(s.p[y][1], q, nv);
                ai += w * inc * inc;
            }
            if (sys == 2) ad += w * dk * dk;
        }
    }
    const double ti = block_sum(ai);
    const double td = block_sum(ad);
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        pinc[p * NBMAX + bx] = ti;
        if (sys == 2) pdiv[p * NBMAX + bx] = td;
    }
    }
};

template <typename R>
void Ops<R>::pressure(const Dims &d, const Geo<R> &g, const Geo<double> &gd, const State<R> &s,
                      int sys, double *pinc, double *pdiv, int *nb, int nring, hipStream_t st)
{
    (void)g;
    int64_t b = col_blocks(d.nt, d.np);        // one thread per (j, k) column
    if (b > NBMAX) b = NBMAX;                   // then blocks loop over tiles
    *nb = (int)b;
    launch<KPressure<R>>(dim3((unsigned)b, d.npatch), dim3(COL_K, COL_J), 0, st,
                         PressArgs<R>{d, gd, s, sys, pinc, pdiv, nring});
}

// ---------------------------------------------------------------------------
// Algorithm step 7 (Sec. 4): the pressure of a patch's outermost cells is
// interpolated from the other patch (cubic Lagrange at the same radial
// index, as every boundary value).  Every target of the launched patches
// is gathered into tmp first ([patch][i][target]) and written afterwards,
// so in the additive mode each patch reads the other's values as its
// pressure update left them (ring cells are donors of the other patch's
// ring).  Thread = (target, radial index).
// ---------------------------------------------------------------------------
#if !defined(YY_ONLY_FLOAT)
__global__ void k_pring_gather(Dims d, const FillScalar *__restrict__ tab, int ntab, const double *a,
                               double *tmp)
{
    const int p = d.p0 + (int)blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntab * d.nr) return;
    const int e = t % ntab, i = t / ntab;
    const FillScalar &f = tab[e];
    tmp[(int64_t)p * ntab * d.nr + t] = gather16(a, ix(d, 1 - p, i, f.dj, f.dk), d.sJ, f.wt, f.wp);
}
#endif

#if !defined(YY_ONLY_FLOAT)
__global__ void k_pring_scatter(Dims d, const FillScalar *__restrict__ tab, int ntab, double *a,
                                const double *tmp)
{
    const int p = d.p0 + (int)blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntab * d.nr) return;
    const int e = t % ntab, i = t / ntab;
    const FillScalar &f = tab[e];
    a[ix(d, p, i, f.tj, f.tk)] = tmp[(int64_t)p * ntab * d.nr + t];
}
#endif

#if !defined(YY_ONLY_FLOAT)
void pressure_exchange(const Dims &d, double *p, const FillScalar *tab, int ntab, double *tmp,
                       hipStream_t st)
{
    if (LaunchRecorder *r = launch_recorder()) {
        r->foreign = true;
        return;
    }
    const int n = ntab * d.nr;
    const dim3 g((unsigned)((n + 255) / 256), (unsigned)d.npatch);
    hipLaunchKernelGGL(k_pring_gather, g, dim3(256), 0, st, d, tab, ntab, (const double *)p, tmp);
    hipLaunchKernelGGL(k_pring_scatter, g, dim3(256), 0, st, d, tab, ntab, p, (const double *)tmp);
}
#endif

// ---------------------------------------------------------------------------
// norms: fixed-order reduction of the per-block partial sums
// ---------------------------------------------------------------------------
struct NB { int n[NSLOT]; };

struct ReduceArgs { const double *partial; NB nb; double *out; };
struct KReduce {
    using Args = ReduceArgs;
    static constexpr int bounds = 1024;
    static constexpr bool xcd = false;
    static __device__ __forceinline__ void body(const Args &a, const Blk &blk)
    {
        const double *partial = a.partial;
        const NB &nb = a.nb;
        double *out = a.out;

    const int slot = blk.x >> 1, p = blk.x & 1;
    const double *src = partial + (int64_t)(slot * 2 + p) * NBMAX;
    double v = 0.0;
    for (int b = threadIdx.x; b < nb.n[slot]; b += blockDim.x) v += src[b];
    const double t = block_sum(v);
    if (threadIdx.x == 0) out[p * NSLOT + slot] = sqrt(t);
    }
};

#if !defined(YY_ONLY_FLOAT)
void reduce_norms(const double *partial, const int *nblocks, double *out, hipStream_t st)
{
    NB nb;
    for (int q = 0; q < NSLOT; q++) nb.n[q] = nblocks[q];
    launch<KReduce>(dim3(2 * NSLOT), dim3(1024), 0, st, ReduceArgs{partial, nb, out});
}
#endif

#if !defined(YY_ONLY_FLOAT)
__global__ void k_zero(double *p, int64_t n)
{
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x)
        p[q] = 0.0;
}
#endif

#if !defined(YY_ONLY_FLOAT)
void zero_doubles(double *p, int64_t n, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero, dim3(grid_for(n)), dim3(256), 0, st, p, n);
}
#endif

// ---------------------------------------------------------------------------
// plain streaming copy in 16-byte words (the HBM ceiling a streaming kernel
// reaches on this part: every word read once and written once)
// ---------------------------------------------------------------------------
#if !defined(YY_ONLY_FLOAT)
// block b copies the 16 KiB chunk [1024 b, 1024 b + 1024) of 16-byte words,
// four coalesced words per thread, all loads in flight before the stores
__global__ void __launch_bounds__(256) k_stream_copy(uint4 *__restrict__ dst, const uint4 *__restrict__ src,
                                                     int64_t n)
{
    const int64_t q = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    if (q + 768 < n) {
        const uint4 a = src[q], b = src[q + 256], c = src[q + 512], e = src[q + 768];
        dst[q] = a;
        dst[q + 256] = b;
        dst[q + 512] = c;
        dst[q + 768] = e;
    } else {
        for (int64_t r = q; r < n && r < q + 1024; r += 256) dst[r] = src[r];
    }
}

void stream_copy(void *dst, const void *src, int64_t words16, hipStream_t st)
{
    const int64_t blocks = (words16 + 1023) / 1024;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, st, (uint4 *)dst, (const uint4 *)src,
                       words16);
}
#endif

// ---------------------------------------------------------------------------
// field I/O: MAC or padded double arrays <-> internal layout
// ---------------------------------------------------------------------------
template <typename TT>
__global__ void k_io(Dims d, TT *in, const double *src, double *dst, int loc, int layout, const double *prof)
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
        const double b = prof ? prof[i + 1] : 0.0;
        if (src) in[q] = (TT)(src[t] - b);
        else dst[t] = (double)in[q] + b;
    }
}

template <typename TT> __global__ void k_add_profile(Dims d, TT *a, const double *prof)
{
    const int nk = d.np + 2, nj = d.nt + 2, ni = d.nr + 2;
    const int64_t n = 2LL * ni * nj * nk;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(t % nk) - 1, j = (int)((t / nk) % nj) - 1, i = (int)((t / ((int64_t)nk * nj)) % ni) - 1;
        const int p = (int)(t / ((int64_t)nk * nj * ni));
        const int64_t q = ix(d, p, i, j, k);
        a[q] = (TT)((double)a[q] + prof[i + 1]);
    }
}

template <typename R>
void Ops<R>::io(const Dims &d, R *internal, const double *src, double *dst, int loc, int layout,
                const double *prof, hipStream_t st)
{
    const int64_t n = 2LL * (d.nr + 2) * (d.nt + 2) * (d.np + 2);
    hipLaunchKernelGGL(k_io<R>, dim3(grid_for(n)), dim3(256), 0, st, d, internal, src, dst, loc, layout, prof);
}

template <typename R> void Ops<R>::add_profile(const Dims &d, R *a, const double *prof, hipStream_t st)
{
    const int64_t n = 2LL * (d.nr + 2) * (d.nt + 2) * (d.np + 2);
    hipLaunchKernelGGL(k_add_profile<R>, dim3(grid_for(n)), dim3(256), 0, st, d, a, prof);
}

#if !defined(YY_ONLY_FLOAT)
void io_double(const Dims &d, double *internal, const double *src, double *dst, int loc, int layout,
               hipStream_t st)
{
    const int64_t n = 2LL * (d.nr + 2) * (d.nt + 2) * (d.np + 2);
    hipLaunchKernelGGL(k_io<double>, dim3(grid_for(n)), dim3(256), 0, st, d, internal, src, dst, loc, layout,
                       (const double *)nullptr);
}
#endif

// ---------------------------------------------------------------------------
// Algorithm step 4 (mass-flux correction of the interpolated boundary data).
// The net outward flux F of a patch's boundary normal data -- u_r on the
// wall faces (Dirichlet data), u_theta on the theta-boundary faces and u_phi
// on the phi-boundary faces (interpolated) -- with the face areas of Div_h
// as weights (r-face r_f^2 sin(theta_j) dtheta dphi, theta-face r_i
// sin(theta_f) dr dphi, phi-face r_i dr dtheta) is removed by the least
// change of the interpolated faces: v = u - (F / S) a, a = outward weights,
// S = a.a.  This is the minimiser of the paper's functional J (quadratic,
// Hessian I + c a a^T, so its conjugate-gradient iteration ends there) in
// the limit of its penalty parameter going to zero.
// ---------------------------------------------------------------------------
struct MfFace {
    int kind, i, j, k;   // 0: r-wall, 1: theta-boundary, 2: phi-boundary face
    double w;            // outward flux weight
};

__device__ __forceinline__ MfFace mf_face(const Dims &d, const Geo<double> &g, int64_t t)
{
    MfFace f;
    const int64_t nA = 2 * (int64_t)d.nt * d.np, nB = 2 * (int64_t)d.nr * d.np;
    if (t < nA) {
        const int side = (int)(t / ((int64_t)d.nt * d.np));
        const int64_t u = t % ((int64_t)d.nt * d.np);
        f.kind = 0; f.j = (int)(u / d.np); f.k = (int)(u % d.np); f.i = side ? d.nr : 0;
        const double rf = g.rf[f.i + 1];
        f.w = (side ? 1.0 : -1.0) * rf * rf * g.sc[f.j + 1] * g.dth * g.dph;
    } else if (t < nA + nB) {
        t -= nA;
        const int side = (int)(t / ((int64_t)d.nr * d.np));
        const int64_t u = t % ((int64_t)d.nr * d.np);
        f.kind = 1; f.i = (int)(u / d.np); f.k = (int)(u % d.np); f.j = side ? d.nt : 0;
        f.w = (side ? 1.0 : -1.0) * g.rc[f.i + 1] * g.sf[f.j + 1] * g.dr * g.dph;
    } else {
        t -= nA + nB;
        const int side = (int)(t / ((int64_t)d.nr * d.nt));
        const int64_t u = t % ((int64_t)d.nr * d.nt);
        f.kind = 2; f.i = (int)(u / d.nt); f.j = (int)(u % d.nt); f.k = side ? d.np : 0;
        f.w = (side ? 1.0 : -1.0) * g.rc[f.i + 1] * g.dr * g.dth;
    }
    return f;
}

__device__ __forceinline__ int64_t mf_count(const Dims &d)
{
    return 2 * ((int64_t)d.nt * d.np + (int64_t)d.nr * d.np + (int64_t)d.nr * d.nt);
}

// blockIdx.y = patch, blockIdx.z = system: partial net fluxes
template <typename R>
__global__ void __launch_bounds__(256) k_mflux(Dims d, Geo<double> g, State<R> s, int lev, double *partial,
                                               int pmask)
{
    const int p = blockIdx.y, y = blockIdx.z;
    if (!((pmask >> p) & 1)) return;
    const R *ur = s.u[y][0][lev], *ut = s.u[y][1][lev], *up = s.u[y][2][lev];
    const int64_t n = mf_count(d);
    double acc = 0.0;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const MfFace f = mf_face(d, g, t);
        const R *a = f.kind == 0 ? ur : (f.kind == 1 ? ut : up);
        acc += f.w * (double)a[ix(d, p, f.i, f.j, f.k)];
    }
    const double tot = block_sum(acc);
    if (threadIdx.x == 0) partial[(y * 2 + p) * MF_BLOCKS + blockIdx.x] = tot;
}

// every block sums the partials (fixed order), then corrects its faces
template <typename R>
__global__ void __launch_bounds__(256) k_mfix(Dims d, Geo<double> g, State<R> s, int lev, double S,
                                              double tol, const double *partial, int pmask)
{
    const int p = blockIdx.y, y = blockIdx.z;
    if (!((pmask >> p) & 1)) return;
    __shared__ double kap;
    if (threadIdx.x < 64) {
        double v = 0.0;
        for (int b = threadIdx.x; b < MF_BLOCKS; b += 64) v += partial[(y * 2 + p) * MF_BLOCKS + b];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (threadIdx.x == 0) kap = fabs(v) < tol ? 0.0 : v / S;
    }
    __syncthreads();
    R *ut = s.u[y][1][lev], *up = s.u[y][2][lev];
    const int64_t nA = 2 * (int64_t)d.nt * d.np, n = mf_count(d);
    for (int64_t t = nA + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const MfFace f = mf_face(d, g, t);
        R *a = f.kind == 1 ? ut : up;
        const int64_t q = ix(d, p, f.i, f.j, f.k);
        a[q] = (R)((double)a[q] - kap * f.w);
    }
}

template <typename R>
void Ops<R>::mass_fix(const Dims &d, const Geo<double> &gd, const State<R> &s, int lev, double S, double tol,
                      double *partial, int pmask, hipStream_t st)
{
    if (LaunchRecorder *r = launch_recorder()) {
        r->foreign = true;
        return;
    }
    const dim3 g(MF_BLOCKS, 2, 2);
    hipLaunchKernelGGL(k_mflux<R>, g, dim3(256), 0, st, d, gd, s, lev, partial, pmask);
    hipLaunchKernelGGL(k_mfix<R>, dim3(64, 2, 2), dim3(256), 0, st, d, gd, s, lev, S, tol,
                       (const double *)partial, pmask);
}

#if !defined(YY_ONLY_FLOAT)
template struct Ops<double>;
#endif
#if !defined(YY_ONLY_DOUBLE)
template struct Ops<float>;
#endif

}  // namespace yy

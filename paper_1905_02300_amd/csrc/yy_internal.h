// yy_internal.h -- types shared by the host orchestrator and the gfx950
// kernels of libyy.so (not part of the public ABI).
//
// Device layout of every field: [patch][i][j][k] with one ghost layer,
// logical index -1..N per direction, k (phi) fastest; face f of a
// face-located field at logical f.  Within a row, k = 0 sits at element ko
// (16 FP64 or 32 FP32 elements: 128 bytes), the ghost k = -1 just before
// it, and the row pitch is a multiple of 128 bytes, so the unknowns of
// every row start on an L2 line.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <vector>

namespace yy {

enum Loc { CC = 0, FR = 1, FT = 2, FP = 3 };   // centre, r-, theta-, phi-face

struct Dims {
    int nr, nt, np;
    int64_t sJ, sI, sP;      // element strides of j, i and patch (k: 1)
    int p0, npatch;          // patches a launch covers: p0 .. p0+npatch-1
    int ko;                  // element of k = 0 within a row
};

__host__ __device__ inline int64_t ix(const Dims &d, int p, int i, int j, int k)
{
    return (int64_t)p * d.sP + (int64_t)(i + 1) * d.sI + (int64_t)(j + 1) * d.sJ + (k + d.ko);
}

// element of k = 0 and row pitch of the layout (FP64 or FP32-mixed; the FP64
// pressures of FP32-mixed share the FP32 indexing)
__host__ __device__ inline int row_origin(int elem_bytes) { return 128 / elem_bytes; }
__host__ __device__ inline int64_t row_pitch(int np, int elem_bytes)
{
    const int64_t a = 128 / elem_bytes;
    return (np + 1 + row_origin(elem_bytes) + a - 1) / a * a;
}

// Pointer to a read-only table.  Device reads go through the constant
// address space: the tables are never written while a kernel runs, so the
// compiler may use scalar loads where the index is wave-uniform (an r-table
// indexed by the marching radial index) and may hoist loop-invariant reads
// past stores to the fields.
template <typename R> struct CPtr {
    const R *p;
    __host__ __device__ CPtr &operator=(const R *q) { p = q; return *this; }
    __host__ __device__ operator const R *() const { return p; }
    __device__ __forceinline__ R operator[](int64_t i) const
    {
        return ((const __attribute__((address_space(4))) R *)p)[i];
    }
};

// metric tables and grid constants in compute precision R
template <typename R> struct Geo {
    CPtr<R> rc;     // r at centres, index i+1, i = -1..nr
    CPtr<R> rf;    // r at faces, index f+1, f = -1..nr+1
    CPtr<R> sc, cc;   // sin, cos theta at centres, index j+1, j = -1..nt
    CPtr<R> sf, cf;   // sin, cos theta at faces, index f+1, f = -1..nt+1
    R dr, dth, dph, r1;
    R cphat;        // 1 / (R1^2 sin^2(theta_1) dphi^2), theta_1 = pi/4 - d
    R ht, tau, inv_tau;
    R pr, ic, prra; // Pr, 1/(2 chi), Pr*Ra
    double inv_chi, prra_d;
    // Coefficient tables of the split operators (unit viscosity, built in
    // FP64 on the host), index i+1 / f+1 / j+1 as above; they replace the
    // per-point divisions of the metric factors.
    CPtr<R> ir_c, ir_f, ir2_c, ir2_f;   // 1/r, 1/r^2 at r-centres, r-faces
    CPtr<R> rc_lo, rc_up;                 // D_rr at r-centres
    CPtr<R> rf_lo, rf_up, rf_di;         // u_r radial viscous operator at r-faces
    CPtr<R> gf_lo, gf_up, gf_di;         // D11 at r-faces
    CPtr<R> tc_lo, tc_up;                 // Dhat_thth at theta-centres
    CPtr<R> tf_lo, tf_up;                 // Dhat_thth at theta-faces
    CPtr<R> ef_lo, ef_up, ef_di;         // u_theta extra viscous terms (x 1/r^2)
    CPtr<R> gt_lo, gt_up, gt_di;         // D22 at theta-faces (x 1/r^2)
    CPtr<R> h2p_c, h2p_f;                 // 1/(2 sin(theta) dphi), centres / faces
    CPtr<R> is2_c, is2_f;                 // 1/sin^2(theta), centres / faces
    CPtr<R> cot_c;                         // cot(theta) at centres
    CPtr<R> dr_p, dr_m;                   // Div_r at r-centre i: rf(i+1)^2, rf(i)^2 over rc^2 dr
    CPtr<R> dt_p, dt_m, dp_c;            // Div_th at theta-centre j (x 1/r); 1/(sin dphi)
    CPtr<R> cot_f, is_c;                  // cot(theta) at faces, 1/sin(theta) at centres
    R h2r, h2t, idph2;                      // 1/(2 dr), 1/(2 dtheta), 1/dphi^2
    R idr, idth, idph, r12;                 // 1/dr, 1/dtheta, 1/dphi, R1^2
    // parameter-dependent combinations (rebuilt when Pr or chi change):
    // Pr * rf_* + ic * gf_* (u_r radial operator) and Pr * ef_* + ic * gt_*
    CPtr<R> fr_lo, fr_up, fr_di, ft_lo, ft_up, ft_di;
    // wall rules of the correction, c_ghost = -rho c_in (1: Dirichlet): T,
    // and the tangential velocity
    R rho_t[2];
    R rho_u[2];
    // FP32-mixed stores T as its deviation T - Tref from the discrete
    // conductive profile Tref(r) of the wall temperatures (tdev = 1): Tref
    // at centres (FP64, index i+1, i = -1..nr) and its centred radial
    // difference (Tref(i+1) - Tref(i-1)) / (2 dr); FP64 keeps T itself
    // (tdev = 0, tables zero)
    int tdev;
    CPtr<double> tref;
    CPtr<R> dtref;
};

// T's Robin walls a T + b dT/dn = g: ghost = cg g - rho T_in (Dirichlet:
// cg = 2, rho = 1)
struct TRobin {
    double cg[2], rho[2];
    // deviation storage of T (FP32-mixed): the ghost of T - Tref is
    // cg g - shift - rho (T - Tref)_in with shift = rho Tref_in + Tref_ghost
    double shift[2];
};
// Robin walls of the tangential velocity a u + b R dn(u/r) = g: ghost =
// cg g - rho u_in (Dirichlet: cg = 2, rho = 1)
struct URobin {
    double cg[2], rho[2];
};
constexpr int NTAB_R = 14;   // per-r coefficient tables (length nr+3)
constexpr int NTAB_T = 20;   // per-theta coefficient tables (length nt+3)

// one interpolation target of a scalar (centre-type in theta and phi)
struct FillScalar {
    int32_t tj, tk;          // target (logical j, k)
    int32_t dj, dk;          // donor window start (logical j, k) in the other patch
    double wt[4], wp[4];     // cubic Lagrange weights along theta, phi
};

// one interpolation target of a tangential velocity component: both of the
// other patch's components are interpolated (each on its own staggered
// grid) and rotated: value = ma * u_theta~ + mb * u_phi~
struct FillVector {
    int32_t tj, tk;
    int32_t tjA, tkA;        // window on the theta-face grid
    int32_t tjB, tkB;        // window on the phi-face grid
    double wtA[4], wpA[4], wtB[4], wpB[4];
    double ma, mb;
};

// line-solver tile choices per location (CC, FR, FT, FP, and 4 for the
// diffusion-only solves of the line-solve workload); 0 = built-in
// default.  Strided r/theta sweeps: rows per chunk m (4, 6, 8, 12, 16; 1 =
// the per-line Thomas kernel), the largest lane width w (64, 32, 16) and
// bl (1: all loads of a chunk issued together); phi sweeps: one wave per
// line and lines per block lpb (1, 2, 4), or wpl (2, 4, 8) waves per line.
struct Tune {
    int8_t m[5][2], w[5][2], bl[5][2], lpb[5], wpl[5];   // [4]: the diffusion-only line solves
    int8_t rt[4];            // residual column tile per location (index into RES_TILES)
    int8_t rseg[4];          // radial segments per residual column (0: chosen from the occupancy)
    int16_t sb[5][3];        // blocks per patch of each partitioned line solve (0: SWEEP_BLOCKS)
};

// Column tiles of the residual kernels: (k extent, j extent) of a block
// and the order in which consecutive blocks take tiles (k-tiles fastest, or
// j-tiles fastest so that blocks sharing theta-halo rows run together);
// lds: the neighbours are staged in LDS planes (64 x cj threads), else read
// from memory (256 threads).  Index 0 is the default.
struct ResTile { int ck, cj, jfast, lds; const char *name; };
constexpr int N_RES_TILES = 12;
constexpr ResTile RES_TILES[N_RES_TILES] = {
    {64, 4, 0, 0, "64x4k"}, {64, 4, 1, 0, "64x4j"}, {128, 2, 1, 0, "128x2j"}, {256, 1, 1, 0, "256x1j"},
    {128, 2, 0, 0, "128x2k"}, {32, 8, 1, 0, "32x8j"}, {32, 8, 0, 0, "32x8k"}, {16, 16, 0, 0, "16x16k"},
    {64, 4, 0, 1, "lds64x4k"}, {64, 8, 0, 1, "lds64x8k"}, {64, 8, 1, 1, "lds64x8j"}, {64, 16, 0, 1, "lds64x16k"}};

// pointers of one step (compute precision R; pressures double)
template <typename R> struct State {
    Tune tune;
    R *T[3];                 // levels n, n-1, working iterate k
    R *Ts;                   // T*
    R *u[2][3][3];           // [system][component r,t,p][level]
    R *us[2][3];             // [system][component] extrapolated
    double *p[2][2];         // [system][level n, working]
    R *force[4];             // T, u_r, u_t, u_p forcing (or null)
    R *res;                  // residual / sweep buffer
    R *cb;                   // Thomas scratch (c')
};

// Dirichlet wall data of one level: T, u_r, u_theta, u_phi x (wall at R1,
// wall at R2), each [patch][j+1][k+1] doubles at the field's own (theta,
// phi) positions, or null (T = the constant wall temperature, u = 0)
struct WallLev {
    const double *v[4][2];
};

constexpr int MF_BLOCKS = 128;       // partial sums per (system, patch) of the mass-flux step
constexpr int NBMAX = 16384;     // partial-sum slots per patch (grid limit of norm launches)
constexpr int SWEEP_BLOCKS = 1024;   // blocks per patch of a sweep (each loops over its tasks)
constexpr int NSLOT = 10;        // norm slots
constexpr int NRING_MAX = 8;     // rings of the pressure exchange

// Step scratch held in a static device array (yy_step_static): the
// residual/correction buffer and the Thomas scratch (each at most
// STATIC_FIELD_BYTES), the norm partial sums and the mass-flux partials.
constexpr int64_t STATIC_FIELD_BYTES = (int64_t)32 << 20;
constexpr int64_t STATIC_PARTIAL_BYTES = (int64_t)NSLOT * 2 * NBMAX * 8;
constexpr int64_t STATIC_MF_BYTES = (int64_t)4 * MF_BLOCKS * 8;
constexpr int64_t STATIC_SCRATCH_BYTES = 2 * STATIC_FIELD_BYTES + STATIC_PARTIAL_BYTES + STATIC_MF_BYTES;

// ---- batched launches (ensembles) ----

// shell q of a batched launch owns the logical blocks [off, off + nx ny) of
// its 1-D grid, which it sees as a grid of nx x ny blocks
// one shell's part of a batched launch: blocks [off, off + padded) of the
// 1-D grid (off and padded multiples of 8), of which the first nx*ny are
// the shell's grid nx x ny
struct BatchEnt {
    int32_t off, nx, ny, padded;
};

// While installed (set_launch_recorder), every kernel launch of the step is
// recorded instead of issued: the batched twin of the kernel (taking a
// device table of argument structs and a BatchEnt table), the shell's grid,
// block and LDS bytes, and its argument struct.
struct LaunchRec {
    const void *multi;       // k_multi<K> instance
    dim3 grid, block;
    size_t lds;
    size_t arg_off, arg_size;   // the argument struct in LaunchRecorder::args
};
struct LaunchRecorder {
    std::vector<LaunchRec> recs;
    std::vector<unsigned char> args;
    bool foreign = false;    // a launch with no batched twin was asked for (and skipped)
    void push(const void *multi, dim3 grid, dim3 block, size_t lds, const void *a, size_t n)
    {
        LaunchRec r{multi, grid, block, lds, args.size(), n};
        const unsigned char *b = (const unsigned char *)a;
        args.insert(args.end(), b, b + n);
        recs.push_back(r);
    }
};
void set_launch_recorder(LaunchRecorder *r);
LaunchRecorder *launch_recorder();

// ---- launchers (yy_kernels.hip) ----
template <typename R> struct Ops {
    // host queries the launchers use (the residuals' resident blocks per
    // device); once per process, outside any stream capture
    static void prepare();
    static void extrap(const Dims &d, const State<R> &s, hipStream_t st);
    // extrap, and the working level k = level n (fields and pressures)
    static void extrap_copy(const Dims &d, const State<R> &s, hipStream_t st);
    static void fill(const Dims &d, const State<R> &s, int level, const FillScalar *cc, int ncc,
                     const FillVector *vt, int nvt, const FillVector *vp, int nvp,
                     double t_in, double t_out, const TRobin &tb, const URobin &ub, const WallLev &walls,
                     int patch_mask, hipStream_t st);
    static void residual(const Dims &d, const Geo<R> &g, const State<R> &s, int field, R *out,
                         hipStream_t st);
    // one sweep; mode 0: y = solve(x); mode 1: psi_k += solve(x) and norm
    static void sweep(const Dims &d, const Geo<R> &g, const Geo<double> &gd, const State<R> &s,
                      int field, int dir, const R *x, R *y, int mode, double *partial,
                      int *nblocks, int diffusion_only, hipStream_t st);
    // nring > 0: the outermost nring cells are left to the pressure exchange
    static void pressure(const Dims &d, const Geo<R> &g, const Geo<double> &gd, const State<R> &s,
                         int sys, double *partial_inc, double *partial_div, int *nblocks, int nring,
                         hipStream_t st);
    // prof (or null): a radial profile (index i+1, i = -1..nr) subtracted
    // on the way in and added on the way out (T's deviation storage)
    static void io(const Dims &d, R *internal, const double *ext, double *ext_out, int field_loc,
                   int layout, const double *prof, hipStream_t st);
    // a[i][j][k] += prof[i+1] over the whole padded array (both patches)
    static void add_profile(const Dims &d, R *a, const double *prof, hipStream_t st);
    // Algorithm step 4 on a filled velocity level: make each patch's boundary
    // normal data carry no net mass flux (both systems); partial: 4 * MF_BLOCKS
    // doubles of scratch; S = sum of the squared boundary flux weights plus
    // eps |dOmega|^2; patches whose |net flux| is below tol are left alone
    static void mass_fix(const Dims &d, const Geo<double> &gd, const State<R> &s, int level,
                         double S, double tol, double *partial, int patch_mask, hipStream_t st);
};
void io_double(const Dims &d, double *internal, const double *ext, double *ext_out, int field_loc,
               int layout, hipStream_t st);
void reduce_norms(const double *partial, const int *nblocks_dev, double *out, hipStream_t st);
// Algorithm step 7: the ring targets tab[0..ntab) of the launched patches
// (d.p0, d.npatch) take the other patch's interpolated pressure p; tmp
// holds 2 * ntab * nr doubles
void pressure_exchange(const Dims &d, double *p, const FillScalar *tab, int ntab, double *tmp,
                       hipStream_t st);
void zero_doubles(double *p, int64_t n, hipStream_t st);
void stream_copy(void *dst, const void *src, int64_t words16, hipStream_t st);
int contig_pitch(int n, int P, int mc, int elem_bytes);
// choose the register-resident partitioned line solver (default) or the
// per-line Thomas kernel
void set_partitioned(bool on);
// block shape of a strided partitioned solve (lines of n, chunks <= M rows,
// at most wmax lanes); false if it does not fit
bool strided_tile(int n, int M, int wmax, int &W, int &P);

}  // namespace yy

struct yy_shell;
namespace yy {
// yy_step with the step's scratch arrays taken from `scratch` (device
// memory of `cap` bytes, 256-byte aligned) instead of the workspace
// (yy_host.cpp)
int step_with_scratch(yy_shell *s, int K, char *scratch, int64_t cap, hipStream_t st);
}  // namespace yy

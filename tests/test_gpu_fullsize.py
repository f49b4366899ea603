"""GPU checks at the benchmarked sizes, in the launch configuration
bench.py times (autotuned tiles).

The 64x192x576 line-solve workload and two steps of the benchmark's
convection workload on 2x64x192x576 (with the benchmark's tile set) are
compared element by element with the oracle.  At 2x128x384x1152 the oracle
needs minutes per step (bench.py --parity-oracle covers it), so the tests
check properties that hold at any size: the
discrete conductive state is steady, and identical data on the two patches
stays bitwise identical (the Yin-Yang construction treats both alike).
"""
import numpy as np
import pytest

from paper_1905_02300_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def yy():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1905_02300_amd import yy as mod
    mod.load()
    return mod


@pytest.mark.parametrize("prec", [0, 1])
def test_line_solve_64x192x576(oracle_lib, yy, prec):
    """(I - tau/2 Pr D) y = x along r, theta, phi on both patches, RHS
    uniform[-1,1] (seed 2), tau = 1e-3, Pr = 1, with the split (hat) and the
    true metric (FP64 at 1e-12; FP32 at the rounding of its inputs, 1e-5)."""
    print(f"case: line solve 64x192x576 prec {prec}", flush=True)
    g = I.Grid(64, 192, 576)
    o = oracle_lib.Shell(64, 192, 576)
    o.set_params(pr=1.0, tau=1e-3)
    o.extrapolate()
    s = yy.Shell(64, 192, 576, prec=prec)
    s.set_params(pr=1.0, dt=1e-3)
    s.autotune()
    x = I.line_rhs(g, seed=2)
    m = np.zeros(x.shape, bool)
    m[:, 1:-1, 1:-1, 1:-1] = True
    tol = 1e-12 if prec == 0 else 1e-5
    ops = [[oracle_lib.OP_DRR, oracle_lib.OP_DTT_HAT, oracle_lib.OP_DPP_HAT],
           [oracle_lib.OP_DRR, oracle_lib.OP_DTT, oracle_lib.OP_DPP]]
    for metric in (0, 1):
        for d in range(3):
            if metric == 1 and d == 0:
                continue                 # D_rr is the same in both metrics
            ref = o.sweep_op(ops[metric][d], x)
            yt = s.internal_tensor()
            s.sweep_diffusion(d, s.to_internal(x), yt, metric=metric)
            got = s.from_internal(yt).double().cpu().numpy()
            err = np.max(np.abs(got[m] - ref[m])) / np.max(np.abs(ref[m]))
            print(f"  metric {metric} dir {d}: relative error {err:.2e}", flush=True)
            assert err <= tol


# the tiles the autotuner chose for the FP64 step on 2x128x384x1152 in the
# benchmark's driver run (lane widths shrink to fit where a line is shorter)
BENCH_TILES = ('{"T.r":"m8w16b","T.t":"m6w32b","T.p":"v4","u_r.r":"m4w32b","u_r.t":"m12w16",'
               '"u_r.p":"v4","u_t.r":"m8w16b","u_t.t":"t","u_t.p":"v4","u_p.r":"m8w16",'
               '"u_p.t":"m6w32b","u_p.p":"v4","D.r":"m8w16b","D.t":"m6w16b","D.p":"v4"}')


# the tiles the autotuner chose for the same workload with the LDS-staged
# residual tiles available (theta/phi neighbours staged in LDS planes)
BENCH_TILES_LDS = ('{"T.r":"m8w16b","T.t":"m12w32","T.p":"v4","u_r.r":"m8w16b","u_r.t":"m12w16",'
                   '"u_r.p":"v4","u_t.r":"m8w16","u_t.t":"m6w16","u_t.p":"v4","u_p.r":"m8w16b",'
                   '"u_p.t":"m12w16b","u_p.p":"v4","D.r":"m16w32b","D.t":"m12w64b","D.p":"v2",'
                   '"res.T":"lds64x8k","res.u_r":"lds64x4k","res.u_t":"lds64x4k","res.u_p":"lds64x4k"}')


_ORACLE_64 = {}     # the oracle's two steps, shared by every tile set


@pytest.mark.timeout(600)
@pytest.mark.parametrize("tiles", ["bench", "bench_lds", "auto"])
def test_convection_steps_64x192x576(oracle_lib, yy, tiles):
    """The benchmark's workload (convection start: conductive T plus seeded
    noise, hydrostatic p, Ra = 1e5, tau = 2e-4, K = 3) on 2x64x192x576:
    two whole steps against the oracle, with two tile sets the autotuner
    picked for the benchmark (memory-read and LDS-staged residuals) and with
    the tiles it picks at this size.  Every field within
    1e-12 relative, the velocities plus the rounding floor of the cancelling
    buoyancy and hydrostatic pressure gradient (as in the small convection
    parity case)."""
    print(f"case: convection 64x192x576 x2 steps, tiles {tiles}", flush=True)
    nr, nt, np_ = 64, 192, 576
    pr, ra, dt, K, nsteps = 1.0, 1e5, 2e-4, 3, 2
    st = I.convection_state(I.Grid(nr, nt, np_), pr, ra, seed=3)
    g = yy.Shell(nr, nt, np_)
    g.set_params(pr=pr, ra=ra, dt=dt, chi=1.0, t_inner=1.0, t_outer=0.0)
    for f in range(9):
        g.set_field(f, 0, st[f])
        if f not in (I.P1, I.P2):
            g.set_field(f, 1, st[f])
    if tiles == "bench":
        g.set_tuning(BENCH_TILES)
    elif tiles == "bench_lds":
        g.set_tuning(BENCH_TILES_LDS)
    else:
        g.autotune()
    for _ in range(nsteps):
        g.step(K)
    got = {f: g.get_field(f).cpu().numpy() for f in range(9)}
    gn = g.norms()
    del g
    if "ref" not in _ORACLE_64:
        o = oracle_lib.Shell(nr, nt, np_)
        o.set_params(pr=pr, ra=ra, tau=dt, chi=1.0, t_inner=1.0, t_outer=0.0)
        for f in range(9):
            o.set_field(f, 0, st[f])
            if f not in (I.P1, I.P2):
                o.set_field(f, 1, st[f])
        for s in range(nsteps):
            o.step(K)
            print(f"  oracle step {s + 1} done", flush=True)
        _ORACLE_64["ref"] = ({f: o.get_field(f) for f in range(9)}, o.norms(K))
    ref, on = _ORACLE_64["ref"]
    M = pr * ra * np.max(np.abs(st[I.T]))
    floor = 16 * np.finfo(float).eps * dt * M * nsteps * K
    for f in range(9):
        b = ref[f]
        err = np.max(np.abs(got[f] - b))
        scale = np.max(np.abs(b))
        print(f"  {I.FIELD_NAMES[f]}: max |gpu - oracle| {err:.2e}, relative {err / scale:.2e}", flush=True)
        lim = 1e-12 * scale + (0.0 if f in (I.T, I.P1, I.P2) else floor)
        assert err <= lim, (I.FIELD_NAMES[f], err, lim)
    assert np.allclose(gn, on, rtol=1e-6, atol=0.0)


def _discrete_conductive(g):
    rf = g.r1 + np.arange(g.nr + 1) * g.dr
    n = g.nr
    A = np.zeros((n, n))
    b = np.zeros(n)
    for i in range(n):
        am, ap = rf[i] ** 2, rf[i + 1] ** 2
        A[i, i] = -(am + ap)
        if i > 0:
            A[i, i - 1] = am
        else:
            A[i, i] -= am
            b[i] -= 2 * am
        if i < n - 1:
            A[i, i + 1] = ap
        else:
            A[i, i] -= ap
    return np.linalg.solve(A, b)


def test_conductive_state_steady_full_size(yy):
    print("case: conductive state 128x384x1152", flush=True)
    nr, nt, np_ = 128, 384, 1152
    g = I.Grid(nr, nt, np_)
    pr, ra = 1.0, 1e5
    prof = _discrete_conductive(g)
    T = torch.tensor(prof, dtype=torch.float64, device="cuda")[None, :, None, None].expand(2, nr, nt, np_).contiguous()
    p = torch.zeros_like(T)
    for i in range(1, nr):
        p[:, i] = p[:, i - 1] + g.dr * pr * ra * 0.5 * (T[:, i - 1] + T[:, i])
    s = yy.Shell(nr, nt, np_)
    s.set_params(pr=pr, ra=ra, dt=2e-4, t_inner=1.0, t_outer=0.0)
    s.autotune()
    for f in range(9):
        z = torch.zeros(s.mac_shape(f), dtype=torch.float64, device="cuda")
        val = T if f == I.T else (p if f in (I.P1, I.P2) else z)
        s.set_field(f, 0, val)
        if f not in (I.P1, I.P2):
            s.set_field(f, 1, val)
    s.step(3)
    assert float((s.get_field(I.T) - T).abs().max()) < 1e-12
    assert float((s.get_field(I.P2) - p).abs().max()) < 1e-12 * float(p.abs().max())
    for f in (I.U1R, I.U1T, I.U1P, I.U2R, I.U2T, I.U2P):
        assert float(s.get_field(f).abs().max()) < 1e-9
    nm = s.norms()
    assert np.all(np.isfinite(nm))


def test_patch_symmetry_full_size(yy):
    print("case: patch symmetry 128x384x1152", flush=True)
    nr, nt, np_ = 128, 384, 1152
    s = yy.Shell(nr, nt, np_)
    s.set_params(pr=1.0, ra=1e5, dt=2e-4, t_inner=1.0, t_outer=0.0)
    s.autotune()
    gen = torch.Generator(device="cuda").manual_seed(11)
    for f in range(9):
        shape = s.mac_shape(f)
        a = 1e-3 * torch.randn(shape[1:], dtype=torch.float64, device="cuda", generator=gen)
        a = a[None].expand(2, *shape[1:]).contiguous()
        s.set_field(f, 0, a)
        if f not in (I.P1, I.P2):
            s.set_field(f, 1, a)
    s.step(3)
    for f in range(9):
        a = s.get_field(f)
        assert torch.equal(a[0], a[1]), I.FIELD_NAMES[f]

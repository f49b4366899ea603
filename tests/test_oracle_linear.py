"""Pins of the oracle's linear algebra against what mathematics fixes:
dense LU on tiny systems, banded LAPACK on long ones, the closed-form
eigen-solution of constant-coefficient lines, the factored operator
assembled densely from Kronecker-structured 1-D factors, and the exact
commutation / positivity statements of the hat operators (Sec. 3.2)."""
import numpy as np
import pytest
import scipy.linalg

from paper_1905_02300_amd import inputs as I


def _rand_tri(rng, n):
    lo = rng.uniform(-1, 1, n)
    up = rng.uniform(-1, 1, n)
    di = 2.5 + rng.uniform(0, 1, n)
    return lo, di, up


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_thomas_matches_dense_lu(oracle_lib, n):
    rng = np.random.default_rng(10 + n)
    lo, di, up = _rand_tri(rng, n)
    rhs = rng.uniform(-1, 1, n)
    A = np.diag(di) + np.diag(lo[1:], -1) + np.diag(up[:-1], 1)
    x = oracle_lib.thomas(lo, di, up, rhs)
    ref = scipy.linalg.lu_solve(scipy.linalg.lu_factor(A), rhs)
    assert np.allclose(x, ref, rtol=1e-13, atol=1e-14)


def test_thomas_matches_solve_banded(oracle_lib):
    n = 1152
    rng = np.random.default_rng(3)
    lo, di, up = _rand_tri(rng, n)
    rhs = rng.uniform(-1, 1, n)
    ab = np.zeros((3, n))
    ab[0, 1:] = up[:-1]
    ab[1] = di
    ab[2, :-1] = lo[1:]
    ref = scipy.linalg.solve_banded((1, 1), ab, rhs)
    x = oracle_lib.thomas(lo, di, up, rhs)
    assert np.max(np.abs(x - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("m", [1, 7, 40])
def test_thomas_toeplitz_eigenvector(oracle_lib, m):
    # (a, b, a) Toeplitz: eigenvectors sin(m pi j/(n+1)), eigenvalues
    # b + 2 a cos(m pi/(n+1)) -- a constant-coefficient phi-line
    n, a, b = 72, -0.37, 1.9
    j = np.arange(1, n + 1)
    v = np.sin(m * np.pi * j / (n + 1))
    lam = b + 2 * a * np.cos(m * np.pi / (n + 1))
    x = oracle_lib.thomas(np.full(n, a), np.full(n, b), np.full(n, a), v)
    assert np.allclose(x, v / lam, rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------------------
def _unknown_mask(sh, field):
    """padded-layout mask of a field's unknowns"""
    nr, nt, np_ = sh.nr, sh.nt, sh.np
    loc = I.LOC[field]
    m = np.zeros(sh.padded_shape(), bool)
    lo = [1 if loc == key else 0 for key in "rtp"]
    hi = [nr, nt, np_]
    m[:, 1 + lo[0]:1 + hi[0], 1 + lo[1]:1 + hi[1], 1 + lo[2]:1 + hi[2]] = True
    return m


def _matrix(sh, field, op, mask):
    """dense matrix of an operator restricted to the unknowns (columns by
    applying it to unit vectors)"""
    idx = np.flatnonzero(mask)
    A = np.zeros((idx.size, idx.size))
    for c, q in enumerate(idx):
        e = np.zeros(sh.padded_shape())
        e.flat[q] = 1.0
        A[:, c] = sh.apply_op(field, op, e).flat[idx]
    return A


def _random_velocity_shell(oracle_lib, seed, nr=3, nt=6, np_=8, tau=0.05):
    sh = oracle_lib.Shell(nr, nt, np_)
    sh.set_params(pr=0.7, ra=3.0, tau=tau, chi=1.3)
    rng = np.random.default_rng(seed)
    for f in range(9):
        for lev in (oracle_lib.LEV_N, oracle_lib.LEV_NM1):
            sh.set_field(f, lev, rng.uniform(-1, 1, sh.padded_shape()), layout=oracle_lib.PADDED)
    sh.extrapolate()
    return sh


SWEEP_ORDER = {I.T: (0, 1, 2), I.U1R: (1, 2, 0), I.U1T: (2, 0, 1), I.U1P: (0, 1, 2)}


@pytest.mark.parametrize("field", [I.T, I.U1R, I.U1T, I.U1P])
def test_three_sweeps_invert_factored_operator(oracle_lib, field):
    """The factor order of eq. Convect_Douglas / r_comp / theta_comp /
    phi_comp: prod_d [I - tau/2 L_d] assembled densely (with advection by a
    random velocity, so the factors do not commute) and solved by LU equals
    the three line sweeps in the field's order."""
    y = oracle_lib
    sh = _random_velocity_shell(y, 7 + field)
    tau = 0.05
    mask = _unknown_mask(sh, field)
    ops = [y.OP_LR, y.OP_LT, y.OP_LP]
    n = mask.sum()
    P = np.eye(n)
    for d in SWEEP_ORDER[field]:
        P = P @ (np.eye(n) - 0.5 * tau * _matrix(sh, field, ops[d], mask))
    rng = np.random.default_rng(1)
    x = np.where(mask, rng.uniform(-1, 1, sh.padded_shape()), 0.0)
    ref = np.linalg.solve(P, x[mask])
    w = x
    for d in SWEEP_ORDER[field]:
        w = sh.sweep(field, d, w)
    assert np.max(np.abs(w[mask] - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.all(w[~mask] == 0.0)


def test_split_operators_reduce_to_paper_heat_operators(oracle_lib):
    """With zero velocity the three T factors are Drr, Dhat_thth, Dhat_phph."""
    y = oracle_lib
    sh = y.Shell(4, 8, 10)
    sh.set_params(tau=0.1)
    sh.extrapolate()
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, sh.padded_shape())
    for a, b in [(y.OP_LR, y.OP_DRR), (y.OP_LT, y.OP_DTT_HAT), (y.OP_LP, y.OP_DPP_HAT)]:
        assert np.array_equal(sh.apply_op(I.T, a, x), sh.apply_op(I.T, b, x))


def test_hat_operators_commute(oracle_lib):
    """Drr, Dhat_thth, Dhat_phph with homogeneous boundary values commute
    exactly (Sec. 3.2); the true D_thth does not commute with Drr."""
    y = oracle_lib
    sh = y.Shell(5, 8, 12)
    rng = np.random.default_rng(4)
    mask = _unknown_mask(sh, I.T)
    x = np.where(mask, rng.uniform(-1, 1, sh.padded_shape()), 0.0)
    A = lambda op, v: sh.apply_op(I.T, op, v)
    scale = np.max(np.abs(A(y.OP_DRR, A(y.OP_DTT_HAT, x))))
    for a, b in [(y.OP_DRR, y.OP_DTT_HAT), (y.OP_DRR, y.OP_DPP_HAT), (y.OP_DTT_HAT, y.OP_DPP_HAT)]:
        d = A(a, A(b, x)) - A(b, A(a, x))
        assert np.max(np.abs(d)) <= 1e-12 * scale
    d = A(y.OP_DRR, A(y.OP_DTT, x)) - A(y.OP_DTT, A(y.OP_DRR, x))
    assert np.max(np.abs(d)) > 1e-3 * scale


def test_hat_operators_over_stabilise(oracle_lib):
    """-(Dhat T, T)_w >= -(D T, T)_w >= 0 for theta and phi with the weight
    w = r^2 sin(theta) (eq. HeatStab2, HeatStab1)."""
    y = oracle_lib
    g = I.Grid(5, 8, 14)
    sh = y.Shell(5, 8, 14)
    mask = _unknown_mask(sh, I.T)
    r, t, _ = g.axes(I.T, padded=True)
    w = (r[:, None, None] ** 2 * np.sin(t)[None, :, None]) * np.ones((1, 1, g.np + 2))
    w = np.broadcast_to(w, sh.padded_shape())
    for seed in range(5):
        x = np.where(mask, np.random.default_rng(seed).standard_normal(sh.padded_shape()), 0.0)
        ip = lambda op: -np.sum(w * sh.apply_op(I.T, op, x) * x)
        assert ip(y.OP_DTT_HAT) >= ip(y.OP_DTT) * (1 - 1e-13) >= 0
        assert ip(y.OP_DPP_HAT) >= ip(y.OP_DPP) * (1 - 1e-13) >= 0
        assert ip(y.OP_DRR) >= 0


def test_sweep_op_line_solves(oracle_lib):
    """The line-solve workload's solves (I - tau/2 Pr D) y = x: with the
    paper's split operators (Drr, Dhat_thth, Dhat_phph) they are the sweeps
    of T at rest (Pr = 1); with the true metric (D_thth, D_phph) they
    invert I - tau/2 Pr D for the operator applied with homogeneous
    neighbours (zero at theta/phi ghosts, reflection at the walls)."""
    y = oracle_lib
    sh = y.Shell(6, 14, 40, 0.5, 1.0)
    tau, pr = 3e-3, 1.3
    sh.set_params(pr=1.0, tau=tau)
    sh.extrapolate()
    rng = np.random.default_rng(8)
    x = rng.uniform(-1, 1, sh.padded_shape())
    m = _unknown_mask(sh, I.T)
    for d, op in enumerate((y.OP_DRR, y.OP_DTT_HAT, y.OP_DPP_HAT)):
        a = sh.sweep_op(op, x)
        b = sh.sweep(I.T, d, x)
        assert np.max(np.abs(a[m] - b[m])) <= 1e-14 * np.max(np.abs(b[m]))
    sh.set_params(pr=pr, tau=tau)
    for op in (y.OP_DRR, y.OP_DTT, y.OP_DPP, y.OP_DTT_HAT, y.OP_DPP_HAT):
        v = sh.sweep_op(op, x)
        back = v - 0.5 * tau * pr * sh.apply_op(I.T, op, v)
        assert np.max(np.abs(back[m] - x[m])) < 1e-12, op


@pytest.mark.parametrize("tau", [0.05, 1.0, 100.0])
def test_heat_split_energy_estimate(oracle_lib, tau):
    """Discrete form of eq. Stability (Sec. 3.2): the split heat scheme
    [I - tau/2 D_rr][I - tau/2 Dhat_thth][I - tau/2 Dhat_phph] dT^{n+1}/tau
    = Lap T* - Lap^ dT^n / 2 on each patch with homogeneous Dirichlet data
    dissipates the energy
      E^n = (-Lap T^n, T^n)_w / 2 + ((-Lap^ dT^n, dT^n)_w - (-Lap dT^n, dT^n)_w) / 4
    (the omega_1, omega_2 terms of the estimate are the last bracket):
    E^{n+1} + tau |dT^{n+1}/tau|_w^2 <= E^n for every tau."""
    y = oracle_lib
    g = I.Grid(6, 12, 36)
    o = y.Shell(g.nr, g.nt, g.np)
    o.set_params(pr=1.0, tau=tau)
    rng = np.random.default_rng(9)
    sh = o.padded_shape()
    mask = np.zeros(sh, bool)
    mask[:, 1:-1, 1:-1, 1:-1] = True

    def rnd():
        a = np.zeros(sh)
        a[mask] = rng.standard_normal(int(mask.sum()))
        return a

    r = g.r1 + (np.arange(-1, g.nr + 1) + 0.5) * g.dr
    th = g.th0 + (np.arange(-1, g.nt + 1) + 0.5) * g.dth
    w = (r[None, :, None, None] ** 2 * np.sin(th)[None, None, :, None] * g.dr * g.dth * g.dph) * mask

    def ip(a, b):
        return float(np.sum(w * a * b))

    def lap(x):
        return sum(o.apply_op(I.T, op, x) for op in (y.OP_DRR, y.OP_DTT, y.OP_DPP))

    def laph(x):
        return sum(o.apply_op(I.T, op, x) for op in (y.OP_DRR, y.OP_DTT_HAT, y.OP_DPP_HAT))

    def energy(tn, tm):
        d = tn - tm
        return 0.5 * ip(-lap(tn), tn) + 0.25 * (ip(-laph(d), d) - ip(-lap(d), d))

    tm = rnd()
    tn = tm + 0.1 * rnd()
    e = energy(tn, tm)
    for _ in range(20):
        rhs = tau * (lap(1.5 * tn - 0.5 * tm) - 0.5 * laph(tn - tm))
        d = o.sweep_op(y.OP_DRR, rhs)
        d = o.sweep_op(y.OP_DTT_HAT, d)
        d = o.sweep_op(y.OP_DPP_HAT, d)
        tp = tn + d * mask
        e1 = energy(tp, tn)
        assert e1 + tau * ip(d / tau, d / tau) <= e * (1 + 1e-12), (tau, e, e1)
        e, tm, tn = e1, tn, tp

"""Pins of the oracle's Robin / stress-free walls for the tangential
velocity (the paper's Introduction: the approach applies to Neumann and
Robin conditions).  Wall condition a u + b R dn(u/r) = g on the cell pair
across a wall of radius R; (0, 1) with g = 0 is the stress-free wall (with
u_r = 0 the tangential stress is proportional to R d(u_t/r)/dr).

Pinned against what the definition and the mechanics fix independently:
the ghost rule satisfies the discrete condition on the cell pair; the
r-line solves with the Robin end rows invert I - tau/2 L_r applied with
that rule; a rigid rotation, an exact steady solution of the equations
with stress-free walls (u = Omega x x, p = Omega^2 (x^2 + y^2)/2), stays
steady up to the second-order truncation error, while no-slip walls drag
it at O(1)."""
import numpy as np
import pytest

from paper_1905_02300_amd import inputs as I


def _rigid_state(g, om):
    st = {}
    for f in range(9):
        out = np.zeros(g.mac_shape(f))
        for patch in range(2):
            X, (er, et, ep) = I.points(g, f, patch)
            x, y, z = X
            U = [-om * y, om * x, 0.0 * z]
            if f in (I.P1, I.P2):
                out[patch] = 0.5 * om * om * (x * x + y * y)
            elif f != I.T:
                e = {"r": er, "t": et, "p": ep}[I.LOC[f]]
                out[patch] = U[0] * e[0] + U[1] * e[1] + U[2] * e[2]
        st[f] = out
    return st


def _rigid_drift(y, m, free):
    g = I.Grid(3 * m, 12 * m, 36 * m)
    sh = y.Shell(g.nr, g.nt, g.np, g.r1, g.r2)
    sh.set_params(pr=1.0, ra=0.0, tau=2e-3, chi=1.0)
    if free:
        sh.set_u_bc(0, 0.0, 1.0)
        sh.set_u_bc(1, 0.0, 1.0)
    st = _rigid_state(g, 0.5)
    for f in range(9):
        sh.set_field(f, y.LEV_N, st[f])
        sh.set_field(f, y.LEV_NM1, st[f])
    for _ in range(5):
        sh.step(3)
    return {f: np.max(np.abs(sh.get_field(f) - st[f])) for f in (I.U2R, I.U2T, I.U2P)}


@pytest.mark.slow
def test_rigid_rotation_steady_under_stress_free_walls(oracle_lib):
    d1 = _rigid_drift(oracle_lib, 1, True)
    d2 = _rigid_drift(oracle_lib, 2, True)
    n1 = _rigid_drift(oracle_lib, 1, False)
    for f in (I.U2T, I.U2P):
        assert d1[f] / d2[f] > 3.0, (I.FIELD_NAMES[f], d1[f], d2[f])   # second order
        assert n1[f] > 1000 * d1[f], (I.FIELD_NAMES[f], n1[f], d1[f])   # no-slip drags


def test_ghost_rule_satisfies_the_wall_condition(oracle_lib):
    """After a fill, each tangential ghost and its interior neighbour
    satisfy a (u_g + u_i)/2 + b R (u_g/r_g - u_i/r_i)/dr = g at both walls
    (stress-free on R1; a Robin condition with wall data on R2)."""
    y = oracle_lib
    g = I.Grid(4, 12, 36)
    sh = y.Shell(g.nr, g.nt, g.np)
    sh.set_params(pr=1.0, ra=0.0, tau=1e-3)
    bc = [(0.0, 1.0), (0.7, 0.4)]
    for w, (a, b) in enumerate(bc):
        sh.set_u_bc(w, a, b)
    rng = np.random.default_rng(5)
    for f in range(9):
        sh.set_field(f, y.LEV_N, rng.uniform(-1, 1, g.mac_shape(f)))
    data = {}
    for f in (I.U1T, I.U1P):
        data[f] = rng.uniform(-1, 1, (2, g.nt + 2, g.np + 2))
        sh.set_wall(f, y.LEV_N, 1, data[f])
    sh.fill(y.LEV_N)
    for f in (I.U1T, I.U1P, I.U2T, I.U2P):
        u = sh.get_field(f, y.LEV_N, layout=y.PADDED)
        for w, (a, b) in enumerate(bc):
            R = g.r1 if w == 0 else g.r2
            ig, ii = (0, 1) if w == 0 else (g.nr + 1, g.nr)
            rg = R - 0.5 * g.dr if w == 0 else R + 0.5 * g.dr
            ri = R + 0.5 * g.dr if w == 0 else R - 0.5 * g.dr
            ug, ui = u[:, ig], u[:, ii]
            lhs = a * 0.5 * (ug + ui) + b * R * (ug / rg - ui / ri) / g.dr
            gw = np.zeros_like(lhs) if w == 0 else data[I.U1T if I.LOC[f] == "t" else I.U1P]
            jt = slice(1 + (1 if I.LOC[f] == "t" else 0), g.nt + 1)
            kp = slice(1 + (1 if I.LOC[f] == "p" else 0), g.np + 1)
            assert np.max(np.abs((lhs - gw)[:, jt, kp])) < 1e-12, (I.FIELD_NAMES[f], w)


def test_r_sweep_end_rows_invert_the_robin_operator(oracle_lib):
    """The r-line solves of u_theta and u_phi with the Robin end rows invert
    I - tau/2 L_r applied with the same homogeneous ghost rule."""
    y = oracle_lib
    g = I.Grid(6, 12, 36)
    sh = y.Shell(g.nr, g.nt, g.np)
    tau = 2e-2
    sh.set_params(pr=0.7, ra=0.0, tau=tau)
    sh.set_u_bc(0, 0.0, 1.0)
    sh.set_u_bc(1, 0.3, 0.8)
    rng = np.random.default_rng(8)
    for f in range(9):
        sh.set_field(f, y.LEV_N, 0.1 * rng.uniform(-1, 1, g.mac_shape(f)))
        sh.set_field(f, y.LEV_NM1, 0.1 * rng.uniform(-1, 1, g.mac_shape(f)))
    sh.extrapolate()
    x = rng.uniform(-1, 1, sh.padded_shape())
    for f in (I.U2T, I.U2P):
        yv = sh.sweep(f, 0, x)
        back = yv - 0.5 * tau * sh.apply_op(f, y.OP_LR, yv)
        m = np.zeros(sh.padded_shape(), bool)
        lo_t = 2 if I.LOC[f] == "t" else 1
        lo_p = 2 if I.LOC[f] == "p" else 1
        m[:, 1:-1, lo_t:-1, lo_p:-1] = True
        assert np.max(np.abs(back[m] - x[m])) < 1e-12, I.FIELD_NAMES[f]

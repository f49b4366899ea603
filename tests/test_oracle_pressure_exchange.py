"""Pins of the oracle's pressure exchange (Algorithm step 7 of Sec. 4: after
each pressure update the pressure near a patch's boundary is interpolated
from the other patch).

In this MAC layout no momentum stencil reads a pressure ghost, so the
exchanged values are placed in the patch's own outermost nring cells,
which then take the other patch's pressure instead of the AC update.  The
pins below check that against what is fixed independently of the oracle's
arithmetic: exact reproduction of constants by the interpolation, the
fourth-order accuracy of cubic Lagrange interpolation of a smooth field at
the ring cells' own centres, an exact discrete steady state, the geometric
limit of the ring, and the paper's remark that the exchange speeds up the
Schwarz iteration."""
import math

import numpy as np
import pytest

from paper_1905_02300_amd import inputs as I
from tests.test_oracle_scheme import _discrete_conductive


def _quiet_shell(y, g, tau, chi=1.0, nring=1, mode=0):
    sh = y.Shell(g.nr, g.nt, g.np, g.r1, g.r2, g.delta)
    sh.set_params(pr=1.0, ra=0.0, tau=tau, chi=chi)
    sh.set_mode(mode)
    sh.set_pressure_exchange(nring)
    return sh


def _ring_mask(g, nring):
    j = np.arange(g.nt)[:, None]
    k = np.arange(g.np)[None, :]
    m = (j < nring) | (j >= g.nt - nring) | (k < nring) | (k >= g.np - nring)
    return np.broadcast_to(m[None, None], (2, g.nr, g.nt, g.np))


@pytest.mark.parametrize("nring", [1, 2])
def test_constant_per_patch_is_exchanged_exactly(oracle_lib, nring):
    """A pressure that is constant on each patch (c0 on Yin, c1 on Yang),
    at rest and without buoyancy: in the first Schwarz iteration u1 stays 0,
    the AC update leaves every other cell at its own constant, and the ring
    cells take the other patch's constant (cubic Lagrange weights sum to
    one).  In the additive mode both patches read the values their pressure
    update left, so a ring cell whose donor window reaches the other
    patch's ring still sees only that patch's constant."""
    y = oracle_lib
    g = I.Grid(4, 24, 72, 0.5, 1.0, 0.12)
    c = (0.75, -1.25)
    p = np.zeros(g.mac_shape(I.P1))
    p[0], p[1] = c
    sh = _quiet_shell(y, g, 1e-2, nring=nring)
    for lev in (y.LEV_N, y.LEV_NM1):
        sh.set_field(I.P1, lev, p)
        sh.set_field(I.P2, lev, p)
    sh.step(1)
    p1 = sh.get_field(I.P1)
    ring = _ring_mask(g, nring)
    for patch in range(2):
        own, other = c[patch], c[1 - patch]
        assert np.max(np.abs(p1[patch][~ring[patch]] - own)) == 0.0
        assert np.max(np.abs(p1[patch][ring[patch]] - other)) < 1e-14
    # the velocity of system 1 never saw a pressure jump
    for f in (I.U1R, I.U1T, I.U1P):
        assert np.max(np.abs(sh.get_field(f))) == 0.0


def _smooth_p(g, patch_points):
    x, y_, z = patch_points
    return np.sin(1.3 * x + 0.4) * np.cos(0.9 * y_) + 0.5 * z * z


def _ring_interp_error(y, m):
    """Max error at the ring cells after one step of a pressure-only state
    whose AC update is negligible (tau = 1e-12): the ring holds the other
    patch's pressure interpolated at the ring centres."""
    g = I.Grid(2, 12 * m, 36 * m, 0.5, 1.0, 0.2)
    p = np.zeros(g.mac_shape(I.P1))
    for patch in range(2):
        X, _ = I.points(g, I.P1, patch)
        p[patch] = _smooth_p(g, X)
    sh = _quiet_shell(y, g, 1e-12, nring=1)
    for lev in (y.LEV_N, y.LEV_NM1):
        sh.set_field(I.P1, lev, p)
    sh.step(1)
    ring = _ring_mask(g, 1)
    err = np.abs(sh.get_field(I.P1) - p)
    return err[ring].max(), err[~ring].max(), np.abs(p).max()


def test_ring_takes_interpolated_pressure_at_its_centres(oracle_lib):
    """With a smooth global pressure, the ring values equal the field at
    the ring cells' own centres up to the cubic interpolation error, which
    falls at fourth order (a target placed at the wrong position, or read
    at the wrong radial index, would leave an O(h) or O(1) error)."""
    e1, o1, scale = _ring_interp_error(oracle_lib, 1)
    e2, o2, _ = _ring_interp_error(oracle_lib, 2)
    assert o1 < 1e-9 and o2 < 1e-9            # other cells: AC update ~ tau
    assert e1 < 1e-3 * scale
    assert math.log2(e1 / e2) > 3.5, (e1, e2)


@pytest.mark.parametrize("mode", [0, 1])
def test_conductive_state_steady_with_exchange(oracle_lib, mode):
    """The discrete conductive state (u = 0, T the discrete conductive
    profile, p its hydrostatic balance) depends on r only, and the exchange
    interpolates at the same radial index, so it stays exactly steady with
    the exchange on, and the tolerance loop stops after one iteration."""
    y = oracle_lib
    g = I.Grid(6, 24, 72, 0.5, 1.0, 0.15)
    pr, ra = 1.0, 1e4
    prof = _discrete_conductive(g, 1.0, 0.0)
    T = np.broadcast_to(prof[None, :, None, None], g.mac_shape(I.T)).copy()
    p = np.zeros_like(T)
    for i in range(1, g.nr):
        p[:, i] = p[:, i - 1] + g.dr * pr * ra * 0.5 * (T[:, i - 1] + T[:, i])
    sh = y.Shell(g.nr, g.nt, g.np, g.r1, g.r2, g.delta)
    sh.set_params(pr=pr, ra=ra, tau=1e-2, t_inner=1.0, t_outer=0.0)
    sh.set_mode(mode)
    sh.set_pressure_exchange(2)
    st = {f: np.zeros(g.mac_shape(f)) for f in range(9)}
    st[I.T], st[I.P1], st[I.P2] = T, p, p
    for f in range(9):
        sh.set_field(f, y.LEV_N, st[f])
        sh.set_field(f, y.LEV_NM1, st[f])
    for _ in range(2):
        sh.step(2)
    assert sh.step_tol(10, 1e-9) == 1
    assert np.max(np.abs(sh.get_field(I.T) - T)) < 1e-12
    for f in (I.P1, I.P2):
        assert np.max(np.abs(sh.get_field(f) - p)) < 1e-12 * np.max(np.abs(p))
    for f in (I.U1R, I.U1T, I.U1P, I.U2R, I.U2T, I.U2P):
        assert np.max(np.abs(sh.get_field(f))) < 1e-11


def test_ring_must_lie_inside_the_other_patch(oracle_lib):
    """Ring cells are interpolation targets, so they must lie inside the
    other patch's span of centres (as every ghost must).  The one-cell
    overlap leaves room for one ring; a wide overlap for more; half a patch
    is never allowed."""
    y = oracle_lib
    sh = y.Shell(10, 46, 96)
    sh.set_pressure_exchange(1)
    with pytest.raises(ValueError):
        sh.set_pressure_exchange(2)
    sh.set_pressure_exchange(0)
    wide = y.Shell(10, 46, 96, 1.0, 2.0, 0.1)
    wide.set_pressure_exchange(3)
    with pytest.raises(ValueError):
        wide.set_pressure_exchange(23)
    with pytest.raises(ValueError):
        wide.set_pressure_exchange(-1)


_WALL_FIELDS = (I.T, I.U1R, I.U1T, I.U1P)


def _paper_counts(y, g, tau, nsteps, chi, nring):
    sh = y.Shell(g.nr, g.nt, g.np, g.r1, g.r2, g.delta)
    sh.set_params(pr=1.0, ra=1.0, tau=tau, chi=chi)
    sh.set_pressure_exchange(nring)

    def walls(level, t):
        for f in _WALL_FIELDS:
            w = I.wall_values(g, t, f, "paper")
            sh.set_wall(f, level, 0, w[0])
            sh.set_wall(f, level, 1, w[1])

    for lev, t in ((y.LEV_N, 0.0), (y.LEV_NM1, -tau)):
        st = I.mms_state(g, t, kind="paper")
        for f in range(9):
            sh.set_field(f, lev, st[f])
        walls(lev, t)
    ks = []
    for s in range(nsteps):
        for f in _WALL_FIELDS:
            sh.set_forcing(f, I.mms_forcing(g, (s + 0.5) * tau, f, 1.0, 1.0, kind="paper"))
        walls(y.LEV_K, (s + 1) * tau)
        ks.append(sh.step_tol(30, 1e-6))
    err = np.max(np.abs(sh.get_field(I.U2R) - I.mms_fields(g, nsteps * tau, I.U2R, kind="paper")))
    return ks, err


def test_exchange_speeds_up_schwarz(oracle_lib):
    """The paper's remark after the Algorithm of Sec. 4: skipping step 7
    can seriously slow the Schwarz iteration.  On its manufactured solution
    (eq. Exact) with the stop test of Sec. 5.1 (tolerance 1e-6), the
    exchange cuts the iteration count of every step, while the solution
    error is unchanged."""
    y = oracle_lib
    g = I.Grid(6, 24, 72, 1.0, 2.0)
    k0, e0 = _paper_counts(y, g, 5e-3, 3, 1.0, 0)
    k1, e1 = _paper_counts(y, g, 5e-3, 3, 1.0, 1)
    assert all(a < b for a, b in zip(k1, k0)), (k0, k1)
    assert abs(e1 - e0) < 0.05 * e0, (e0, e1)

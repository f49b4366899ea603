"""Pins of the oracle's Yin-Yang geometry and overlap interpolation
(Sec. 2 transforms; Sec. 4 Lagrange interpolation of boundary data)."""
import math

import numpy as np
import pytest

from paper_1905_02300_amd import inputs as I


def test_involution_twice_is_identity(oracle_lib):
    rng = np.random.default_rng(0)
    for _ in range(200):
        th = rng.uniform(0.1, math.pi - 0.1)
        ph = rng.uniform(-math.pi + 0.01, math.pi - 0.01)
        a, b = oracle_lib.involution(th, ph)
        c, d = oracle_lib.involution(a, b)
        assert abs(c - th) < 1e-12 and abs(d - ph) < 1e-12


def test_involution_maps_same_cartesian_point(oracle_lib):
    # Yin (th, ph) and Yang (th2, ph2) name one point: x = r sin cos ... and
    # x = -r sin th2 cos ph2, y = r cos th2, z = r sin th2 sin ph2 (Sec. 2)
    rng = np.random.default_rng(1)
    for _ in range(50):
        th, ph = rng.uniform(0.2, 2.9), rng.uniform(-3.0, 3.0)
        a, b = oracle_lib.involution(th, ph)
        yin = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        yang = np.array([-math.sin(a) * math.cos(b), math.cos(a), math.sin(a) * math.sin(b)])
        assert np.allclose(yin, yang, atol=1e-13)


def _basis(th, ph, patch):
    st, ct, sp, cp = math.sin(th), math.cos(th), math.sin(ph), math.cos(ph)
    et = np.array([ct * cp, ct * sp, -st])
    ep = np.array([-sp, cp, 0.0])
    if patch == 1:
        et, ep = np.array([-et[0], et[2], et[1]]), np.array([-ep[0], ep[2], ep[1]])
    return et, ep


def test_rotation_is_orthogonal_and_projects(oracle_lib):
    rng = np.random.default_rng(2)
    for _ in range(50):
        th, ph = rng.uniform(0.6, 2.5), rng.uniform(-2.4, 2.4)
        M = oracle_lib.rotation(th, ph)
        assert np.allclose(M @ M.T, np.eye(2), atol=1e-13)
        a, b = oracle_lib.involution(th, ph)
        V = rng.standard_normal(3)
        et, ep = _basis(th, ph, 0)
        et2, ep2 = _basis(a, b, 1)
        # the tangential part of V is the same vector in both bases
        v_yang = np.array([V @ et2, V @ ep2])
        assert np.allclose(M @ v_yang, [V @ et, V @ ep], atol=1e-13)


def _target_mask(g, field):
    """padded-layout mask of the interpolation targets of a field"""
    m = np.zeros((2, g.nr + 2, g.nt + 2, g.np + 2), bool)
    loc = I.LOC[field]
    nr, nt, np_ = g.nr, g.nt, g.np
    ir = slice(2, nr + 1) if loc == "r" else slice(1, nr + 1)
    if loc in ("c", "r"):
        m[:, ir, [0, nt + 1], 1:np_ + 1] = True
        m[:, ir, 1:nt + 1, [0, np_ + 1]] = True
    elif loc == "t":
        m[:, ir, [1, nt + 1], 1:np_ + 1] = True
        m[:, ir, 2:nt + 1, [0, np_ + 1]] = True
    else:
        m[:, ir, 1:nt + 1, [1, np_ + 1]] = True
        m[:, ir, [0, nt + 1], 2:np_ + 1] = True
    return m


def _fill_error(oracle_lib, nt, fields):
    g = I.Grid(3, nt, 3 * nt)
    sh = oracle_lib.Shell(3, nt, 3 * nt)
    st = I.mms_state(g, 1.0)
    for f in range(9):
        sh.set_field(f, oracle_lib.LEV_N, st[f])
    sh.fill(oracle_lib.LEV_N)
    ex = I.mms_state(g, 1.0, padded=True)
    err = {}
    for f in fields:
        m = _target_mask(g, f)
        got = sh.get_field(f, oracle_lib.LEV_N, layout=oracle_lib.PADDED)
        err[f] = np.max(np.abs(got[m] - ex[f][m])) / np.max(np.abs(ex[f][m]))
    return err


def test_interpolation_fourth_order(oracle_lib):
    """Tensor cubic Lagrange interpolation converges at O(h^4) for scalar
    and (rotated) vector fields."""
    fields = [I.T, I.P1, I.U1R, I.U1T, I.U1P]
    e1 = _fill_error(oracle_lib, 16, fields)
    e2 = _fill_error(oracle_lib, 32, fields)
    for f in fields:
        rate = math.log2(e1[f] / e2[f])
        assert rate > 3.5, (I.FIELD_NAMES[f], e1[f], e2[f])
        assert e2[f] < 1e-4


def test_interpolation_reproduces_constants(oracle_lib):
    g = I.Grid(3, 12, 36)
    sh = oracle_lib.Shell(3, 12, 36)
    sh.set_field(I.T, oracle_lib.LEV_N, np.full(g.mac_shape(I.T), 2.5))
    sh.set_params(t_inner=2.5, t_outer=2.5)
    sh.fill(oracle_lib.LEV_N)
    got = sh.get_field(I.T, oracle_lib.LEV_N, layout=oracle_lib.PADDED)
    m = _target_mask(g, I.T)
    assert np.max(np.abs(got[m] - 2.5)) < 1e-14


def test_wall_rules(oracle_lib):
    g = I.Grid(4, 8, 24)
    sh = oracle_lib.Shell(4, 8, 24)
    sh.set_params(t_inner=1.0, t_outer=0.25)
    rng = np.random.default_rng(5)
    for f in range(9):
        sh.set_field(f, oracle_lib.LEV_N, rng.standard_normal(g.mac_shape(f)))
    sh.fill(oracle_lib.LEV_N)
    T = sh.get_field(I.T, oracle_lib.LEV_N, layout=oracle_lib.PADDED)
    assert np.allclose(T[:, 0], 2 * 1.0 - T[:, 1], rtol=0, atol=1e-15)
    assert np.allclose(T[:, -1], 2 * 0.25 - T[:, -2], rtol=0, atol=1e-15)
    for f in (I.U1R, I.U2R):
        u = sh.get_field(f, oracle_lib.LEV_N, layout=oracle_lib.PADDED)
        assert np.all(u[:, 1] == 0.0) and np.all(u[:, g.nr + 1] == 0.0)
    for f in (I.U1T, I.U1P, I.U2T, I.U2P):
        u = sh.get_field(f, oracle_lib.LEV_N, layout=oracle_lib.PADDED)
        assert np.array_equal(u[:, 0], -u[:, 1]) and np.array_equal(u[:, -1], -u[:, -2])


def test_geometry_rejects_extrapolating_overlap(oracle_lib):
    # a negative overlap (gap between the patches) leaves targets outside
    # every donor window
    with pytest.raises(ValueError):
        oracle_lib.Shell(4, 12, 36, delta=1e-9)


def _nominal(th, ph):
    """inside a patch's nominal region (overlap delta = 0, Sec. 2)"""
    return (th >= math.pi / 4) & (th <= 3 * math.pi / 4) & (ph >= -3 * math.pi / 4) & (ph <= 3 * math.pi / 4)


def test_nominal_patches_cover_the_sphere(oracle_lib):
    """Every point of S^2 lies in Yin's nominal region or, mapped by the
    oracle's involution, in Yang's (Sec. 2); the part covered twice has the
    area 2 (3 pi / 2) sqrt(2) - 4 pi of the two regions' excess over the
    sphere (each nominal region has area (3 pi / 2)(cos pi/4 - cos 3pi/4))."""
    rng = np.random.default_rng(7)
    n = 40000
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    th = np.arccos(np.clip(v[:, 2], -1, 1))
    ph = np.arctan2(v[:, 1], v[:, 0])
    yin = _nominal(th, ph)
    yang = np.array([_nominal(*oracle_lib.involution(a, b)) for a, b in zip(th, ph)])
    assert np.all(yin | yang)
    both = np.mean(yin & yang)
    expect = (3 * math.sqrt(2) * math.pi - 4 * math.pi) / (4 * math.pi)
    assert abs(both - expect) < 4 * math.sqrt(expect * (1 - expect) / n), (both, expect)


def test_partitioned_area_converges_to_the_sphere(oracle_lib):
    """Summing both patches' cell areas sin(theta) dtheta dphi with weight 1
    where a cell centre is in its own nominal region only, 1/2 where it is
    in both (the oracle's involution decides the other's), gives the
    sphere's 4 pi; the sharp weights leave an O(h) boundary error, which
    falls under refinement."""
    errs = []
    for m in (1, 2, 4, 8):
        g = I.Grid(2, 12 * m, 36 * m)
        _, t, p = g.axes(I.T)
        TT, PP = np.meshgrid(t, p, indexing="ij")
        own = _nominal(TT, PP)
        oth = np.zeros_like(own)
        for a in range(TT.shape[0]):
            for b in range(TT.shape[1]):
                oth[a, b] = _nominal(*oracle_lib.involution(TT[a, b], PP[a, b]))
        w = np.where(own & oth, 0.5, np.where(own, 1.0, 0.0))
        area = 2 * np.sum(w * np.sin(TT)) * g.dth * g.dph
        errs.append(abs(area / (4 * math.pi) - 1))
        assert errs[-1] < 2.0 * g.dth, (m, errs[-1])
    assert errs[-1] < errs[0] / 8, errs

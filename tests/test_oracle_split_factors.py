"""Independent pin of which implicit term sits in which split factor.

The split operators L_{psi,r}, L_{psi,theta}, L_{psi,phi} of T (eq.
Convect_Douglas) and of u_r, u_theta, u_phi (eq. r_comp, theta_comp,
phi_comp, with every grad-div block carrying 1/(2 chi), the viscosity Pr,
the nonlinear metric terms linearised with the advecting velocity and the
hat metrics of Sec. 3.2 in the theta/phi diffusion) are assembled here as
dense matrices on a small two-patch grid from one-dimensional difference
matrices written for this test: flux-form second differences, centred first
differences, and the grad-div blocks as products of a gradient and a
divergence matrix (D_cc = G_c Div_c), combined by Kronecker products with
diagonal metric and advecting-velocity factors.  Nothing is taken from the
oracle except its apply_op, which is compared against them.

Moving any term from one factor to another leaves the sum Lhat (and so
every consistency pin of the scheme) unchanged but changes these matrices;
the last test plants such a move in a copy of the oracle and checks that
this pin catches it.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1905_02300_amd import inputs as I

NR, NT, NP = 3, 6, 8
PR, CHI, TAU = 0.7, 1.3, 0.05


class Geom:
    def __init__(self, nr=NR, nt=NT, np_=NP, r1=0.5, r2=1.0):
        self.nr, self.nt, self.np = nr, nt, np_
        self.r1 = r1
        self.delta = np.pi / (2 * (nt - 2))
        self.dr = (r2 - r1) / nr
        self.th0 = np.pi / 4 - self.delta
        self.ph0 = -3 * np.pi / 4 - self.delta
        self.dth = (np.pi / 2 + 2 * self.delta) / nt
        self.dph = (1.5 * np.pi + 2 * self.delta) / np_
        self.th1 = np.pi / 4 - self.delta

    def n(self, d):
        return (self.nr, self.nt, self.np)[d]

    def h(self, d):
        return (self.dr, self.dth, self.dph)[d]

    def x0(self, d):
        return (self.r1, self.th0, self.ph0)[d]

    def centres(self, d):
        return self.x0(d) + (np.arange(self.n(d)) + 0.5) * self.h(d)

    def faces(self, d):
        return self.x0(d) + np.arange(self.n(d) + 1) * self.h(d)

    def unknowns(self, loc, d):
        """logical indices and positions of the unknowns of a location along d"""
        if loc == "rtp"[d]:
            idx = np.arange(1, self.n(d))
            return idx, self.faces(d)[idx]
        idx = np.arange(self.n(d))
        return idx, self.centres(d)[idx]


def _tri_matrix(lo, di, up, reflect):
    """rows (lo, di, up) acting on consecutive unknowns; neighbours outside
    the set are zero, or (reflect) the negative of the end unknown"""
    n = len(di)
    A = np.diag(np.asarray(di, float).copy())
    for m in range(n):
        if m > 0:
            A[m, m - 1] += lo[m]
        elif reflect:
            A[m, m] -= lo[m]
        if m < n - 1:
            A[m, m + 1] += up[m]
        elif reflect:
            A[m, m] -= up[m]
    return A


def second_diff(x, xlo, xhi, w, s, h, reflect):
    """(1/(s h^2)) [w(xhi)(psi_{m+1} - psi_m) - w(xlo)(psi_m - psi_{m-1})]"""
    a, b = w(xlo) / (s * h * h), w(xhi) / (s * h * h)
    return _tri_matrix(a, -(a + b), b, reflect)


def centred_diff(n, h, reflect):
    return _tri_matrix(np.full(n, -1 / (2 * h)), np.zeros(n), np.full(n, 1 / (2 * h)), reflect)


def grad_div(g, d, scale_div=None):
    """1-D G_d Div_d on the face unknowns of direction d (faces 1..N-1; the
    boundary faces are zero): Div maps faces to centres, G centres to faces"""
    n = g.n(d)
    fc = g.faces(d)
    cc = g.centres(d)
    Div = np.zeros((n, n - 1))          # centres x interior faces
    for c in range(n):
        for f in (c, c + 1):
            if 1 <= f <= n - 1:
                sgn = 1.0 if f == c + 1 else -1.0
                if d == 0:
                    Div[c, f - 1] += sgn * fc[f] ** 2 / (cc[c] ** 2 * g.dr)
                elif d == 1:
                    Div[c, f - 1] += sgn * np.sin(fc[f]) / (np.sin(cc[c]) * g.dth)
                else:
                    Div[c, f - 1] += sgn / g.dph
    G = np.zeros((n - 1, n))           # interior faces x centres
    for f in range(1, n):
        G[f - 1, f] += 1.0 / g.h(d)
        G[f - 1, f - 1] -= 1.0 / g.h(d)
    return G @ Div


def kron3(A, d, g, loc):
    """a 1-D matrix along d as an operator on the 3-D unknowns of loc"""
    mats = []
    for e in range(3):
        n = len(g.unknowns(loc, e)[0])
        mats.append(A if e == d else np.eye(n))
    return np.kron(np.kron(mats[0], mats[1]), mats[2])


def point_values(g, loc):
    """(r, theta) at every unknown of loc, flattened in (i, j, k) order"""
    (_, r), (_, t), (_, p) = (g.unknowns(loc, d) for d in range(3))
    R, T, _ = np.meshgrid(r, t, p, indexing="ij")
    return R.ravel(), T.ravel()


def advecting(g, ustar, loc):
    """a = u2* averaged from its faces to the unknowns of loc: the mean of
    the nearest stored points (2 or 4), per component, flattened"""
    (ii, _), (jj, _), (kk, _) = (g.unknowns(loc, d) for d in range(3))
    out = []
    for c in range(3):
        offs = []
        for d in range(3):
            cface, lface = d == c, loc == "rtp"[d]
            offs.append((0, 1) if cface and not lface else ((-1, 0) if lface and not cface else (0,)))
        acc = 0.0
        cnt = 0
        for a in offs[0]:
            for b in offs[1]:
                for e in offs[2]:
                    acc = acc + ustar[c][np.ix_(ii + a + 1, jj + b + 1, kk + e + 1)]
                    cnt += 1
        out.append((acc / cnt).ravel())
    return out


def split_operators(g, loc, a):
    """the three factors L_r, L_theta, L_phi of one unknown (one patch)"""
    nu = 1.0 if loc == "c" else PR
    ic = 1.0 / (2 * CHI)
    r, th = point_values(g, loc)
    ar, at, ap = a
    D = lambda v: np.diag(v)
    (ri, rx), (ti, tx), (pi_, px) = (g.unknowns(loc, d) for d in range(3))
    # flux-form second differences along each direction
    if loc == "r":
        d2r = second_diff(rx, g.centres(0)[ri - 1], g.centres(0)[ri], lambda x: x ** 2, rx ** 2, g.dr, False)
    else:
        d2r = second_diff(rx, g.faces(0)[ri], g.faces(0)[ri + 1], lambda x: x ** 2, rx ** 2, g.dr, True)
    if loc == "t":
        d2t = second_diff(tx, g.centres(1)[ti - 1], g.centres(1)[ti], np.sin, g.r1 ** 2 * np.sin(tx), g.dth, False)
    else:
        d2t = second_diff(tx, g.faces(1)[ti], g.faces(1)[ti + 1], np.sin, g.r1 ** 2 * np.sin(tx), g.dth, False)
    shat = g.r1 ** 2 * np.sin(g.th1) ** 2
    d2p = second_diff(px, px, px, lambda x: np.ones_like(x), np.full(len(px), shat), g.dph, False)
    c1r = centred_diff(len(rx), g.dr, loc != "r")
    c1t = centred_diff(len(tx), g.dth, False)
    c1p = centred_diff(len(px), g.dph, False)
    Lr = nu * kron3(d2r, 0, g, loc) - D(ar) @ kron3(c1r, 0, g, loc)
    Lt = nu * kron3(d2t, 1, g, loc) - D(at / r) @ kron3(c1t, 1, g, loc)
    Lp = nu * kron3(d2p, 2, g, loc) - D(ap / (r * np.sin(th))) @ kron3(c1p, 2, g, loc)
    if loc == "r":
        # Pr[-2/r^2 + (2/r^3) d_r(r^2 .)] + D11/(2 chi)
        extra = -np.diag(2 / rx ** 2) + np.diag(2 / rx ** 3) @ c1r @ np.diag(rx ** 2)
        Lr = Lr + nu * kron3(extra, 0, g, loc) + ic * kron3(grad_div(g, 0), 0, g, loc)
    elif loc == "t":
        # Pr[-1/(r^2 sin^2) + (2 cos/(r^2 sin^2)) d_th(sin .)] - a_r/r + D22/(2 chi)
        Lt = Lt + nu * (D(-1 / (r * np.sin(th)) ** 2)
                        + D(2 * np.cos(th) / (r * np.sin(th)) ** 2) @ kron3(c1t @ np.diag(np.sin(tx)), 1, g, loc))
        Lt = Lt - D(ar / r) + ic * D(1 / r ** 2) @ kron3(grad_div(g, 1), 1, g, loc)
    elif loc == "p":
        # -Pr/(r^2 sin^2) - (a_r + a_th cot)/r + D33/(2 chi)
        Lp = Lp - nu * D(1 / (r * np.sin(th)) ** 2) - D((ar + at * np.cos(th) / np.sin(th)) / r)
        Lp = Lp + ic * D(1 / (r * np.sin(th)) ** 2) @ kron3(grad_div(g, 2), 2, g, loc)
    return Lr, Lt, Lp


def _random_shell(y, seed, lib=None):
    sh = y.Shell(NR, NT, NP, _lib=lib)
    sh.set_params(pr=PR, ra=3.0, tau=TAU, chi=CHI)
    rng = np.random.default_rng(seed)
    levels = {}
    for f in range(9):
        for lev in (y.LEV_N, y.LEV_NM1):
            a = rng.uniform(-1, 1, sh.padded_shape())
            levels[(f, lev)] = a
            sh.set_field(f, lev, a, layout=y.PADDED)
    sh.extrapolate()
    ustar = [1.5 * levels[(f, y.LEV_N)] - 0.5 * levels[(f, y.LEV_NM1)] for f in (I.U2R, I.U2T, I.U2P)]
    return sh, ustar


def _oracle_matrix(sh, field, op, mask):
    idx = np.flatnonzero(mask)
    A = np.zeros((idx.size, idx.size))
    for c, q in enumerate(idx):
        e = np.zeros(sh.padded_shape())
        e.flat[q] = 1.0
        A[:, c] = sh.apply_op(field, op, e).flat[idx]
    return A


def _mask(g, loc):
    m = np.zeros((2, g.nr + 2, g.nt + 2, g.np + 2), bool)
    (ri, _), (ti, _), (pi_, _) = (g.unknowns(loc, d) for d in range(3))
    m[np.ix_([0, 1], ri + 1, ti + 1, pi_ + 1)] = True
    return m


def _compare(y, sh, ustar, field):
    g = Geom()
    loc = I.LOC[field]
    mask = _mask(g, loc)
    n1 = mask[0].sum()
    worst = {}
    for d, op in enumerate((y.OP_LR, y.OP_LT, y.OP_LP)):
        A = _oracle_matrix(sh, field, op, mask)
        for p in range(2):
            a = advecting(g, [u[p] for u in ustar], loc)
            B = split_operators(g, loc, a)[d]
            blk = A[p * n1:(p + 1) * n1, p * n1:(p + 1) * n1]
            worst[(d, p)] = np.max(np.abs(blk - B)) / np.max(np.abs(B))
        # no coupling between the patches
        assert np.all(A[:n1, n1:] == 0) and np.all(A[n1:, :n1] == 0)
    return worst


@pytest.mark.parametrize("field", [I.T, I.U2R, I.U2T, I.U2P])
def test_split_factors_match_independent_assembly(oracle_lib, field):
    sh, ustar = _random_shell(oracle_lib, 40 + field)
    worst = _compare(oracle_lib, sh, ustar, field)
    assert max(worst.values()) <= 1e-13, worst


def test_system_one_uses_the_same_factors(oracle_lib):
    """u1 and u2 share one matrix (Sec. 3.3): the factors of u1 equal
    those of u2, advected by u2*."""
    sh, ustar = _random_shell(oracle_lib, 77)
    for f1, f2 in ((I.U1R, I.U2R), (I.U1T, I.U2T), (I.U1P, I.U2P)):
        mask = _mask(Geom(), I.LOC[f1])
        for op in (oracle_lib.OP_LR, oracle_lib.OP_LT, oracle_lib.OP_LP):
            assert np.array_equal(_oracle_matrix(sh, f1, op, mask), _oracle_matrix(sh, f2, op, mask))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_pin_catches_a_term_moved_between_factors(oracle_lib, tmp_path):
    """Plant a mistake in a copy of the oracle: move the implicit -a_r u/r
    term of u_theta from its theta factor to its phi factor.  The sum of the
    factors is unchanged (so the residual is identical), but this pin fails."""
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = open(os.path.join(here, "oracle", "yyo.c")).read()
    a = "            /* -a_r u / r */\n            t.di += -a[0] / r;\n"
    b = "        t = tri_add(z, op_dpp_hat(h), nu);\n"
    assert src.count(a) == 1 and src.count(b) == 1
    src = src.replace(a, "").replace(b, b + "        if (loc == FT) t.di += -a[0] / r;\n")
    (tmp_path / "yyo.h").write_text(open(os.path.join(here, "oracle", "yyo.h")).read())
    (tmp_path / "yyo.c").write_text(src)
    so = str(tmp_path / "libyyo_planted.so")
    subprocess.run(["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fPIC", "-shared", "-o", so,
                    str(tmp_path / "yyo.c"), "-lm"], check=True)
    bad = oracle_lib.load_library(so)
    sh_bad, ustar = _random_shell(oracle_lib, 40 + I.U2T, lib=bad)
    sh_ok, _ = _random_shell(oracle_lib, 40 + I.U2T)
    # the residual (which holds only the sum of the factors) is the same
    assert np.allclose(sh_bad.residual(I.U2T), sh_ok.residual(I.U2T), rtol=0, atol=1e-12)
    worst = _compare(oracle_lib, sh_bad, ustar, I.U2T)
    assert max(worst.values()) > 1e-3, worst
